"""Benchmark: 3D VGF solves/s at N=256^3, FP32 and FP64, with the HBM roofline.

Workload (synthetic, seeded): beam_3d_256 -- 3D grid of 256^3 points on
[-1,1]^3, one unit anisotropic Gaussian sigma = (0.05, 0.05, 0.3) whose
centroid is drawn uniformly in the ball of radius 0.05 (seed 0). One step is
one VGF solve on a fixed plan: pruned R2C along axis 2, C2C along axis 1, the
fused axis-0 pass (forward FFT, spectral multiply by the kernel spectrum and
by -i k_0 times it, two inverse FFTs), inverse C2C along axis 1 (phi's
spectrum also yields E_1) and C2R along axis 2 (phi's spectrum also yields
E_2), producing phi and E (the one-time FP64 kernel precompute runs
at plan creation and is not part of a step). rho is resident in HBM before
the timed region.

Printed JSON line (one, rank 0):
  value        FP32 solves/s (whole job, one GPU)
  fp64         the same for FP64 solves
  roofline     for the dominant kernel (the pass with the largest mean
               duration): its algorithmic bytes per launch divided by its mean
               duration measured with HIP events recorded by the library on
               the solve stream during the timed region, against the MI355X's
               8 TB/s HBM peak
  pass_model   the whole solve against the same peak, using one HBM read and
               write per axis pass of the pruned arrays
  cpu_baseline the FP64 CPU oracle's 2N FFT path on the same input, timed on
               the host cores for one solve (its values also give the stated
               rel-L2 of the GPU results)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "3D VGF solves/s at N=256^3 FP32 vs FP64 + HBM GB/s, at stated rel-L2 error"


def pass_model_bytes(n, prec_bytes, nf=4):
    """The fixed pass model: one HBM read and write per axis pass of the pruned
    arrays with one inverse per field on every axis (the kernel spectrum
    octant read once). This is the reference accounting for the whole solve;
    any fusion that moves fewer bytes raises the fraction honestly."""
    N0, N1, N2 = n
    P1, H = 2 * N1, N2 + 1
    rb, cb = prec_bytes, 2 * prec_bytes
    x1 = N0 * N1 * H * cb
    x2 = N0 * P1 * H * cb
    spec = (N0 + 1) * (N1 + 1) * (N2 + 1) * rb
    real = N0 * N1 * N2 * rb
    return (real + x1) + (x1 + x2) + (x2 + spec + nf * x2) + nf * (x2 + x1) + nf * (x1 + real)


def kernel_bytes(n, prec_bytes):
    """Algorithmic HBM bytes of each pass as this library structures the solve
    (phi + E): the axis-0 pass writes the spectra of phi and E_0 only, the
    axis-1 inverse writes phi, E_1 (from phi) and E_0, and the last pass
    writes phi, E_2 (from phi), E_1 and E_0."""
    N0, N1, N2 = n
    P1, H = 2 * N1, N2 + 1
    rb, cb = prec_bytes, 2 * prec_bytes
    x1 = N0 * N1 * H * cb
    x2 = N0 * P1 * H * cb
    spec = (N0 + 1) * (N1 + 1) * (N2 + 1) * rb
    real = N0 * N1 * N2 * rb
    return {
        "r2c": real + x1,
        "c2c_fwd": x1 + x2,
        "fused_axis0": x2 + spec + 2 * x2,
        "c2c_inv": 2 * x2 + 3 * x1,
        "c2r": 3 * x1 + 4 * real,
    }


def run_precision(vgf, torch, ch, rho64, precision, steps, warmup):
    dt = torch.float32 if precision == "f32" else torch.float64
    plan = vgf.Plan(ch.n, ch.h, method="vgf", precision=precision)
    rho = torch.from_numpy(rho64).to(device="cuda", dtype=dt)
    phi = torch.empty(ch.n, dtype=dt, device="cuda")
    E = torch.empty((3,) + ch.n, dtype=dt, device="cuda")
    for _ in range(warmup):
        plan.solve(rho, phi, E)
    torch.cuda.synchronize()
    plan.profile_begin(steps)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        plan.solve(rho, phi, E)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    passes, nsolves = plan.profile_end()
    wall_ms = (t1 - t0) * 1e3 / steps
    ev_ms = ev0.elapsed_time(ev1) / steps
    out = {"phi": phi.double().cpu().numpy(), "E": E.double().cpu().numpy()}
    L = plan.L
    plan.close()
    del rho, phi, E
    torch.cuda.empty_cache()
    return {"wall_ms": wall_ms, "event_ms": ev_ms, "passes": passes, "nsolves": nsolves,
            "out": out, "L": L}


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))


def cpu_baseline(ch, rho64, L, results):
    """FP64 oracle, 2N FFT path, one full solve (phi + E) on the host cores."""
    import oracle as orc
    w = orc.vgf_kernel(ch.n, ch.h, L)  # plan-time precompute: not timed
    t0 = time.perf_counter()
    phi_o, E_o = orc.solve_fft2n(ch.n, ch.h, w, rho64)
    t = time.perf_counter() - t0
    acc = {}
    for prec, r in results.items():
        acc[prec] = {"phi": rel_l2(r["out"]["phi"], phi_o),
                     "E": rel_l2(r["out"]["E"], E_o)}
    base = {"value": 1.0 / t, "unit": "solves/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": "one full 256^3 FP64 solve (phi + E) by the oracle's naive 2N FFT path, "
                      "including its FFT of the kernel; kernel precompute excluded; %.1f s" % t}
    return base, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the solves, copy 256 MiB device-to-device once (a plain copy "
                         "kernel of known size, to scale HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solve path runs on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_08531_amd import vgf, workloads
    torch.cuda.set_device(0)
    ch = workloads.beam_3d_256(seed=args.seed)
    rho64 = ch.rho()

    results = {}
    for prec in ("f32", "f64"):
        results[prec] = run_precision(vgf, torch, ch, rho64, prec, args.steps, args.warmup)
        print("[bench] %s: %.3f ms/solve (events %.3f), passes %s" % (
            prec, results[prec]["wall_ms"], results[prec]["event_ms"],
            {k: round(v, 4) for k, v in results[prec]["passes"].items()}), file=sys.stderr, flush=True)

    f32 = results["f32"]
    f64 = results["f64"]
    kb32 = kernel_bytes(ch.n, 4)
    kb64 = kernel_bytes(ch.n, 8)
    pm32 = pass_model_bytes(ch.n, 4)
    pm64 = pass_model_bytes(ch.n, 8)
    # dominant kernel: the pass with the largest mean duration
    dom = max(f32["passes"], key=lambda k: f32["passes"][k])
    dom_ms = f32["passes"][dom]
    achieved = kb32[dom] / (dom_ms * 1e-3) / 1e9
    dom64 = max(f64["passes"], key=lambda k: f64["passes"][k])
    ach64 = kb64[dom64] / (f64["passes"][dom64] * 1e-3) / 1e9

    line = {
        "metric": METRIC,
        "value": 1e3 / f32["wall_ms"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["wall_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "beam_3d_256", "grid": list(ch.n), "domain": "[-1,1]^3",
                   "method": "vgf", "outputs": "phi+E", "sigma": [0.05, 0.05, 0.3],
                   "seed": args.seed, "L": f32["L"], "parallelism": "single GPU"},
        "fp64": {"value": 1e3 / f64["wall_ms"], "unit": "solves/s", "ms_per_step": f64["wall_ms"],
                 "dtype": "f64"},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": kb32[dom], "mean_launch_ms": dom_ms,
                     "fp64": {"kernel": dom64, "achieved": ach64, "mean_launch_ms": f64["passes"][dom64],
                              "algorithmic_bytes_per_launch": kb64[dom64],
                              "frac": ach64 / HBM_PEAK_GBS}},
        "pass_model": {"bytes_per_solve_f32": pm32, "bytes_per_solve_f64": pm64,
                       "frac_f32": pm32 / (f32["wall_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "frac_f64": pm64 / (f64["wall_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "passes": {"bytes_f32": kb32, "bytes_f64": kb64,
                   "moved_bytes_per_solve_f32": sum(kb32.values()),
                   "moved_bytes_per_solve_f64": sum(kb64.values()),
                   "ms_f32": f32["passes"], "ms_f64": f64["passes"],
                   "gbs_f32": {k: kb32[k] / (f32["passes"][k] * 1e-3) / 1e9 for k in kb32},
                   "gbs_f64": {k: kb64[k] / (f64["passes"][k] * 1e-3) / 1e9 for k in kb64}},
        "accuracy": {"f32_vs_f64_gpu": {"phi": rel_l2(f32["out"]["phi"], f64["out"]["phi"]),
                                        "E": rel_l2(f32["out"]["E"], f64["out"]["E"])}},
    }
    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = src.numel() * 4
        del src, dst
    if not args.no_cpu_baseline:
        base, acc = cpu_baseline(ch, rho64, f64["L"], results)
        line["cpu_baseline"] = base
        line["accuracy"]["vs_oracle"] = acc
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
