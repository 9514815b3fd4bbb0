"""Benchmark: 3D VGF solves/s at N=256^3, FP32 and FP64, with the HBM roofline.

Workload (synthetic, seeded): beam_3d_256 -- 3D grid of 256^3 points on
[-1,1]^3, one unit anisotropic Gaussian sigma = (0.05, 0.05, 0.3) whose
centroid is drawn uniformly in the ball of radius 0.05 (seed 0). One step is
one VGF solve on a fixed plan: pruned R2C along axis 0, C2C along axis 1,
the multiply pass along the contiguous axis 2 (forward FFT, multiply by the
kernel spectrum and by -i k_2 times it, two inverse FFTs), inverse C2C along
axis 1 (phi's spectrum also yields E_1) and C2R along axis 0 (phi's spectrum
also yields E_0), producing phi and E (the one-time FP64 kernel precompute
runs at plan creation and is not part of a step). rho is resident in HBM
before the timed region.

Printed JSON line (one, rank 0):
  value        FP32 solves/s (whole job, one GPU)
  fp64         the same for FP64 solves
  roofline     for the dominant kernel (the launch with the largest mean
               duration): its algorithmic bytes per launch divided by its mean
               duration measured with HIP events recorded by the library after
               every launch on the solve stream during the timed region,
               against the MI355X's 8 TB/s HBM peak
  pass_model   the whole solve against the same peak, using one HBM read and
               write per axis pass of the pruned arrays
  cpu_baseline the FP64 CPU oracle's 2N FFT path on the same input, timed on
               the host cores for one solve (its values also give the stated
               rel-L2 of the GPU results)
  batch        batch_3d_mixed (64 FP32 grids of uneven N): one solve per
               entry vs one launch per pass and grid size vs the same as one
               replayed hipGraph, before and after autotuning the groups' tile
               schedules, in ms per batch and solves/s
  other_workloads  gaussian_3d_32 and mixture_2d_512 (FP64, VGF and HE)
               solves/s, launched pass by pass and replayed as one graph,
               diff_3d_128 (8 FP32 forward solves + 8 adjoints, one by one
               and batched) ms, and
               variants_256: the beam_3d_256 input through every method,
               field mode and layout, and a rectangular grid, FP32, phi + E
The 256^3 plans are autotuned (tile schedule per pass, bit-identical results)
before the warm-up; the chosen schedules are reported.

roofline.traffic is the dominant kernel's HBM bytes per launch from two
rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE), each scaled by what the
same counter reads for a plain 256 MiB device-to-device copy in the same run
(--copy-calibration). `--digest-counters FETCH_CSV FETCH_OUT WRITE_CSV WRITE_OUT` turns the two
counter files (with the two profiled runs' outputs, which must carry the
current source hash) into profiles/vgf_solve_beam_3d_256_traffic.{json,md},
stamped with a hash of the library code (comments and whitespace ignored); a
bench run reports the traffic only while the code still hashes the same, else null. `--digest-trace STATS_CSV` turns a
`rocprofv3 --kernel-trace --stats` summary into
profiles/vgf_solve_beam_3d_256_kernel_trace.md.
"""
import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "3D VGF solves/s at N=256^3 FP32 vs FP64 + HBM GB/s, at stated rel-L2 error"
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_JSON = os.path.join(PROFILES, "vgf_solve_beam_3d_256_traffic.json")
TRACE_MD = os.path.join(PROFILES, "vgf_solve_beam_3d_256_kernel_trace.md")
CALIB_BYTES = 256 * 1024 * 1024
def _code_only(text):
    """C/C++ source without comments and with whitespace collapsed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(root=None):
    """sha256 over the library's code (comments and whitespace ignored) and
    its build script: counter data taken from other code no longer describe
    the kernels that run."""
    h = hashlib.sha256()
    pkg = os.path.join(root or ROOT, "paper_2103_08531_amd")
    csrc = os.path.join(pkg, "csrc")
    for name in sorted(os.listdir(csrc)):
        if not os.path.isfile(os.path.join(csrc, name)) or name.endswith(".pyc"):
            continue  # caches a test run may leave beside the sources
        with open(os.path.join(csrc, name)) as f:
            h.update(name.encode() + b"\0" + _code_only(f.read()).encode())
    with open(os.path.join(pkg, "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def _short_name(kname):
    name = kname.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
    return name.replace("vgf::", "")


def _read_counter(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _bench_line(path):
    """The JSON line a bench run printed (its output may hold other lines)."""
    for ln in reversed(open(path).read().splitlines()):
        if ln.startswith("{"):
            return json.loads(ln)
    raise SystemExit("no bench output line in %s" % path)


def digest_counters(fetch_csv, fetch_out, write_csv, write_out):
    """Per-kernel HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by the factor that maps the counter's reading for
    the calibration copy (the last copyBuffer dispatch of the run) to its
    known 256 MiB. Both profiled bench runs must have run these sources."""
    src = kernel_source_hash()
    for path in (fetch_out, write_out):
        if _bench_line(path).get("source_hash") != src:
            raise SystemExit("%s was measured on other sources than these" % path)
    out = {"source_hash": src, "calibration_bytes": CALIB_BYTES, "kernels": {},
           "schedule": _bench_line(fetch_out).get("schedule")}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _read_counter(path, counter)
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not copies:
            raise SystemExit("no calibration copy in %s (run bench.py with --copy-calibration)" % path)
        kib = float(copies[-1]["Counter_Value"])
        factor = CALIB_BYTES / 1024.0 / kib
        out[counter.lower() + "_calibration"] = {"copy_kib": kib, "factor": factor}
        for r in rows:
            if "vgf::" not in r["Kernel_Name"]:
                continue
            name = _short_name(r["Kernel_Name"])
            per.setdefault(name, {}).setdefault(counter, []).append(float(r["Counter_Value"]))
    ff = out["fetch_size_calibration"]["factor"]
    fw = out["write_size_calibration"]["factor"]
    for name, d in per.items():
        if "FETCH_SIZE" not in d or "WRITE_SIZE" not in d:
            continue
        fk = sum(d["FETCH_SIZE"]) / len(d["FETCH_SIZE"])
        wk = sum(d["WRITE_SIZE"]) / len(d["WRITE_SIZE"])
        out["kernels"][name] = {"dispatches": len(d["FETCH_SIZE"]), "fetch_kib": fk, "write_kib": wk,
                                "read_bytes": fk * 1024 * ff, "write_bytes": wk * 1024 * fw,
                                "traffic_bytes": fk * 1024 * ff + wk * 1024 * fw}
    return out


def load_traffic():
    """The committed counter digest, if it still describes these sources."""
    try:
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return d if d.get("source_hash") == kernel_source_hash() else None


PASS_INDEX = {"r2c": 0, "c2c_fwd": 1, "fused": 2, "c2c_inv": 3, "c2r": 4}


def write_traffic_profile(fetch_csv, fetch_out, write_csv, write_out, command):
    d = digest_counters(fetch_csv, fetch_out, write_csv, write_out)
    d["command"] = command
    os.makedirs(PROFILES, exist_ok=True)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    # algorithmic bytes per launch of every kernel a solve launches, both tile variants
    alg_of = {}
    for prec in ("f32", "f64"):
        for pname, pattern, nbytes in launch_model((256, 256, 256), 4 if prec == "f32" else 8):
            for v in (0, 1):
                alg_of[launch_kernel_name(pattern, prec, [3 * v] * 5, pname)] = nbytes
    md = [ "# HBM traffic per launch: VGF solve kernels, beam_3d_256 (3D 256^3, phi+E), FP32 and FP64", "",
          "Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), one rocprofv3 run each, averaged over "
          "the dispatches of each kernel. Each is scaled by the factor that maps its reading for a plain "
          "256 MiB device-to-device copy in the same run to 256 MiB (FETCH_SIZE counts each 128-byte read "
          "request as 64 bytes, so its factor is about 2; WRITE_SIZE reads true).", "",
          "Commands:", "", "```", command, "```", "",
          "| counter | copy reads (KiB) | factor |", "|---|---|---|",
          "| FETCH_SIZE | %.1f | %.4f |" % (d["fetch_size_calibration"]["copy_kib"],
                                         d["fetch_size_calibration"]["factor"]),
          "| WRITE_SIZE | %.1f | %.4f |" % (d["write_size_calibration"]["copy_kib"],
                                         d["write_size_calibration"]["factor"]), "",
          "| kernel | launches | read MB | write MB | traffic MB | algorithmic MB | traffic / algorithmic |",
          "|---|---|---|---|---|---|---|"]
    for name in sorted(d["kernels"]):
        v = d["kernels"][name]
        alg = alg_of.get(name)
        md.append("| %s | %d | %.1f | %.1f | %.1f | %s | %s |" % (
            name, v["dispatches"], v["read_bytes"] / 1e6, v["write_bytes"] / 1e6, v["traffic_bytes"] / 1e6,
            "%.1f" % (alg / 1e6) if alg else "-", "%.3f" % (v["traffic_bytes"] / alg) if alg else "-"))
    md += ["", "The run autotunes each plan's tile schedule first, so both variants of the strided kernels "
           "(last template argument) appear above. Per solve and pass, with the launches of one solve and "
           "the schedule the timed solves used (%s):" % json.dumps(d["schedule"]), "",
           "| pass | precision | traffic MB | algorithmic MB | traffic / algorithmic |", "|---|---|---|---|---|"]
    for prec, label in (("f32", "FP32"), ("f64", "FP64")):
        sched = (d["schedule"] or {}).get(prec)
        if not sched:
            continue
        tot, alg = {}, {}
        model = launch_model((256, 256, 256), 4 if prec == "f32" else 8)
        for (pname, pattern, nbytes), idx in zip(model, launch_indices(model)):
            v = d["kernels"].get(launch_kernel_name(pattern, prec, sched, pname, idx))
            if v is None:
                continue
            tot[pname] = tot.get(pname, 0.0) + v["traffic_bytes"]
            alg[pname] = alg.get(pname, 0) + nbytes
        for pname in tot:
            md.append("| %s | %s | %.1f | %.1f | %.3f |" % (pname, label, tot[pname] / 1e6, alg[pname] / 1e6,
                                                           tot[pname] / alg[pname]))
    md += ["", "Source hash (sha256 of the library code, comments and whitespace ignored, and its build script, that the counters describe): `%s`"
           % d["source_hash"], ""]
    with open(TRAFFIC_JSON[:-5] + ".md", "w") as f:
        f.write("\n".join(md))
    print(TRAFFIC_JSON)


COUNTERS_MD = os.path.join(PROFILES, "vgf_solve_beam_3d_256_counters.md")
# one rocprofv3 --pmc run per set (at most 8 SQ counters per run)
PMC_SETS = (("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CU_CYCLES", "SQ_WAVE_CYCLES"),
            ("SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS",
             "SQ_WAIT_INST_ANY"))


def digest_pmc(csvs, outs):
    """Per-kernel means over the dispatches of the SQ counters of rocprofv3
    --pmc runs of the bench (one counter set per run). Every profiled run
    must have run these sources."""
    src = kernel_source_hash()
    for path in outs:
        if _bench_line(path).get("source_hash") != src:
            raise SystemExit("%s was measured on other sources than these" % path)
    per = {}
    for path in csvs:
        for r in csv.DictReader(open(path)):
            if "vgf::" not in r["Kernel_Name"]:
                continue
            d = per.setdefault(_short_name(r["Kernel_Name"]), {"vgpr": r["VGPR_Count"], "lds": r["LDS_Block_Size"]})
            d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = {}
    for name, d in per.items():
        out[name] = {"vgpr_field": d.pop("vgpr"), "lds_bytes": d.pop("lds")}
        for c, v in d.items():
            out[name][c] = sum(v) / len(v)
            out[name]["dispatches"] = len(v)
    return src, out


def write_counters_profile(csvs, outs, command):
    src, per = digest_pmc(csvs, outs)
    nlines = 257 * 512  # multiply-pass lines of a 256^3 solve (H0 x P1)
    md = ["# SQ counters per kernel: VGF solve, beam_3d_256 (3D 256^3, phi+E), FP32 and FP64", "",
          "rocprofv3 --pmc runs of the bench, one counter set per run, means over each kernel's dispatches "
          "(the run autotunes the tile schedules, so both variants of the strided kernels appear). Counts are "
          "wave-level instructions summed over the chip; SQ_ACTIVE_INST_* and SQ_LDS_BANK_CONFLICT are "
          "cycles. Per-line figures divide by the 131 584 lines of the multiply pass.", "",
          "Commands:", "", "```", command, "```", "",
          "| kernel | VALU instr | VALU instr per line | LDS instr | LDS active | bank-conflict cycles | "
          "conflict / LDS active | wait LDS / wait any | busy CU cycles | VGPR field |",
          "|---|---|---|---|---|---|---|---|---|---|"]
    for name in sorted(per):
        v = per[name]
        g = lambda c: v.get(c, float("nan"))
        q = lambda a, b: g(a) / g(b) if g(b) else float("nan")
        per_line = "%.0f" % (g("SQ_INSTS_VALU") / nlines) if "fused_c" in name else "-"
        md.append("| %s | %.3g | %s | %.3g | %.3g | %.3g | %.2f | %.2f | %.3g | %s |" % (
            name, g("SQ_INSTS_VALU"), per_line, g("SQ_INSTS_LDS"), g("SQ_ACTIVE_INST_LDS"),
            g("SQ_LDS_BANK_CONFLICT"), q("SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS"),
            q("SQ_WAIT_INST_LDS", "SQ_WAIT_INST_ANY"), g("SQ_BUSY_CU_CYCLES"), v["vgpr_field"]))
    md += ["", "VGPR field: rocprofv3's VGPR_Count column, which counts registers in units of two here "
           "(a kernel the compiler reports at 80 VGPRs shows 40).", "",
           "Source hash (sha256 of the library code, comments and whitespace ignored, and its build script, "
           "that the counters describe): `%s`" % src, ""]
    with open(COUNTERS_MD, "w") as f:
        f.write("\n".join(md))
    print(COUNTERS_MD)


WORKLOAD_TITLES = {
    "batch_3d_mixed": "64 FP32 grids of N in {32, 48, 64, 96, 128}, phi + E: one solve per grid, grouped "
                      "launches, one replayed graph, and the graph after autotuning",
    "diff_3d_128": "8 FP32 right-hand sides at 128^3, E only: forward solves and adjoints one by one, then "
                   "one batched solve (graph) and one batched adjoint",
}


def write_workload_trace_profile(trace_csv, name, bench_json, command):
    """Per-kernel durations from a rocprofv3 --kernel-trace run of
    `bench.py --only-workload NAME`, next to the times that run printed."""
    rows = list(csv.DictReader(open(trace_csv)))
    agg = {}
    for r in rows:
        k = _short_name(r["Kernel_Name"])
        if k.startswith("at::") or "elementwise" in k or "distribution" in k:
            k = "torch " + k[:40]
        agg.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(d) for d in agg.values())
    md = ["# Kernel trace: %s" % name, "", WORKLOAD_TITLES.get(name, name) + ".", "",
          "rocprofv3 kernel trace of the whole run (plans, autotuning, warm-up and timed repetitions of "
          "every mode). Durations in microseconds.", "", "Command:", "", "```", command, "```", "",
          "| kernel | calls | mean us | total ms | share |", "|---|---|---|---|---|"]
    for k, d in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        md.append("| %s | %d | %.1f | %.3f | %.1f%% |" % (k, len(d), sum(d) / len(d), sum(d) / 1e3,
                                                         100.0 * sum(d) / total))
    if bench_json:
        line = json.loads(open(bench_json).read().strip().splitlines()[-1])
        md += ["", "Times the same (profiled) run measured:", "", "```", json.dumps(line, indent=1), "```"]
    path = os.path.join(PROFILES, "%s_kernel_trace.md" % name)
    with open(path, "w") as f:
        f.write("\n".join(md) + "\n")
    print(path)


def write_trace_profile(trace_csv, bench_json, command):
    """Per-kernel durations from a rocprofv3 --kernel-trace run, next to the
    per-pass means the same bench run measured live with HIP events."""
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    agg = {}
    for r in rows:
        name = _short_name(r["Kernel_Name"])
        if name.startswith("at::") or "elementwise" in name:
            name = "torch " + name[:40]
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = agg.setdefault(name, {"d": [], "wg": r["Workgroup_Size_X"], "grid": r["Grid_Size_X"],
                                  "lds": r["LDS_Block_Size"], "vgpr": r["VGPR_Count"],
                                  "agpr": r["Accum_VGPR_Count"], "scratch": r["Scratch_Size"]})
        a["d"].append(dur)
    md = ["# Kernel trace: VGF solve, beam_3d_256 (3D 256^3, phi+E), FP32 and FP64", "",
          "rocprofv3 kernel trace of one bench run (plan precompute, warm-up and timed solves of both "
          "precisions). Durations in microseconds.", "", "Command:", "", "```", command, "```", "",
          "| kernel | calls | mean us | min us | max us | total ms | grid | wg | LDS B | VGPR | AGPR | scratch |",
          "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, a in sorted(agg.items(), key=lambda kv: -sum(kv[1]["d"])):
        d = a["d"]
        md.append("| %s | %d | %.1f | %.1f | %.1f | %.3f | %s | %s | %s | %s | %s | %s |" % (
            name, len(d), sum(d) / len(d), min(d), max(d), sum(d) / 1e3, a["grid"], a["wg"], a["lds"],
            a["vgpr"], a["agpr"], a["scratch"]))
    if bench_json:
        line = json.loads(open(bench_json).read().strip().splitlines()[-1])
        md += ["", "Per-pass mean durations the same run measured live (HIP events on the solve stream, "
               "timed solves only), in microseconds:", "",
               "| pass | FP32 | FP64 |", "|---|---|---|"]
        for k in line["passes"]["ms_f32"]:
            md.append("| %s | %.1f | %.1f |" % (k, 1e3 * line["passes"]["ms_f32"][k],
                                               1e3 * line["passes"]["ms_f64"][k]))
        if "launches_ms_f32" in line["passes"]:
            md += ["", "Per-launch mean durations of the same timed solves, with the kernel each launch "
                   "runs under the tuned schedule (%s), in microseconds:" % json.dumps(line.get("schedule")), "",
                   "live: HIP events of the bench; trace: the same kernel's last dispatches in this trace "
                   "(the timed solves run last in each precision).", "",
                   "| launch | pass | FP32 kernel | FP32 live | FP32 trace | FP64 kernel | FP64 live | FP64 trace |",
                   "|---|---|---|---|---|---|---|---|"]
            model = launch_model(tuple(line["config"]["grid"]), 4)
            steps = int(line["steps"])

            idxs = launch_indices(model)

            def timed_mean(kname):
                prec = "f32" if "float" in kname else "f64"
                per_solve = sum(1 for (pn, pt, _), ix in zip(model, idxs)
                                if launch_kernel_name(pt, prec, line["schedule"][prec], pn, ix) == kname)
                d = agg.get(kname, {"d": []})["d"][-steps * per_solve:]
                return sum(d) / len(d) if d else float("nan")

            for i, ((pname, pat, _), a, b) in enumerate(zip(model, line["passes"]["launches_ms_f32"],
                                                            line["passes"]["launches_ms_f64"])):
                k32 = launch_kernel_name(pat, "f32", line["schedule"]["f32"], pname, idxs[i])
                k64 = launch_kernel_name(pat, "f64", line["schedule"]["f64"], pname, idxs[i])
                md.append("| %d | %s | %s | %.1f | %.1f | %s | %.1f | %.1f |" % (
                    i, pname, k32, 1e3 * a[1], timed_mean(k32), k64, 1e3 * b[1], timed_mean(k64)))
    md.append("")
    with open(TRACE_MD, "w") as f:
        f.write("\n".join(md))
    print(TRACE_MD)


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


def launch_model(n, prec_bytes):
    """The launches of one 3D solve (phi + E) in the default layout, in order:
    (pass, kernel name pattern at P = 2N, algorithmic HBM bytes). The
    multiply pass runs along the last axis and writes the spectra of phi and
    E_2; the axis-1 inverse writes phi and E_1 (from phi) and E_2 in one
    launch; the axis-0 complex-to-real pass writes phi and E_0 (from phi),
    E_1 and E_2 in one launch. Arrays: X1 = [N0+1][N1][N2],
    X2 = [N0+1][2 N1][N2] complex."""
    N0, N1, N2 = n
    P = 2 * N2
    rb, cb = prec_bytes, 2 * prec_bytes
    x1 = (N0 + 1) * N1 * N2 * cb
    x2 = (N0 + 1) * 2 * N1 * N2 * cb
    spec = (N0 + 1) * (N1 + 1) * (N2 + 1) * rb
    real = N0 * N1 * N2 * rb
    return [
        ("r2c", "k_r2c_s<{t}, %d, 1, {v}>" % P, real + x1),
        ("c2c_fwd", "k_c2c_fwd<{t}, %d, 1, {v}>" % P, x1 + x2),
        ("fused", "k_fused_c{fc}<{t}, %d, {fv}>" % P, x2 + spec + 2 * x2),
        ("c2c_inv", "k_c2c_inv<{t}, %d, 3, {v}>" % P, 2 * x2 + 3 * x1),
        ("c2r", "k_c2r_s<{t}, %d, 4, {v}>" % P, 3 * x1 + 4 * real),
    ]


def kernel_bytes(n, prec_bytes):
    """Algorithmic HBM bytes of each pass (sum over its launches)."""
    out = {}
    for pname, _, b in launch_model(n, prec_bytes):
        out[pname] = out.get(pname, 0) + b
    return out


# vector FMA rate without packed FP32 instructions (which this library does
# not use): 256 CUs x 64 lanes x 2 flops x 2.4 GHz, in FP32 and in FP64
VECTOR_PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}


def multiply_pass_flops(n):
    """Conventional flop count of one multiply-pass launch (3D phi + E): per
    line of the last axis, a forward and two inverse P-point complex
    transforms at 5 P log2 P each, plus 2 P for the kernel multiply and 2 P
    for -i k_last."""
    N0, N1, N2 = n
    P = 2 * N2
    lines = (N0 + 1) * 2 * N1
    return lines * (3 * 5 * P * np.log2(P) + 4 * P)


def launch_indices(model):
    """Index of each launch among the launches of its pass (0 = the first)."""
    seen, out = {}, []
    for pname, _, _ in model:
        out.append(seen.get(pname, 0))
        seen[pname] = out[-1] + 1
    return out


def wave_lanes(P):
    """Lanes that share one line in the contiguous multiply pass (a power of
    two up to P/8 and 64)."""
    nq = 1
    while nq * 2 <= P // 8 and nq * 2 <= 64:
        nq *= 2
    return nq


def launch_kernel_name(name_pattern, prec, schedule, pass_name, idx=0):
    """Concrete kernel name of a pass's launch number idx under a schedule.
    Strided passes: bit 0 of the pass's value is the tile width of its first
    launch, bit 1 that of the later ones. The contiguous multiply pass takes
    its value whole: bit 0 halves the lanes per line where four such tiles
    fit 64 KiB of LDS; one line per wavefront (64 lanes) runs k_fused_c1 with
    the field count (2) as template argument, otherwise k_fused_c with the
    lane variant."""
    t = "float" if prec == "f32" else "double"
    value = schedule[PASS_INDEX[pass_name]]
    if pass_name == "fused":
        P = int(re.search(r", (\d+), \{fv\}", name_pattern).group(1))
        nq = wave_lanes(P)
        cb = 8 if prec == "f32" else 16
        half = (value & 1) and nq > 1 and 4 * (128 // nq) * (P + P // 8) * cb <= 65536
        if nq // (2 if half else 1) == 64:
            return name_pattern.format(fc="1", t=t, fv=2)
        return name_pattern.format(fc="", t=t, fv=1 if half else 0)
    v = (value >> (1 if idx > 0 else 0)) & 1
    return name_pattern.format(t=t, v=v)


def run_precision(vgf, torch, ch, rho64, precision, steps, warmup, tune=True):
    dt = torch.float32 if precision == "f32" else torch.float64
    torch.cuda.synchronize()
    t_plan = time.perf_counter()
    plan = vgf.Plan(ch.n, ch.h, method="vgf", precision=precision)  # FP64 precompute, synchronous
    plan_ms = 1e3 * (time.perf_counter() - t_plan)
    rho = torch.from_numpy(rho64).to(device="cuda", dtype=dt)
    phi = torch.empty(ch.n, dtype=dt, device="cuda")
    E = torch.empty((3,) + ch.n, dtype=dt, device="cuda")
    schedule = plan.autotune(rho, phi, E, reps=5) if tune else plan.schedule
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
    passes, launches, nsolves = plan.profile_end()
    wall_ms = (t1 - t0) * 1e3 / steps
    ev_ms = ev0.elapsed_time(ev1) / steps
    out = {"phi": phi.double().cpu().numpy(), "E": E.double().cpu().numpy()}
    L = plan.L
    plan.close()
    del rho, phi, E
    torch.cuda.empty_cache()
    return {"wall_ms": wall_ms, "event_ms": ev_ms, "passes": passes, "launches": launches,
            "nsolves": nsolves, "out": out, "L": L, "schedule": list(schedule), "plan_ms": plan_ms}


def run_batch(vgf, torch, workloads, steps, warmup, seed):
    """batch_3d_mixed: 64 FP32 right-hand sides of uneven N in
    {32, 48, 64, 96, 128}, phi + E, three ways on the same plans and buffers:
    one vgf_solve per entry (its passes launched one entry at a time), one
    launch per pass and per grid size (vgf_batch, direct launches), and the
    same launches replayed as one captured hipGraph."""
    charges = workloads.batch_3d_mixed(seed=seed, count=64)
    plans = {}
    for ch in charges:
        if ch.n not in plans:
            plans[ch.n] = vgf.Plan(ch.n, ch.h, method="vgf", precision="f32")
    pl = [plans[ch.n] for ch in charges]
    rhos = [torch.from_numpy(ch.rho()).to("cuda", torch.float32) for ch in charges]
    phis = [torch.empty(ch.n, dtype=torch.float32, device="cuda") for ch in charges]
    Es = [torch.empty((3,) + ch.n, dtype=torch.float32, device="cuda") for ch in charges]
    grouped = vgf.Batch(pl, graph=False)
    graphed = vgf.Batch(pl, graph=True)

    def single():
        for p, r, ph, E in zip(pl, rhos, phis, Es):
            p.solve(r, ph, E)

    runs = {"single": single, "grouped": lambda: grouped.solve(rhos, phis, Es),
            "graph": lambda: graphed.solve(rhos, phis, Es),
            "graph_tuned": lambda: graphed.solve(rhos, phis, Es)}
    out = {}
    schedules = None
    for name, fn in runs.items():
        if name == "graph_tuned":
            schedules = graphed.autotune(rhos, phis, Es, reps=3)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        out[name] = {"ms_per_batch": wall, "event_ms_per_batch": e0.elapsed_time(e1) / steps,
                     "solves_per_s": len(charges) * 1e3 / wall}
    moved = sum(sum(kernel_bytes(ch.n, 4).values()) for ch in charges)
    sizes = {}
    for ch in charges:
        sizes[str(ch.n[0])] = sizes.get(str(ch.n[0]), 0) + 1
    res = {"workload": "batch_3d_mixed", "entries": len(charges), "precision": "f32",
           "outputs": "phi+E", "sizes": sizes, "groups": graphed.groups, "schedules": schedules, "modes": out,
           "moved_bytes_per_batch": moved,
           "graph_gbs": moved / (out["graph_tuned"]["ms_per_batch"] * 1e-3) / 1e9,
           "speedup_graph_vs_single": out["single"]["ms_per_batch"] / out["graph_tuned"]["ms_per_batch"]}
    grouped.close()
    graphed.close()
    for p in plans.values():
        p.close()
    del rhos, phis, Es
    torch.cuda.empty_cache()
    return res


def time_fn(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def run_small_configs(vgf, torch, workloads, steps, warmup, seed):
    """The other workloads, timed on their own plans (rho resident in HBM):
    gaussian_3d_32 (3D 32^3, FP64, phi + E) and mixture_2d_512 (2D 512^2,
    FP64, phi + E), each with VGF and HE; diff_3d_128 (8 right-hand sides at
    128^3, FP32, E only): one step is the 8 forward solves plus the 8
    adjoints of the loss gradient."""
    out = {}
    for name, ch in (("gaussian_3d_32", workloads.gaussian_3d_32()),
                     ("mixture_2d_512", workloads.mixture_2d_512(seed=seed))):
        rho = torch.from_numpy(ch.rho()).to("cuda", torch.float64)
        res = {"grid": list(ch.n), "precision": "f64", "outputs": "phi+E"}
        for method in ("vgf", "he"):
            plan = vgf.Plan(ch.n, ch.h, method=method, precision="f64")
            phi = torch.empty(ch.n, dtype=torch.float64, device="cuda")
            E = torch.empty((len(ch.n),) + ch.n, dtype=torch.float64, device="cuda")
            sched = plan.autotune(rho, phi, E, reps=3)
            ms = time_fn(torch, lambda: plan.solve(rho, phi, E), max(steps, 50), warmup)
            res[method] = {"ms_per_solve": ms, "solves_per_s": 1e3 / ms, "schedule": list(sched)}
            if any(sched):
                # what the tuned schedule gains over the default one
                plan.schedule = (0, 0, 0, 0, 0)
                ms0 = time_fn(torch, lambda: plan.solve(rho, phi, E), max(steps, 50), warmup)
                plan.schedule = sched
                res[method]["ms_per_solve_default_schedule"] = ms0
            # the same solve replayed as one captured graph (a one-entry batch);
            # the first graph replays of a process carry a one-time runtime
            # set-up, so the replays are warmed up longer
            batch = vgf.Batch([plan], graph=True)
            ms_g = time_fn(torch, lambda: batch.solve([rho], [phi], [E]), max(steps, 50), max(warmup, 50))
            res[method + "_graph"] = {"ms_per_solve": ms_g, "solves_per_s": 1e3 / ms_g}
            batch.close()
            plan.close()
        out[name] = res
    out["diff_3d_128"] = run_diff(vgf, torch, workloads, steps, warmup, seed)
    torch.cuda.empty_cache()
    return out


def run_diff(vgf, torch, workloads, steps, warmup, seed):
    """diff_3d_128: 8 right-hand sides at 128^3, FP32, E only; one step is
    the 8 forward solves plus the 8 adjoints of the loss gradient, one by one
    and as one batched solve (graph) + one batched adjoint."""
    rhs, _ = workloads.diff_3d_128(seed=seed)
    n, h = rhs[0].n, rhs[0].h
    plan = vgf.Plan(n, h, method="vgf", precision="f32", outputs=("E",))
    rhos = [torch.from_numpy(c.rho()).to("cuda", torch.float32) for c in rhs]
    Es = [torch.empty((3,) + n, dtype=torch.float32, device="cuda") for _ in rhs]
    gEs = [torch.randn((3,) + n, dtype=torch.float32, device="cuda") for _ in rhs]
    grs = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in rhs]
    plan.autotune(rhos[0], None, Es[0], reps=3)

    def step():
        for r, E in zip(rhos, Es):
            plan.solve(r, None, E, want_phi=False)
        for gE, gr in zip(gEs, grs):
            plan.adjoint(None, gE, gr)

    ms = time_fn(torch, step, steps, warmup)
    # the same step through one batch: each pass one launch over the 8 entries
    batch = vgf.Batch([plan] * len(rhs), graph=True)

    def step_batched():
        batch.solve(rhos, None, Es)
        batch.adjoint(None, gEs, grs)

    ms_b = time_fn(torch, step_batched, steps, warmup)
    res = {"grid": list(n), "batch": len(rhs), "precision": "f32", "outputs": "E",
           "ms_per_step": ms, "rhs_per_s": len(rhs) * 1e3 / ms,
           "ms_per_step_batched": ms_b, "rhs_per_s_batched": len(rhs) * 1e3 / ms_b,
           "step": "8 forward solves (E only) + 8 adjoints; batched: one vgf_batch_solve "
                   "(graph) + one vgf_batch_adjoint"}
    batch.close()
    plan.close()
    return res


def run_variants(vgf, torch, ch, rho64, steps, warmup):
    """The comparison variants at the headline size, FP32, phi + E, each on
    its own autotuned plan: the HE methods (same passes, another kernel
    spectrum), the finite-difference and gradient-kernel fields (the latter
    in both layouts), the axis-0 layout, and a rectangular grid (256 x 128 x 192 points, spacing 2/255 on
    every axis, the beam's leading block of points)."""
    rho = torch.from_numpy(rho64).to("cuda", torch.float32)
    cases = [("vgf", {}), ("vgf_axis0_layout", {"layout": "axis0"}), ("he", {"method": "he"}),
             ("he_nearby", {"method": "he_nearby"}), ("he_cellavg", {"method": "he_cellavg"}),
             ("vgf_fd_field", {"field": "centered"}), ("vgf_gradient_kernel", {"field": "gradient_kernel"}),
             ("vgf_gradient_kernel_axis0_layout", {"field": "gradient_kernel", "layout": "axis0"})]
    out = {"grid": list(ch.n), "precision": "f32", "outputs": "phi+E"}

    def timed(plan, r):
        phi = torch.empty(plan.n, dtype=torch.float32, device="cuda")
        E = torch.empty((plan.dim,) + plan.n, dtype=torch.float32, device="cuda")
        plan.autotune(r, phi, E, reps=3)
        ms = time_fn(torch, lambda: plan.solve(r, phi, E), steps, warmup)
        return {"ms_per_solve": ms, "solves_per_s": 1e3 / ms}

    for name, kw in cases:
        args = {"method": "vgf", "precision": "f32"}
        args.update(kw)
        plan = vgf.Plan(ch.n, ch.h, **args)
        out[name] = timed(plan, rho)
        plan.close()
    n_r = (256, 128, 192)
    rho_r = rho[:n_r[0], :n_r[1], :n_r[2]].contiguous()
    plan = vgf.Plan(n_r, ch.h, method="vgf", precision="f32")
    out["vgf_rectangular"] = dict(timed(plan, rho_r), grid=list(n_r))
    plan.close()
    del rho, rho_r
    torch.cuda.empty_cache()
    return out


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))


def cpu_baseline(ch, rho64, L, results):
    """FP64 oracle, 2N FFT path, one full solve (phi + E) on the host cores."""
    import oracle as orc
    w = orc.vgf_kernel(ch.n, ch.h, L)  # plan-time precompute: not timed
    times = []
    for _ in range(2):  # two solves: about 25 s of host work on 16 threads
        t0 = time.perf_counter()
        phi_o, E_o = orc.solve_fft2n(ch.n, ch.h, w, rho64)
        times.append(time.perf_counter() - t0)
    t = sum(times) / len(times)
    acc = {}
    for prec, r in results.items():
        acc[prec] = {"phi": rel_l2(r["out"]["phi"], phi_o),
                     "E": rel_l2(r["out"]["E"], E_o)}
    # the untruncated analytic potential and field of the Gaussian on a
    # stride-8 subsample (limited by the charge outside the box)
    sub = tuple(slice(0, x, 8) for x in ch.n)
    n_s = tuple(len(range(0, x, 8)) for x in ch.n)
    pa, Ea = orc.gauss_mixture_grid(n_s, ch.x0, tuple(8 * x for x in ch.h), ch.centers, ch.sigmas,
                                    ch.weights, iso=False)
    ana = {"sample": "stride-8 subsample, %s points" % "x".join(map(str, n_s))}
    for prec, r in results.items():
        ana[prec] = {"phi": rel_l2(r["out"]["phi"][sub], pa),
                     "E": rel_l2(r["out"]["E"][(slice(None),) + sub], Ea)}
    acc["vs_analytic"] = ana
    base = {"value": 1.0 / t, "unit": "solves/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": "two full 256^3 FP64 solves (phi + E) by the oracle's naive 2N FFT path, "
                      "each including its FFT of the kernel; kernel precompute excluded; %s s"
                      % ", ".join("%.1f" % x for x in times),
            "host": host_info()}
    return base, acc


def host_info():
    """CPU model, logical CPUs and memory of the machine running the oracle."""
    model, mem = "?", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count(), "mem_gib": round(mem / 2**30, 1)}


def oracle_timing(seed):
    """The oracle's 2N FFT path per workload on the host cores, with all of
    the oracle's threads and with one (kernel precompute excluded, as in
    the CPU baseline). The batch and the differentiable step are timed on one
    grid of each size they hold and summed over their draws."""
    import oracle as orc
    from paper_2103_08531_amd import workloads as W

    def solve_time(ch, want_phi=True, want_E=True, adjoint=False):
        w = orc.vgf_kernel(ch.n, ch.h, orc.default_L(ch.n, ch.h))
        rho = ch.rho()
        t0 = time.perf_counter()
        orc.solve_fft2n(ch.n, ch.h, w, rho, want_phi=want_phi, want_E=want_E)
        if adjoint:
            orc.adjoint_fft2n(ch.n, ch.h, w, None, np.stack([rho] * len(ch.n)))
        return time.perf_counter() - t0

    batch = W.batch_3d_mixed(seed)
    rhs, _ = W.diff_3d_128(seed)
    full = orc.num_threads()
    rows = []
    for threads in (full, 1):
        orc.set_num_threads(threads)
        r = {"threads": threads}
        r["gaussian_3d_32"] = solve_time(W.gaussian_3d_32(seed))
        print("[oracle %d threads] gaussian_3d_32 %.2f s" % (threads, r["gaussian_3d_32"]), file=sys.stderr, flush=True)
        r["mixture_2d_512"] = solve_time(W.mixture_2d_512(seed))
        print("[oracle %d threads] mixture_2d_512 %.2f s" % (threads, r["mixture_2d_512"]), file=sys.stderr, flush=True)
        per_size = {}
        for ch in batch:
            N = ch.n[0]
            if N not in per_size:
                per_size[N] = solve_time(ch)
                print("[oracle %d threads] batch grid %d^3 %.2f s" % (threads, N, per_size[N]),
                      file=sys.stderr, flush=True)
        r["batch_3d_mixed"] = sum(per_size[ch.n[0]] for ch in batch)
        r["diff_3d_128"] = len(rhs) * solve_time(rhs[0], want_phi=False, want_E=True, adjoint=True)
        print("[oracle %d threads] diff_3d_128 %.2f s" % (threads, r["diff_3d_128"]), file=sys.stderr, flush=True)
        if threads == full:
            r["beam_3d_256"] = solve_time(W.beam_3d_256(seed))
            print("[oracle %d threads] beam_3d_256 %.2f s" % (threads, r["beam_3d_256"]), file=sys.stderr,
                  flush=True)
        rows.append(r)
    orc.set_num_threads(full)
    return {"host": host_info(), "seconds": rows,
            "note": "seconds per solve (gaussian_3d_32, mixture_2d_512, beam_3d_256: phi + E), per batch of "
                    "64 grids (batch_3d_mixed, phi + E), per step of 8 E-only solves and 8 adjoints "
                    "(diff_3d_128); the 256^3 solve runs with all threads only"}


PLAN_TRACE_MD = os.path.join(PROFILES, "vgf_plan_precompute_kernel_trace.md")
PLAN_GRIDS = ((256, 256, 256), (512, 512))


def plan_gemm_model(n):
    """The FP64 GEMM launches of one VGF plan's precompute, in order:
    (label, rows x k x columns, flops). Restricted inverse DFT: axis a maps
    2N_a + 1 samples to N_a; spectrum: N_a to N_a + 1."""
    d = len(n)
    out = []
    for stage, (m_of, j_of) in (("restricted", (lambda N: 2 * N + 1, lambda N: N)),
                                ("spectrum", (lambda N: N, lambda N: N + 1))):
        cur = [m_of(N) for N in n]
        for a in range(d):
            M, J = m_of(n[a]), j_of(n[a])
            rest = 1
            for b in range(d):
                if b != a:
                    rest *= cur[b]
            out.append(("%s axis %d" % (stage, a), "%d x %d x %d" % (J, M, rest), 2 * M * J * rest))
            cur[a] = J
    return out


def plan_only():
    """Create each PLAN_GRIDS plan twice (FP32 plans; the precompute is FP64
    either way) and print the creation wall times."""
    import torch
    from paper_2103_08531_amd import vgf
    torch.cuda.synchronize()
    out = {}
    for n in PLAN_GRIDS:
        h = tuple(2.0 / (x - 1) for x in n)
        ts = []
        for _ in range(2):
            t0 = time.perf_counter()
            p = vgf.Plan(n, h, precision="f32")
            ts.append(1e3 * (time.perf_counter() - t0))
            p.close()
        out["x".join(map(str, n))] = ts
    print(json.dumps({"plan_ms": out}), flush=True)


def write_plan_trace_profile(trace_csv, command):
    """Durations of the precompute GEMMs from a kernel trace of --plan-only,
    with each launch's FP64 rate against the 78.6 TFLOP/s MFMA peak."""
    rows = [r for r in csv.DictReader(open(trace_csv)) if "k_gemm_f64" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    model, keep = [], []
    for n in PLAN_GRIDS:
        for rep in range(2):
            for m in plan_gemm_model(n):
                model.append(("x".join(map(str, n)),) + m)
                keep.append(rep == 1)
    if len(rows) != len(model):
        raise SystemExit("expected %d GEMM launches, found %d" % (len(model), len(rows)))
    md = ["# Plan precompute on the matrix cores: FP64 GEMMs of the separable transforms", "",
          "Kernel trace of plan creation (each grid twice; the second creation of each grid is listed). "
          "Each launch is one axis of the restricted inverse DFT or of the kernel spectrum as a batched "
          "FP64 GEMM (k_gemm_f64, v_mfma_f64_16x16x4f64). Flops = 2 x rows x k x columns.", "",
          "Command:", "", "```", command, "```", "",
          "| grid | transform | rows x k x columns | GFLOP | us | TFLOP/s | frac of 78.6 |",
          "|---|---|---|---|---|---|---|"]
    for (grid, label, shape, flops), r, k in zip(model, rows, keep):
        if k:
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            md.append("| %s | %s | %s | %.2f | %.1f | %.1f | %.2f |" % (
                grid, label, shape, flops / 1e9, us, flops / us / 1e6, flops / us / 1e6 / 78.6))
    md.append("")
    with open(PLAN_TRACE_MD, "w") as f:
        f.write("\n".join(md))
    print(PLAN_TRACE_MD)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch_3d_mixed comparison and the other workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the solves, copy 256 MiB device-to-device once (a plain copy "
                         "kernel of known size, to scale HBM byte counters)")
    ap.add_argument("--digest-counters", nargs=4, metavar=("FETCH_CSV", "FETCH_OUT", "WRITE_CSV", "WRITE_OUT"),
                    help="write the traffic profile from two rocprofv3 counter_collection.csv files and "
                         "the outputs of the two profiled bench runs")
    ap.add_argument("--digest-trace", nargs=2, metavar=("TRACE_CSV", "BENCH_JSON"),
                    help="write the kernel-trace profile from a rocprofv3 kernel_trace.csv file")
    ap.add_argument("--digest-pmc", nargs="+", metavar="CSV_OR_OUT",
                    help="write profiles/vgf_solve_beam_3d_256_counters.md from rocprofv3 --pmc "
                         "counter_collection.csv files and the outputs of their profiled bench runs "
                         "(all CSV files first, then the same number of outputs)")
    ap.add_argument("--command", default="", help="the profiling command, recorded in the profile")
    ap.add_argument("--plan-only", action="store_true",
                    help="create the 256^3 and 512^2 plans twice each, print their creation times, exit")
    ap.add_argument("--only-workload", choices=["batch_3d_mixed", "diff_3d_128"],
                    help="time only this workload (for a kernel trace of it), print one JSON line, exit")
    ap.add_argument("--digest-workload-trace", nargs=3, metavar=("TRACE_CSV", "WORKLOAD", "BENCH_JSON"),
                    help="write profiles/WORKLOAD_kernel_trace.md from a kernel trace of --only-workload")
    ap.add_argument("--digest-plan-trace", metavar="TRACE_CSV",
                    help="write the precompute GEMM profile from a kernel trace of --plan-only")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the oracle's 2N FFT path on every workload (all threads and one), "
                         "print one JSON line and exit (no GPU)")
    args = ap.parse_args()
    if args.digest_plan_trace:
        write_plan_trace_profile(args.digest_plan_trace, args.command)
        return
    if args.digest_workload_trace:
        write_workload_trace_profile(args.digest_workload_trace[0], args.digest_workload_trace[1],
                                     args.digest_workload_trace[2], args.command)
        return
    if args.plan_only:
        plan_only()
        return
    if args.oracle_timing:
        print(json.dumps(oracle_timing(args.seed)), flush=True)
        return
    if args.digest_counters:
        write_traffic_profile(*args.digest_counters, command=args.command)
        return
    if args.digest_pmc:
        half = len(args.digest_pmc) // 2
        write_counters_profile(args.digest_pmc[:half], args.digest_pmc[half:], args.command)
        return
    if args.digest_trace:
        write_trace_profile(args.digest_trace[0], args.digest_trace[1], args.command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solve path runs on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_08531_amd import vgf, workloads
    torch.cuda.set_device(0)
    if args.only_workload:
        if args.only_workload == "batch_3d_mixed":
            res = run_batch(vgf, torch, workloads, args.steps, args.warmup, args.seed)
        else:
            res = run_diff(vgf, torch, workloads, args.steps, args.warmup, args.seed)
        print(json.dumps({"workload": args.only_workload, "result": res}), flush=True)
        return
    ch = workloads.beam_3d_256(seed=args.seed)
    rho64 = ch.rho()
    # one small plan first, so that the timed plan creations exclude the
    # library's one-time start-up (code object loading, first allocations)
    vgf.Plan((16, 16, 16), (2.0 / 15,) * 3, precision="f32").close()

    results = {}
    for prec in ("f32", "f64"):
        results[prec] = run_precision(vgf, torch, ch, rho64, prec, args.steps, args.warmup)
        print("[bench] %s: %.3f ms/solve (events %.3f), passes %s" % (
            prec, results[prec]["wall_ms"], results[prec]["event_ms"],
            {k: round(v, 4) for k, v in results[prec]["passes"].items()}), file=sys.stderr, flush=True)

    others = None
    if not args.no_batch:
        others = run_small_configs(vgf, torch, workloads, args.steps, args.warmup, args.seed)
        others["variants_256"] = run_variants(vgf, torch, ch, rho64, args.steps, args.warmup)
        print("[bench] other workloads: %s" % json.dumps(others), file=sys.stderr, flush=True)
    batch = None
    if not args.no_batch:
        batch = run_batch(vgf, torch, workloads, args.steps, args.warmup, args.seed)
        print("[bench] batch_3d_mixed: %s" % {k: round(v["ms_per_batch"], 3) for k, v in batch["modes"].items()},
              file=sys.stderr, flush=True)

    f32 = results["f32"]
    f64 = results["f64"]
    kb32 = kernel_bytes(ch.n, 4)
    kb64 = kernel_bytes(ch.n, 8)
    pm32 = pass_model_bytes(ch.n, 4)
    pm64 = pass_model_bytes(ch.n, 8)
    traffic = load_traffic()

    def dominant(res, prec):
        """The launch with the largest mean duration, its algorithmic bytes
        and, when the committed counters describe these sources, its HBM
        traffic per launch."""
        model = launch_model(ch.n, 4 if prec == "f32" else 8)
        if len(res["launches"]) != len(model):
            raise SystemExit("unexpected launch sequence %s" % res["launches"])
        k = max(range(len(model)), key=lambda i: res["launches"][i][1])
        pname, pattern, nbytes = model[k]
        assert res["launches"][k][0] == pname, (res["launches"], model)
        ms = res["launches"][k][1]
        name = launch_kernel_name(pattern, prec, res["schedule"], pname, launch_indices(model)[k])
        tr = None
        if traffic is not None and name in traffic["kernels"]:
            tr = traffic["kernels"][name]["traffic_bytes"]
        out = {"kernel": name, "pass": pname, "launch": k, "achieved": nbytes / (ms * 1e-3) / 1e9,
               "mean_launch_ms": ms, "algorithmic_bytes_per_launch": nbytes, "traffic": tr}
        if pname == "fused":
            fl = multiply_pass_flops(ch.n)
            peak = VECTOR_PEAK_TFLOPS[prec]
            out["alu"] = {"achieved": fl / (ms * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                          "frac": fl / (ms * 1e-3) / 1e12 / peak, "flops_per_launch": fl,
                          "count": "5 P log2 P per P-point complex transform (three per line) + 4 P "
                                   "for the kernel multiply and -i k; peak: non-packed vector FMA rate"}
        return out

    d32 = dominant(f32, "f32")
    d64 = dominant(f64, "f64")

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
        "source_hash": kernel_source_hash(),
        "config": {"workload": "beam_3d_256", "grid": list(ch.n), "domain": "[-1,1]^3",
                   "method": "vgf", "outputs": "phi+E", "sigma": [0.05, 0.05, 0.3],
                   "seed": args.seed, "L": f32["L"], "parallelism": "single GPU"},
        "fp64": {"value": 1e3 / f64["wall_ms"], "unit": "solves/s", "ms_per_step": f64["wall_ms"],
                 "dtype": "f64"},
        "schedule": {"f32": f32["schedule"], "f64": f64["schedule"]},
        "plan_ms": {"f32": f32["plan_ms"], "f64": f64["plan_ms"]},
        "roofline": {"bound": "hbm", "kernel": d32["kernel"],
                     "achieved": d32["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": d32["achieved"] / HBM_PEAK_GBS, "traffic": d32["traffic"],
                     "traffic_unit": "bytes/launch",
                     "algorithmic_bytes_per_launch": d32["algorithmic_bytes_per_launch"],
                     "mean_launch_ms": d32["mean_launch_ms"], "alu": d32.get("alu"),
                     "fp64": dict(d64, peak=HBM_PEAK_GBS, frac=d64["achieved"] / HBM_PEAK_GBS)},
        "pass_model": {"bytes_per_solve_f32": pm32, "bytes_per_solve_f64": pm64,
                       "frac_f32": pm32 / (f32["wall_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "frac_f64": pm64 / (f64["wall_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "passes": {"bytes_f32": kb32, "bytes_f64": kb64,
                   "moved_bytes_per_solve_f32": sum(kb32.values()),
                   "moved_bytes_per_solve_f64": sum(kb64.values()),
                   "ms_f32": f32["passes"], "ms_f64": f64["passes"],
                   "launches_ms_f32": f32["launches"], "launches_ms_f64": f64["launches"],
                   "gbs_f32": {k: kb32[k] / (f32["passes"][k] * 1e-3) / 1e9 for k in kb32},
                   "gbs_f64": {k: kb64[k] / (f64["passes"][k] * 1e-3) / 1e9 for k in kb64}},
        "accuracy": {"f32_vs_f64_gpu": {"phi": rel_l2(f32["out"]["phi"], f64["out"]["phi"]),
                                        "E": rel_l2(f32["out"]["E"], f64["out"]["E"])}},
    }
    line["batch"] = batch
    line["other_workloads"] = others
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
        line["accuracy"]["vs_analytic"] = acc.pop("vs_analytic")
        line["accuracy"]["vs_oracle"] = acc
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
