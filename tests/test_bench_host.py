"""Host logic of bench.py (no GPU): its byte models against figures fixed
elsewhere (the reference pass model's published totals, the committed HBM
counter digest), the counter scaling, the source hash and the one-GPU rule."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N256 = (256, 256, 256)


def test_pass_model_matches_the_reference_totals():
    """One HBM read and write per axis pass of the pruned arrays, one inverse
    per field, the kernel octant read once: 4 445.7 MB (FP32) and 8 891.4 MB
    (FP64) per 256^3 solve with phi + E, 1 819.0 / 3 638.0 MB for phi alone."""
    assert round(bench.pass_model_bytes(N256, 4) / 1e6, 1) == 4445.7
    assert round(bench.pass_model_bytes(N256, 8) / 1e6, 1) == 8891.4
    assert round(bench.pass_model_bytes(N256, 4, nf=1) / 1e6, 1) == 1819.0
    assert round(bench.pass_model_bytes(N256, 8, nf=1) / 1e6, 1) == 3638.0


def test_launch_model_is_below_the_pass_model_and_scales_with_precision():
    for prec_bytes in (4, 8):
        model = bench.launch_model(N256, prec_bytes)
        assert [m[0] for m in model] == ["r2c", "c2c_fwd", "fused", "c2c_inv", "c2r"]
        total = sum(b for _, _, b in model)
        assert total < bench.pass_model_bytes(N256, prec_bytes)
        assert sum(bench.kernel_bytes(N256, prec_bytes).values()) == total
    f32 = sum(b for _, _, b in bench.launch_model(N256, 4))
    f64 = sum(b for _, _, b in bench.launch_model(N256, 8))
    assert f64 == 2 * f32
    assert round(f32 / 1e6, 1) == 3098.3


def test_launch_model_agrees_with_the_measured_traffic():
    """The committed counter digest (FETCH_SIZE / WRITE_SIZE of a 256^3 run)
    is an independent measurement of the bytes each launch moves: the passes
    that read and write every array once agree with the model within 1%
    (the multiply pass re-reads kernel-octant rows, and the FP32 C2R reads
    phi's spectrum twice, by design)."""
    with open(bench.TRAFFIC_JSON) as f:
        d = json.load(f)
    checked = 0
    for prec, b in (("f32", 4), ("f64", 8)):
        for pname, pattern, nbytes in bench.launch_model(N256, b):
            if pname == "fused" or (pname == "c2r" and prec == "f32"):
                continue
            name = bench.launch_kernel_name(pattern, prec, d["schedule"][prec], pname)
            tr = d["kernels"][name]["traffic_bytes"]
            assert abs(tr / nbytes - 1) < 0.01, (name, tr, nbytes)
            checked += 1
    assert checked == 7


def test_multiply_pass_flop_count():
    # 257 x 512 lines, each three 512-point transforms (5 P log2 P) + 4 P
    assert bench.multiply_pass_flops(N256) == 257 * 512 * (3 * 5 * 512 * 9 + 4 * 512)


def test_source_hash_ignores_comments_and_whitespace(tmp_path):
    pkg = tmp_path / "paper_2103_08531_amd"
    shutil.copytree(os.path.join(ROOT, "paper_2103_08531_amd", "csrc"), pkg / "csrc")
    shutil.copy(os.path.join(ROOT, "paper_2103_08531_amd", "build.py"), pkg / "build.py")
    h0 = bench.kernel_source_hash(str(tmp_path))
    assert h0 == bench.kernel_source_hash(ROOT)
    f = pkg / "csrc" / "vgf_fd.hip"
    text = f.read_text()
    f.write_text("// a new comment\n/* and a block\n comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash(str(tmp_path)) == h0
    f.write_text(text.replace("T(4)", "T(5)", 1))
    assert bench.kernel_source_hash(str(tmp_path)) != h0


def _write_csv(path, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, c, v) in enumerate(rows):
            f.write('%d,"%s",%s,%s\n' % (i, k, c, v))


def test_counter_digest_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """FETCH_SIZE reads 128 MiB for the 256 MiB calibration copy (factor 2),
    WRITE_SIZE reads true (factor 1); each kernel's mean per dispatch is
    scaled by its counter's factor."""
    kern = "void vgf::k_c2c_fwd<float, 512, 1, 0>(vgf::C2CFwdArgs<float>, HIP_vector_type<float, 2u> const*)"
    copy = "__amd_rocclr_copyBuffer"
    _write_csv(tmp_path / "f.csv", [(kern, "FETCH_SIZE", 100.0), (kern, "FETCH_SIZE", 110.0),
                                    (copy, "FETCH_SIZE", 131072.0)])
    _write_csv(tmp_path / "w.csv", [(kern, "WRITE_SIZE", 300.0), (kern, "WRITE_SIZE", 300.0),
                                    (copy, "WRITE_SIZE", 262144.0)])
    line = json.dumps({"source_hash": bench.kernel_source_hash(), "schedule": {"f32": [0] * 5}})
    for name in ("f.out", "w.out"):
        (tmp_path / name).write_text("noise\n" + line + "\n")
    d = bench.digest_counters(str(tmp_path / "f.csv"), str(tmp_path / "f.out"),
                              str(tmp_path / "w.csv"), str(tmp_path / "w.out"))
    assert d["fetch_size_calibration"]["factor"] == pytest.approx(2.0)
    assert d["write_size_calibration"]["factor"] == pytest.approx(1.0)
    k = d["kernels"]["k_c2c_fwd<float, 512, 1, 0>"]
    assert k["dispatches"] == 2
    assert k["read_bytes"] == pytest.approx(105.0 * 1024 * 2)
    assert k["write_bytes"] == pytest.approx(300.0 * 1024)
    # counters of other sources are refused
    (tmp_path / "w.out").write_text(json.dumps({"source_hash": "0" * 64}) + "\n")
    with pytest.raises(SystemExit):
        bench.digest_counters(str(tmp_path / "f.csv"), str(tmp_path / "f.out"),
                              str(tmp_path / "w.csv"), str(tmp_path / "w.out"))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
