"""Host-side accounting of bench.py: algorithmic work and bytes per stage, and
the rule that a committed HBM-traffic record is used only while the kernel
sources it was taken on are unchanged."""
import hashlib
import importlib.util
import json
import os
import shutil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(path):
    spec = importlib.util.spec_from_file_location("bench_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_stage_units_of_the_bench_configuration():
    b = _load(os.path.join(ROOT, "bench.py"))
    nao, naux, nocc = 768, 3072, 96
    # X at s = 7: 28 digit pairs, each 2 naux nao^2 nocc int8 ops; the stored
    # (lower-triangle) B read once plus C, X a streamed workspace
    ops, byts = b.stage_units("x", 7, nao, naux, nocc)
    assert ops == 28 * 2 * naux * nao * nao * nocc == 9_740_985_827_328
    assert byts == 8 * naux * nao * (nao + 1) // 2 + 8 * nao * nocc == 7_257_784_320
    # the digits of X: X read once, 7 planes written once
    _, byts = b.stage_units("slice_x", 7, nao, naux, nocc)
    assert byts == 15 * naux * nao * nocc
    # K at s = 7: the symmetric products over nao (nao + 1) / 2 pairs, x2 ops per MAC
    ops, byts = b.stage_units("k", 7, nao, naux, nocc)
    assert ops == 28 * nao * (nao + 1) * naux * nocc == 4_876_834_701_312
    assert byts == 7 * naux * nao * nocc
    # J reads the lower triangle of B once
    _, byts = b.stage_units("j", 7, nao, naux, nocc)
    assert byts == 8 * naux * nao * (nao + 1) // 2 == 7_257_194_496
    # the FP64-equivalent work that the bench's TFLOP/s divides by
    assert b.flops_alg(nao, naux, nocc) == 529_312_776_192


def test_roofline_picks_the_binding_roof():
    b = _load(os.path.join(ROOT, "bench.py"))
    # X at s = 7: 9.74e12 int8 ops take 1.95 ms at 5 POPS, its 7.26 GB 0.91 ms
    # at 8 TB/s: the matrix cores bind
    r = b.roofline_of("x", 6.0, 7, 768, 3072, 96)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 5000.0
    assert abs(r["achieved"] - 9_740_985_827_328 / 6e-3 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 5000.0) < 1e-12
    # at s = 1 the bytes bind
    r = b.roofline_of("x", 2.0, 1, 768, 3072, 96)
    assert r["bound"] == "hbm" and r["peak"] == 8000.0
    r = b.roofline_of("k", 2.0, 7, 768, 3072, 96, {"int8": 4000.0})
    assert r["bound"] == "mfma" and r["peak"] == 5000.0
    assert abs(r["frac_of_measured_peak"] - r["achieved"] / 4000.0) < 1e-12
    # J and the slicing of X are byte-bound; the FP64 X product is flop-bound
    assert b.roofline_of("j", 1.0, 7, 768, 3072, 96)["bound"] == "hbm"
    assert b.roofline_of("slice_x", 1.0, 7, 768, 3072, 96)["bound"] == "hbm"
    assert b.roofline_of("x", 9.0, 0, 768, 3072, 96)["bound"] == "mfma"


def test_traffic_record_used_only_while_sources_unchanged(tmp_path):
    shutil.copy(os.path.join(ROOT, "bench.py"), tmp_path / "bench.py")
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\n")
    (tmp_path / "profiles").mkdir()
    rec = {"stage": "x", "slices": 7, "traffic_bytes_per_launch": 123,
           "sources_sha256": {"kernel.hip": hashlib.sha256(src.read_bytes()).hexdigest()}}
    (tmp_path / "profiles" / "traffic_x.json").write_text(json.dumps(rec))
    b = _load(str(tmp_path / "bench.py"))
    assert b.measured_traffic("x", 7) == 123
    assert b.measured_traffic("x", 5) is None      # another slice count
    assert b.measured_traffic("k", 7) is None      # another stage
    src.write_text("// kernel v2\n")               # the kernel changed since
    assert b.measured_traffic("x", 7) is None


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says so
    (before touching torch or the GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
