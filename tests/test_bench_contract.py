"""CPU checks of the benchmark's contract: the algorithmic bytes it divides by (the
figures of one even-odd hop launch on the 24^3 x 48 workload, worked out by hand below),
the gate that reports measured traffic only for the kernel source it was measured on, the
mappings it fixes for the 12-rhs launches, and its refusal of more than one GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

V = 24 ** 3 * 48          # 663 552 sites


def test_algorithmic_bytes_per_launch():
    # even-odd half hop, 12 rhs: links 4 V x 18 reals once, and per rhs V/2 input and V/2
    # output sites of 24 reals (FP16: 24 halves and a 4-byte norm)
    #   FP32: 191 102 976 + 12 x 331 776 x 2 x  96 =   955 514 880
    #   FP64: 382 205 952 + 12 x 331 776 x 2 x 192 = 1 911 029 760
    #   FP16:  95 551 488 + 12 x 331 776 x 2 x  52 =   509 607 936
    assert bench.eo_bytes(V, "f32", 12) == 955_514_880
    assert bench.eo_bytes(V, "f64", 12) == 1_911_029_760
    assert bench.eo_bytes(V, "f16", 12) == 509_607_936
    # single rhs
    assert bench.eo_bytes(V, "f32", 1) == 191_102_976 + 331_776 * 2 * 96
    # apply_M per site: 4 links of 18 reals + spinor in and out
    assert [bench.apply_M_bytes(V, p) // V for p in ("f64", "f32", "f16")] == [960, 480, 248]


def test_traffic_is_reported_only_for_the_measured_kernel_source(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "hop_traffic_24x24x24x48.json")) as fh:
        rec = json.load(fh)
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_0710_0066_amd", "csrc", f)), f
    key = "eo_f32_12rhs"
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["kernel_source_hash"])
    assert bench.committed_traffic(key) == rec[key]["traffic_bytes_per_launch"] > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.committed_traffic(key) is None


def test_headline_mappings_exist():
    import paper_0710_0066_amd as sap
    assert set(bench.HEADLINE_MAPS) == {"f64", "f32", "f16"}
    for prec, name in bench.HEADLINE_MAPS.items():
        assert 0 <= bench.hop_map_id(sap, name) < sap.HOP_NMAP, (prec, name)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
