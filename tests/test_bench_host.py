"""Host logic of bench.py (no GPU): the measured-traffic lookup in the
committed counter summaries, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

LAUNCH = dict(tile_rows=4, schedule=4, persist_blocks_per_cu=4, graph_steps=64, fp64_arith=1, chunk_rows=12)


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    """A repository root whose profiles/ holds one counter summary of the
    current kernel sources, taken at chunk 12, with chunk 8 as a second entry."""
    os.makedirs(tmp_path / "profiles")
    d = {"kernel_source_sha256_16": bench.kernel_source_hash(), "launch": dict(LAUNCH),
         "hbm_bytes_per_launch": 1200,
         "other_launches": [{"launch": dict(LAUNCH, chunk_rows=8), "hbm_bytes_per_launch": 1300}]}
    (tmp_path / "profiles" / "lb_wide_bin_sweep_counters.json").write_text(json.dumps(d))
    real = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: real)
    return tmp_path


def test_traffic_is_looked_up_by_launch_shape(fake_root):
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", LAUNCH) == 1200
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", dict(LAUNCH, chunk_rows=8)) == 1300
    # graph steps and persistent blocks do not change the kernel's traffic
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", dict(LAUNCH, graph_steps=0)) == 1200
    # another chunking, schedule or arithmetic: not measured
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", dict(LAUNCH, chunk_rows=16)) is None
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", dict(LAUNCH, schedule=3)) is None
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", dict(LAUNCH, fp64_arith=0)) is None
    assert bench.traffic_from_profiles("lb_wide_bin", "vdw16k", LAUNCH) is None


def test_traffic_of_other_kernel_sources_is_not_used(fake_root, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    assert bench.traffic_from_profiles("lb_wide_bin", "sweep", LAUNCH) is None


def test_committed_summaries_name_their_launch_and_commands():
    """The counter summaries of the two hot kernels: their launch shape
    named, every command a rocprofv3 call of committed files.  The fused van der Waals sweep moves its populations once
    per two steps (traffic below the two steps' algorithmic bytes); the
    moment-storage sweep re-reads strip and chunk halos (above)."""
    for name, schedule, lo, hi in (("lb_wmom_bin_sweep_counters.json", 6, 0.8, 1.2),
                                   ("lb_wide2_vdw_vdw16k_counters.json", 5, 0.5, 0.8)):
        d = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert d["launch"]["schedule"] == schedule
        assert lo < d["hbm_bytes_per_launch"] / d["algorithmic_bytes_per_launch"] < hi
        assert all(c.startswith(("cd ", "rocprofv3 ")) for c in d["commands"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_algorithmic_and_stored_bytes():
    """The method's algorithmic bytes per update (every population, and phi,
    read and written once: 72 B vdW, 80 B binary) are the roofline's; the
    binary moment storage (schedule 6) itself moves 64 B."""
    import bench
    assert bench.BYTES_PER_LUP == {"vdw": 72, "binary": 80}
    assert bench.stored_bytes_per_lup("vdw", 5) == 36
    assert bench.stored_bytes_per_lup("binary", 5) == 40
    assert bench.stored_bytes_per_lup("vdw", 4) == 72
    assert bench.stored_bytes_per_lup("binary", 4) == 80
    assert bench.stored_bytes_per_lup("binary", 6) == 64


def test_kernel_hash_ignores_comments_only():
    """The counter summaries are tied to the kernels' code: editing a comment
    keeps them, changing code drops them."""
    a = "int f(int x) { // one\n  return x + 1; /* two\n lines */ }\n"
    b = "int f(int x) {\n  // another comment\n  return x + 1;\n}\n"
    c = "int f(int x) { return x + 2; }"
    assert bench.code_of(a) == bench.code_of(b)
    assert bench.code_of(a) != bench.code_of(c)
