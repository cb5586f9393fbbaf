"""CPU checks of the benchmark's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_traffic_is_null_for_changed_or_missing_kernels(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    # an instantiation without a committed counter run
    assert bench.counter_traffic("interact_f64", 3, 1) is None
    # a stale source hash is ignored
    fake = tmp_path / "profiles"
    fake.mkdir()
    (fake / "interact_uniform-1M_counters.md").write_text(
        "traffic_bytes interact_mixed<8, 0> 1.0e+09 source 0000000000000000\n")
    csrc = tmp_path / "paper_2003_01836_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES["interact_mixed"]:
        (csrc / f).write_text("x")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("interact_mixed", 8, 0) is None


def test_issue_model_from_the_committed_counters(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    # FP64 kernels and uncounted instantiations have no model
    assert bench.issue_model("interact_f64", 8, 0, 1, 10 ** 9, 1.0) is None
    assert bench.issue_model("interact_mixed", 3, 1, 2, 10 ** 9, 1.0) is None
    # a counted kernel: (VALU - trans) FMA-class cycles + trans transcendental cycles
    csrc = tmp_path / "paper_2003_01836_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES["near_pairs_mixed"]:
        (csrc / f).write_text("x")
    import hashlib
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES["near_pairs_mixed"]:
        h.update(b"x")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "interact_uniform-1M_valu_counters.md").write_text(
        f"valu_insts near_pairs_mixed<0> 1.0e+09 source {h.hexdigest()[:16]}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    m = bench.issue_model("near_pairs_mixed", 8, 0, 1, 64 * 10 ** 8, 2.0)
    cycles = (1e9 - 1e8) * bench.CYCLES_FMA32 + 1e8 * bench.CYCLES_TRANS32
    assert abs(m["t_min_ms"] - cycles / bench.SIMDS / bench.CLOCK_HZ * 1e3) < 1e-9
    assert abs(m["frac"] - m["t_min_ms"] / 2.0) < 1e-12


def test_committed_profiles_cover_the_headline_kernels():
    """The counters the bench line reads (HBM traffic, instruction counts, clocks)
    exist for the headline kernels as they are now: every interaction kernel at
    2 and 4 threads per target, the pair kernels, both upward instantiations.
    A kernel source edited after the counters were taken fails here."""
    sys.path.insert(0, ROOT)
    import bench
    for kernel in ("interact_f64", "interact_mixed"):
        for tpt in (2, 4):
            assert bench.counter_value("traffic_bytes", "interact_uniform-1M_counters.md",
                                       kernel, 8, 0, tpt) is not None, (kernel, tpt)
            assert bench.counter_value("valu_insts", "interact_uniform-1M_valu_counters.md",
                                       kernel, 8, 0, tpt) is not None, (kernel, tpt)
            assert bench.counter_value("clock_hz", "interact_uniform-1M_valu_counters.md",
                                       kernel, 8, 0, tpt) is not None, (kernel, tpt)
    for kernel in ("near_pairs_f64", "near_pairs_mixed"):
        assert bench.counter_value("traffic_bytes", "interact_uniform-1M_counters.md",
                                   kernel, 8, 0) is not None, kernel
        assert bench.counter_value("valu_insts", "interact_uniform-1M_valu_counters.md",
                                   kernel, 8, 0) is not None, kernel
    for ker_id in (0, 1):
        assert bench.counter_value("mfma_busy_cycles", "upward_uniform-1M_mfma_counters.md",
                                   "upward_single", 8, ker_id) is not None, ker_id
