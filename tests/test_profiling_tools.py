"""CPU tests of the measurement plumbing: the rocprofv3 summariser, the
counter calibration, the traffic lookup's source check, and bench.py's
single-GPU guard."""
import csv
import os
import subprocess
import sys

import pytest

from paper_1607_06156_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counters(path, counter, rows):
    path.mkdir(parents=True, exist_ok=True)
    with open(path / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for did, name, val in rows:
            w.writerow([did, name, counter, val])


def test_pmc_calibration_and_averages(tmp_path, capsys):
    # a 1024 MiB copy reads as 524288 KiB (half) and writes as 1048576 KiB
    _counters(tmp_path / "f", "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 524288.0), (2, "__amd_rocclr_copyBuffer", 4.0),
                                             (3, "void ccmi::sv_pass_kernel<true>(int)", 1000.0),
                                             (4, "void ccmi::sv_pass_kernel<false>(int)", 3000.0)])
    _counters(tmp_path / "w", "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 1048576.0),
                                             (3, "void ccmi::sv_pass_kernel<true>(int)", 10.0),
                                             (4, "void ccmi::sv_pass_kernel<false>(int)", 30.0)])
    rs.main(["pmc", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--kernel", "sv_pass_kernel",
             "--cls", "sv_pass", "--copy-mib", "1024"])
    out = capsys.readouterr().out
    p = tmp_path / "s.txt"
    p.write_text(out)
    d = rs.read_pmc_file(str(p))
    assert float(d["fetch_scale_bytes_per_kib"]) == pytest.approx(2048.0)
    assert float(d["write_scale_bytes_per_kib"]) == pytest.approx(1024.0)
    # two dispatches averaged: fetch (1000 + 3000) / 2 KiB x 2048, write (10 + 30) / 2 KiB x 1024
    assert int(d["fetch_bytes_per_launch"]) == 2000 * 2048
    assert int(d["write_bytes_per_launch"]) == 20 * 1024
    assert int(d["traffic_bytes_per_launch"]) == 2000 * 2048 + 20 * 1024
    assert d["source_sha256"] == rs.source_sha256("sv_pass")


def test_pmc_needs_the_calibration_copy(tmp_path):
    _counters(tmp_path / "f", "FETCH_SIZE", [(3, "sv_pass_kernel", 1.0)])
    _counters(tmp_path / "w", "WRITE_SIZE", [(3, "sv_pass_kernel", 1.0)])
    with pytest.raises(SystemExit):
        rs.main(["pmc", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--kernel", "sv_pass_kernel",
                 "--cls", "sv_pass", "--copy-mib", "1024"])


def test_stats_table(tmp_path):
    with open(tmp_path / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void ccmi::sv_pass_kernel<true>(int const*)", 4, 4000000, 1000000, 90.0, 900000, 1100000, 1.0])
    t = rs.stats_table(str(tmp_path))
    assert "| sv_pass_kernel<true> | 4 | 4.000 | 1000.0 | 900.0 | 1100.0 | 90.00 |" in t


def test_source_hash_tracks_the_sources():
    h = rs.source_sha256("sv_pass")
    assert len(h) == 64 and h == rs.source_sha256("sv_pass")
    assert h != rs.source_sha256("degree")


def test_bench_traffic_lookup_rejects_stale_counters(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "pmc_sv_pass_demo.txt").write_text("source_sha256: %s\ntraffic_bytes_per_launch: 1234\n"
                                               % rs.source_sha256("sv_pass"))
    (prof / "pmc_degree_demo.txt").write_text("source_sha256: deadbeef\ntraffic_bytes_per_launch: 99\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("sv_pass", "demo") == 1234.0
    assert bench.measured_traffic("degree", "demo") is None       # sources changed since
    assert bench.measured_traffic("sv_pass", "other") is None     # never measured


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_router_weights_save_load_roundtrip(tmp_path):
    """The router tool's text format keeps every float32 parameter exactly and
    refuses a file with the wrong parameter count."""
    import numpy as np
    from paper_1607_06156_amd import router_train as rt
    import paper_1607_06156_amd as ccmi
    w = np.random.default_rng(7).standard_normal(ccmi.ROUTER_NPARAMS).astype(np.float32)
    p = tmp_path / "w.txt"
    rt.save(w, str(p), "test weights\nsecond line")
    assert np.array_equal(rt.load(str(p)), w)
    shipped = rt.load(os.path.join(ROOT, "paper_1607_06156_amd", "router_weights.txt"))
    assert shipped.shape == (ccmi.ROUTER_NPARAMS,) and np.isfinite(shipped).all()
    (tmp_path / "short.txt").write_text("# two\n1 2\n")
    with pytest.raises(ValueError):
        rt.load(str(tmp_path / "short.txt"))


def test_counters_table(tmp_path, capsys):
    _counters(tmp_path / "a", "TCC_ATOMIC_sum", [(1, "void ccmi::sv_pass_kernel<true, true>(int)", 10.0),
                                                 (2, "void ccmi::sv_pass_kernel<true, true>(int)", 30.0),
                                                 (3, "ccmi::giant_pick_kernel(int)", 0.0)])
    _counters(tmp_path / "b", "SQ_INSTS_VALU_MFMA_MOPS_F32", [(1, "void ccmi::sv_pass_kernel<true, true>(int)", 0.0)])
    rs.main(["counters", str(tmp_path / "a"), str(tmp_path / "b"), "--title", "t"])
    out = capsys.readouterr().out
    assert "| sv_pass_kernel<true, true> | TCC_ATOMIC_sum | 2 | 40 | 20 |" in out
    assert "| sv_pass_kernel<true, true> | SQ_INSTS_VALU_MFMA_MOPS_F32 | 1 | 0 | 0 |" in out
    assert "| giant_pick_kernel | TCC_ATOMIC_sum | 1 | 0 | 0 |" in out
