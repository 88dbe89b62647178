"""Host logic of bench.py (no GPU): the algorithmic byte model, the counter
databases' reduction to HBM bytes per launch, and the refusal of several GPUs."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes():
    n, z, k = 1000, 7000, 16
    # FP64: values + column indices + row pointers, P read once, Q written once
    assert bench.algorithmic_bytes("spmm", n, z, k, "fp64") == 8 * z + 4 * z + 4 * (n + 1) + 2 * 8 * n * k
    assert bench.algorithmic_bytes("spmm", n, z, k, "fp32_reliable") == 4 * z + 4 * z + 4 * (n + 1) + 2 * 4 * n * k
    assert bench.algorithmic_bytes("update_r", n, z, k, "fp64") == 3 * 8 * n * k
    assert bench.algorithmic_bytes("update_xp", n, z, k, "fp32_refine") == 5 * 4 * n * k
    with pytest.raises(ValueError):
        bench.algorithmic_bytes("reduce", n, z, k, "fp64")


def test_solve_bytes():
    n, z, k = 1000, 7000, 16
    kernels = {"spmm": {"launches": 10}, "update_r": {"launches": 10}, "update_xp": {"launches": 11},
               "small": {"launches": 20}}
    want = (10 * bench.algorithmic_bytes("spmm", n, z, k, "fp64") + 10 * bench.algorithmic_bytes("update_r", n, z, k, "fp64")
            + 11 * bench.algorithmic_bytes("update_xp", n, z, k, "fp64"))
    assert bench.solve_bytes(kernels, n, z, k, "fp64") == want
    assert bench.solve_bytes({}, n, z, k, "fp64") == 0


def _db(path, rows):
    """A counters_collection table as rocprofv3 writes it (the columns read)."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
                "counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_from_scales_and_picks_the_iteration_kernel(tmp_path):
    d = tmp_path / "traffic"
    copy_kib = bench.COPY_BYTES / 1024
    # the copy reports half its reads and all its writes
    _db(str(d / "copy_fetch" / "run_results.db"), [(1, "copy", "FETCH_SIZE", copy_kib / 2)])
    _db(str(d / "copy_write" / "run_results.db"), [(1, "copy", "WRITE_SIZE", copy_kib)])
    spmm64 = "void bcg::k_spmm_mfma<double, 16, 16, true, false>(Plan)"
    resid = "void bcg::k_spmm_fast<double, 16, 16, 1>(Plan)"   # a residual mode: few launches
    spmm32 = "void bcg::k_spmm_mfma_f32<16, 16, true, false>(Plan)"
    upd32 = "void bcg::k_update_xp_mfma<float, 16, 16, true, 2>(Plan)"
    fetch, write = [], []
    disp = 0
    for name, kib, launches in ((spmm64, 100.0, 10), (resid, 900.0, 2), (spmm32, 50.0, 10), (upd32, 70.0, 10)):
        for i in range(launches):
            disp += 1
            fetch.append((disp, name, "FETCH_SIZE", kib))
            write.append((disp, name, "WRITE_SIZE", kib / 2))
        # a launch that returned at entry is left out of the mean
        disp += 1
        fetch.append((disp, name, "FETCH_SIZE", 0.0))
        write.append((disp, name, "WRITE_SIZE", 0.0))
    _db(str(d / "fetch" / "run_results.db"), fetch)
    _db(str(d / "write" / "run_results.db"), write)
    out = tmp_path / "traffic.json"
    assert bench.traffic_from(str(d), "wl", "hybrid", path=str(out)) == 0
    rec = json.load(open(out))
    s64 = rec["spmm/wl/hybrid/fp64"]
    assert s64["read_bytes"] == pytest.approx(100.0 * 1024 * 2)   # not the residual mode's 900
    assert s64["write_bytes"] == pytest.approx(50.0 * 1024)
    assert s64["kernel_hash"] == bench.kernel_hash()
    assert rec["spmm/wl/hybrid/fp32"]["bytes_per_launch"] == pytest.approx(50 * 1024 * 2 + 25 * 1024)
    assert rec["update_xp/wl/hybrid/fp32"]["read_bytes"] == pytest.approx(70 * 1024 * 2)
    assert "update_r/wl/hybrid/fp64" not in rec


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert json.loads(r.stdout.strip().splitlines()[-1])["n_gpus"] == 2
