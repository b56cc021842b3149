"""Host arithmetic of bench.py's roofline objects (no GPU): which kernel is
priced as dominant, its share of the step's kernel time, and the algorithmic
bytes per launch, and the parsing and copy calibration of the counter passes."""
import os

import pytest

import bench
import fdlb_inputs as I


def _prof(table, upd, prec):
    # [table, update 1..3 FP64, update 1..3 FP32] in ms, as fdlb_profile returns them
    p = [table, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    p[1 + 3 * prec:4 + 3 * prec] = upd
    return p


@pytest.mark.parametrize("prec", [0, 1])
def test_dominant_kernel_and_its_share(prec):
    cfg = I.config("C2", precision=prec)
    nodes = cfg["nx"] * 2 * cfg["qx_half"] * cfg["qy"] * cfg["qz"]
    # table pass larger: 3 x 0.008 against 3 x 0.005
    r = bench.dominant_roofline((1, 8), _prof(0.008, [0.005] * 3, prec), cfg, nodes, prec, "C2")
    assert r["kernel"].startswith("k_table")
    assert r["share_of_kernel_time"] == pytest.approx(0.024 / 0.039, abs=1e-3)
    assert r["other_kernel"]["kernel"].startswith("k_update")
    # update larger
    r = bench.dominant_roofline((1, 8), _prof(0.004, [0.005, 0.006, 0.007], prec), cfg, nodes, prec, "C2")
    assert r["kernel"].startswith("k_update")
    assert r["share_of_kernel_time"] == pytest.approx(0.018 / 0.030, abs=1e-3)
    # stage 2 is priced: three passes of the population element size over every node
    s = 8 if prec == 0 else 4
    assert r["algorithmic_bytes_per_launch"] == 3 * s * nodes
    assert r["achieved"] == pytest.approx(3 * s * nodes / 0.006e-3 / 1e9, rel=1e-3)


def test_mlp_flops_per_step():
    # 10 -> 256 -> 256 -> 256 -> 256 -> 640 at batch 2: forward + weight gradient for every
    # layer, input gradient for all but the first
    macs = [10 * 256, 256 * 256, 256 * 256, 256 * 256, 256 * 640]
    want = 2 * 2 * (2 * macs[0] + 3 * sum(macs[1:]))
    assert bench.mlp_flops_per_step(2) == want


def test_measure_traffic_scales_each_counter_by_the_copy(monkeypatch):
    """The two counter passes are parsed from the profiler's result database
    and each is scaled by the copy kernel's reading of the same counter
    (262144 KiB moved per copy); the profiler itself is replaced here by a
    stand-in that writes such a database."""
    import sqlite3
    import subprocess

    readings = {"FETCH_SIZE": (5000.0, 131072.0), "WRITE_SIZE": (3700.0, 262144.0)}

    def fake_run(cmd, **kw):
        counter = cmd[cmd.index("--pmc") + 1]
        d = cmd[cmd.index("-d") + 1]
        os.makedirs(os.path.join(d, "host"), exist_ok=True)
        con = sqlite3.connect(os.path.join(d, "host", "pmc_results.db"))
        con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
        k, copy = readings[counter]
        for v in (k - 10.0, k + 10.0):
            con.execute("insert into counters_collection values (?, ?, ?)",
                        ("void fdlb::k_update<double, 2, true, 8>(x)", counter, v))
        con.execute("insert into counters_collection values (?, ?, ?)",
                    ("void fdlb::k_update<double, 1, true, 8>(x)", counter, 1e9))   # another stage
        con.execute("insert into counters_collection values (?, ?, ?)", ("fdlb::k_copy_probe(x)", counter, copy))
        con.commit()
        con.close()
        return subprocess.CompletedProcess(cmd, 139)   # the profiler may exit non-zero after a full run

    monkeypatch.setattr(subprocess, "run", fake_run)
    t, detail = bench.measure_traffic("C3", 0, (2, 8))
    fetch = 5000.0 * (262144.0 / 131072.0) * 1024
    write = 3700.0 * (262144.0 / 262144.0) * 1024
    assert detail["FETCH_SIZE"]["bytes"] == round(fetch) and detail["WRITE_SIZE"]["bytes"] == round(write)
    assert t == round(fetch) + round(write)


def test_measure_traffic_reports_a_missing_profiler(monkeypatch):
    import subprocess
    monkeypatch.setattr(subprocess, "run", lambda cmd, **kw: subprocess.CompletedProcess(cmd, 127))
    t, detail = bench.measure_traffic("R2", 1, (8, 4))
    assert t is None and "no result file" in detail


def test_more_than_one_gpu_is_refused_with_a_message():
    """bench.py measures one GPU: any other --gpus exits 2 with a message,
    before it touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
