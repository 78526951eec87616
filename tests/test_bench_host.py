"""Host logic of bench.py that needs no GPU: the one-GPU refusal, the
per-workload launch defaults, and the guard that reports the HBM traffic of
the dominant kernel only for the sources and configuration it was measured
with."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_workload_defaults():
    b = _bench()
    for name, op in b.OPERATING_POINT.items():
        assert 1 <= op["leaf_max"] <= 255 and op["leaf_max"] <= op["group_max"] <= 4096
        assert 0 <= op["theta"] < 1 and op["err_tol"] >= 0
        assert name in b.ETA_GRID and len(b.ETA_GRID[name]) > 0
    for name, w in b.WORKLOADS.items():
        assert os.path.exists(os.path.join(ROOT, "tests", "golden", w["ref"]))
        if w["heldout"]:
            assert os.path.exists(os.path.join(ROOT, "tests", "golden", w["heldout"]))
    # each counter record was taken at its workload's operating point
    for t in b.TRAFFIC:
        op = b.OPERATING_POINT[t["workload"]]
        assert all(op[k] == t["config"][k] for k in op)


def test_heldout_targets_are_disjoint_from_selection():
    """The 128^3 held-out targets share none with the 10^4 selection targets
    the operating point was chosen on."""
    import numpy as np
    g = os.path.join(ROOT, "tests", "golden")
    sel = np.load(os.path.join(g, "zeldovich128_ref.npz"))["targets"]
    held = np.load(os.path.join(g, "zeldovich128_heldout.npz"))["targets"]
    assert len(held) >= 1000
    assert len(np.intersect1d(sel, held)) == 0


@pytest.mark.parametrize("rec", [0, -1])
def test_traffic_reported_only_for_its_configuration(rec):
    import hashlib
    b = _bench()
    t = b.TRAFFIC[rec]
    prm = dict(t["config"], box=1.0, G=1.0, periodic=1)
    wl = t["workload"]
    h = hashlib.sha256()
    for f in b.TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1407_2600_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    saved = t["sha256"]
    try:
        if h.hexdigest() != saved:
            # sources changed since the counter runs: nothing is reported
            assert b.measured_traffic(prm, wl) is None
            t["sha256"] = h.hexdigest()
        assert b.measured_traffic(prm, wl) == t["bytes_per_eval"]
        assert b.measured_traffic(dict(prm, group_max=prm["group_max"] * 2), wl) is None
        assert b.measured_traffic(dict(prm, err_tol=prm["err_tol"] * 1.5), wl) is None
        assert b.measured_traffic(prm, "nfw256") is None
        t["sha256"] = "0" * 64  # sources changed since the counter runs
        assert b.measured_traffic(prm, wl) is None
    finally:
        t["sha256"] = saved
