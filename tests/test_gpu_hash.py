"""The hashed oct-tree (paper Sec. 2.1: keys translate into cell storage
through a hash table), built by every force evaluation and queried through
hot_cell_lookup: for every cell key of the oracle's tree the library returns
the cell with the same key, level, first particle and count, and for keys of
cells the tree does not have (daughters of leaves, empty octants of split
cells, random keys, key 0) it returns -1.  Bit-exact against the oracle's
key -> cell map, at small sizes and at the full 128^3 benchmark
configuration."""
import numpy as np
import pytest

import oracle
import workloads
from _gpu import operating_point, run_gpu

pytestmark = pytest.mark.gpu


def _absent_keys(cells, rng, nrand=2000):
    present = set(int(k) for k in cells["key"])
    out = set()
    for k, lvl, leaf in zip(cells["key"], cells["level"], cells["is_leaf"]):
        if lvl >= 21:
            continue
        for o in range(8):
            kk = (int(k) << 3) | o
            if kk not in present:
                out.add(kk)        # a leaf's daughter or an empty octant
    lv = rng.integers(1, 22, size=nrand)
    for lev in lv:
        kk = (1 << (3 * int(lev))) | int(rng.integers(0, 1 << (3 * int(lev)), dtype=np.uint64))
        if kk not in present:
            out.add(kk)
    out.add(0)
    return np.array(sorted(out), dtype=np.uint64)


def _check(name, ns, prm_over, precision="fp64"):
    import torch
    pos, mass, prm = workloads.make(name, n_side=ns)
    prm = dict(prm, **prm_over)
    T = oracle.Tree(pos, mass, prm)
    c = T.cells()
    r = run_gpu(pos, mass, prm, precision, lists=False)
    g, dbg = r["grav"], r["dbg"]
    keys = c["key"].astype(np.uint64)
    got = g.cell_lookup(torch.as_tensor(keys.view(np.int64), device="cuda")).cpu().numpy()
    assert np.all(got >= 0)
    np.testing.assert_array_equal(dbg["cell_key"][got], keys)
    np.testing.assert_array_equal(dbg["cell_level"][got], c["level"])
    np.testing.assert_array_equal(dbg["cell_first"][got].astype(np.int64), c["first"])
    np.testing.assert_array_equal(dbg["cell_count"][got].astype(np.int64), c["count"])
    assert len(np.unique(got)) == len(got) == len(dbg["cell_key"])
    absent = _absent_keys(c, np.random.default_rng(ns))
    miss = g.cell_lookup(torch.as_tensor(absent.view(np.int64), device="cuda")).cpu().numpy()
    assert np.all(miss == -1)
    print(f"{name} n_side={ns}: {len(keys)} cells found, {len(absent)} absent keys refused",
          flush=True)


@pytest.mark.parametrize("name,ns,over", [
    ("zeldovich128", 20, dict(leaf_max=8, group_max=32)),
    ("nfw256", 16, dict(leaf_max=4, group_max=16)),
    ("lattice16", 16, dict(leaf_max=1, group_max=8)),
])
def test_hash_matches_oracle_key_map(name, ns, over):
    _check(name, ns, over)


def test_hash_full_size_benchmark_configuration():
    _check("zeldovich128", None, operating_point("zeldovich128"), precision="fp32")


def test_hash_coincident_particles_level21():
    """Coincident particles give level-21 leaves above leaf_max: their keys
    too are found."""
    import torch
    from paper_1407_2600_amd import Gravity
    rng = np.random.default_rng(9)
    pos = rng.random((3, 2000))
    pos[:, 10:200] = pos[:, 10:11]
    mass = np.full(2000, 1 / 2000)
    prm = dict(box=1.0, G=1.0, eps=0.01, theta=0.5, order=4, periodic=1, leaf_max=8,
               group_max=32, far_order=6)
    T = oracle.Tree(pos, mass, prm)
    c = T.cells()
    assert np.any(c["level"] == 21)
    r = run_gpu(pos, mass, prm, "fp64", lists=False)
    keys = c["key"].astype(np.uint64)
    got = r["grav"].cell_lookup(torch.as_tensor(keys.view(np.int64), device="cuda")).cpu().numpy()
    np.testing.assert_array_equal(r["dbg"]["cell_key"][got], keys)
