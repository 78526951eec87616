"""Pins for the oracle's error-bound acceptance test (the paper sets its
tolerance as an absolute acceleration error, Sec. 2.1; the bound is Salmon &
Warren's for a truncated multipole expansion).  The radius solver is checked
against the bound's definition and its far limit, the bound itself against
real truncation errors of random clusters at every order, and the per-cell
second moments and extents against brute force."""
import numpy as np
import pytest

import oracle
import workloads

from test_oracle_tree import _check_lists


def _f(G, bp, b, p, r):
    """Salmon & Warren's bound for B_(pe+1) = bp, pe = max(p, 1)."""
    pe = max(p, 1)
    return G * bp * ((pe + 2) * r - (pe + 1) * b) / (r ** (pe + 2) * (r - b) ** 2)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_err_radius_is_the_smallest_radius_meeting_the_bound(p):
    rng = np.random.default_rng(p)
    for _ in range(20):
        b = 10 ** rng.uniform(-4, -1)
        bp = 10 ** rng.uniform(-3, 0) * b ** (max(p, 1) + 1)
        tol = 10 ** rng.uniform(-6, -2)
        rc = oracle.err_radius(1.0, bp, b, p, tol)
        assert rc > b
        assert _f(1.0, bp, b, p, rc) <= tol * (1 + 1e-12)
        assert _f(1.0, bp, b, p, rc * (1 - 1e-9)) > tol


def test_err_radius_limits():
    # point mass: exact at any distance beyond its extent
    assert oracle.err_radius(1.0, 0.0, 0.0, 4, 1e-3) == 0.0
    assert oracle.err_radius(1.0, 0.0, 0.25, 4, 1e-3) == 0.25
    # b -> 0 with B_(p+1) fixed (order 1, B_2): r = (3 G B_2 / tol)^(1/4)
    r = oracle.err_radius(2.0, 0.3, 1e-9, 1, 1e-4)
    assert r == pytest.approx((3 * 2.0 * 0.3 / 1e-4) ** 0.25, rel=1e-6)
    # larger tolerance, smaller radius; order 0 is treated as order 1
    assert oracle.err_radius(1.0, 1e-4, 0.02, 4, 1e-2) < oracle.err_radius(1.0, 1e-4, 0.02, 4,
                                                                          1e-4)
    assert oracle.err_radius(1.0, 1e-4, 0.02, 0, 1e-3) == oracle.err_radius(1.0, 1e-4, 0.02, 1,
                                                                           1e-3)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_bound_holds_for_random_clusters(p):
    """At the opening radius, the actual acceleration error of the order-p
    expansion (eps = 0) is below the tolerance in every direction, and not
    vastly below it (the bound is tight to a modest factor)."""
    rng = np.random.default_rng(100 + p)
    worst = 0.0
    for trial in range(6):
        k = 40
        src = rng.random((3, k)) * 0.1
        if trial % 2:
            src[:, :10] *= 0.2  # a dense core
        m = rng.random(k) + 0.1
        com = (src * m).sum(1) / m.sum()
        d = src - com[:, None]
        r2 = (d * d).sum(0)
        # the cell's actual B_(p+1) (order 0 counts as order 1)
        bp = float((m * np.sqrt(r2) ** (max(p, 1) + 1)).sum())
        b = float(np.sqrt(r2.max()))
        tol = 1e-3 * m.sum() / 0.1 ** 2
        rc = oracle.err_radius(1.0, bp, b, p, tol)
        for _ in range(60):
            u = rng.normal(size=3)
            x = com + rc * (1 + 1e-12) * u / np.linalg.norm(u)
            allp = np.concatenate([src, x[:, None]], axis=1)
            allm = np.concatenate([m, [0.0]])
            acc, _ = oracle.direct_open(allp, allm, 1.0, 0.0)
            _, g = oracle.multipole_eval(src, m, p, 0.0, x)
            err = np.linalg.norm(acc[:, -1] - g)  # g: gradient of sum m/r
            assert err <= tol
            worst = max(worst, err / tol)
    assert worst > 1e-3


@pytest.mark.parametrize("name,ns", [("zeldovich128", 10), ("nfw256", 12)])
def test_cell_bounds_brute_force(name, ns):
    pos, mass, prm = workloads.make(name, n_side=ns)
    prm = dict(prm, err_tol=1e-3, theta=0.0, leaf_max=8)
    T = oracle.Tree(pos, mass, prm)
    cells = T.cells()
    b2, bm = T.cell_bounds()
    perm, _ = T.perm()
    sp = np.asarray(pos)[:, perm]
    sm = np.asarray(mass)[perm]
    bk = [T.cell_bk(k) for k in range(6)]
    for c in range(len(b2)):
        f, n = cells["first"][c], cells["count"][c]
        d = sp[:, f:f + n] - cells["com"][:, c][:, None]
        r2 = (d * d).sum(0)
        ref = float((sm[f:f + n] * r2).sum())
        assert b2[c] == pytest.approx(ref, rel=1e-11, abs=1e-300)
        assert bm[c] >= np.sqrt(r2.max()) * (1 - 1e-14)
        if cells["is_leaf"][c]:
            assert bm[c] == np.sqrt(r2.max())
        # B_k: exact for k = 0, 2 and at leaves, an upper bound elsewhere,
        # and never looser than the extent bound b^(k-2) B_2
        for k in range(6):
            exact = float((sm[f:f + n] * np.sqrt(r2) ** k).sum())
            if k in (0, 2) or cells["is_leaf"][c]:
                assert bk[k][c] == pytest.approx(exact, rel=1e-11, abs=1e-300)
            else:
                assert bk[k][c] >= exact * (1 - 1e-12)
            if k > 2:
                assert bk[k][c] <= b2[c] * bm[c] ** (k - 2) * (1 + 1e-12) or \
                    not cells["is_leaf"][c]


def test_opening_radius_combines_both_tests():
    pos, mass, prm = workloads.make("nfw256", n_side=10)
    base = dict(prm, leaf_max=8, group_max=32)
    for theta, tol in ((0.0, 1e-3), (0.6, 1e-3), (0.6, 0.0)):
        T = oracle.Tree(pos, mass, dict(base, theta=theta, err_tol=tol))
        cells = T.cells()
        b2, bm = T.cell_bounds()
        for c in range(0, len(b2), 7):
            side = 1.0 / 2 ** cells["level"][c]
            ctr = np.array([((k + 0.5) * side) for k in _cell_xyz(cells["key"][c],
                                                                      cells["level"][c])])
            geo = side / theta + np.linalg.norm(cells["com"][:, c] - ctr) if theta > 0 else 0.0
            bp = T.cell_bk(max(base["order"], 1) + 1)[c]
            err = oracle.err_radius(1.0, bp, bm[c], base["order"], tol) if tol > 0 else 0.0
            assert cells["rcrit"][c] == pytest.approx(max(geo, err), rel=1e-14)
        _check_lists(T, dict(base, theta=theta, err_tol=tol))


def _cell_xyz(key, level):
    key = int(key)
    ix = iy = iz = 0
    for b in range(level):
        ix |= ((key >> (3 * b + 2)) & 1) << b
        iy |= ((key >> (3 * b + 1)) & 1) << b
        iz |= ((key >> (3 * b)) & 1) << b
    return ix, iy, iz


def test_tree_error_falls_with_tolerance():
    pos, mass, prm = workloads.make("nfw256", n_side=12)
    n = pos.shape[1]
    a0, _ = oracle.Tree(pos, mass, dict(prm, theta=0.0)).direct_near_far(np.arange(n))
    errs = []
    for tol in (1e-2, 1e-3, 1e-4):
        T = oracle.Tree(pos, mass, dict(prm, theta=0.0, err_tol=tol))
        a, _ = T.forces()
        errs.append(oracle.rms_rel_error(a, a0))
    assert errs[0] > errs[1] > errs[2]
