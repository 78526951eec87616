"""Pins for the oracle's adjoint (vector-Jacobian product of the forces with
respect to positions and masses; an extension beyond the paper).  At theta=0
the gather-form adjoint is the exact derivative of the 27-image + far-field
sum, checked against central finite differences of the oracle's own forward
and by the adjoint dot-product identity; for theta > 0 its error against the
exact derivative falls with theta and with the multipole order."""
import numpy as np
import pytest

import oracle
import workloads


def _setup(n_side=5, **over):
    pos, mass, prm = workloads.make("zeldovich128", n_side=n_side)
    n = pos.shape[1]
    rng = np.random.default_rng(0)
    mass = mass * (0.5 + rng.random(n))
    prm = dict(prm, **dict(dict(theta=0.0, leaf_max=4, group_max=8, far_order=6), **over))
    ga = rng.normal(size=(3, n))
    gp = rng.normal(size=n)
    return pos, mass, prm, ga, gp


def _loss(pos, mass, prm, ga, gp):
    a, ph = oracle.Tree(pos, mass, prm).forces()
    return np.sum(ga * a) + np.sum(gp * ph)


@pytest.mark.parametrize("periodic", [1, 0])
def test_vjp_matches_finite_differences(periodic):
    pos, mass, prm, ga, gp = _setup(periodic=periodic)
    xb, mb = oracle.Tree(pos, mass, prm).vjp(ga, gp)
    h = 1e-6
    for a, k in [(0, 3), (1, 17), (2, 60), (0, 100), (1, 124)]:
        pp = pos.copy()
        pp[a, k] += h
        pm = pos.copy()
        pm[a, k] -= h
        fd = (_loss(pp, mass, prm, ga, gp) - _loss(pm, mass, prm, ga, gp)) / (2 * h)
        assert xb[a, k] == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.max(np.abs(xb)))
    for k in (5, 77):
        dm = 1e-7 * mass[k]
        mp = mass.copy()
        mp[k] += dm
        mm = mass.copy()
        mm[k] -= dm
        fd = (_loss(pos, mp, prm, ga, gp) - _loss(pos, mm, prm, ga, gp)) / (2 * dm)
        assert mb[k] == pytest.approx(fd, rel=1e-6)


def test_vjp_dot_product_identity():
    """<gacc, J v> (by a central difference along v) equals <xbar, v>."""
    pos, mass, prm, ga, gp = _setup()
    rng = np.random.default_rng(4)
    v = rng.normal(size=pos.shape)
    xb, _ = oracle.Tree(pos, mass, prm).vjp(ga, gp)
    h = 1e-7
    fd = (_loss(pos + h * v, mass, prm, ga, gp) - _loss(pos - h * v, mass, prm, ga, gp)) / (2 * h)
    assert np.sum(xb * v) == pytest.approx(fd, rel=1e-6)


def test_tree_vjp_error_falls_with_theta_and_order():
    pos, mass, prm, ga, gp = _setup(n_side=8)
    x0, m0 = oracle.Tree(pos, mass, prm).vjp(ga, gp)
    errs = {}
    for order in (2, 4):
        for th in (0.3, 0.5, 0.7):
            xb, mb = oracle.Tree(pos, mass, dict(prm, theta=th, order=order)).vjp(ga, gp)
            errs[(order, th)] = (oracle.rms_rel_error(xb, x0), oracle.rms_rel_error(mb, m0))
    for order in (2, 4):
        for k in (0, 1):
            assert errs[(order, 0.3)][k] < errs[(order, 0.5)][k] < errs[(order, 0.7)][k]
    for th in (0.3, 0.5):
        assert errs[(4, th)][0] < errs[(2, th)][0]
    assert errs[(4, 0.5)][0] < 1e-3


def test_vjp_sampled_groups_agree_with_full():
    pos, mass, prm, ga, gp = _setup(n_side=6, theta=0.5)
    T = oracle.Tree(pos, mass, prm)
    xb, mb = T.vjp(ga, gp)
    gsel = [0, 3, 7]
    xs, ms = oracle.Tree(pos, mass, prm).vjp(ga, gp, groups=gsel)
    sel = ~np.isnan(ms)
    assert sel.sum() > 0
    np.testing.assert_allclose(xs[:, sel], xb[:, sel], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ms[sel], mb[sel], rtol=1e-13, atol=1e-13)
