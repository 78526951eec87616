"""Pins of the oracle's Dehnen K1 softening (paper Sec. 2.1: the compensating
smoothing kernel used for small-scale force softening).  The paper names the
kernel and gives no form; the oracle reads it as the compact density
rho ~ (1 - x^2)^2 (1 - 11 x^2/5), x = r/h < 1, with h = (945/256) eps for the
"Plummer equivalent" softening eps.  These tests check that reading through
what it must satisfy, from the oracle's pair function alone: unit mass
(exactly Newtonian beyond h), zero second moment (compensating), continuity
at h, potential and force consistent, the Plummer-equivalent central
potential; then the tree built on it: theta = 0 equals the direct sum, every
accepted cell lies beyond the kernel radius, and the tree error falls with
theta."""
import numpy as np
import pytest

import oracle
import workloads

EPS = 0.01


def _M(r, eps=EPS):
    """enclosed kernel mass at r from the pair force: a = -G m r f, and the
    enclosed mass of a unit point mass spread by the kernel is r^3 f"""
    g, f = oracle.pair_kernel("k1", r * r, eps)
    return r ** 3 * f


def test_exactly_newtonian_beyond_radius():
    h = oracle.k1_radius(EPS)
    assert h == pytest.approx(945.0 / 256.0 * EPS, rel=1e-15)
    for r in (h * (1 + 1e-12), 1.5 * h, 3.0 * h, 17.0 * h):
        g, f = oracle.pair_kernel("k1", r * r, EPS)
        assert g == pytest.approx(1.0 / r, rel=1e-14)
        assert f == pytest.approx(1.0 / r ** 3, rel=1e-14)


def test_unit_mass_and_continuity_at_radius():
    h = oracle.k1_radius(EPS)
    # the enclosed mass reaches exactly 1 at the radius, from inside
    assert _M(h * (1 - 1e-12)) == pytest.approx(1.0, rel=1e-9)
    gi, fi = oracle.pair_kernel("k1", (h * (1 - 1e-12)) ** 2, EPS)
    assert gi == pytest.approx(1.0 / h, rel=1e-9)
    assert fi == pytest.approx(1.0 / h ** 3, rel=1e-9)


def test_compensating_second_moment_vanishes():
    """int rho r^2 dV = int_0^h r^2 dM = h^2 M(h) - 2 int_0^h r M(r) dr = 0,
    by Gauss-Legendre quadrature of the enclosed mass taken from the force;
    the plain (uncompensated) (1 - x^2)^2 kernel would leave 1/9 h^2."""
    h = oracle.k1_radius(EPS)
    x, w = np.polynomial.legendre.leggauss(40)
    r = 0.5 * h * (x + 1.0)
    I = 0.5 * h * float(np.sum(w * r * np.array([_M(v) for v in r])))
    assert abs(h * h - 2.0 * I) <= 1e-12 * h * h
    # and its density is negative beyond sqrt(5/11) h (the compensating part):
    # dM/dr changes sign there
    dr = 1e-7 * h
    def dM(v):
        return (_M(v + dr) - _M(v - dr)) / (2 * dr)
    assert dM(0.5 * h) > 0 and dM(0.8 * h) < 0
    assert abs(dM(np.sqrt(5.0 / 11.0) * h)) < 1e-6 / h


def test_potential_is_integral_of_force_and_plummer_equivalent():
    h = oracle.k1_radius(EPS)
    for r in (0.1 * h, 0.37 * h, 0.8 * h, 0.999 * h):
        d = 1e-6 * h
        gp, _ = oracle.pair_kernel("k1", (r + d) ** 2, EPS)
        gm, _ = oracle.pair_kernel("k1", (r - d) ** 2, EPS)
        _, f = oracle.pair_kernel("k1", r * r, EPS)
        # -dg/dr = r f
        assert -(gp - gm) / (2 * d) == pytest.approx(r * f, rel=1e-7)
    g0, f0 = oracle.pair_kernel("k1", 0.0, EPS)
    assert g0 == pytest.approx(1.0 / EPS, rel=1e-14)     # Plummer's central potential
    gp, fp = oracle.pair_kernel("plummer", 0.0, EPS)
    assert g0 == pytest.approx(gp, rel=1e-14)
    assert np.isfinite(f0) and f0 > 0


def _k1_case(ns=12, **over):
    pos, mass, prm = workloads.make("zeldovich128", n_side=ns)
    prm = dict(prm, kernel="k1", leaf_max=8, group_max=32, **over)
    return pos, mass, prm


def test_tree_theta_zero_is_direct_sum_k1():
    pos, mass, prm = _k1_case(theta=0.0)
    T = oracle.Tree(pos, mass, prm)
    a, p = T.forces()
    a0, p0 = T.direct_near_far(np.arange(pos.shape[1]))
    assert oracle.rms_rel_error(a, a0) < 1e-13
    # the potential: a sum of same-signed terms the far field cancels
    # (summation order differs between the two)
    assert oracle.rms_rel_error(p, p0) < 1e-11
    # open boundaries: the plain K1 direct sum
    po = dict(prm, periodic=0)
    To = oracle.Tree(pos, mass, po)
    ao, pt = To.forces()
    ad, pd = oracle.direct_open(pos, mass, 1.0, prm["eps"], kernel="k1")
    assert oracle.rms_rel_error(ao, ad) < 1e-13


def test_k1_changes_only_the_near_pairs():
    """K1 and Plummer differ only for pairs closer than the K1 radius: with
    every pair farther apart, the two direct sums agree to the Plummer
    softening's own far-field deviation."""
    rng = np.random.default_rng(3)
    pos = rng.random((3, 300))
    mass = rng.random(300)
    eps = 1e-4  # h = 3.7e-4, far below the typical separation
    d = pos[:, :, None] - pos[:, None, :]
    r = np.sqrt(np.sum(d ** 2, 0)) + np.eye(300)
    assert r.min() > oracle.k1_radius(eps)
    a1, _ = oracle.direct_open(pos, mass, 1.0, eps, kernel="k1")
    a0, _ = oracle.direct_open(pos, mass, 1.0, 0.0)
    assert oracle.rms_rel_error(a1, a0) < 1e-13


def test_accepted_cells_lie_beyond_kernel_radius():
    pos, mass, prm = _k1_case(theta=0.7)
    prm["eps"] = 0.5 / 12  # a large kernel, so that the separation term decides
    T = oracle.Tree(pos, mass, prm)
    T.forces()
    c = T.cells()
    b2, bmax = T.cell_bounds()
    h = oracle.k1_radius(prm["eps"])
    gcell, lo, hi = T.groups()
    L = prm["box"]
    nacc = 0
    for g in range(len(gcell)):
        img, cell = T.group_list(g, 1)
        for i, B in zip(img, cell):
            n = np.array([i // 9 - 1, (i // 3) % 3 - 1, i % 3 - 1])
            ctr = c["com"][:, B] + n * L
            dd = np.maximum(0.0, np.maximum(lo[:, g] - ctr, ctr - hi[:, g]))
            assert np.sqrt(np.sum(dd ** 2)) > bmax[B] + h
            nacc += 1
    assert nacc > 0


def test_k1_tree_error_falls_with_theta():
    pos, mass, prm = _k1_case()
    a0, _ = oracle.Tree(pos, mass, dict(prm, theta=0.0)).forces()
    errs = [oracle.rms_rel_error(oracle.Tree(pos, mass, dict(prm, theta=th)).forces()[0], a0)
            for th in (0.8, 0.6, 0.4)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3
