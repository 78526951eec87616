"""Pins for the oracle's Green's-function Taylor coefficients and multipole
interactions (paper Sec. 2.1: truncated multipole expansions; quadrupole and
hexadecapole interactions near the leaves).  Each check is against a closed
form, an identity or a convergence law, never against the oracle itself."""
import numpy as np
import pytest

import oracle


def test_green_taylor_low_orders_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(5):
        R = rng.normal(size=3)
        eps = 0.3
        T = oracle.green_taylor(4, R, eps)
        mi = oracle.mi_list(4)
        u = R @ R + eps * eps
        assert T[mi.index((0, 0, 0))] == pytest.approx(u ** -0.5, rel=1e-15)
        for a, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            assert T[mi.index(e)] == pytest.approx(-R[a] / u ** 1.5, rel=1e-14)
        # second derivatives / k!
        assert T[mi.index((2, 0, 0))] == pytest.approx((3 * R[0] ** 2 - u) / (2 * u ** 2.5), rel=1e-13)
        assert T[mi.index((1, 1, 0))] == pytest.approx(3 * R[0] * R[1] / u ** 2.5, rel=1e-13)
        # d^3/dx dy dz g = -15 x y z / u^(7/2)
        assert T[mi.index((1, 1, 1))] == pytest.approx(-15 * R[0] * R[1] * R[2] / u ** 3.5, rel=1e-13)


@pytest.mark.parametrize("D", [3, 6, 9])
def test_green_taylor_reproduces_function(D):
    """sum_k T_k(R) h^k must equal g(R+h) up to O(|h|^(D+1))."""
    rng = np.random.default_rng(D)
    R = np.array([0.7, -0.4, 0.5])
    eps = 0.2
    T = oracle.green_taylor(D, R, eps)
    mi = np.array(oracle.mi_list(D))
    errs = []
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    for scale in (0.04, 0.02):
        h = scale * direction
        series = np.sum(T * np.prod(h[None, :] ** mi, axis=1))
        exact = 1.0 / np.sqrt(np.sum((R + h) ** 2) + eps * eps)
        errs.append(abs(series - exact))
    # halving |h| must shrink the truncation error by ~2^(D+1)
    assert errs[0] < 1e-5
    if errs[1] > 1e-15:
        assert errs[0] / errs[1] > 0.5 * 2 ** (D + 1)


def test_green_taylor_harmonic_when_unsoftened():
    """For eps=0, 1/r is harmonic: sum_a (k_a+1)(k_a+2) T_{k+2e_a} = 0."""
    R = np.array([0.3, 0.8, -0.6])
    D = 8
    T = oracle.green_taylor(D, R, 0.0)
    mi = oracle.mi_list(D)
    idx = {m: i for i, m in enumerate(mi)}
    worst = 0.0
    for k in oracle.mi_list(D - 2):
        s = 0.0
        scale = 0.0
        for a in range(3):
            kk = list(k)
            kk[a] += 2
            c = (k[a] + 1) * (k[a] + 2)
            s += c * T[idx[tuple(kk)]]
            scale += abs(c * T[idx[tuple(kk)]])
        if scale > 0:
            worst = max(worst, abs(s) / scale)
    assert worst < 1e-12


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4, 6])
def test_one_particle_cell_equals_direct(order):
    """A cell of one particle has only the monopole: its multipole interaction
    equals the softened pair interaction exactly, at every order."""
    pos = np.array([[0.31], [0.52], [0.27]])
    mass = np.array([0.7])
    x = np.array([0.9, -0.2, 0.4])
    eps = 0.05
    phi, g = oracle.multipole_eval(pos, mass, order, eps, x)
    d = pos[:, 0] - x
    s = np.sqrt(d @ d + eps * eps)
    assert phi == pytest.approx(mass[0] / s, rel=1e-14)
    np.testing.assert_allclose(g, mass[0] * d / s ** 3, rtol=1e-13)


@pytest.mark.parametrize("ratio", [0.5, 0.25])
def test_multipole_error_falls_with_order(ratio):
    """K particles in a cube of side s at distance d: the expansion error falls
    monotonically with p, roughly like (sqrt(3) s / (2 d))^(p+1)."""
    rng = np.random.default_rng(7)
    K = 40
    s = 1.0
    dist = s / ratio
    pos = rng.random((3, K)) * s
    mass = rng.random(K) + 0.5
    eps = 0.01
    dirs = rng.normal(size=(6, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    errs = []
    for p in range(0, 6):
        e = 0.0
        ref = 0.0
        for dvec in dirs:
            x = 0.5 * s + dist * dvec
            phi, g = oracle.multipole_eval(pos, mass, p, eps, x)
            dd = pos - x[:, None]
            r = np.sqrt(np.sum(dd ** 2, 0) + eps * eps)
            gref = np.sum(mass * dd / r ** 3, axis=1)
            e += np.sum((g - gref) ** 2)
            ref += np.sum(gref ** 2)
        errs.append(np.sqrt(e / ref))
    # dipole about the centre of mass vanishes: p=0 and p=1 agree
    assert errs[1] == pytest.approx(errs[0], rel=1e-8)
    for p in range(1, 5):
        assert errs[p + 1] < errs[p]
    bound = (np.sqrt(3) / 2 * ratio)
    # error at p=4 within a modest factor of the geometric law
    assert errs[4] < 10 * bound ** 5


def test_dipole_about_com_vanishes():
    rng = np.random.default_rng(3)
    pos = rng.random((3, 30))
    mass = rng.random(30)
    T = oracle.Tree(pos, mass, dict(box=1.0, eps=0.0, theta=0.5, order=2, periodic=0,
                                    leaf_max=4, group_max=8))
    cells = T.cells()
    mi = oracle.mi_list(2)
    for c in range(len(cells["key"])):
        M = T.cell_moments(c)
        m0 = M[mi.index((0, 0, 0))]
        assert m0 == pytest.approx(cells["mass"][c], rel=1e-14)
        for e in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
            assert abs(M[mi.index(e)]) <= 1e-14 * m0
