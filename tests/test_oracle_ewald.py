"""Pins for the oracle's periodic sums (paper Sec. 2.1: uniform background
subtracted; periodic images beyond the nearest via a high-order local
expansion).  The Ewald form is the textbook one; the checks are closed forms
(Madelung constant, tidal trace 4 pi/3, two-body limit), symmetries (half-box
separations, perfect lattice, cubic symmetry, odd orders), alpha-independence
and brute-force lattice sums."""
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _madelung():
    vals = {}
    for line in open(os.path.join(GOLDEN, "madelung_sc.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals["xi"], vals["tolerance"]


def test_xi_matches_literature_and_is_alpha_independent():
    xi_ref, tol = _madelung()
    vals = [oracle.ewald_xi(1.0, a, 5, 14) for a in (1.5, 2.0, 3.0)]
    for v in vals:
        assert abs(v - xi_ref) < tol
    assert max(vals) - min(vals) < 1e-12
    # scales as 1/L
    assert oracle.ewald_xi(2.5, 2.0 / 2.5, 5, 14) == pytest.approx(vals[1], abs=1e-12)


def test_psi_E_alpha_independent():
    rng = np.random.default_rng(5)
    for _ in range(4):
        r = rng.random(3) - 0.5
        p1, g1 = oracle.ewald_psi(r, 1.0, 1.5, 5, 8)
        p2, g2 = oracle.ewald_psi(r, 1.0, 3.0, 3, 14)
        assert p1 == pytest.approx(p2, abs=1e-12)
        np.testing.assert_allclose(g1, g2, atol=1e-11)


def test_psi_E_cell_average_zero_and_periodic():
    """Neutralising background: psi_E has zero mean over the cell; it is
    periodic and even."""
    r = np.array([0.13, 0.41, -0.27])
    p, g = oracle.ewald_psi(r)
    p2, g2 = oracle.ewald_psi(r + np.array([1.0, -1.0, 2.0]))
    p3, g3 = oracle.ewald_psi(-r)
    assert p == pytest.approx(p2, abs=1e-12)
    assert p == pytest.approx(p3, abs=1e-13)
    np.testing.assert_allclose(g, -g3, atol=1e-12)
    # mean over a midpoint grid (the 1/r singularity is integrable; use an
    # offset grid and compare with the leading term's known integral)
    n = 24
    grid = (np.arange(n) + 0.5) / n - 0.5
    tot = 0.0
    for x in grid:
        for y in grid:
            for z in grid[::4]:
                tot += oracle.ewald_psi(np.array([x, y, z]))[0]
    assert abs(tot / (n * n * n / 4)) < 0.05


def test_psi_table_closed_forms():
    """Psi(0) L = xi - (6 + 12/sqrt2 + 8/sqrt3); d^2 Psi(0) = 4pi/(3L^3) I;
    odd orders vanish; cubic symmetry."""
    xi_ref, tol = _madelung()
    L = 1.0
    T = oracle.psi_table(16, L)
    mi = oracle.mi_list(16)
    idx = {m: i for i, m in enumerate(mi)}
    assert T[0] * L == pytest.approx(xi_ref - (6 + 12 / np.sqrt(2) + 8 / np.sqrt(3)), abs=tol)
    for e in [(2, 0, 0), (0, 2, 0), (0, 0, 2)]:
        # T_{2e_a} = (1/2) d^2 Psi / dx_a^2 = 2 pi / (3 L^3)
        assert T[idx[e]] == pytest.approx(2 * np.pi / (3 * L ** 3), rel=1e-13)
    for e in [(1, 1, 0), (1, 0, 1), (0, 1, 1)]:
        assert abs(T[idx[e]]) < 1e-13
    scale = np.max(np.abs(T))
    for m, i in idx.items():
        if sum(m) % 2:
            assert abs(T[i]) < 1e-12 * scale
        a, b, c = m
        for q in [(b, a, c), (c, b, a), (a, c, b)]:
            assert T[idx[q]] == pytest.approx(T[i], abs=1e-11 * scale)


def test_psi_table_box_scaling():
    T1 = oracle.psi_table(10, 1.0)
    L = 3.0
    T3 = oracle.psi_table(10, L)
    deg = np.array([sum(m) for m in oracle.mi_list(10)])
    np.testing.assert_allclose(T3, T1 / L ** (deg + 1), rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("deg", [8, 10])
def test_psi_table_vs_bare_lattice_sum(deg):
    """For |s| >= 3 the coefficients are absolutely convergent lattice sums
    of the bare 1/r Taylor coefficients over the images |n|_inf >= 2; compare
    with a brute-force sum to |n|_inf <= K plus its tail bound."""
    T = oracle.psi_table(deg, 1.0)
    mi = oracle.mi_list(deg)
    sel = [i for i, m in enumerate(mi) if sum(m) == deg]
    K = 12
    S = np.zeros(len(mi))
    for nx in range(-K, K + 1):
        for ny in range(-K, K + 1):
            for nz in range(-K, K + 1):
                if max(abs(nx), abs(ny), abs(nz)) < 2:
                    continue
                S += oracle.green_taylor(deg, np.array([nx, ny, nz], float), 0.0)
    # tail: sum over |n| > K of C(deg) |n|^-(deg+1) ~ 4 pi C K^(2-deg-1)/(deg-2)
    coef_bound = 3.0 ** deg  # crude bound on |T_s| * r^(deg+1) for 1/r
    tail = 4 * np.pi * coef_bound * K ** (2 - deg) / (deg - 2)
    err = np.max(np.abs(T[sel] - S[sel]))
    assert err < tail
    assert err < 1e-4 * np.max(np.abs(T[sel])) + 1e-12


def test_two_body_periodic_small_separation():
    """Two bodies at separation r << L (unsoftened): a = G m [r/|r|^3 -
    (4 pi / 3 L^3) r] + O(r^3 / L^5); the remainder scales as r^3."""
    L = 1.0
    res = []
    for r in (0.01, 0.02, 0.04):
        pos = np.array([[0.3, 0.3 + r], [0.4, 0.4], [0.5, 0.5]])
        mass = np.array([1.0, 1.0])
        acc, pot = oracle.direct_ewald(pos, mass, dict(box=L, eps=0.0), targets=[0])
        lead = 1.0 / r ** 2 - 4 * np.pi / 3 * r
        res.append(acc[0, 0] - lead)
        assert abs(acc[1, 0]) < 1e-10 and abs(acc[2, 0]) < 1e-10
    ratios = [res[1] / res[0], res[2] / res[1]]
    for q in ratios:
        assert q == pytest.approx(8.0, rel=0.02)


@pytest.mark.parametrize("sep", [(0.5, 0, 0), (0.5, 0.5, 0), (0.5, 0.5, 0.5)])
def test_half_box_separation_zero_force(sep):
    pos = np.array([[0.1, 0.1 + sep[0]], [0.2, 0.2 + sep[1]], [0.3, 0.3 + sep[2]]])
    mass = np.array([1.0, 1.0])
    acc, pot = oracle.direct_ewald(pos, mass, dict(box=1.0, eps=0.0))
    assert np.max(np.abs(acc)) < 1e-12


@pytest.mark.parametrize("n", [4, 8])
def test_perfect_lattice_zero_force_and_madelung(n):
    xi_ref, tol = _madelung()
    g = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    N = pos.shape[1]
    mass = np.full(N, 1.0 / N)
    acc, pot = oracle.direct_ewald(pos, mass, dict(box=1.0, eps=0.0))
    a_unit = (1.0 / N) * n * n  # G m / a^2
    assert np.max(np.abs(acc)) < 1e-12 * a_unit
    # phi_i = -G m xi n / L
    np.testing.assert_allclose(pot, -(1.0 / N) * xi_ref * n, rtol=2 * tol / abs(xi_ref))


def test_momentum_conservation_and_translation_invariance():
    pos, mass, prm = workloads.make("lattice16", n_side=8)
    rng = np.random.default_rng(11)
    mass = mass * (0.5 + rng.random(mass.size))
    acc, pot = oracle.direct_ewald(pos, mass, prm)
    net = np.abs(np.sum(mass * acc, axis=1))
    assert np.all(net <= 1e-13 * np.sum(mass * np.linalg.norm(acc, axis=0)))
    # with softening only on the 27 images of the wrapped positions, a shift
    # that wraps a particle changes which images are softened; unsoftened, the
    # sum is exactly periodic
    prm = dict(prm, eps=0.0)
    acc, pot = oracle.direct_ewald(pos, mass, prm)
    shift = np.array([0.137, -0.291, 0.55])[:, None]
    acc2, pot2 = oracle.direct_ewald(pos + shift, mass, prm)
    np.testing.assert_allclose(acc2, acc, atol=1e-12 * np.max(np.abs(acc)))
    np.testing.assert_allclose(pot2, pot, atol=1e-12 * np.max(np.abs(pot)))


OFFSETS = [(1, 0, 0), (1, 1, 0), (1, 1, 1), (-1, 0, 1)]


@pytest.mark.parametrize("off", OFFSETS)
def test_psi_table_at_reproduces_psi(off):
    """The table about r0 = off * L/2 must reproduce
    Psi(r) = psi_E(r) - sum_{|n|inf<=1} 1/|r + nL| near r0, with the
    truncation error falling like |h|^(D+1)."""
    L = 1.0
    r0 = np.array(off, float) * 0.5 * L
    D = 12
    T = oracle.psi_table_at(D, r0, L)
    mi = np.array(oracle.mi_list(D))

    def psi_direct(r):
        p, _ = oracle.ewald_psi(r, L, 2.0, 5, 12)
        for nx in (-1, 0, 1):
            for ny in (-1, 0, 1):
                for nz in (-1, 0, 1):
                    p -= 1.0 / np.linalg.norm(r + np.array([nx, ny, nz]) * L)
        return p

    direction = np.array([0.3, -0.5, 0.8])
    direction /= np.linalg.norm(direction)
    errs = []
    for hs in (0.1, 0.05):
        h = hs * direction
        series = np.sum(T * np.prod(h[None, :] ** mi, axis=1))
        errs.append(abs(series - psi_direct(r0 + h)))
    assert errs[0] < 1e-9
    assert errs[1] <= errs[0] + 1e-13


@pytest.mark.parametrize("off", OFFSETS)
def test_psi_table_at_symmetries(off):
    """Psi is even in each coordinate: reflecting r0 in axis a multiplies
    T_s by (-1)^{s_a}; inverting r0 multiplies it by (-1)^{|s|}."""
    L = 1.0
    D = 10
    r0 = np.array(off, float) * 0.5 * L
    T = oracle.psi_table_at(D, r0, L)
    mi = np.array(oracle.mi_list(D))
    scale = np.max(np.abs(T))
    Tm = oracle.psi_table_at(D, -r0, L)
    np.testing.assert_allclose(Tm, T * (-1.0) ** mi.sum(1), atol=1e-11 * scale)
    rx = r0 * np.array([-1, 1, 1])
    Tx = oracle.psi_table_at(D, rx, L)
    np.testing.assert_allclose(Tx, T * (-1.0) ** mi[:, 0], atol=1e-11 * scale)
    # permuting the axes of r0 permutes the multi-indices:
    # Psi(rp + h) with rp = (y0, z0, x0) equals Psi(r0 + (h3, h1, h2)), so
    # the coefficient of h^(b,c,a) about rp is that of h^(a,b,c) about r0
    rp = r0[[1, 2, 0]]
    Tp = oracle.psi_table_at(D, rp, L)
    idx = {tuple(m): i for i, m in enumerate(mi.tolist())}
    for i, (a, b, c) in enumerate(mi.tolist()):
        assert Tp[idx[(b, c, a)]] == pytest.approx(T[i], abs=1e-11 * scale)


@pytest.mark.parametrize("off", [(1, 0, 0), (1, 1, 1)])
def test_psi_table_at_vs_bare_lattice_sum(off):
    """Degree >= 3 coefficients about r0 are absolutely convergent sums of the
    bare 1/r coefficients over the images |n|_inf >= 2 (expanded about
    r0 + nL)."""
    deg = 8
    r0 = np.array(off, float) * 0.5
    T = oracle.psi_table_at(deg, r0, 1.0)
    mi = oracle.mi_list(deg)
    sel = [i for i, m in enumerate(mi) if sum(m) == deg]
    K = 12
    S = np.zeros(len(mi))
    for nx in range(-K, K + 1):
        for ny in range(-K, K + 1):
            for nz in range(-K, K + 1):
                if max(abs(nx), abs(ny), abs(nz)) < 2:
                    continue
                S += oracle.green_taylor(deg, r0 + np.array([nx, ny, nz], float), 0.0)
    tail = 4 * np.pi * 3.0 ** deg * (K - 1) ** (2 - deg) / (deg - 2)
    err = np.max(np.abs(T[sel] - S[sel]))
    assert err < tail
    assert err < 1e-4 * np.max(np.abs(T[sel])) + 1e-12
