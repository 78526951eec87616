"""Pins for the oracle's tree (paper Sec. 2.1: Morton keys, hashed oct-tree,
sink groups sharing interaction lists, multipole acceptance test, 27-image
periodic walk plus high-order far field).  Structural facts are checked by
brute force with numpy; forces by limits (theta -> 0), exact cases and
convergence trends against the direct Ewald sum."""
import numpy as np
import pytest

import oracle
import workloads


def _deinterleave(key, level):
    ix = iy = iz = 0
    for b in range(level):
        ix |= ((key >> (3 * b + 2)) & 1) << b
        iy |= ((key >> (3 * b + 1)) & 1) << b
        iz |= ((key >> (3 * b)) & 1) << b
    return ix, iy, iz


def test_keys_known_values_and_wrap():
    L = 2.0
    pos = np.array([[0.0, L - 1e-12, L / 2, -0.5, L + 0.25],
                    [0.0, L - 1e-12, 0.0, 0.0, 0.0],
                    [0.0, L - 1e-12, 0.0, 0.0, 0.0]])
    k, w = oracle.keys(pos, L)
    assert int(k[0]) == 1 << 63
    assert int(k[1]) == (1 << 64) - 1
    # x = L/2: octant 0b100 at level 1 -> bit 62
    assert int(k[2]) == (1 << 63) | (1 << 62)
    assert w[0, 3] == L - 0.5 and w[0, 4] == 0.25


def test_keys_contain_particles_geometrically():
    rng = np.random.default_rng(2)
    L = 1.7
    pos = rng.random((3, 500)) * 3 * L - L  # needs wrapping, |x| < 2L
    k, w = oracle.keys(pos, L)
    assert np.all((w >= 0) & (w < L))
    for i in range(0, 500, 7):
        for level in (1, 5, 13, 21):
            ck = int(k[i]) >> (3 * (21 - level))
            assert ck >> (3 * level) == 1  # placeholder bit on top
            ix, iy, iz = _deinterleave(ck, level)
            s = L / 2 ** level
            for a, ia in enumerate((ix, iy, iz)):
                # quantisation is floor(x * 2^21 / L): containment up to one
                # rounding of the product
                assert ia * s <= w[a, i] * (1 + 1e-15) + 1e-300
                assert w[a, i] < (ia + 1) * s * (1 + 1e-15)


def test_sort_is_stable_key_order():
    rng = np.random.default_rng(4)
    pos = np.floor(rng.random((3, 2000)) * 8) / 8  # many equal keys
    T = oracle.Tree(pos, np.ones(2000), dict(box=1.0, leaf_max=8, group_max=16))
    perm, sk = T.perm()
    k, _ = oracle.keys(pos, 1.0)
    ref = np.lexsort((np.arange(2000), k))
    np.testing.assert_array_equal(perm, ref)
    np.testing.assert_array_equal(sk, k[ref])


@pytest.mark.parametrize("name,ns,leaf", [("zeldovich128", 12, 8), ("nfw256", 16, 16),
                                          ("lattice16", 16, 16)])
def test_cells_brute_force(name, ns, leaf):
    pos, mass, prm = workloads.make(name, n_side=ns)
    prm = dict(prm, leaf_max=leaf)
    T = oracle.Tree(pos, mass, prm)
    c = T.cells()
    perm, sk = T.perm()
    n = pos.shape[1]
    sk_int = sk.astype(np.uint64)
    seen = set()
    for i in range(len(c["key"])):
        lev = int(c["level"][i])
        key = np.uint64(c["key"][i])
        pref = sk_int >> np.uint64(3 * (21 - lev))
        members = np.nonzero(pref == key)[0]
        assert members.size == c["count"][i]
        assert members[0] == c["first"][i] and members[-1] == c["first"][i] + c["count"][i] - 1
        if c["is_leaf"][i]:
            assert c["count"][i] <= leaf or lev == 21
        else:
            assert c["count"][i] > leaf and lev < 21
        if lev > 0:
            parent = (int(key) >> 3, lev - 1)
            assert parent in seen  # pre-order: parent listed before child
        seen.add((int(key), lev))
        # centre of mass
        orig = perm[members]
        _, w = oracle.keys(pos[:, orig], 1.0)
        com = (w * mass[orig]).sum(1) / mass[orig].sum()
        np.testing.assert_allclose(c["com"][:, i], com, rtol=1e-13, atol=1e-15)
    # canonical order is (first, level)
    order = np.lexsort((c["level"], c["first"]))
    np.testing.assert_array_equal(order, np.arange(len(order)))
    # leaves partition the particles
    leaves = np.nonzero(c["is_leaf"])[0]
    assert np.sum(c["count"][leaves]) == n


def test_groups_partition_and_rule():
    pos, mass, prm = workloads.make("nfw256", n_side=16)
    prm = dict(prm, leaf_max=8, group_max=48)
    T = oracle.Tree(pos, mass, prm)
    c = T.cells()
    gcell, lo, hi = T.groups()
    firsts = c["first"][gcell]
    counts = c["count"][gcell]
    assert firsts[0] == 0
    np.testing.assert_array_equal(firsts[1:], (firsts + counts)[:-1])
    assert firsts[-1] + counts[-1] == pos.shape[1]
    key_of = {(int(k), int(l)): i for i, (k, l) in enumerate(zip(c["key"], c["level"]))}
    perm, _ = T.perm()
    _, w = oracle.keys(pos, 1.0)
    for g, ci in enumerate(gcell):
        assert c["count"][ci] <= 48 or c["is_leaf"][ci]
        if c["level"][ci] > 0:
            pi = key_of[(int(c["key"][ci]) >> 3, int(c["level"][ci]) - 1)]
            assert c["count"][pi] > 48
        idx = perm[c["first"][ci]:c["first"][ci] + c["count"][ci]]
        np.testing.assert_array_equal(lo[:, g], w[:, idx].min(1))
        np.testing.assert_array_equal(hi[:, g], w[:, idx].max(1))


def _check_lists(T, prm, check_geometry=True):
    c = T.cells()
    gcell, lo, hi = T.groups()
    n = T.n
    L = prm["box"]
    perm, _ = T.perm()
    _, w = oracle.keys(T.pos, L)
    ws = w[:, perm]
    offs = {}
    for kind in (0, 1):
        offs[kind] = T.lists(kind)
    for g in range(len(gcell)):
        A = gcell[g]
        cover = np.zeros((27, n), np.int32)
        cover[13, c["first"][A]:c["first"][A] + c["count"][A]] += 1
        for kind in (0, 1):
            off, img, cell = offs[kind]
            for e in range(off[g], off[g + 1]):
                B = cell[e]
                cover[img[e], c["first"][B]:c["first"][B] + c["count"][B]] += 1
                if kind == 0:
                    assert c["is_leaf"][B]
                if kind == 1 and check_geometry:
                    # convergence geometry: every target is farther from the
                    # expansion centre than every source of the cell
                    sh = np.array([img[e] // 9 - 1, (img[e] // 3) % 3 - 1, img[e] % 3 - 1]) * L
                    cen = c["com"][:, B] + sh
                    src = ws[:, c["first"][B]:c["first"][B] + c["count"][B]] + sh[:, None]
                    tgt = ws[:, c["first"][A]:c["first"][A] + c["count"][A]]
                    rs = np.max(np.linalg.norm(src - cen[:, None], axis=0))
                    rt = np.min(np.linalg.norm(tgt - cen[:, None], axis=0))
                    assert rt > rs
        if prm.get("periodic", 1):
            assert np.all(cover == 1)
        else:
            assert np.all(cover[13] == 1)


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7, 0.9])
def test_lists_tile_every_image_exactly_once(theta):
    pos, mass, prm = workloads.make("zeldovich128", n_side=10)
    prm = dict(prm, theta=theta, leaf_max=8, group_max=32)
    T = oracle.Tree(pos, mass, prm)
    _check_lists(T, prm)


def test_lists_open_boundary():
    pos, mass, prm = workloads.make("nfw256", n_side=10)
    prm = dict(prm, periodic=0, leaf_max=4, group_max=16)
    T = oracle.Tree(pos, mass, prm)
    _check_lists(T, prm)


def test_theta_zero_is_direct_sum():
    pos, mass, prm = workloads.make("zeldovich128", n_side=8)
    prm = dict(prm, theta=0.0, leaf_max=8, group_max=32)
    T = oracle.Tree(pos, mass, prm)
    assert T.lists(1)[1].size == 0
    a, p = T.forces()
    a0, p0 = T.direct_near_far(np.arange(pos.shape[1]))
    assert oracle.rms_rel_error(a, a0) < 1e-12
    assert oracle.rms_rel_error(p, p0) < 1e-12


def test_open_boundary_two_body_and_momentum():
    pos = np.array([[0.2, 0.7], [0.4, 0.45], [0.5, 0.55]])
    mass = np.array([0.3, 0.6])
    eps = 0.05
    T = oracle.Tree(pos, mass, dict(box=1.0, eps=eps, theta=0.5, order=4, periodic=0,
                                    leaf_max=1, group_max=1))
    a, p = T.forces()
    d = pos[:, 1] - pos[:, 0]
    s3 = (d @ d + eps * eps) ** 1.5
    np.testing.assert_allclose(a[:, 0], 0.6 * d / s3, rtol=1e-14)
    np.testing.assert_allclose(a[:, 1], -0.3 * d / s3, rtol=1e-14)
    rng = np.random.default_rng(9)
    pos = rng.random((3, 300))
    mass = rng.random(300)
    a, p = oracle.direct_open(pos, mass, 1.0, 0.01)
    net = np.abs(np.sum(mass * a, axis=1))
    assert np.all(net < 1e-13 * np.sum(mass * np.linalg.norm(a, axis=0)))
    T = oracle.Tree(pos, mass, dict(box=1.0, eps=0.01, theta=0.0, order=2, periodic=0,
                                    leaf_max=4, group_max=8))
    a2, p2 = T.forces()
    np.testing.assert_allclose(a2, a, rtol=1e-12, atol=1e-12 * np.max(np.abs(a)))


def test_far_field_converges_to_ewald():
    """theta=0 tree (27 softened images + far-field local expansions about
    the octant centres) against the exact direct Ewald sum: the truncation
    error falls with the expansion order (measured on the 16^3 set: p=4
    1.1e-3, p=6 3.8e-5, p=8 2.9e-7 -- the paper's one part in 1e7)."""
    pos, mass, prm = workloads.make("lattice16", n_side=12)
    n = pos.shape[1]
    tg = np.arange(0, n, 3)
    a1, p1 = oracle.direct_ewald(pos, mass, prm, targets=tg)
    errs = []
    for pf in (4, 6, 8):
        T = oracle.Tree(pos, mass, dict(prm, theta=0.0, far_order=pf))
        a0, p0 = T.direct_near_far(tg)
        errs.append(oracle.rms_rel_error(a0, a1))
    assert all(errs[i + 1] < errs[i] for i in range(2))
    assert errs[-1] < 2e-6


def test_tree_error_falls_with_theta_and_order():
    pos, mass, prm = workloads.make("zeldovich128", n_side=14)
    n = pos.shape[1]
    T0 = oracle.Tree(pos, mass, dict(prm, theta=0.0))
    a0, _ = T0.direct_near_far(np.arange(n))
    errs = {}
    for order in (2, 4):
        for th in (0.3, 0.5, 0.7):
            T = oracle.Tree(pos, mass, dict(prm, theta=th, order=order))
            a, _ = T.forces()
            errs[(order, th)] = oracle.rms_rel_error(a, a0)
    for order in (2, 4):
        assert errs[(order, 0.3)] < errs[(order, 0.5)] < errs[(order, 0.7)]
    for th in (0.3, 0.5, 0.7):
        assert errs[(4, th)] < errs[(2, th)]
    assert errs[(4, 0.5)] < 1e-3


def test_perfect_lattice_tree_residual():
    """A perfect lattice feels no force; the tree's residual is pure
    approximation error and falls as theta decreases."""
    n = 8
    g = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    N = pos.shape[1]
    mass = np.full(N, 1.0 / N)
    res = []
    for th in (0.7, 0.5, 0.3):
        T = oracle.Tree(pos, mass, dict(box=1.0, eps=0.0, theta=th, order=4, leaf_max=8,
                                        group_max=8, far_order=8))
        a, p = T.forces()
        res.append(np.max(np.abs(a)) / ((1.0 / N) * n * n))
    assert res[2] < res[1] < res[0] < 1e-2


def test_tree_potential_matches_ewald():
    """The tree's potential against the exact periodic sum (the plain
    definition, pinned itself by the Madelung constant): the 27-image softened
    sum plus the far field about the octant centres reaches the direct Ewald
    potential to the far-field floor, for targets in every octant.  This pins
    the far field's constant terms (one per octant pair, which enter the
    potential alone) and the self-image term Psi(0) carried by the octant
    moments (paper Sec. 2.1: periodic local expansion, background
    subtraction)."""
    pos, mass, prm = workloads.make("lattice16", n_side=12)
    n = pos.shape[1]
    tg = np.arange(0, n, 3)
    a1, p1 = oracle.direct_ewald(pos, mass, prm, targets=tg)
    errs = []
    for pf in (4, 6, 8):
        T = oracle.Tree(pos, mass, dict(prm, theta=0.0, far_order=pf))
        _, p0 = T.direct_near_far(tg)
        errs.append(oracle.rms_rel_error(p0, p1))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= 1e-6
    # the whole tree pipeline at theta = 0 (walk, direct lists, far field)
    T = oracle.Tree(pos, mass, dict(prm, theta=0.0, far_order=8))
    _, pt = T.forces()
    assert oracle.rms_rel_error(pt[tg], p1) <= 1e-6
    # every octant holds targets and sources
    octs = (pos[0, tg] >= 0.5) * 4 + (pos[1, tg] >= 0.5) * 2 + (pos[2, tg] >= 0.5)
    assert len(np.unique(octs)) == 8


@pytest.mark.parametrize("n", [4, 8])
def test_perfect_lattice_potential_is_madelung(n):
    """Unsoftened simple-cubic lattice of n^3 equal masses m: every particle
    has phi = -G m xi n / L (xi the lattice's self constant, from the
    literature); the theta = 0 tree reaches it to the far-field floor and the
    tree at theta > 0 to its own (small, falling) approximation error."""
    xi = -2.837297479
    g = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    N = pos.shape[1]
    m = 1.0 / N
    want = -m * xi * n
    prm = dict(box=1.0, G=1.0, eps=0.0, order=4, leaf_max=8, group_max=8, far_order=8)
    T = oracle.Tree(pos, np.full(N, m), dict(prm, theta=0.0))
    _, p0 = T.direct_near_far(np.arange(N))
    assert np.max(np.abs(p0 - want)) <= 1e-7 * abs(want)
    res = []
    for th in (0.7, 0.5, 0.3):
        _, p = oracle.Tree(pos, np.full(N, m), dict(prm, theta=th)).forces()
        res.append(np.max(np.abs(p - want)) / abs(want))
    assert res[2] < res[1] < res[0] < 1e-2


def test_pair_count_closed_form_and_lists():
    """Direct pairs: at theta = 0 every (target, source image) pair but the
    self pair is direct, N (27 N - 1) periodic and N (N - 1) open; at theta >
    0 the count equals the sum over groups of targets x (own sources + listed
    leaves' sources), counted from the lists by brute force."""
    pos, mass, prm = workloads.make("nfw256", n_side=8)
    n = pos.shape[1]
    for periodic, want in ((1, n * (27 * n - 1)), (0, n * (n - 1))):
        T = oracle.Tree(pos, mass, dict(prm, theta=0.0, periodic=periodic, leaf_max=8,
                                        group_max=32))
        assert T.pair_count() == want
    T = oracle.Tree(pos, mass, dict(prm, theta=0.5, leaf_max=8, group_max=32))
    c = T.cells()
    gcell, _, _ = T.groups()
    off, _, cell = T.lists(0)
    want = 0
    for g, A in enumerate(gcell):
        src = c["count"][A] - 1 + int(np.sum(c["count"][cell[off[g]:off[g + 1]]]))
        want += int(c["count"][A]) * src
    assert T.pair_count() == want


def test_far_field_moments_and_local_coefficients():
    """Octant moments M^o_k = sum_{j in o} m_j (x_j - c_o)^k by brute force,
    and the local coefficients of one particle: sum_q Lam_q h^q at a target
    in every octant equals m Psi(x - y), the Ewald potential minus the 27
    nearest bare images, to the order-8 truncation."""
    rng = np.random.default_rng(31)
    pos = rng.random((3, 200))
    mass = rng.random(200)
    prm = dict(box=1.0, G=1.0, eps=0.0, theta=0.5, order=2, leaf_max=8, group_max=16,
               far_order=6)
    T = oracle.Tree(pos, mass, prm)
    _, M, _ = T.far()
    mi = oracle.mi_list(6)
    octs = (pos[0] >= 0.5) * 4 + (pos[1] >= 0.5) * 2 + (pos[2] >= 0.5)
    for o in range(8):
        cen = 0.25 + 0.5 * np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1])
        d = pos[:, octs == o] - cen[:, None]
        want = [np.sum(mass[octs == o] * d[0] ** a * d[1] ** b * d[2] ** cc) for a, b, cc in mi]
        np.testing.assert_allclose(M[o], want, rtol=1e-12, atol=1e-14)
    # one source particle: the local coefficients reproduce m Psi
    y = np.array([0.31, 0.72, 0.44])
    m = 0.7
    T1 = oracle.Tree(y[:, None], np.array([m]), dict(prm, far_order=8))
    _, _, Lam = T1.far()
    mi8 = oracle.mi_list(8)
    for o in range(8):
        cen = 0.25 + 0.5 * np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1])
        x = cen + np.array([0.11, -0.07, 0.09])
        h = x - cen
        phi = sum(Lam[o, k] * h[0] ** a * h[1] ** b * h[2] ** cc for k, (a, b, cc) in
                  enumerate(mi8))
        r = x - y
        psi_e, _ = oracle.ewald_psi(r)
        bare = sum(1.0 / np.linalg.norm(r + np.array([i, j, k]))
                   for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1))
        assert phi == pytest.approx(m * (psi_e - bare), rel=1e-6, abs=1e-7)
