"""Pins of the oracle's group-level local expansions (the dual-tree route of
paper Sec. 2.1: source cells bundled with the sinks of a sink group; here a
cell far from the whole group is re-expanded once about the group's centre).

The route expands the Newtonian kernel.  It must reproduce what the cell's
multipole expansion gives, up to a truncation and a softening difference that
the acceptance bound controls:
- at the expansion centre, orders 0 and 1 of the local expansion are the
  multipole field's value and gradient there (no truncation yet), and order
  2 holds its Hessian (checked against finite differences of the multipole
  gradient);
- the local expansion converges to the multipole field as its order grows,
  geometrically in (group radius / distance);
- for a point mass (where the multipole field is exact) the acceleration
  error never exceeds the truncation bound the walk uses, and against the
  Plummer-softened field the truncation bound plus 1.5 G m eps^2 / (u-a)^4;
- in the tree, the local list and the multipole list together are exactly
  the multipole list without local expansions, and the forces move by no
  more than the bound summed over the group's local cells."""
import numpy as np
import pytest

import oracle
import workloads

RNG = np.random.default_rng(77)


def _cluster(n, scale=0.05, centre=(0.0, 0.0, 0.0), rng=RNG):
    pos = rng.normal(0.0, scale, (3, n)) + np.array(centre)[:, None]
    mass = rng.uniform(0.5, 1.5, n)
    return pos, mass


def _bound(m, a, u, q, G=1.0, eps=0.0):
    """Acceleration bound of the order-q truncation for mass m whose
    particles are all at least u from the centre, sinks within a of it, plus
    the change of leaving out Plummer softening eps."""
    t = a / u
    return (G * m * t ** q * ((q + 2) - (q + 1) * t) / (u * u * (1 - t) ** 2) +
            1.5 * G * m * eps ** 2 / (u - a) ** 4)


@pytest.mark.parametrize("order", [0, 2, 4])
@pytest.mark.parametrize("q", [0, 1, 2, 4])
def test_value_and_gradient_at_centre(order, q):
    pos, mass = _cluster(20)
    c = np.array([2.0, -1.2, 0.7])
    phi_l, g_l = oracle.local_eval(pos, mass, order, q, 0.01, c, c)
    phi_m, g_m = oracle.multipole_eval(pos, mass, order, 0.01, c)
    assert abs(phi_l - phi_m) <= 1e-13 * abs(phi_m)
    if q >= 1:
        np.testing.assert_allclose(g_l, g_m, rtol=1e-12, atol=1e-15 * np.abs(g_m).max())
    else:
        assert np.all(g_l == 0.0)


@pytest.mark.parametrize("order", [2, 4])
def test_hessian_at_centre(order):
    """Order 2: the local gradient is linear in y, so its difference quotient
    is the Hessian exactly; it must match central differences of the
    multipole gradient."""
    pos, mass = _cluster(15)
    c = np.array([1.5, 0.9, -1.1])
    h = 1e-4
    _, g0 = oracle.local_eval(pos, mass, order, 2, 0.0, c, c)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        _, gl = oracle.local_eval(pos, mass, order, 2, 0.0, c, c + e)
        _, gp = oracle.multipole_eval(pos, mass, order, 0.0, c + e)
        _, gm = oracle.multipole_eval(pos, mass, order, 0.0, c - e)
        H_loc = (gl - g0) / h
        H_fd = (gp - gm) / (2 * h)
        np.testing.assert_allclose(H_loc, H_fd, rtol=1e-6, atol=1e-8 * np.abs(H_fd).max())


def test_converges_to_multipole_field_with_order():
    """Sinks within a = 0.3 of the centre, the cell 2 away: the error of the
    local route against the multipole field falls at least like (a/u)^q."""
    pos, mass = _cluster(30, scale=0.04)
    c = np.array([2.0, 0.0, 0.0])
    rng = np.random.default_rng(5)
    xs = []
    while len(xs) < 40:
        y = rng.uniform(-0.3, 0.3, 3)
        if np.linalg.norm(y) <= 0.3:
            xs.append(c + y)
    errs = []
    for q in (2, 4, 6, 8, 10):
        e = 0.0
        for x in xs:
            _, gl = oracle.local_eval(pos, mass, 4, q, 0.0, c, x)
            _, gm = oracle.multipole_eval(pos, mass, 4, 0.0, x)
            e = max(e, np.linalg.norm(gl - gm))
        errs.append(e)
    t = 0.3 / (2.0 - 0.2)
    for i in range(len(errs) - 1):
        assert errs[i + 1] < errs[i] * 6 * t ** 2, errs
    assert errs[-1] < 1e-6 * np.linalg.norm(oracle.multipole_eval(pos, mass, 4, 0.0, c)[1])


@pytest.mark.parametrize("eps_frac", [0.0, 0.05, 0.2])
@pytest.mark.parametrize("q", [1, 2, 4, 6])
def test_point_mass_error_within_bound(q, eps_frac):
    """One particle: the multipole field is exact, and the acceleration error
    of the (Newtonian) local route against the particle's Plummer-softened
    field is at most the truncation bound plus the softening term, for sinks
    anywhere in the ball of radius a."""
    rng = np.random.default_rng(100 + q)
    worst = 0.0
    for _ in range(300):
        z = rng.normal(0, 1, 3)
        m = rng.uniform(0.1, 2.0)
        c = np.zeros(3)
        u = np.linalg.norm(z)
        a = u * rng.uniform(0.05, 0.6)
        eps = eps_frac * (u - a)
        y = rng.normal(0, 1, 3)
        y *= a * rng.uniform(0, 1) ** (1 / 3) / np.linalg.norm(y)
        _, gl = oracle.local_eval(z[:, None], np.array([m]), 0, q, 0.0, c, c + y)
        d = z - (c + y)
        g_exact = m * d / (d @ d + eps * eps) ** 1.5
        err = np.linalg.norm(gl - g_exact)
        b = _bound(m, a, u, q, eps=eps)
        assert err <= b * (1 + 1e-9) + 1e-15, (err, b)
        worst = max(worst, err / b)
    assert worst > 1e-3  # the bound is not vacuous


def _small_tree(local_order, local_tol, err_tol=None, ns=16):
    pos = workloads.zeldovich(ns, 1002, rms_frac=0.5)
    n = pos.shape[1]
    mass = np.full(n, 1.0 / n)
    prm = dict(box=1.0, G=1.0, eps=0.02 / ns, order=4, leaf_max=8, group_max=32, far_order=6,
               theta=0.8, err_tol=err_tol if err_tol is not None else 0.02, periodic=1,
               local_order=local_order, local_tol=local_tol)
    return pos, mass, prm


def test_lists_partition_the_multipole_list():
    pos, mass, prm = _small_tree(4, 0.01)
    T_on = oracle.Tree(pos, mass, prm)
    T_off = oracle.Tree(pos, mass, dict(prm, local_order=0))
    o0, i0, c0 = T_off.lists(0)
    o0b, i0b, c0b = T_on.lists(0)
    np.testing.assert_array_equal(o0, o0b)
    np.testing.assert_array_equal(c0, c0b)
    om, im, cm = T_off.lists(1)
    pm, jm, dm = T_on.lists(1)
    pl, jl, dl = T_on.lists(2)
    assert len(dl) > 0.3 * len(cm)  # the route takes a good share
    for g in range(len(om) - 1):
        want = sorted(zip(im[om[g]:om[g + 1]], cm[om[g]:om[g + 1]]))
        got = sorted(list(zip(jm[pm[g]:pm[g + 1]], dm[pm[g]:pm[g + 1]])) +
                     list(zip(jl[pl[g]:pl[g + 1]], dl[pl[g]:pl[g + 1]])))
        assert got == want, g


def test_no_local_route_without_tolerance_or_at_theta_zero():
    pos, mass, prm = _small_tree(4, 0.0)
    assert oracle.Tree(pos, mass, prm).lists(2)[2].size == 0
    pos, mass, prm = _small_tree(4, 1.0, err_tol=0.0)
    assert oracle.Tree(pos, mass, dict(prm, theta=0.0)).lists(2)[2].size == 0


def test_tree_forces_move_within_summed_bound():
    """Per target, the local route changes the acceleration by at most the
    truncation bound summed over the group's local cells (each cell's
    particles all lie at least u = |c - z| - b from the centre)."""
    pos, mass, prm = _small_tree(4, 0.005)
    eps = prm["eps"]
    T_on = oracle.Tree(pos, mass, prm)
    T_off = oracle.Tree(pos, mass, dict(prm, local_order=0))
    a_on, _ = T_on.forces()
    a_off, _ = T_off.forces()
    cells = T_on.cells()
    _, bmax = T_on.cell_bounds()
    gcell, lo, hi = T_on.groups()
    perm, _ = T_on.perm()
    off, img, cl = T_on.lists(2)
    checked = 0
    for g in range(len(gcell)):
        if off[g + 1] == off[g]:
            continue
        c = 0.5 * (lo[:, g] + hi[:, g])
        a = np.linalg.norm(hi[:, g] - c)
        bsum = 0.0
        for e in range(off[g], off[g + 1]):
            i = img[e]
            sh = np.array([i // 9 - 1, (i // 3) % 3 - 1, i % 3 - 1], float)
            B = cl[e]
            u = np.linalg.norm(c - (cells["com"][:, B] + sh)) - bmax[B]
            bsum += _bound(cells["mass"][B], a, u, 4, eps=eps)
        A = gcell[g]
        idx = perm[cells["first"][A]:cells["first"][A] + cells["count"][A]]
        d = np.linalg.norm(a_on[:, idx] - a_off[:, idx], axis=0)
        assert np.all(d <= 1.05 * bsum + 1e-14), (g, d.max(), bsum)
        checked += 1
    assert checked > 10


def test_local_error_falls_with_tolerance():
    pos, mass, _ = _small_tree(4, 0.0)
    errs = []
    for tol in (0.05, 0.005, 0.0005):
        _, _, prm = _small_tree(4, tol)
        a_on, _ = oracle.Tree(pos, mass, prm).forces()
        a_off, _ = oracle.Tree(pos, mass, dict(prm, local_order=0)).forces()
        errs.append(oracle.rms_rel_error(a_on, a_off))
    assert errs[0] > errs[1] > errs[2], errs
    # a_rms is 0.43 here: the smallest tolerance is 1.2e-3 of it
    assert errs[-1] < 1e-3


def test_adjoint_refuses_local_route():
    pos, mass, prm = _small_tree(4, 0.01)
    T = oracle.Tree(pos, mass, prm)
    with pytest.raises(NotImplementedError):
        T.vjp(np.zeros((3, pos.shape[1])))
