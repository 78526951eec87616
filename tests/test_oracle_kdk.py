"""Pins for the oracle's kick-drift-kick leapfrog: time reversibility and a
bounded energy error on a softened two-body orbit (open boundaries)."""
import numpy as np
import pytest

import oracle
import workloads


def test_kdk_time_reversible():
    pos, mass, prm = workloads.make("zeldovich128", n_side=6)
    rng = np.random.default_rng(3)
    vel = 0.05 * rng.normal(size=pos.shape)
    p1, v1, a1, _ = oracle.kdk(pos, vel, mass, prm, 0.01, 5)
    p2, v2, _, _ = oracle.kdk(p1, -v1, mass, prm, 0.01, 5, acc=a1)
    d = p2 - pos
    d -= np.round(d)  # periodic distance
    assert np.max(np.abs(d)) < 1e-12
    np.testing.assert_allclose(-v2, vel, atol=1e-11)


def test_kdk_two_body_energy_bounded():
    """Circular orbit of two unit masses at separation 1 (open boundaries):
    the leapfrog energy error stays bounded and small (no drift)."""
    prm = dict(box=100.0, G=1.0, eps=0.0, theta=0.0, order=0, periodic=0, leaf_max=1,
               group_max=1)
    pos = np.array([[49.5, 50.5], [50.0, 50.0], [50.0, 50.0]])
    v = np.sqrt(0.5) / 1.0  # v^2 = G m / (4 r_half) * 2 ... circular: v = sqrt(G m / (2 d))
    vel = np.array([[0.0, 0.0], [-v, v], [0.0, 0.0]])
    mass = np.array([1.0, 1.0])

    def energy(p, u):
        d = np.linalg.norm(p[:, 0] - p[:, 1])
        return 0.5 * np.sum(mass * np.sum(u ** 2, 0)) - 1.0 / d

    e0 = energy(pos, vel)
    es = []
    acc = None
    p, u = pos, vel
    for _ in range(40):
        p, u, acc, _ = oracle.kdk(p, u, mass, prm, 0.05, 5, acc=acc)
        es.append(energy(p, u))
    es = np.array(es)
    assert np.max(np.abs(es - e0)) < 2e-3 * abs(e0)
    # bounded: the error in the second half is not larger than in the first
    half = len(es) // 2
    assert np.max(np.abs(es[half:] - e0)) < 1.5 * np.max(np.abs(es[:half] - e0)) + 1e-12


def _kdk_loss_setup(theta):
    pos, mass, prm = workloads.make("zeldovich128", n_side=4)
    prm = dict(prm, theta=theta, far_order=6)
    rng = np.random.default_rng(11)
    mass = mass * (0.5 + rng.random(mass.size))
    vel = 0.3 * rng.normal(size=pos.shape)
    cx = rng.normal(size=pos.shape)
    cv = rng.normal(size=pos.shape)
    return pos, vel, mass, prm, cx, cv


def _loss(pos, vel, mass, prm, cx, cv, dt, nsteps):
    p, v, _, _ = oracle.kdk(pos, vel, mass, prm, dt, nsteps)
    return float(np.sum(cx * p) + np.sum(cv * v))


def test_kdk_vjp_matches_finite_differences():
    """theta = 0: the reverse sweep is the exact derivative of the leapfrog map
    (positions, velocities and masses), checked by central differences."""
    dt, ns = 0.01, 3
    pos, vel, mass, prm, cx, cv = _kdk_loss_setup(0.0)
    xs, _ = oracle.kdk_trajectory(pos, vel, mass, prm, dt, ns)
    xb, vb, mb = oracle.kdk_vjp(xs, mass, prm, dt, cx, cv)
    h = 1e-6
    for what, arr, grad in (("x", pos, xb), ("v", vel, vb)):
        for a, k in [(0, 3), (1, 17), (2, 40), (0, 63)]:
            up = arr.copy()
            dn = arr.copy()
            up[a, k] += h
            dn[a, k] -= h
            args_up = (up, vel) if what == "x" else (pos, up)
            args_dn = (dn, vel) if what == "x" else (pos, dn)
            fd = (_loss(*args_up, mass, prm, cx, cv, dt, ns) -
                  _loss(*args_dn, mass, prm, cx, cv, dt, ns)) / (2 * h)
            assert grad[a, k] == pytest.approx(fd, rel=1e-6, abs=1e-8), (what, a, k)
    for k in (5, 33):
        up = mass.copy()
        dn = mass.copy()
        up[k] += h * mass[k]
        dn[k] -= h * mass[k]
        fd = (_loss(pos, vel, up, prm, cx, cv, dt, ns) -
              _loss(pos, vel, dn, prm, cx, cv, dt, ns)) / (2 * h * mass[k])
        assert mb[k] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_kdk_vjp_zero_steps_and_free_drift():
    """No steps: identity.  G = 0: x1 = x + v dt exactly, so
    x0bar = xbar and v0bar = vbar + n dt xbar."""
    pos, vel, mass, prm, cx, cv = _kdk_loss_setup(0.5)
    xb, vb, mb = oracle.kdk_vjp([pos], mass, prm, 0.01, cx, cv)
    np.testing.assert_array_equal(xb, cx)
    np.testing.assert_array_equal(vb, cv)
    np.testing.assert_array_equal(mb, 0.0)
    prm0 = dict(prm, G=0.0)
    xs, _ = oracle.kdk_trajectory(pos, 0.01 * vel, mass, prm0, 0.01, 4)
    xb, vb, mb = oracle.kdk_vjp(xs, mass, prm0, 0.01, cx, cv)
    np.testing.assert_allclose(xb, cx, rtol=0, atol=1e-15)
    np.testing.assert_allclose(vb, cv + 4 * 0.01 * cx, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mb, 0.0, atol=1e-15)


def test_wrap_box_lands_in_box_and_keeps_residue():
    """wrap_box maps any coordinate into [0, L) by a whole number of box
    lengths (values within rounding of L land on 0)."""
    rng = np.random.default_rng(3)
    L = 1.3
    x = np.concatenate([rng.normal(0.0, 5.0, 500), [0.0, L, -L, 2 * L, -1e-18, L * (1 - 1e-17)]])
    w = oracle.wrap_box(x, L)
    assert np.all((w >= 0.0) & (w < L))
    k = (x - w) / L
    np.testing.assert_allclose(k, np.round(k), atol=1e-9)
    inside = (x >= 0.0) & (x < L)
    np.testing.assert_array_equal(w[inside], x[inside])
