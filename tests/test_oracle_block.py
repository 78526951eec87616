"""Pins of the oracle's block-timestep integrator (paper Sec. 2.1: an
adaptive symplectic integrator, read as hierarchical kick-drift-kick on
power-of-two rungs): one rung is the plain leapfrog; with fixed rungs the
scheme is time-reversible; the rung rule is the step criterion it states;
and on an eccentric two-body orbit the adaptive steps are about as accurate
as the finest fixed step and far more than the coarsest."""
import math

import numpy as np
import pytest

import oracle
import workloads


def test_one_rung_is_the_leapfrog():
    pos, mass, prm = workloads.make("zeldovich128", n_side=8)
    prm = dict(prm, theta=0.6, leaf_max=8, group_max=32)
    vel = np.random.default_rng(1).normal(scale=0.05, size=pos.shape)
    x1, v1, a1, _ = oracle.kdk(pos, vel, mass, prm, 0.01, 3)
    x2, v2, a2, _, r, _ = oracle.kdk_block(pos, vel, mass, prm, 0.03, 0, 0.1, 1)
    # three leapfrog steps of 0.01 against one block step of 0.03 with one rung
    # is not the same; one step each is
    x1, v1, a1, _ = oracle.kdk(pos, vel, mass, prm, 0.03, 1)
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(v1, v2)
    np.testing.assert_array_equal(a1, a2)
    assert np.all(r == 0)


def test_rung_rule():
    dt, R, eta, eps = 0.1, 6, 0.2, 0.01
    a = np.array([[0.0, 1e-6, 0.3, 2.0, 50.0, 1e6], [0.0] * 6, [0.0] * 6])
    r = oracle.rung_of(a, dt, R, eta, eps)
    for k in range(a.shape[1]):
        amag = abs(a[0, k])
        want = math.inf if amag == 0 else eta * math.sqrt(eps / amag)
        expect = 0 if want >= dt else min(R, math.ceil(math.log2(dt / want)))
        assert r[k] == expect
        if r[k] < R:
            assert dt / 2 ** r[k] <= want


def test_fixed_rungs_are_time_reversible():
    pos, mass, prm = workloads.make("nfw256", n_side=8)
    prm = dict(prm, theta=0.0, leaf_max=8, group_max=32, eps=0.3 / 8)
    vel = np.zeros_like(pos)
    rung = np.random.default_rng(4).integers(0, 3, size=pos.shape[1])
    x1, v1, a1, p1, r1, _ = oracle.kdk_block(pos, vel, mass, prm, 0.002, 2, 0.1, 2, rung=rung,
                                             fixed=True)
    np.testing.assert_array_equal(r1, rung)
    x2, v2, _, _, _, _ = oracle.kdk_block(x1, -v1, mass, prm, 0.002, 2, 0.1, 2, acc=a1, pot=p1,
                                          rung=rung, fixed=True)
    d = x2 - pos
    d -= np.round(d)
    assert np.max(np.abs(d)) < 1e-13
    assert np.max(np.abs(v2 + vel)) < 1e-10 * max(1.0, np.max(np.abs(v1)))


def _two_body(e=0.9):
    """Unit masses on an orbit of eccentricity e, semi-major axis 0.05, at
    apocentre, open boundaries; returns pos, vel, mass, period."""
    G, m, a = 1.0, 0.5, 0.05
    M = 2 * m
    ra = a * (1 + e)
    va = math.sqrt(G * M * (1 - e) / (a * (1 + e)))
    pos = np.array([[0.5 - ra / 2, 0.5 + ra / 2], [0.5, 0.5], [0.5, 0.5]])
    vel = np.array([[0.0, 0.0], [-va / 2, va / 2], [0.0, 0.0]])
    period = 2 * math.pi * math.sqrt(a ** 3 / (G * M))
    return pos, vel, np.array([m, m]), period


def _energy(x, v, m, eps):
    r = np.linalg.norm(x[:, 0] - x[:, 1])
    return 0.5 * np.sum(m * np.sum(v * v, 0)) - m[0] * m[1] / np.sqrt(r * r + eps * eps)


def test_adaptive_steps_on_an_eccentric_orbit():
    """Pericentre 0.005, apocentre 0.095: the criterion puts the pair on the
    coarse rungs near apocentre and on the finest near pericentre.  Over one
    orbit the energy error is four orders of magnitude below the coarsest
    fixed step's, with a fraction of the finest fixed step's force
    evaluations."""
    x0, v0, m, T = _two_body()
    eps = 1e-3
    prm = dict(box=1.0, G=1.0, eps=eps, theta=0.0, order=2, periodic=0, leaf_max=1,
               group_max=1, far_order=0)
    E0 = _energy(x0, v0, m, eps)
    nbig, R, eta = 16, 6, 0.2
    dt = T / nbig
    rungs, nev = set(), 0
    x, v, a, p, r = x0, v0, None, None, None
    for _ in range(nbig):  # one orbit, one big step at a time, recording the rungs
        x, v, a, p, r, k = oracle.kdk_block(x, v, m, prm, dt, R, eta, 1, acc=a, pot=p, rung=r)
        rungs.update(int(q) for q in r)
        nev += k
    e_ad = abs(_energy(x, v, m, eps) - E0) / abs(E0)
    x, v, _, _, _, _ = oracle.kdk_block(x0, v0, m, prm, dt, 0, eta, nbig)
    e_coarse = abs(_energy(x, v, m, eps) - E0) / abs(E0)
    assert min(rungs) <= 3 and max(rungs) == R
    assert e_ad < 1e-4 * e_coarse and e_ad < 3e-3
    assert nev < 0.3 * nbig * 2 ** R  # the finest fixed step's evaluations
