"""Pins for the oracle's kick-drift-kick leapfrog: time reversibility and a
bounded energy error on a softened two-body orbit (open boundaries)."""
import numpy as np

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
