"""GPU parity of the block-timestep integrator (hot_kdk_block; paper Sec. 2.1,
the adaptive symplectic integrator read as hierarchical kick-drift-kick on
power-of-two rungs) against the oracle's: the same rungs, positions and
velocities; one rung is hot_kdk's leapfrog bit for bit."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _case():
    pos, mass, prm = workloads.make("nfw256", n_side=10)
    prm = dict(prm, theta=0.5, leaf_max=8, group_max=32, eps=0.3 / 10)
    vel = np.random.default_rng(2).normal(scale=0.01, size=pos.shape)
    return pos, vel, mass, prm


def _gpu(pos, vel, mass, prm, precision, **kw):
    import torch
    from paper_1407_2600_amd import Gravity
    dt_ = torch.float32 if precision == "fp32" else torch.float64
    g = Gravity(precision=precision, **prm)
    P = torch.as_tensor(pos, device="cuda").contiguous()
    V = torch.as_tensor(vel, dtype=dt_, device="cuda").contiguous()
    M = torch.as_tensor(mass, dtype=dt_, device="cuda")
    A = torch.empty_like(V)
    R = torch.as_tensor(kw.pop("rung", np.zeros(pos.shape[1])), dtype=torch.uint8,
                        device="cuda").contiguous()
    g.kdk_block(P, V, M, A, R, acc_valid=False, **kw)
    torch.cuda.synchronize()
    return (P.cpu().numpy(), V.double().cpu().numpy(), A.double().cpu().numpy(),
            R.cpu().numpy().astype(np.int64), g)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_one_rung_is_kdk(precision):
    import torch
    from paper_1407_2600_amd import Gravity
    pos, vel, mass, prm = _case()
    x1, v1, a1, r1, _ = _gpu(pos, vel, mass, prm, precision, dt=0.01, max_rung=0, eta=0.1,
                             nsteps=2, rung_valid=False)
    dt_ = torch.float32 if precision == "fp32" else torch.float64
    g = Gravity(precision=precision, **prm)
    P = torch.as_tensor(pos, device="cuda").contiguous()
    V = torch.as_tensor(vel, dtype=dt_, device="cuda").contiguous()
    M = torch.as_tensor(mass, dtype=dt_, device="cuda")
    A = torch.empty_like(V)
    g.kdk(P, V, M, A, 0.01, 2, acc_valid=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(x1, P.cpu().numpy())
    np.testing.assert_array_equal(v1, V.double().cpu().numpy())
    assert np.all(r1 == 0)


def test_adaptive_fp64_matches_oracle():
    pos, vel, mass, prm = _case()
    dt, R, eta = 0.01, 3, 0.1
    xo, vo, ao, po, ro, nev = oracle.kdk_block(pos, vel, mass, prm, dt, R, eta, 2)
    x, v, a, r, g = _gpu(pos, vel, mass, prm, "fp64", dt=dt, max_rung=R, eta=eta, nsteps=2,
                         rung_valid=False)
    print(f"rungs {np.bincount(ro, minlength=R + 1)}, oracle force evaluations {nev}",
          flush=True)
    assert len(np.unique(ro)) >= 3
    np.testing.assert_array_equal(r, ro)
    d = x - xo
    d -= np.round(d)
    assert np.max(np.abs(d)) < 1e-11
    assert oracle.rms_rel_error(v, vo) < 1e-9
    assert oracle.rms_rel_error(a, ao) < 1e-9


def test_fixed_rungs_fp32_matches_oracle():
    pos, vel, mass, prm = _case()
    dt, R = 0.01, 2
    rung = np.random.default_rng(6).integers(0, R + 1, size=pos.shape[1])
    mo = mass.astype(np.float32).astype(np.float64)
    vo32 = vel.astype(np.float32).astype(np.float64)
    xo, vo, ao, po, ro, _ = oracle.kdk_block(pos, vo32, mo, prm, dt, R, 0.1, 1, rung=rung,
                                             fixed=True)
    x, v, a, r, g = _gpu(pos, vel, mass, prm, "fp32", dt=dt, max_rung=R, eta=0.1, nsteps=1,
                         rung=rung, rung_valid=True, fixed_rungs=True)
    np.testing.assert_array_equal(r, rung)
    d = x - xo
    d -= np.round(d)
    ev = oracle.rms_rel_error(v - vo32, vo - vo32)   # the change of velocity over the step
    print(f"fp32 fixed rungs: max |dx| {np.max(np.abs(d)):.2e}, velocity change err {ev:.2e}",
          flush=True)
    assert np.max(np.abs(d)) < 1e-7
    assert ev < 1e-4
    assert oracle.rms_rel_error(a, ao) < 2e-5
