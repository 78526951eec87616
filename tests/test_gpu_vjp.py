"""GPU parity of the adjoint (hot_vjp): against the oracle's gather-form
adjoint over the same lists (exact derivative at theta = 0), against central
finite differences of the GPU forward at theta = 0, and through the
torch.autograd.Function wrapper."""
import numpy as np
import pytest

import oracle
import workloads
from _gpu import oracle_mass

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-5, "fp32": 2e-5}


def _case(n_side=8, **over):
    pos, mass, prm = workloads.make("zeldovich128", n_side=n_side)
    rng = np.random.default_rng(17)
    mass = mass * (0.5 + rng.random(mass.size))
    prm = dict(prm, **over)
    ga = rng.normal(size=pos.shape)
    gp = rng.normal(size=mass.size)
    return pos, mass, prm, ga, gp


def _gpu_vjp(pos, mass, prm, ga, gp, precision):
    import torch
    from paper_1407_2600_amd import Gravity
    g = Gravity(precision=precision, **prm)
    dt = torch.float32 if precision == "fp32" else torch.float64
    P = torch.as_tensor(pos, dtype=torch.float64, device="cuda")
    M = torch.as_tensor(mass, dtype=dt, device="cuda")
    GA = torch.as_tensor(ga, dtype=dt, device="cuda")
    GP = None if gp is None else torch.as_tensor(gp, dtype=dt, device="cuda")
    xb, mb = g.vjp(P, M, GA, GP)
    torch.cuda.synchronize()
    return xb.cpu().numpy(), mb.double().cpu().numpy()


def _oracle_inputs(ga, gp, precision):
    if precision == "fp32":
        ga = ga.astype(np.float32).astype(np.float64)
        gp = None if gp is None else gp.astype(np.float32).astype(np.float64)
    return ga, gp


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("theta,order", [(0.0, 4), (0.5, 4), (0.6, 2), (0.4, 3)])
def test_vjp_matches_oracle(theta, order, precision):
    pos, mass, prm, ga, gp = _case(theta=theta, order=order, leaf_max=8, group_max=32)
    print(f"vjp theta={theta} order={order} {precision}", flush=True)
    mo = oracle_mass(mass, precision)
    gao, gpo = _oracle_inputs(ga, gp, precision)
    xo, mbo = oracle.Tree(pos, mo, prm).vjp(gao, gpo)
    xg, mbg = _gpu_vjp(pos, mass, prm, ga, gp, precision)
    ex = oracle.rms_rel_error(xg, xo)
    em = oracle.rms_rel_error(mbg, mbo)
    print(f"  xbar err {ex:.3e} mbar err {em:.3e}", flush=True)
    assert ex <= TOL[precision]
    assert em <= TOL[precision]


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4])
def test_vjp_every_order_fp64(order):
    pos, mass, prm, ga, gp = _case(n_side=7, theta=0.5, order=order, leaf_max=4, group_max=16)
    xo, mbo = oracle.Tree(pos, mass, prm).vjp(ga, gp)
    xg, mbg = _gpu_vjp(pos, mass, prm, ga, gp, "fp64")
    assert oracle.rms_rel_error(xg, xo) < 1e-9
    assert oracle.rms_rel_error(mbg, mbo) < 1e-9


def test_vjp_without_potential_cotangent_and_open_boundaries():
    pos, mass, prm, ga, _ = _case(n_side=7, theta=0.5, periodic=0)
    xo, mbo = oracle.Tree(pos, mass, prm).vjp(ga, None)
    xg, mbg = _gpu_vjp(pos, mass, prm, ga, None, "fp64")
    assert oracle.rms_rel_error(xg, xo) < 1e-9
    assert oracle.rms_rel_error(mbg, mbo) < 1e-9


def test_vjp_vs_finite_differences_of_gpu_forward():
    """theta = 0: the adjoint is the exact derivative of the GPU forward."""
    import torch
    from paper_1407_2600_amd import Gravity
    pos, mass, prm, ga, gp = _case(n_side=5, theta=0.0, leaf_max=4, group_max=8, far_order=6)
    g = Gravity(precision="fp64", **prm)
    M = torch.as_tensor(mass, device="cuda")

    def loss(p):
        a, ph = g.forces(torch.as_tensor(p, device="cuda"), M)
        return float(np.sum(ga * a.cpu().numpy()) + np.sum(gp * ph.cpu().numpy()))

    xg, mbg = _gpu_vjp(pos, mass, prm, ga, gp, "fp64")
    h = 1e-6
    for a, k in [(0, 2), (1, 40), (2, 99), (0, 120)]:
        pp = pos.copy()
        pp[a, k] += h
        pm = pos.copy()
        pm[a, k] -= h
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert xg[a, k] == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.max(np.abs(xg)))


def test_autograd_function_backward():
    import torch
    from paper_1407_2600_amd import Gravity, gravity_forces
    pos, mass, prm, ga, gp = _case(n_side=6, theta=0.5)
    g = Gravity(precision="fp64", **prm)
    P = torch.as_tensor(pos, device="cuda").requires_grad_(True)
    M = torch.as_tensor(mass, device="cuda").requires_grad_(True)
    acc, pot = gravity_forces(g, P, M)
    L = (acc * torch.as_tensor(ga, device="cuda")).sum() + (pot * torch.as_tensor(gp, device="cuda")).sum()
    L.backward()
    xo, mbo = oracle.Tree(pos, mass, prm).vjp(ga, gp)
    assert oracle.rms_rel_error(P.grad.cpu().numpy(), xo) < 1e-9
    assert oracle.rms_rel_error(M.grad.cpu().numpy(), mbo) < 1e-9


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_vjp_after_forces_matches_vjp(precision):
    """hot_vjp_after_forces after a force evaluation at the same point uses
    that evaluation's tree and lists and gives bit-identical results to
    hot_vjp (same lists, same summation order), also when repeated; after an
    evaluation at other positions it builds its own tree and again matches;
    and the adjoint still matches the oracle's."""
    import torch
    from paper_1407_2600_amd import Gravity
    pos, mass, prm, ga, gp = _case(n_side=20, theta=0.6, leaf_max=8, group_max=48)
    dt = torch.float32 if precision == "fp32" else torch.float64
    g = Gravity(precision=precision, **prm)
    P = torch.as_tensor(pos, dtype=torch.float64, device="cuda")
    M = torch.as_tensor(mass, dtype=dt, device="cuda")
    GA = torch.as_tensor(ga, dtype=dt, device="cuda")
    GP = torch.as_tensor(gp, dtype=dt, device="cuda")
    P2 = torch.remainder(P + 0.013, 1.0)
    print(f"vjp after forces {precision}: n={pos.shape[1]}", flush=True)
    xr, mr = g.vjp(P, M, GA, GP)
    xr2, mr2 = g.vjp(P2, M, GA, GP)
    ref = [(xr.cpu().numpy(), mr.double().cpu().numpy()),
           (xr2.cpu().numpy(), mr2.double().cpu().numpy())]
    for pp, (xe, me) in ((P, ref[0]), (P2, ref[1])):
        g.forces(pp, M)
        for _ in range(2):
            xb, mb = g.vjp(pp, M, GA, GP, after_forces=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(xb.cpu().numpy(), xe)
            np.testing.assert_array_equal(mb.double().cpu().numpy(), me)
    # the last evaluation was at P2: at P the library rebuilds the tree
    xb, mb = g.vjp(P, M, GA, GP, after_forces=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(xb.cpu().numpy(), ref[0][0])
    np.testing.assert_array_equal(mb.double().cpu().numpy(), ref[0][1])
    gao, gpo = _oracle_inputs(ga, gp, precision)
    xo, mbo = oracle.Tree(pos, oracle_mass(mass, precision), prm).vjp(gao, gpo)
    assert oracle.rms_rel_error(ref[0][0], xo) <= TOL[precision]
    assert oracle.rms_rel_error(ref[0][1], mbo) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autograd_interleaved_forwards_noncontiguous(precision):
    """Two differentiable force evaluations on one context with
    non-contiguous positions (a transposed (N, 3) tensor), then the backward
    of the first: the first forward's tree and lists are no longer in the
    workspace, so the backward must build its own tree; its gradients equal
    hot_vjp's at the first positions, bit for bit."""
    import torch
    from paper_1407_2600_amd import Gravity, gravity_forces
    pos, mass, prm, ga, gp = _case(n_side=14, theta=0.6, leaf_max=8, group_max=32)
    dt = torch.float32 if precision == "fp32" else torch.float64
    g = Gravity(precision=precision, **prm)
    X1 = torch.as_tensor(pos.T.copy(), dtype=torch.float64, device="cuda").requires_grad_(True)
    X2 = torch.remainder(X1.detach() + 0.021, 1.0).requires_grad_(True)
    M = torch.as_tensor(mass, dtype=dt, device="cuda")
    GA = torch.as_tensor(ga, dtype=dt, device="cuda")
    GP = torch.as_tensor(gp, dtype=dt, device="cuda")
    a1, p1 = gravity_forces(g, X1.T, M)   # X1.T is a non-contiguous (3, N) view
    a2, p2 = gravity_forces(g, X2.T, M)
    ((a1 * GA).sum() + (p1 * GP).sum()).backward()
    torch.cuda.synchronize()
    xr, _ = g.vjp(X1.detach().T.contiguous(), M, GA, GP)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(X1.grad.T.cpu().numpy(), xr.cpu().numpy())
    # the second forward's backward right after it may reuse its tree
    ((a2 * GA).sum() + (p2 * GP).sum()).backward()
    xr2, _ = g.vjp(X2.detach().T.contiguous(), M, GA, GP)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(X2.grad.T.cpu().numpy(), xr2.cpu().numpy())
