"""GPU parity of the differentiated leapfrog (hot_kdk_vjp behind
checkpointed_kdk): against the oracle's step-by-step reverse sweep on the
oracle's own trajectory, and, for the trajectory loss of the differentiation
workload (sum of squared minimum-image distances to a target configuration
after 10 steps of dt = 0.01), against central finite differences of the GPU
forward in FP64."""
import numpy as np
import pytest

import oracle
import workloads
from _gpu import oracle_mass

pytestmark = pytest.mark.gpu


def _setup(n_side, theta, seed_shift=0, **over):
    pos, mass, prm = workloads.make("zeldovich128", n_side=n_side)
    prm = dict(prm, theta=theta, **over)
    rng = np.random.default_rng(23 + seed_shift)
    vel = 0.2 * rng.normal(size=pos.shape)
    return pos, vel, mass, prm


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 2e-5)])
@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_kdk_vjp_matches_oracle(theta, precision, tol):
    import torch
    from paper_1407_2600_amd import Gravity
    pos, vel, mass, prm = _setup(6, theta, leaf_max=8, group_max=32)
    dt, ns = 0.01, 3
    print(f"kdk_vjp theta={theta} {precision}", flush=True)
    mo = oracle_mass(mass, precision)
    xs, _ = oracle.kdk_trajectory(pos, vel, mo, prm, dt, ns)
    rng = np.random.default_rng(5)
    cx = rng.normal(size=pos.shape)
    cv = rng.normal(size=pos.shape)
    if precision == "fp32":
        cv = cv.astype(np.float32).astype(np.float64)
    xo, vo, mbo = oracle.kdk_vjp(xs, mo, prm, dt, cx, cv)
    g = Gravity(precision=precision, **prm)
    dtp = g.dtype
    ck = torch.as_tensor(np.stack(xs), device="cuda")
    xb = torch.as_tensor(cx, device="cuda").contiguous()
    vb = torch.as_tensor(cv, dtype=dtp, device="cuda").contiguous()
    mb = g.kdk_vjp(ck, torch.as_tensor(mass, dtype=dtp, device="cuda"), dt, xb, vb)
    torch.cuda.synchronize()
    ex = oracle.rms_rel_error(xb.cpu().numpy(), xo)
    ev = oracle.rms_rel_error(vb.double().cpu().numpy(), vo)
    em = oracle.rms_rel_error(mb.double().cpu().numpy(), mbo)
    print(f"  xbar {ex:.2e} vbar {ev:.2e} mbar {em:.2e}", flush=True)
    assert ex <= tol and ev <= tol and em <= tol


def test_kdk_vjp_zero_steps():
    import torch
    from paper_1407_2600_amd import Gravity
    pos, vel, mass, prm = _setup(4, 0.5)
    g = Gravity(precision="fp64", **prm)
    ck = torch.as_tensor(pos[None], device="cuda")
    x = torch.randn((3, pos.shape[1]), dtype=torch.float64, device="cuda")
    v = torch.randn((3, pos.shape[1]), dtype=torch.float64, device="cuda")
    x0, v0 = x.clone(), v.clone()
    mb = g.kdk_vjp(ck, torch.as_tensor(mass, device="cuda"), 0.01, x, v)
    torch.cuda.synchronize()
    assert torch.equal(x, x0) and torch.equal(v, v0)
    assert torch.count_nonzero(mb).item() == 0


def _trajectory_loss_case(n_side, theta, nsteps=10, dt=0.01):
    """Differentiation workload: Zel'dovich start at rest, loss on the
    minimum-image distance to the end state of a second seed's run."""
    import torch
    from paper_1407_2600_amd import Gravity, checkpointed_kdk
    pos, mass, prm = workloads.make("adjoint64", n_side=n_side)
    pos_t, _, _ = workloads.make("adjoint64", n_side=n_side,
                                 seed=workloads.WORKLOADS["adjoint64"]["seed"] + 100)
    prm = dict(prm, theta=theta)
    g = Gravity(precision="fp64", **prm)
    M = torch.as_tensor(mass, device="cuda")
    V0 = torch.zeros((3, pos.shape[1]), dtype=torch.float64, device="cuda")
    with torch.no_grad():
        xt, _ = checkpointed_kdk(g, torch.as_tensor(pos_t, device="cuda"), V0, M, dt, nsteps)
    L = float(prm["box"])

    def loss_of(x_final):
        d = x_final - xt
        d = d - L * torch.round(d / L)
        return (d * d).sum()

    def loss(p_np):
        with torch.no_grad():
            xf, _ = checkpointed_kdk(g, torch.as_tensor(p_np, device="cuda"), V0, M, dt, nsteps)
            return float(loss_of(xf))

    P = torch.as_tensor(pos, device="cuda").requires_grad_(True)
    xf, _ = checkpointed_kdk(g, P, V0, M, dt, nsteps)
    loss_of(xf).backward()
    return pos, P.grad.cpu().numpy(), loss, prm


def _fd_check(pos, grad, loss, prm, comps, h):
    out = []
    for a, k in comps:
        up = pos.copy()
        dn = pos.copy()
        up[a, k] += h
        dn[a, k] -= h
        fd = (loss(up) - loss(dn)) / (2 * h)
        out.append((grad[a, k], fd))
    return np.array(out)


def test_trajectory_gradient_theta_zero_fd():
    """theta = 0 (27-image direct sum + far field), 8^3 particles: the
    checkpointed reverse sweep is the exact gradient of the GPU trajectory."""
    pos, grad, loss, prm = _trajectory_loss_case(8, 0.0)
    rng = np.random.default_rng(2)
    comps = [(int(rng.integers(3)), int(rng.integers(pos.shape[1]))) for _ in range(16)]
    r = _fd_check(pos, grad, loss, prm, comps, h=1e-6 / 8)
    rel = np.abs(r[:, 0] - r[:, 1]) / np.max(np.abs(r[:, 1]))
    print(f"theta=0 8^3: max rel err {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-5


def test_trajectory_gradient_c4_fd():
    """64^3, theta = 0.5, order 4, 10 steps: gradient with respect to the
    initial displacements against FP64 finite differences of the tree
    trajectory on 16 sampled components.  For theta > 0 the adjoint of the
    tree forces is the tree approximation of the exact derivative, so the
    two agree to the tree's own error level."""
    pos, grad, loss, prm = _trajectory_loss_case(64, 0.5)
    rng = np.random.default_rng(3)
    comps = [(int(rng.integers(3)), int(rng.integers(pos.shape[1]))) for _ in range(16)]
    r = _fd_check(pos, grad, loss, prm, comps, h=1e-5 / 64)
    rel = np.sqrt(np.sum((r[:, 0] - r[:, 1]) ** 2) / np.sum(r[:, 1] ** 2))
    print(f"C4 64^3 theta=0.5: rms rel err over 16 components {rel:.2e}", flush=True)
    assert rel <= 1e-3
