"""hot_forces_noalloc (the entry point for callers that cannot allocate
device memory) against hot_forces: the same kernels on the library's fixed
device scratch instead of a workspace, so the results must be bit-identical.
Two calls in a row on that one array, the second with fewer particles (the
array keeps the first call's contents), in both precisions; a size beyond
the array is refused before any kernel runs."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_forces(precision):
    import torch
    from paper_1407_2600_amd import Gravity
    dt = torch.float32 if precision == "fp32" else torch.float64
    for name, ns, over in (("zeldovich128", 40, dict(theta=0.8, err_tol=4.88e-3, leaf_max=16,
                                                        group_max=128)),
                           ("nfw256", 24, dict(theta=0.5, leaf_max=8, group_max=32))):
        pos, mass, prm = workloads.make(name, n_side=ns)
        prm = dict(prm, **over)
        n = pos.shape[1]
        print(f"noalloc {precision} {name} n={n}", flush=True)
        g = Gravity(precision=precision, **prm)
        P = torch.as_tensor(pos, device="cuda")
        M = torch.as_tensor(mass, dtype=dt, device="cuda")
        a1, p1 = g.forces(P, M)
        a2 = torch.empty_like(a1)
        p2 = torch.empty_like(p1)
        g.forces_noalloc(P, M, a2, p2)
        torch.cuda.synchronize()
        st = g.stats()
        print(f"  list chunks {st['list_chunks']}", flush=True)
        assert torch.equal(a1, a2) and torch.equal(p1, p2)
        # without potentials
        a3 = torch.empty_like(a1)
        g.forces_noalloc(P, M, a3, None)
        torch.cuda.synchronize()
        assert torch.equal(a1, a3)


def test_noalloc_refuses_too_many_particles():
    import torch
    from paper_1407_2600_amd import Gravity, HotError
    n = 1 << 22
    g = Gravity(precision="fp32", box=1.0, eps=1e-4, leaf_max=16, group_max=128)
    P = torch.rand((3, n), dtype=torch.float64, device="cuda")
    M = torch.full((n,), 1.0 / n, dtype=torch.float32, device="cuda")
    A = torch.empty((3, n), dtype=torch.float32, device="cuda")
    with pytest.raises(HotError, match="ENOMEM"):
        g.forces_noalloc(P, M, A)
    # a size that fits still works afterwards, and matches hot_forces
    k = 20000
    a1, _ = g.forces(P[:, :k].contiguous(), M[:k].contiguous())
    a2 = torch.empty_like(a1)
    g.forces_noalloc(P[:, :k].contiguous(), M[:k].contiguous(), a2)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)
