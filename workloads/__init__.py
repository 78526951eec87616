"""Seeded synthetic particle sets shaped like the paper's cosmological workloads.

These generators are shared by the oracle-side tests, the GPU-side tests and the
benchmark.  They hold none of the force method's arithmetic: they only draw
positions, masses and the physical parameters (softening, opening angle,
multipole order) that go with each workload.  Positions are returned as an SoA
float64 array of shape (3, N) wrapped into [0, L); masses are 1/N.

Workloads (seed = 1000 + workload number):

* ``lattice16``   16^3 simple-cubic lattice at (i+1/2)a plus Gaussian jitter of
  0.1a per component; quadrupole order (p=2), theta=0.5.
* ``zeldovich``   n^3 Zel'dovich displacements of a Gaussian random field with
  P(k) ~ k^-1.5 cut at the Nyquist sphere, rms displacement 0.5a (128^3 is the
  headline size); order 4, theta=0.5.
* ``nfw``         70% of particles in NFW halos (counts drawn from
  dN/dM ~ M^-1.9 on [1e2, 1e5] particles, concentration 8, r_vir from a
  200x mean-density sphere), 30% uniform background (256^3 is the full size).
* ``adjoint64``   64^3 Zel'dovich as above, for the differentiation workload.

The paper's own initial conditions (2LPTic with a CLASS power spectrum) and its
data products are not used; these seeded sets stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = ["lattice_jitter", "zeldovich", "zeldovich_torch", "nfw_background", "uniform", "make",
           "WORKLOADS"]


def _spacing(n_side: int, box: float) -> float:
    return box / n_side


def _wrap(x: np.ndarray, box: float) -> np.ndarray:
    x = np.mod(x, box)
    # np.mod can return exactly `box` for tiny negative inputs; fold it to 0.
    x[x >= box] -= box
    return x


def uniform(n: int, seed: int, box: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((3, n)) * box


def lattice_jitter(n_side: int, seed: int, sigma_frac: float = 0.1, box: float = 1.0,
                   order: str = "C") -> np.ndarray:
    """Simple-cubic lattice at (i+1/2)a plus N(0, (sigma_frac*a)^2) jitter, wrapped."""
    a = _spacing(n_side, box)
    g = (np.arange(n_side) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(order), Y.ravel(order), Z.ravel(order)])
    if sigma_frac > 0:
        rng = np.random.default_rng(seed)
        pos = pos + rng.normal(0.0, sigma_frac * a, size=pos.shape)
    return _wrap(pos, box)


def zeldovich(n_side: int, seed: int, slope: float = -1.5, rms_frac: float = 0.5,
              box: float = 1.0) -> np.ndarray:
    """Zel'dovich displacements of a Gaussian field with P(k) ~ k^slope.

    White noise on the n^3 grid is Fourier transformed and multiplied by
    |k|^(slope/2) for 0 < |k| <= k_Nyquist (spherical cut, Nyquist planes
    zeroed); the displacement is psi_k = i k delta_k / k^2, scaled so that the
    rms of |psi| is ``rms_frac`` times the grid spacing.
    """
    n = n_side
    a = _spacing(n, box)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kny = n // 2
    keep = (k2 > 0) & (k2 <= kny * kny)
    keep &= (np.abs(KX) < kny) & (np.abs(KY) < kny) & (np.abs(KZ) < kny)
    amp = np.zeros_like(k2)
    amp[keep] = k2[keep] ** (slope / 4.0)
    dk = wk * amp
    del wk, amp
    disp = []
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_k2 = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    for K in (KX, KY, KZ):
        psik = 1j * K * dk * inv_k2
        disp.append(np.fft.irfftn(psik, s=(n, n, n), axes=(0, 1, 2)))
    disp = np.stack([d.ravel() for d in disp])
    rms = np.sqrt(np.mean(np.sum(disp ** 2, axis=0)))
    disp *= (rms_frac * a) / rms
    q = lattice_jitter(n, seed, sigma_frac=0.0, box=box)
    return _wrap(q + disp, box)


def zeldovich_torch(n_side: int, seed: int, slope: float = -1.5, rms_frac: float = 0.5,
                    box: float = 1.0, device="cuda"):
    """The recipe of ``zeldovich`` evaluated with torch on a device, for grids
    too large for host memory (1024^3: about 60 GB of FP64 temporaries).
    torch's generator draws a different realisation of the same field (same
    spectrum, cut, normalisation and lattice order).  Returns a (3, n^3)
    FP64 tensor on the device."""
    import torch
    n = n_side
    a = _spacing(n, box)
    f64 = torch.float64
    gen = torch.Generator(device=device).manual_seed(seed)
    w = torch.randn((n, n, n), generator=gen, dtype=f64, device=device)
    dk = torch.fft.rfftn(w)
    del w
    kx = torch.fft.fftfreq(n, d=1.0 / n, dtype=f64, device=device)
    kz = torch.fft.rfftfreq(n, d=1.0 / n, dtype=f64, device=device)
    KX, KY, KZ = kx[:, None, None], kx[None, :, None], kz[None, None, :]
    k2 = KX * KX + KY * KY + KZ * KZ
    kny = n // 2
    keep = (k2 > 0) & (k2 <= kny * kny)
    keep &= (KX.abs() < kny) & (KY.abs() < kny) & (KZ.abs() < kny)
    dk *= torch.where(keep, k2.clamp_min(1.0) ** (slope / 4.0), torch.zeros_like(k2))
    del keep
    inv_k2 = torch.where(k2 > 0, 1.0 / k2.clamp_min(1.0), torch.zeros_like(k2))
    del k2
    dk *= inv_k2
    del inv_k2
    pos = torch.empty((3, n ** 3), dtype=f64, device=device)
    for axis, K in enumerate((KX, KY, KZ)):
        psik = dk * (1j * K)
        pos[axis] = torch.fft.irfftn(psik, s=(n, n, n), dim=(0, 1, 2)).reshape(-1)
        del psik
    del dk
    rms = torch.sqrt(torch.mean(torch.sum(pos * pos, dim=0)))
    pos *= (rms_frac * a) / rms
    g = (torch.arange(n, dtype=f64, device=device) + 0.5) * a
    pos[0] += g[:, None, None].expand(n, n, n).reshape(-1)
    pos[1] += g[None, :, None].expand(n, n, n).reshape(-1)
    pos[2] += g[None, None, :].expand(n, n, n).reshape(-1)
    pos = torch.remainder(pos, box)
    for r in pos:  # row by row and without a mask index (over 2^31 elements at 1024^3)
        r.sub_((r >= box).to(f64) * box)
    return pos


def _nfw_radii(rng, count: int, c: float) -> np.ndarray:
    """Radii x=r/r_vir in [0,1] with enclosed mass ~ ln(1+cx) - cx/(1+cx)."""
    def m(x):
        return np.log1p(c * x) - c * x / (1.0 + c * x)
    u = rng.random(count) * m(1.0)
    lo = np.zeros(count)
    hi = np.ones(count)
    for _ in range(60):  # bisection to ~1e-18
        mid = 0.5 * (lo + hi)
        below = m(mid) < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def nfw_background(n_side: int, seed: int, halo_frac: float = 0.7, slope: float = -1.9,
                   m_lo: float = 1e2, m_hi: float = 1e5, conc: float = 8.0,
                   box: float = 1.0) -> np.ndarray:
    """NFW halos (halo_frac of particles) plus a uniform background."""
    n = n_side ** 3
    rng = np.random.default_rng(seed)
    n_halo_total = int(round(halo_frac * n))
    e = slope + 1.0  # -0.9
    counts = []
    total = 0
    while total < n_halo_total:
        u = rng.random()
        mass = (m_lo ** e + u * (m_hi ** e - m_lo ** e)) ** (1.0 / e)
        k = max(1, int(round(mass)))
        k = min(k, n_halo_total - total)
        counts.append(k)
        total += k
    counts = np.asarray(counts)
    rho = n / box ** 3
    parts = []
    centres = rng.random((len(counts), 3)) * box
    for cnt, cen in zip(counts, centres):
        r_vir = (3.0 * cnt / (4.0 * np.pi * 200.0 * rho)) ** (1.0 / 3.0)
        x = _nfw_radii(rng, cnt, conc) * r_vir
        v = rng.standard_normal((cnt, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        parts.append(cen + v * x[:, None])
    halo = np.concatenate(parts, axis=0).T if parts else np.zeros((3, 0))
    bg = rng.random((3, n - n_halo_total)) * box
    pos = np.concatenate([halo, bg], axis=1)
    perm = rng.permutation(n)
    return _wrap(pos[:, perm], box)


# name -> (generator, n_side, params).  Softening is 0.02 of the mean spacing.
WORKLOADS = {
    "lattice16": dict(kind="lattice", n_side=16, seed=1001, order=2, theta=0.5),
    "zeldovich128": dict(kind="zeldovich", n_side=128, seed=1002, order=4, theta=0.5),
    "nfw256": dict(kind="nfw", n_side=256, seed=1003, order=4, theta=0.5),
    # sink groups of up to 96: 20% faster forward and backward than 64 on
    # this workload
    "adjoint64": dict(kind="zeldovich", n_side=64, seed=1004, order=4, theta=0.5, group_max=96),
    "zeldovich1024": dict(kind="zeldovich", n_side=1024, seed=1005, order=4, theta=0.5,
                          rms_frac=1.5),
}


def make(name: str, n_side: int | None = None, box: float = 1.0, seed: int | None = None):
    """Return (pos[3,N] float64, mass[N] float64, params dict) for a workload.

    ``n_side`` overrides the size (same recipe, smaller or larger grid), which
    the tests use to get cases the oracle finishes in seconds; ``seed``
    overrides the workload's seed (a second realisation of the same recipe).
    """
    spec = dict(WORKLOADS[name])
    if seed is not None:
        spec["seed"] = int(seed)
    ns = n_side or spec["n_side"]
    kind = spec["kind"]
    if kind == "lattice":
        pos = lattice_jitter(ns, spec["seed"], box=box)
    elif kind == "zeldovich":
        pos = zeldovich(ns, spec["seed"], rms_frac=spec.get("rms_frac", 0.5), box=box)
    elif kind == "nfw":
        pos = nfw_background(ns, spec["seed"], box=box)
    else:
        raise ValueError(kind)
    n = pos.shape[1]
    mass = np.full(n, 1.0 / n)
    params = dict(box=box, G=1.0, eps=0.02 * box / ns, theta=spec["theta"],
                  order=spec["order"], periodic=1, leaf_max=16,
                  group_max=spec.get("group_max", 64), far_order=8)
    return np.ascontiguousarray(pos), mass, params
