"""FP64 CPU oracle for the periodic tree-gravity force evaluation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
(``paper_1407_2600_amd``) never imports, links or calls it, and the two share
no code: the oracle is plain C (``oracle/*.c``, built with gcc) behind this
ctypes wrapper.

What it computes (paper Sec. 2.1, "2HOT"):

* ``direct_ewald``   -- the plain definition: periodic, Plummer-softened,
  background-neutralised accelerations and potentials by direct summation with
  the textbook Ewald split (real space + structure factors);
* ``Tree``           -- the same-acceptance-test FP64 tree: Morton keys, sort,
  oct-tree, moments, sink groups, 27-image walk, direct and multipole
  interactions, and the periodic far field as local expansions of the Ewald
  remainder about the centres of the box's 8 octants (the paper's high-order
  periodic expansion);
* ``direct_near_far`` -- the tree result at theta=0 for sampled targets
  (27-image softened direct sum plus far field);
* ``green_taylor``, ``psi_table``, ``ewald_psi``, ``ewald_xi``,
  ``multipole_eval``, ``direct_open`` -- the building blocks, exposed so the
  tests can pin each one to closed forms.

Every function here is pinned by ``tests/test_oracle_*.py`` against closed
forms, literature constants, brute force or limits (the tree's accelerations
and potentials against the direct Ewald sum, whose potential is pinned by the
Madelung constant); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["series.c", "kernel.c", "ewald.c", "tree.c"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no fused multiply-add)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(_HERE, "oracle.h")])
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB_PATH)
        vp, i64, dp, i64p, u64p, i32p = (C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_int32))
        L.or_tree_build.restype = vp
        L.or_tree_build.argtypes = [i64, dp, dp, C.c_void_p]
        L.or_tree_free.argtypes = [vp]
        L.or_tree_ncells.restype = i64
        L.or_tree_ncells.argtypes = [vp]
        L.or_tree_ngroups.restype = i64
        L.or_tree_ngroups.argtypes = [vp]
        L.or_tree_perm.argtypes = [vp, i64p, u64p]
        L.or_tree_cells.argtypes = [vp, u64p, i32p, i64p, i64p, i32p, dp, dp, dp]
        L.or_tree_cell_moments.argtypes = [vp, i64, dp]
        L.or_tree_cell_bounds.argtypes = [vp, dp, dp]
        L.or_tree_cell_bk.argtypes = [vp, C.c_int, dp]
        L.or_err_radius.restype = C.c_double
        L.or_err_radius.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_double]
        L.or_tree_groups.argtypes = [vp, i64p, dp, dp]
        L.or_tree_walk.argtypes = [vp]
        L.or_tree_list_total.restype = i64
        L.or_tree_list_total.argtypes = [vp, C.c_int]
        L.or_tree_lists.argtypes = [vp, C.c_int, i64p, i32p, i64p]
        L.or_tree_group_list.restype = i64
        L.or_tree_group_list.argtypes = [vp, i64, C.c_int, i32p, i64p]
        L.or_tree_pair_count.restype = i64
        L.or_tree_pair_count.argtypes = [vp]
        L.or_tree_forces.argtypes = [vp, i64, i64p, dp, dp]
        L.or_tree_far.argtypes = [vp, dp, dp, dp]
        L.or_tree_vjp.argtypes = [vp, dp, dp, i64, i64p, dp, dp]
        L.or_direct_near_far.argtypes = [vp, i64, i64p, dp, dp]
        L.or_direct_open.argtypes = [i64, dp, dp, C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_pair_kernel.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.or_k1_radius.restype = C.c_double
        L.or_k1_radius.argtypes = [C.c_double]
        L.or_direct_ewald.argtypes = [i64, dp, dp, i64, i64p, C.c_double, C.c_double,
                                      C.c_double, C.c_int, C.c_double, C.c_int, C.c_int, dp, dp]
        L.or_keys.argtypes = [i64, dp, C.c_double, u64p, dp]
        L.or_sort.argtypes = [i64, u64p, i64p]
        L.or_green_taylor.argtypes = [C.c_int, dp, C.c_double, dp]
        L.or_psi_table.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, dp]
        L.or_psi_table_at.argtypes = [C.c_int, C.c_double, dp, C.c_double, C.c_int, C.c_int, dp]
        L.or_ewald_psi.argtypes = [dp, C.c_double, C.c_double, C.c_int, C.c_int, dp, dp]
        L.or_ewald_xi.restype = C.c_double
        L.or_ewald_xi.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
        L.or_multipole_eval.argtypes = [i64, dp, dp, C.c_int, C.c_double, dp, dp, dp]
        L.or_local_eval.argtypes = [i64, dp, dp, C.c_int, C.c_int, C.c_double, dp, dp, dp, dp]
        L.or_nterms.restype = C.c_int
        L.or_nterms.argtypes = [C.c_int]
        L.or_mi_get.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int)]
        _lib = L
    return _lib


def _p(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


class _Params(C.Structure):
    _fields_ = [("box", C.c_double), ("G", C.c_double), ("eps", C.c_double),
                ("theta", C.c_double), ("order", C.c_int), ("periodic", C.c_int),
                ("leaf_max", C.c_int), ("group_max", C.c_int), ("far_order", C.c_int),
                ("err_tol", C.c_double), ("kernel", C.c_int), ("local_order", C.c_int),
                ("local_tol", C.c_double)]

# softening kernels: Plummer, or Dehnen's compensating K1 (kernel.c)
KERNELS = {"plummer": 0, "k1": 1, 0: 0, 1: 1}


def kernel_id(p: dict) -> int:
    return KERNELS[p.get("kernel", 0)]


def _params(p: dict) -> _Params:
    return _Params(float(p.get("box", 1.0)), float(p.get("G", 1.0)), float(p.get("eps", 0.0)),
                   float(p.get("theta", 0.5)), int(p.get("order", 2)),
                   int(p.get("periodic", 1)), int(p.get("leaf_max", 16)),
                   int(p.get("group_max", 64)), int(p.get("far_order", 8)),
                   float(p.get("err_tol", 0.0)), kernel_id(p), int(p.get("local_order", 0)),
                   float(p.get("local_tol", 0.0)))


def pair_kernel(kernel, r2: float, eps: float):
    """(g, f) of one pair at squared separation r2: potential -G m g and
    acceleration -G m r f toward the source (kernel.c)."""
    g, f = C.c_double(), C.c_double()
    lib().or_pair_kernel(KERNELS[kernel], float(r2), float(eps), C.byref(g), C.byref(f))
    return g.value, f.value


def k1_radius(eps: float) -> float:
    """Support radius of the K1 kernel for Plummer-equivalent softening eps."""
    return lib().or_k1_radius(float(eps))


def err_radius(G: float, bp: float, b: float, order: int, tol: float) -> float:
    """Opening radius of the error-bound acceptance test for a cell of extent
    b with B_(p+1) = bp (p = max(order, 1))."""
    return float(lib().or_err_radius(G, bp, b, order, tol))


def mi_list(D: int) -> list[tuple[int, int, int]]:
    """Multi-indices |k| <= D in the oracle's order (degree, then a, b descending)."""
    L = lib()
    out = []
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    for i in range(L.or_nterms(D)):
        L.or_mi_get(i, C.byref(a), C.byref(b), C.byref(c))
        out.append((a.value, b.value, c.value))
    return out


def green_taylor(D: int, R, eps: float) -> np.ndarray:
    """Taylor coefficients d^k g(R)/k! of g = (|r|^2+eps^2)^-1/2, |k| <= D."""
    L = lib()
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.zeros(L.or_nterms(D))
    L.or_green_taylor(D, _p(R), float(eps) ** 2, _p(out))
    return out


def psi_table(D: int, box: float = 1.0, alpha: float | None = None, nreal: int = 5,
              kmax: int = 6) -> np.ndarray:
    """Taylor coefficients d^s Psi(0)/s! of the periodic remainder, |s| <= D."""
    L = lib()
    alpha = 2.0 / box if alpha is None else alpha
    out = np.zeros(L.or_nterms(D))
    L.or_psi_table(D, box, alpha, nreal, kmax, _p(out))
    return out


def psi_table_at(D: int, r0, box: float = 1.0, alpha: float | None = None, nreal: int = 5,
                 kmax: int = 6) -> np.ndarray:
    """Taylor coefficients d^s Psi(r0)/s! of the periodic remainder about r0."""
    L = lib()
    alpha = 2.0 / box if alpha is None else alpha
    r0 = np.ascontiguousarray(r0, dtype=np.float64)
    out = np.zeros(L.or_nterms(D))
    L.or_psi_table_at(D, box, _p(r0), alpha, nreal, kmax, _p(out))
    return out


def ewald_psi(r, box: float = 1.0, alpha: float | None = None, nreal: int = 4, kmax: int = 10):
    L = lib()
    alpha = 2.0 / box if alpha is None else alpha
    r = np.ascontiguousarray(r, dtype=np.float64)
    psi = np.zeros(1)
    g = np.zeros(3)
    L.or_ewald_psi(_p(r), box, alpha, nreal, kmax, _p(psi), _p(g))
    return psi[0], g


def ewald_xi(box: float = 1.0, alpha: float | None = None, nreal: int = 4, kmax: int = 10) -> float:
    alpha = 2.0 / box if alpha is None else alpha
    return lib().or_ewald_xi(box, alpha, nreal, kmax)


def multipole_eval(pos, mass, order: int, eps: float, x):
    """Phi and grad Phi at x of one cell's order-p expansion about its COM."""
    L = lib()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    phi = np.zeros(1)
    g = np.zeros(3)
    L.or_multipole_eval(pos.shape[1], _p(pos), _p(mass), order, eps, _p(x), _p(phi), _p(g))
    return phi[0], g


def local_eval(pos, mass, order: int, q: int, eps: float, c, x):
    """Phi and grad Phi at x of one cell's order-p expansion (about its COM)
    re-expanded to order q about c: the tree's group-level local route."""
    L = lib()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    phi = np.zeros(1)
    g = np.zeros(3)
    L.or_local_eval(pos.shape[1], _p(pos), _p(mass), order, q, eps, _p(c), _p(x), _p(phi),
                    _p(g))
    return phi[0], g


def direct_open(pos, mass, G: float = 1.0, eps: float = 0.0, kernel=0):
    """Open-boundary softened direct sum; returns (acc[3,N], pot[N])."""
    L = lib()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[1]
    acc = np.zeros((3, n))
    pot = np.zeros(n)
    L.or_direct_open(n, _p(pos), _p(mass), G, eps, KERNELS[kernel], _p(acc), _p(pot))
    return acc, pot


def direct_ewald(pos, mass, params: dict, targets=None, alpha: float | None = None,
                 nreal: int = 1, kmax: int | None = None):
    """Exact periodic direct sum (the plain definition) at the targets.

    Returns (acc[3,T], pot[T]).  Default split alpha = 4/L with the real-space
    sum over the 27 images of the minimum-image separation and |k|_inf <= 8.
    """
    L = lib()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[1]
    box = float(params.get("box", 1.0))
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    alpha = 4.0 / box if alpha is None else alpha
    if kmax is None:
        kmax = int(np.ceil(np.sqrt(40.0) * alpha * box / np.pi)) + 1
    nt = len(targets)
    acc = np.zeros((3, nt))
    pot = np.zeros(nt)
    L.or_direct_ewald(n, _p(pos), _p(mass), nt, _p(targets, C.c_int64), box,
                      float(params.get("G", 1.0)), float(params.get("eps", 0.0)),
                      kernel_id(params), alpha, nreal, kmax, _p(acc), _p(pot))
    return acc, pot


def keys(pos, box: float = 1.0):
    L = lib()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[1]
    k = np.zeros(n, dtype=np.uint64)
    w = np.zeros((3, n))
    L.or_keys(n, _p(pos), box, _p(k, C.c_uint64), _p(w))
    return k, w


class Tree:
    """The same-acceptance-test FP64 tree (build on construction)."""

    def __init__(self, pos, mass, params: dict):
        self.lib = lib()
        self.params = dict(params)
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.n = self.pos.shape[1]
        self._prm = _params(params)
        self.h = self.lib.or_tree_build(self.n, _p(self.pos), _p(self.mass), C.byref(self._prm))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_tree_free(h)
            self.h = None

    # structure -----------------------------------------------------------
    def perm(self):
        perm = np.zeros(self.n, dtype=np.int64)
        sk = np.zeros(self.n, dtype=np.uint64)
        self.lib.or_tree_perm(self.h, _p(perm, C.c_int64), _p(sk, C.c_uint64))
        return perm, sk

    def cells(self) -> dict:
        nc = self.lib.or_tree_ncells(self.h)
        d = dict(key=np.zeros(nc, np.uint64), level=np.zeros(nc, np.int32),
                 first=np.zeros(nc, np.int64), count=np.zeros(nc, np.int64),
                 is_leaf=np.zeros(nc, np.int32), mass=np.zeros(nc), com=np.zeros((3, nc)),
                 rcrit=np.zeros(nc))
        self.lib.or_tree_cells(self.h, _p(d["key"], C.c_uint64), _p(d["level"], C.c_int32),
                               _p(d["first"], C.c_int64), _p(d["count"], C.c_int64),
                               _p(d["is_leaf"], C.c_int32), _p(d["mass"]), _p(d["com"]),
                               _p(d["rcrit"]))
        return d

    def cell_bounds(self):
        """(B_2[ncells], bmax[ncells]): sum m |x - com|^2 and the extent bound
        the error-bound acceptance test uses."""
        nc = self.lib.or_tree_ncells(self.h)
        b2 = np.zeros(nc)
        bm = np.zeros(nc)
        self.lib.or_tree_cell_bounds(self.h, _p(b2), _p(bm))
        return b2, bm

    def cell_bk(self, k: int):
        """The bound on B_k = sum m |x - com|^k per cell (exact at leaves and
        for k = 0, 2), k = 0..5."""
        out = np.zeros(self.lib.or_tree_ncells(self.h))
        self.lib.or_tree_cell_bk(self.h, int(k), _p(out))
        return out

    def cell_moments(self, c: int) -> np.ndarray:
        nm = self.lib.or_nterms(int(self.params.get("order", 2)))
        M = np.zeros(nm)
        self.lib.or_tree_cell_moments(self.h, int(c), _p(M))
        return M

    def groups(self):
        ng = self.lib.or_tree_ngroups(self.h)
        cell = np.zeros(ng, np.int64)
        lo = np.zeros((3, ng))
        hi = np.zeros((3, ng))
        self.lib.or_tree_groups(self.h, _p(cell, C.c_int64), _p(lo), _p(hi))
        return cell, lo, hi

    def lists(self, kind: int):
        """(offsets[ng+1], image[E], cell[E]) for kind 0 (direct), 1 (multipole)
        or 2 (cells taken through the group's local expansion)."""
        tot = self.lib.or_tree_list_total(self.h, kind)
        ng = self.lib.or_tree_ngroups(self.h)
        off = np.zeros(ng + 1, np.int64)
        img = np.zeros(tot, np.int32)
        cell = np.zeros(tot, np.int64)
        self.lib.or_tree_lists(self.h, kind, _p(off, C.c_int64), _p(img, C.c_int32),
                               _p(cell, C.c_int64))
        return off, img, cell

    def group_list(self, g: int, kind: int):
        """(image[E], cell[E]) of group g's list of a kind (walks g only)."""
        m = self.lib.or_tree_group_list(self.h, int(g), kind, None, None)
        img = np.zeros(m, np.int32)
        cell = np.zeros(m, np.int64)
        self.lib.or_tree_group_list(self.h, int(g), kind, _p(img, C.c_int32), _p(cell, C.c_int64))
        return img, cell

    def pair_count(self) -> int:
        return int(self.lib.or_tree_pair_count(self.h))

    def far(self):
        """(Tpsi[27, nt(2p)], M[8, nt(p)], Lam[8, nt(p)]): the 27 offset tables,
        octant moments and octant local coefficients."""
        pf = int(self.params.get("far_order", 8))
        T = np.zeros((27, self.lib.or_nterms(2 * pf)))
        M = np.zeros((8, self.lib.or_nterms(pf)))
        Lm = np.zeros((8, self.lib.or_nterms(pf)))
        self.lib.or_tree_far(self.h, _p(T), _p(M), _p(Lm))
        return T, M, Lm

    # forces ---------------------------------------------------------------
    def forces(self, groups=None):
        """(acc[3,N], pot[N]) in original order; with ``groups`` only the
        particles of those groups are filled (the rest are NaN)."""
        acc = np.full((3, self.n), np.nan)
        pot = np.full(self.n, np.nan)
        if groups is None:
            self.lib.or_tree_forces(self.h, -1, None, _p(acc), _p(pot))
        else:
            g = np.ascontiguousarray(groups, dtype=np.int64)
            self.lib.or_tree_forces(self.h, len(g), _p(g, C.c_int64), _p(acc), _p(pot))
        return acc, pot

    def vjp(self, gacc, gpot=None, groups=None):
        """(xbar[3,N], mbar[N]) for cotangents (gacc[3,N], gpot[N]) of the
        forces: the gather-form adjoint over the same lists (exact derivative
        of the direct sum at theta = 0).  With ``groups`` only their particles
        are filled (NaN elsewhere).  Plummer softening only."""
        if kernel_id(self.params) != 0:
            raise NotImplementedError("the adjoint is built for Plummer softening only")
        if int(self.params.get("local_order", 0)) > 0 and float(self.params.get("local_tol", 0)) > 0:
            raise NotImplementedError("the adjoint is built without group local expansions")
        ga = np.ascontiguousarray(gacc, dtype=np.float64)
        gp = None if gpot is None else np.ascontiguousarray(gpot, dtype=np.float64)
        xb = np.full((3, self.n), np.nan)
        mb = np.full(self.n, np.nan)
        if groups is None:
            self.lib.or_tree_vjp(self.h, _p(ga), None if gp is None else _p(gp), -1, None,
                                 _p(xb), _p(mb))
        else:
            g = np.ascontiguousarray(groups, dtype=np.int64)
            self.lib.or_tree_vjp(self.h, _p(ga), None if gp is None else _p(gp), len(g),
                                 _p(g, C.c_int64), _p(xb), _p(mb))
        return xb, mb

    def direct_near_far(self, targets):
        t = np.ascontiguousarray(targets, dtype=np.int64)
        acc = np.zeros((3, len(t)))
        pot = np.zeros(len(t))
        self.lib.or_direct_near_far(self.h, len(t), _p(t, C.c_int64), _p(acc), _p(pot))
        return acc, pot


def rms_rel_error(a, ref) -> float:
    """sqrt(sum |a-ref|^2 / sum |ref|^2) over targets (the rms force error)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((a - ref) ** 2) / np.sum(ref ** 2)))


def wrap_box(x, box: float):
    """Wrap into [0, L) with the floor form (any displacement)."""
    x = x - box * np.floor(x / box)
    x = np.where(x >= box, x - box, x)
    return np.where(x < 0.0, 0.0, x)


def kdk(pos, vel, mass, params: dict, dt: float, nsteps: int, acc=None):
    """Fixed-step kick-drift-kick leapfrog (the single-rung case of the
    paper's adaptive symplectic integrator, Sec. 2.1):
    v += a dt/2; x = wrap(x + v dt); a = forces(x); v += a dt/2.
    Returns (pos, vel, acc, pot) after nsteps."""
    box = float(params.get("box", 1.0))
    periodic = int(params.get("periodic", 1))
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    pot = None
    if acc is None:
        acc, pot = Tree(pos, mass, params).forces()
    for _ in range(nsteps):
        vel = vel + (0.5 * dt) * acc
        pos = pos + dt * vel
        if periodic:
            pos = wrap_box(pos, box)
        acc, pot = Tree(pos, mass, params).forces()
        vel = vel + (0.5 * dt) * acc
    return pos, vel, acc, pot


def hubble(a, omega_m: float, omega_l: float, h0: float):
    """H(a) = h0 sqrt(omega_m a^-3 + omega_k a^-2 + omega_l), omega_k =
    1 - omega_m - omega_l: the expansion rate of the background of the
    paper's comoving volumes (Sec. 3: omega_m 0.295, omega_lambda 0.705)."""
    return h0 * np.sqrt(omega_m / a ** 3 + (1.0 - omega_m - omega_l) / a ** 2 + omega_l)


def comoving_factors(a1: float, a2: float, omega_m: float, omega_l: float, h0: float):
    """(K, D) over [a1, a2]: K = int da / (a^2 H(a)) = int dt / a (the kick of
    the canonical momentum p = a^2 dx/dt under dp/dt = -grad(phi) / a) and
    D = int da / (a^3 H(a)) = int dt / a^2 (the drift, dx/dt = p / a^2),
    by adaptive quadrature in a."""
    from scipy.integrate import quad
    k = quad(lambda a: 1.0 / (a * a * hubble(a, omega_m, omega_l, h0)), a1, a2,
             epsabs=0.0, epsrel=2e-14, limit=200)[0]
    d = quad(lambda a: 1.0 / (a ** 3 * hubble(a, omega_m, omega_l, h0)), a1, a2,
             epsabs=0.0, epsrel=2e-14, limit=200)[0]
    return k, d


def kdk_comoving(pos, vel, mass, params: dict, a0: float, da: float, nsteps: int,
                 omega_m: float, omega_l: float, h0: float, acc=None):
    """Kick-drift-kick leapfrog in comoving coordinates (paper Sec. 2.1's
    symplectic integrator for the comoving volumes of Sec. 3): pos comoving,
    vel the canonical momenta p = a^2 dx/dt, steps of da in the scale factor;
    per step, with a_h the middle of [a_k, a_k+1],
    p += acc K(a_k, a_h); x = wrap(x + p D(a_k, a_k+1)); acc = forces(x);
    p += acc K(a_h, a_k+1).  Returns (pos, vel, acc, pot)."""
    box = float(params.get("box", 1.0))
    periodic = int(params.get("periodic", 1))
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    pot = None
    if acc is None:
        acc, pot = Tree(pos, mass, params).forces()
    for k in range(nsteps):
        ak, a1 = a0 + k * da, a0 + (k + 1) * da
        ah = ak + 0.5 * da
        vel = vel + comoving_factors(ak, ah, omega_m, omega_l, h0)[0] * acc
        pos = pos + comoving_factors(ak, a1, omega_m, omega_l, h0)[1] * vel
        if periodic:
            pos = wrap_box(pos, box)
        acc, pot = Tree(pos, mass, params).forces()
        vel = vel + comoving_factors(ah, a1, omega_m, omega_l, h0)[0] * acc
    return pos, vel, acc, pot


def rung_of(acc, dt: float, max_rung: int, eta: float, eps: float):
    """Block-timestep rung of each particle from its acceleration: the
    largest step dt/2^r, r <= max_rung, not above eta sqrt(eps/|a|) (the
    acceleration criterion of multiple-timestep tree codes)."""
    acc = np.asarray(acc, dtype=np.float64)
    a2 = acc[0] * acc[0]
    a2 = a2 + acc[1] * acc[1]
    a2 = a2 + acc[2] * acc[2]
    with np.errstate(divide="ignore"):
        want = eta * np.sqrt(eps / np.sqrt(a2))
    r = np.zeros(acc.shape[1], dtype=np.int64)
    for k in range(max_rung):
        r += (np.ldexp(dt, -r) > want) & (r == k)
    return r


def _ctz(q: int) -> int:
    return (q & -q).bit_length() - 1


def kdk_block(pos, vel, mass, params: dict, dt: float, max_rung: int, eta: float, nsteps: int,
              acc=None, pot=None, rung=None, fixed: bool = False):
    """Block (multiple) timesteps, the paper's adaptive symplectic integrator
    (Sec. 2.1) read as hierarchical kick-drift-kick on power-of-two rungs:
    particle i steps dt/2^rung_i; time advances in substeps dt/2^max_rung
    through which every particle drifts; at each substep boundary the
    particles whose step ends there take their new acceleration, a closing
    half kick and (unless fixed) a new rung no coarser than the steps that
    can start there; the particles starting a step take an opening half
    kick.  A substep boundary where no particle is due only drifts.  Returns
    (pos, vel, acc, pot, rung, force evaluations)."""
    box = float(params.get("box", 1.0))
    periodic = int(params.get("periodic", 1))
    eps = float(params.get("eps", 0.0))
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    if acc is None:
        acc, pot = Tree(pos, mass, params).forces()
    acc = np.array(acc, dtype=np.float64)
    pot = None if pot is None else np.array(pot, dtype=np.float64)
    rung = (rung_of(acc, dt, max_rung, eta, eps) if rung is None
            else np.array(rung, dtype=np.int64))
    S = 1 << max_rung
    sub = np.ldexp(dt, -max_rung)
    nev = 0
    for _ in range(nsteps):
        for q in range(S):
            rstart = 0 if q == 0 else max_rung - _ctz(q)
            m = rung >= rstart
            vel[:, m] = vel[:, m] + acc[:, m] * (0.5 * np.ldexp(dt, -rung[m]))
            pos = pos + vel * sub
            if periodic:
                pos = wrap_box(pos, box)
            rend = 0 if q + 1 == S else max_rung - _ctz(q + 1)
            m = rung >= rend
            if not np.any(m):
                continue
            a_new, p_new = Tree(pos, mass, params).forces()
            nev += 1
            acc[:, m] = a_new[:, m]
            if pot is None:
                pot = np.zeros(pos.shape[1])
            pot[m] = p_new[m]
            vel[:, m] = vel[:, m] + acc[:, m] * (0.5 * np.ldexp(dt, -rung[m]))
            if not fixed:
                rung[m] = np.maximum(rung_of(acc[:, m], dt, max_rung, eta, eps), rend)
    return pos, vel, acc, pot, rung, nev


def kdk_trajectory(pos, vel, mass, params: dict, dt: float, nsteps: int):
    """Positions at the start of every step and at the end, [x_0 .. x_n]
    (each 3 x N), and the final velocities, of ``kdk``."""
    xs = [np.array(pos, dtype=np.float64)]
    p, v, acc = xs[0], np.array(vel, dtype=np.float64), None
    for _ in range(nsteps):
        p, v, acc, _ = kdk(p, v, mass, params, dt, 1, acc=acc)
        xs.append(p)
    return xs, v


def kdk_vjp(xs, mass, params: dict, dt: float, xbar, vbar):
    """Reverse-mode derivative of ``kdk`` over len(xs) - 1 steps, taken one
    operation at a time backwards through each step
        v' = v + a(x) dt/2,  x1 = wrap(x + v' dt),  v1 = v' + a(x1) dt/2
    (the wrap has unit derivative).  xs are the step-start positions and the
    final ones; xbar, vbar the cotangents of the final positions and
    velocities.  Returns the cotangents (x0bar, v0bar, mbar) of the initial
    positions, the initial velocities and the masses.  The force derivative
    is Tree.vjp (exact for theta = 0)."""
    xb = np.array(xbar, dtype=np.float64)
    vb = np.array(vbar, dtype=np.float64)
    mb = np.zeros(len(mass))
    for k in range(len(xs) - 2, -1, -1):
        # v1 = v' + a(x1) dt/2
        vpb = vb.copy()
        tx, tm = Tree(xs[k + 1], mass, params).vjp(0.5 * dt * vb)
        xb = xb + tx
        mb = mb + tm
        # x1 = wrap(x + v' dt)
        vpb = vpb + dt * xb
        # v' = v + a(x) dt/2
        tx, tm = Tree(xs[k], mass, params).vjp(0.5 * dt * vpb)
        xb = xb + tx
        mb = mb + tm
        vb = vpb
    return xb, vb, mb
