"""ctypes binding of libhot (include/hot.h): argument marshalling only.

Every step of the force evaluation runs in the HIP library; PyTorch provides
device memory (tensors) and the stream.  Importing works without a GPU (so the
symbol table can be checked on a CPU-only machine); any compute call raises
if the library or a GPU is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhot.so")

HOT_OK, HOT_EINVAL, HOT_ENOMEM, HOT_EOVERFLOW, HOT_EDEVICE, HOT_EUNSUPPORTED = range(6)
HOT_FP64, HOT_FP32 = 0, 1
HOT_ACC_VALID = 1
HOT_KDK_NO_SNAPSHOT = 2
HOT_RUNG_VALID = 4
HOT_RUNG_FIXED = 8
HOT_CALL_FORCES, HOT_CALL_KDK, HOT_CALL_VJP, HOT_CALL_KDK_VJP = 1, 2, 4, 8
STATUS_NAMES = {0: "HOT_OK", 1: "HOT_EINVAL", 2: "HOT_ENOMEM", 3: "HOT_EOVERFLOW",
                4: "HOT_EDEVICE", 5: "HOT_EUNSUPPORTED"}

# symbols declared in include/hot.h
EXPORTED = ["hot_create", "hot_destroy", "hot_workspace_size", "hot_workspace_size_min",
            "hot_forces", "hot_forces_noalloc", "hot_kdk", "hot_kdk_comoving",
            "hot_comoving_factors", "hot_kdk_block",
            "hot_vjp", "hot_vjp_after_forces", "hot_kdk_vjp", "hot_get_stats", "hot_debug_sizes", "hot_debug_export",
            "hot_debug_list_range", "hot_cell_lookup", "hot_last_error", "hot_version",
            "hot_far_table"]


class HotError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class hot_params(C.Structure):
    _fields_ = [("box", C.c_double), ("G", C.c_double), ("eps", C.c_double),
                ("theta", C.c_double), ("order", C.c_int), ("periodic", C.c_int),
                ("leaf_max", C.c_int), ("group_max", C.c_int), ("far_order", C.c_int),
                ("precision", C.c_int), ("err_tol", C.c_double), ("kernel", C.c_int),
                ("local_order", C.c_int), ("local_tol", C.c_double)]


class hot_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncells", C.c_int64), ("ngroups", C.c_int64),
                ("nlevels", C.c_int64), ("p2p_entries", C.c_int64), ("m2p_entries", C.c_int64),
                ("p2p_pairs", C.c_int64), ("m2p_pairs", C.c_int64), ("flops_p2p", C.c_double),
                ("flops_m2p", C.c_double), ("ms_total", C.c_double), ("ms_sort", C.c_double),
                ("ms_build", C.c_double), ("ms_walk", C.c_double), ("ms_p2p", C.c_double),
                ("ms_m2p", C.c_double), ("ms_far", C.c_double), ("ws_bytes_needed", C.c_size_t),
                ("kdk_steps_done", C.c_int64), ("list_chunks", C.c_int64),
                ("m2p_lanes_main", C.c_int64), ("m2p_lanes_tail", C.c_int64),
                ("m2p_pairs_tail", C.c_int64), ("m2l_entries", C.c_int64),
                ("m2l_pairs", C.c_int64), ("flops_m2l", C.c_double), ("ms_m2l", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class hot_debug(C.Structure):
    _fields_ = [("sorted_keys", C.c_void_p), ("perm", C.c_void_p), ("cell_key", C.c_void_p),
                ("cell_level", C.c_void_p), ("cell_first", C.c_void_p),
                ("cell_count", C.c_void_p), ("cell_com", C.c_void_p), ("cell_mass", C.c_void_p),
                ("group_cell", C.c_void_p), ("p2p_offset", C.c_void_p),
                ("p2p_entry", C.c_void_p), ("m2p_offset", C.c_void_p),
                ("m2p_entry", C.c_void_p), ("m2l_offset", C.c_void_p),
                ("m2l_entry", C.c_void_p)]


_lib = None


def lib():
    """Load libhot.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                              "python paper_1407_2600_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.hot_create.restype = C.c_int
        L.hot_create.argtypes = [C.POINTER(hot_params), C.POINTER(vp)]
        L.hot_destroy.argtypes = [vp]
        L.hot_workspace_size.restype = sz
        L.hot_workspace_size.argtypes = [vp, sz]
        L.hot_workspace_size_min.restype = sz
        L.hot_workspace_size_min.argtypes = [vp, sz, C.c_uint]
        L.hot_forces.restype = C.c_int
        L.hot_forces.argtypes = [vp, sz, vp, vp, vp, vp, vp, sz, vp]
        L.hot_forces_noalloc.restype = C.c_int
        L.hot_forces_noalloc.argtypes = [vp, sz, vp, vp, vp, vp, vp]
        L.hot_kdk.restype = C.c_int
        L.hot_kdk.argtypes = [vp, sz, vp, vp, vp, vp, vp, C.c_double, C.c_int, C.c_uint, vp, sz,
                              vp]
        L.hot_kdk_block.restype = C.c_int
        L.hot_kdk_block.argtypes = [vp, sz, vp, vp, vp, vp, vp, vp, C.c_double, C.c_int,
                                    C.c_double, C.c_int, C.c_uint, vp, sz, vp]
        L.hot_vjp.restype = C.c_int
        L.hot_vjp.argtypes = [vp, sz, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.hot_vjp_after_forces.restype = C.c_int
        L.hot_vjp_after_forces.argtypes = [vp, sz, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.hot_kdk_vjp.restype = C.c_int
        L.hot_kdk_vjp.argtypes = [vp, sz, C.c_int, vp, vp, C.c_double, vp, vp, vp, vp, sz, vp]
        L.hot_get_stats.restype = C.c_int
        L.hot_get_stats.argtypes = [vp, C.POINTER(hot_stats)]
        L.hot_debug_sizes.restype = C.c_int
        L.hot_debug_sizes.argtypes = [vp] + [C.POINTER(C.c_int64)] * 5
        L.hot_debug_export.restype = C.c_int
        L.hot_debug_export.argtypes = [vp, vp, C.POINTER(hot_debug)]
        L.hot_cell_lookup.restype = C.c_int
        L.hot_cell_lookup.argtypes = [vp, vp, sz, vp, vp, vp]
        L.hot_debug_list_range.restype = C.c_int
        L.hot_debug_list_range.argtypes = [vp, vp, C.c_int, C.c_int64, C.c_int64, vp]
        L.hot_last_error.restype = C.c_char_p
        L.hot_version.restype = C.c_char_p
        L.hot_kdk_comoving.restype = C.c_int
        L.hot_kdk_comoving.argtypes = [vp, sz, vp, vp, vp, vp, vp, C.c_double, C.c_double,
                                       C.c_int, C.c_double, C.c_double, C.c_double, C.c_uint,
                                       vp, sz, vp]
        L.hot_comoving_factors.restype = C.c_int
        L.hot_comoving_factors.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)]
        L.hot_far_table.restype = C.c_int
        L.hot_far_table.argtypes = [C.c_int, C.c_double, C.c_int, C.POINTER(C.c_double), sz]
        _lib = L
    return _lib


def check(status: int):
    if status != HOT_OK:
        raise HotError(status, lib().hot_last_error().decode())


HOT_KERNEL_PLUMMER, HOT_KERNEL_K1 = 0, 1
KERNELS = {"plummer": HOT_KERNEL_PLUMMER, "k1": HOT_KERNEL_K1, 0: 0, 1: 1}


def make_params(box=1.0, G=1.0, eps=0.0, theta=0.5, order=4, periodic=1, leaf_max=16,
                group_max=64, far_order=8, precision="fp64", err_tol=0.0, kernel="plummer",
                local_order=0, local_tol=0.0, **_ignored) -> hot_params:
    prec = precision
    if isinstance(prec, str):
        prec = {"fp64": HOT_FP64, "fp32": HOT_FP32}[prec]
    return hot_params(float(box), float(G), float(eps), float(theta), int(order), int(periodic),
                      int(leaf_max), int(group_max), int(far_order), int(prec), float(err_tol),
                      KERNELS[kernel], int(local_order), float(local_tol))


def comoving_factors(a1: float, a2: float, omega_m: float, omega_l: float, h0: float):
    """(K, D): the kick and drift factors of hot_kdk_comoving over [a1, a2]
    (host-only)."""
    out = (C.c_double * 2)()
    check(lib().hot_comoving_factors(float(a1), float(a2), float(omega_m), float(omega_l),
                                     float(h0), out))
    return out[0], out[1]


def far_table(far_order: int, box: float = 1.0, offset: int = 13):
    """The library's Taylor table of the periodic remainder about the octant
    offset (dx,dy,dz) L/2, offset = (dx+1)*9+(dy+1)*3+(dz+1) (host code)."""
    import numpy as np
    n = (2 * far_order + 1) * (2 * far_order + 2) * (2 * far_order + 3) // 6
    out = np.zeros(n)
    check(lib().hot_far_table(int(far_order), float(box), int(offset),
                              out.ctypes.data_as(C.POINTER(C.c_double)), n))
    return out


class Gravity:
    """One libhot context: parameters, Ewald table and a cached workspace."""

    def __init__(self, device=None, workspace_bytes=None, list_bytes=None, **params):
        """workspace_bytes caps the device workspace (at least the library's
        minimum for the call is used); list_bytes instead sizes it as that
        minimum plus a list region of this many bytes.  Interaction lists
        that do not fit are processed in chunks of sink groups."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libhot needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.params = dict(params)
        self.prm = make_params(**params)
        self.fp32 = self.prm.precision == HOT_FP32
        self.dtype = torch.float32 if self.fp32 else torch.float64
        self.L = lib()
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(self.L.hot_create(C.byref(self.prm), C.byref(h)))
        self.h = h
        self.ws = None
        self.ws_cap = workspace_bytes
        self.list_bytes = list_bytes
        # compute calls made on this context; the autograd backward reuses a
        # forward evaluation's tree and lists only if no call came after it
        self.evals = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h and getattr(self, "L", None) is not None:
            self.L.hot_destroy(h)
            self.h = None

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _workspace(self, n: int, calls: int = HOT_CALL_FORCES):
        need = self.L.hot_workspace_size(self.h, n)
        lo = self.L.hot_workspace_size_min(self.h, n, calls)
        if self.list_bytes is not None:
            need = min(need, lo + int(self.list_bytes))
        if self.ws_cap is not None:
            need = max(min(need, int(self.ws_cap)), lo)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self.ws

    def _check_inputs(self, pos, mass):
        t = self.torch
        if pos.device != self.device or mass.device != self.device:
            raise ValueError("pos and mass must be on the context's device")
        if pos.dtype != t.float64 or pos.dim() != 2 or pos.shape[0] != 3:
            raise ValueError("pos must be a (3, N) float64 tensor")
        if mass.dtype != self.dtype or mass.shape != (pos.shape[1],):
            raise ValueError(f"mass must be a (N,) {self.dtype} tensor")
        return pos.contiguous(), mass.contiguous()

    def _call_retry(self, fn, n, calls=HOT_CALL_FORCES):
        self.evals += 1
        for _ in range(6):
            ws = self._workspace(n, calls)
            st = fn(ws)
            if st != HOT_EOVERFLOW:
                check(st)
                return
        check(st)

    def forces(self, pos, mass, out_acc=None, out_pot=None, want_pot=True):
        """(acc[3,N], pot[N]) in the context's precision."""
        t = self.torch
        pos, mass = self._check_inputs(pos, mass)
        n = pos.shape[1]
        acc = out_acc if out_acc is not None else t.empty((3, n), dtype=self.dtype,
                                                          device=self.device)
        pot = out_pot if out_pot is not None else (
            t.empty(n, dtype=self.dtype, device=self.device) if want_pot else None)
        if n == 0:
            return acc, pot
        s = self._stream()

        def run(ws):
            return self.L.hot_forces(self.h, n, C.c_void_p(pos.data_ptr()),
                                     C.c_void_p(mass.data_ptr()), C.c_void_p(acc.data_ptr()),
                                     C.c_void_p(pot.data_ptr() if pot is not None else 0),
                                     C.c_void_p(ws.data_ptr()), ws.numel(), s)
        self._call_retry(run, n)
        return acc, pot

    def forces_noalloc(self, pos, mass, out_acc, out_pot=None):
        """forces() through hot_forces_noalloc: the library's fixed device
        scratch instead of a workspace; the caller passes the outputs, so
        nothing is allocated."""
        pos, mass = self._check_inputs(pos, mass)
        n = pos.shape[1]
        for name, a, shape in (("out_acc", out_acc, (3, n)), ("out_pot", out_pot, (n,))):
            if a is not None and (a.dtype != self.dtype or tuple(a.shape) != shape or
                                  not a.is_contiguous() or a.device != self.device):
                raise ValueError(f"{name} must be a contiguous {shape} {self.dtype} tensor "
                                 "on the context's device")
        if out_acc is None:
            raise ValueError("out_acc is required")
        self.evals += 1
        check(self.L.hot_forces_noalloc(self.h, n, C.c_void_p(pos.data_ptr()),
                                        C.c_void_p(mass.data_ptr()),
                                        C.c_void_p(out_acc.data_ptr()),
                                        C.c_void_p(out_pot.data_ptr() if out_pot is not None
                                                   else 0), self._stream()))
        return out_acc, out_pot

    def kdk(self, pos, vel, mass, acc, dt: float, nsteps: int, acc_valid: bool, pot=None,
            snapshot: bool = True):
        """In-place leapfrog steps on pos (FP64), vel and acc (precision).
        snapshot=False saves 36 bytes per particle of workspace; a failed
        step then raises with pos and vel undefined (no resumption)."""
        pos_c, mass = self._check_inputs(pos, mass)
        if not (pos_c.data_ptr() == pos.data_ptr()):
            raise ValueError("pos must be contiguous (it is updated in place)")
        for name, a in (("vel", vel), ("acc", acc)):
            if a.dtype != self.dtype or a.shape != pos.shape or not a.is_contiguous():
                raise ValueError(f"{name} must be a contiguous (3, N) {self.dtype} tensor")
        n = pos.shape[1]
        s = self._stream()
        self.evals += 1
        left, valid = int(nsteps), bool(acc_valid)
        # after HOT_EOVERFLOW the library has restored the state at the end of
        # the last completed step; resume from there with a larger workspace
        for _ in range(6):
            ws = self._workspace(n, HOT_CALL_KDK if snapshot else HOT_CALL_FORCES)
            st = self.L.hot_kdk(self.h, n, C.c_void_p(pos.data_ptr()),
                                C.c_void_p(vel.data_ptr()), C.c_void_p(mass.data_ptr()),
                                C.c_void_p(acc.data_ptr()),
                                C.c_void_p(pot.data_ptr() if pot is not None else 0),
                                float(dt), left,
                                (HOT_ACC_VALID if valid else 0) |
                                (0 if snapshot else HOT_KDK_NO_SNAPSHOT),
                                C.c_void_p(ws.data_ptr()), ws.numel(), s)
            if st != HOT_EOVERFLOW or not snapshot:
                check(st)
                return
            done = self.stats()["kdk_steps_done"]
            valid = valid or done > 0
            left -= done
        check(st)

    def kdk_comoving(self, pos, vel, mass, acc, a0: float, da: float, nsteps: int,
                     omega_m: float, omega_l: float, h0: float, acc_valid: bool, pot=None,
                     snapshot: bool = True):
        """In-place leapfrog steps in comoving coordinates (pos comoving, vel
        the canonical momenta p = a^2 dx/dt), nsteps steps of da in the scale
        factor from a0 (hot_kdk_comoving).  Resumes after HOT_EOVERFLOW like
        kdk()."""
        pos_c, mass = self._check_inputs(pos, mass)
        if not (pos_c.data_ptr() == pos.data_ptr()):
            raise ValueError("pos must be contiguous (it is updated in place)")
        for name, a in (("vel", vel), ("acc", acc)):
            if a.dtype != self.dtype or a.shape != pos.shape or not a.is_contiguous():
                raise ValueError(f"{name} must be a contiguous (3, N) {self.dtype} tensor")
        n = pos.shape[1]
        s = self._stream()
        self.evals += 1
        left, valid, a = int(nsteps), bool(acc_valid), float(a0)
        for _ in range(6):
            ws = self._workspace(n, HOT_CALL_KDK if snapshot else HOT_CALL_FORCES)
            st = self.L.hot_kdk_comoving(self.h, n, C.c_void_p(pos.data_ptr()),
                                         C.c_void_p(vel.data_ptr()), C.c_void_p(mass.data_ptr()),
                                         C.c_void_p(acc.data_ptr()),
                                         C.c_void_p(pot.data_ptr() if pot is not None else 0),
                                         a, float(da), left, float(omega_m), float(omega_l),
                                         float(h0),
                                         (HOT_ACC_VALID if valid else 0) |
                                         (0 if snapshot else HOT_KDK_NO_SNAPSHOT),
                                         C.c_void_p(ws.data_ptr()), ws.numel(), s)
            if st != HOT_EOVERFLOW or not snapshot:
                check(st)
                return
            done = self.stats()["kdk_steps_done"]
            valid = valid or done > 0
            left -= done
            a += done * float(da)
        check(st)

    def kdk_block(self, pos, vel, mass, acc, rung, dt: float, max_rung: int, eta: float,
                  nsteps: int, acc_valid: bool, rung_valid: bool, fixed_rungs: bool = False,
                  pot=None):
        """In-place block-timestep steps (hot_kdk_block) on pos (FP64), vel,
        acc (precision) and rung (uint8).  The workspace is first sized by a
        force evaluation when it has not been yet (no snapshots are kept)."""
        t = self.torch
        pos_c, mass = self._check_inputs(pos, mass)
        if not (pos_c.data_ptr() == pos.data_ptr()):
            raise ValueError("pos must be contiguous (it is updated in place)")
        n = pos.shape[1]
        for name, a in (("vel", vel), ("acc", acc)):
            if a.dtype != self.dtype or a.shape != pos.shape or not a.is_contiguous():
                raise ValueError(f"{name} must be a contiguous (3, N) {self.dtype} tensor")
        if rung.dtype != t.uint8 or rung.shape != (n,) or not rung.is_contiguous():
            raise ValueError("rung must be a contiguous (N,) uint8 tensor")
        if self.ws is None:
            a0, p0 = self.forces(pos, mass)
            if not acc_valid:
                acc.copy_(a0)
                if pot is not None:
                    pot.copy_(p0)
                acc_valid = True
        self.evals += 1
        ws = self._workspace(n, HOT_CALL_FORCES)
        flags = ((HOT_ACC_VALID if acc_valid else 0) | (HOT_RUNG_VALID if rung_valid else 0) |
                 (HOT_RUNG_FIXED if fixed_rungs else 0))
        check(self.L.hot_kdk_block(self.h, n, C.c_void_p(pos.data_ptr()),
                                   C.c_void_p(vel.data_ptr()), C.c_void_p(mass.data_ptr()),
                                   C.c_void_p(acc.data_ptr()),
                                   C.c_void_p(pot.data_ptr() if pot is not None else 0),
                                   C.c_void_p(rung.data_ptr()), float(dt), int(max_rung),
                                   float(eta), int(nsteps), flags, C.c_void_p(ws.data_ptr()),
                                   ws.numel(), self._stream()))

    def kdk_vjp(self, pos_ckpt, mass, dt: float, xbar, vbar):
        """Reverse sweep over len(pos_ckpt) - 1 leapfrog steps (hot_kdk_vjp).
        pos_ckpt: (S+1, 3, N) FP64 positions at each step start and the end;
        xbar (FP64) and vbar (precision): cotangents of the final state,
        updated in place to those of the initial state.  Returns mbar."""
        t = self.torch
        if pos_ckpt.dtype != t.float64 or pos_ckpt.dim() != 3 or pos_ckpt.shape[1] != 3:
            raise ValueError("pos_ckpt must be a (S+1, 3, N) float64 tensor")
        pos_ckpt = pos_ckpt.contiguous()
        n = pos_ckpt.shape[2]
        _, mass = self._check_inputs(pos_ckpt[0], mass)
        for name, a, dt_ in (("xbar", xbar, t.float64), ("vbar", vbar, self.dtype)):
            if a.dtype != dt_ or a.shape != (3, n) or not a.is_contiguous():
                raise ValueError(f"{name} must be a contiguous (3, N) {dt_} tensor")
        mbar = t.empty(n, dtype=self.dtype, device=self.device)
        s = self._stream()

        def run(ws):
            return self.L.hot_kdk_vjp(self.h, n, pos_ckpt.shape[0] - 1,
                                      C.c_void_p(pos_ckpt.data_ptr()),
                                      C.c_void_p(mass.data_ptr()), float(dt),
                                      C.c_void_p(xbar.data_ptr()), C.c_void_p(vbar.data_ptr()),
                                      C.c_void_p(mbar.data_ptr()), C.c_void_p(ws.data_ptr()),
                                      ws.numel(), s)
        self._call_retry(run, n, HOT_CALL_KDK_VJP)
        return mbar

    def vjp(self, pos, mass, gacc, gpot=None, after_forces=False):
        """(xbar[3,N] FP64, mbar[N]) for cotangents of (acc, pot).  With
        after_forces the caller guarantees that pos and mass hold the values
        of this object's last evaluation, whose tree and lists the library
        then reuses when it can (hot_vjp_after_forces)."""
        t = self.torch
        pos, mass = self._check_inputs(pos, mass)
        n = pos.shape[1]
        gacc = gacc.to(self.dtype).contiguous()
        gpot = gpot.to(self.dtype).contiguous() if gpot is not None else None
        xbar = t.empty((3, n), dtype=t.float64, device=self.device)
        mbar = t.empty(n, dtype=self.dtype, device=self.device)
        s = self._stream()

        fn = self.L.hot_vjp_after_forces if after_forces else self.L.hot_vjp

        def run(ws):
            return fn(self.h, n, C.c_void_p(pos.data_ptr()),
                                  C.c_void_p(mass.data_ptr()), C.c_void_p(gacc.data_ptr()),
                                  C.c_void_p(gpot.data_ptr() if gpot is not None else 0),
                                  C.c_void_p(xbar.data_ptr()), C.c_void_p(mbar.data_ptr()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), s)
        self._call_retry(run, n, HOT_CALL_VJP)
        return xbar, mbar

    def stats(self) -> dict:
        st = hot_stats()
        check(self.L.hot_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def cell_lookup(self, keys):
        """Cell index (library order) of each key in the last evaluation's
        hashed oct-tree, -1 where the tree has no such cell.  keys: int64
        tensor on the device holding the uint64 key bit patterns."""
        t = self.torch
        keys = keys.to(self.device, dtype=t.int64).contiguous()
        out = t.empty(keys.numel(), dtype=t.int32, device=self.device)
        check(self.L.hot_cell_lookup(self.h, C.c_void_p(self.ws.data_ptr()), keys.numel(),
                                     C.c_void_p(keys.data_ptr()), C.c_void_p(out.data_ptr()),
                                     self._stream()))
        return out

    def debug_list_range(self, kind: int, first: int, count: int):
        """count entries of the last forces() call's direct (kind 0),
        multipole (kind 1) or local (kind 2) list, from entry first (host
        uint32 array)."""
        import numpy as np
        out = np.zeros(int(count), np.uint32)
        check(self.L.hot_debug_list_range(self.h, C.c_void_p(self.ws.data_ptr()), int(kind),
                                          int(first), int(count),
                                          C.c_void_p(out.ctypes.data if count else None)))
        return out

    def debug_export(self, lists: bool = True) -> dict:
        """Host copies of keys, permutation, cells, groups, the per-group list
        offsets and (unless lists is False) the interaction lists of the last
        forces() call."""
        import numpy as np
        sizes = [C.c_int64() for _ in range(5)]
        check(self.L.hot_debug_sizes(self.h, *[C.byref(x) for x in sizes]))
        n, nc, ng, tp, tm = [x.value for x in sizes]
        st = self.stats()
        single = st["list_chunks"] == 1
        tl = st["m2l_entries"]
        if not lists:
            tp = tm = tl = 0
        out = dict(sorted_keys=np.zeros(n, np.uint64), perm=np.zeros(n, np.uint32),
                   cell_key=np.zeros(nc, np.uint64), cell_level=np.zeros(nc, np.int32),
                   cell_first=np.zeros(nc, np.int32), cell_count=np.zeros(nc, np.int32),
                   cell_com=np.zeros((3, nc)), cell_mass=np.zeros(nc),
                   group_cell=np.zeros(ng, np.int32), p2p_offset=np.zeros(ng + 1, np.int64),
                   p2p_entry=np.zeros(tp, np.uint32), m2p_offset=np.zeros(ng + 1, np.int64),
                   m2p_entry=np.zeros(tm, np.uint32), m2l_offset=np.zeros(ng + 1, np.int64),
                   m2l_entry=np.zeros(tl, np.uint32))
        skip = () if lists else ("p2p_entry", "m2p_entry", "m2l_entry")
        if not single:
            skip = skip + ("p2p_offset", "m2p_offset", "m2l_offset")
        dbg = hot_debug(*[C.c_void_p(None if f in skip else out[f].ctypes.data)
                          for f, _ in hot_debug._fields_])
        check(self.L.hot_debug_export(self.h, C.c_void_p(self.ws.data_ptr()), C.byref(dbg)))
        return out


def _autograd():
    import torch

    class GravityForces(torch.autograd.Function):
        """acc, pot = GravityForces.apply(gravity, pos, mass); backward runs
        the library's adjoint (hot_vjp)."""

        @staticmethod
        def forward(ctx, grav, pos, mass):
            # the exact (contiguous) tensors the library reads are kept alive
            # until the backward, so no later allocation can take their
            # addresses
            pos_c = pos.detach().contiguous()
            mass_c = mass.detach().contiguous()
            acc, pot = grav.forces(pos_c, mass_c)
            ctx.grav = grav
            ctx.eval_id = grav.evals
            ctx.save_for_backward(pos_c, mass_c)
            return acc, pot

        @staticmethod
        def backward(ctx, gacc, gpot):
            pos, mass = ctx.saved_tensors
            grav = ctx.grav
            if gacc is None:
                gacc = torch.zeros((3, pos.shape[1]), dtype=grav.dtype, device=pos.device)
            # the saved tensors' version check guarantees unchanged positions
            # and masses; the forward's tree and lists are reused only when no
            # other compute call on this context came in between (otherwise
            # the workspace holds that call's structures and the adjoint
            # builds its own tree)
            reuse = grav.evals == ctx.eval_id
            xbar, mbar = grav.vjp(pos, mass, gacc, gpot, after_forces=reuse)
            return None, xbar, mbar

    return GravityForces


_GF = None
_CK = None


def _checkpointed():
    import torch

    class CheckpointedKDK(torch.autograd.Function):
        """(pos_n, vel_n) = CheckpointedKDK.apply(gravity, pos0, vel0, mass,
        dt, nsteps): nsteps leapfrog steps that keep only the positions of
        every step for the backward pass (hot_kdk_vjp rebuilds each tree)."""

        @staticmethod
        def forward(ctx, grav, pos0, vel0, mass, dt, nsteps):
            pos = pos0.detach().clone().contiguous()
            vel = vel0.detach().to(grav.dtype).clone().contiguous()
            mass_d = mass.detach()
            ck = torch.empty((nsteps + 1,) + tuple(pos.shape), dtype=torch.float64,
                             device=pos.device)
            ck[0].copy_(pos)
            acc = torch.empty_like(vel)
            grav.kdk(pos, vel, mass_d, acc, dt, 0, acc_valid=False)
            for k in range(nsteps):
                grav.kdk(pos, vel, mass_d, acc, dt, 1, acc_valid=True)
                ck[k + 1].copy_(pos)
            ctx.grav, ctx.dt = grav, float(dt)
            ctx.save_for_backward(ck, mass_d)
            return pos, vel

        @staticmethod
        def backward(ctx, gpos, gvel):
            ck, mass = ctx.saved_tensors
            grav = ctx.grav
            xbar = (gpos.to(torch.float64).clone() if gpos is not None
                    else torch.zeros(ck.shape[1:], dtype=torch.float64, device=ck.device))
            vbar = (gvel.to(grav.dtype).clone() if gvel is not None
                    else torch.zeros(ck.shape[1:], dtype=grav.dtype, device=ck.device))
            xbar = xbar.contiguous()
            vbar = vbar.contiguous()
            mbar = grav.kdk_vjp(ck, mass, ctx.dt, xbar, vbar)
            return None, xbar, vbar, mbar, None, None

    return CheckpointedKDK


def checkpointed_kdk(grav: Gravity, pos0, vel0, mass, dt: float, nsteps: int):
    """Differentiable nsteps-step leapfrog trajectory with per-step
    checkpointing: (pos_n, vel_n) with gradients to pos0, vel0 and mass."""
    global _CK
    if _CK is None:
        _CK = _checkpointed()
    return _CK.apply(grav, pos0, vel0, mass, dt, int(nsteps))


def gravity_forces(grav: Gravity, pos, mass):
    """Differentiable forces: (acc, pot) with gradients to pos and mass."""
    global _GF
    if _GF is None:
        _GF = _autograd()
    return _GF.apply(grav, pos, mass)
