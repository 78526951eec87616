"""ctypes binding of libhotref (include/hotref.h): exact periodic forces of
selected targets by direct Ewald summation in FP64 on the GPU, the accuracy
reference for evaluations too large for a CPU reference.  Argument
marshalling only; raises if the library or a GPU is missing."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhotref.so")
EXPORTED = ["hotref_scratch_size", "hotref_ewald", "hotref_valu_probe_scratch",
            "hotref_valu_probe", "hotref_last_error"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.hotref_scratch_size.restype = sz
        L.hotref_scratch_size.argtypes = [sz, sz]
        L.hotref_ewald.restype = C.c_int
        L.hotref_ewald.argtypes = [sz, vp, vp, C.c_int, sz, vp, C.c_double, C.c_double,
                                   C.c_double, vp, vp, vp, sz, vp]
        L.hotref_last_error.restype = C.c_char_p
        L.hotref_valu_probe_scratch.restype = sz
        L.hotref_valu_probe.restype = C.c_int
        L.hotref_valu_probe.argtypes = [C.c_int, vp, sz, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        _lib = L
    return _lib


def ewald_reference(pos, mass, targets, box=1.0, G=1.0, eps=0.0):
    """(acc[3, T], pot[T]) FP64 at the targets (int64 indices) for positions
    pos (3, N) FP64 and masses (N,) FP32 or FP64, all on one GPU."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libhotref needs a ROCm GPU")
    dev = pos.device
    if pos.dtype != torch.float64 or pos.dim() != 2 or pos.shape[0] != 3:
        raise ValueError("pos must be a (3, N) float64 tensor")
    if mass.dtype not in (torch.float32, torch.float64) or mass.shape != (pos.shape[1],):
        raise ValueError("mass must be an (N,) float32 or float64 tensor")
    pos = pos.contiguous()
    mass = mass.contiguous()
    tg = torch.as_tensor(targets, dtype=torch.int64, device=dev).contiguous()
    n, nt = pos.shape[1], tg.numel()
    if nt and (int(tg.min()) < 0 or int(tg.max()) >= n):
        raise ValueError("target index out of range")
    acc = torch.empty((3, nt), dtype=torch.float64, device=dev)
    pot = torch.empty(nt, dtype=torch.float64, device=dev)
    L = lib()
    scratch = torch.empty(L.hotref_scratch_size(n, nt), dtype=torch.uint8, device=dev)
    s = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    st = L.hotref_ewald(n, C.c_void_p(pos.data_ptr()), C.c_void_p(mass.data_ptr()),
                        int(mass.dtype == torch.float32), nt, C.c_void_p(tg.data_ptr()),
                        float(box), float(G), float(eps), C.c_void_p(acc.data_ptr()),
                        C.c_void_p(pot.data_ptr()), C.c_void_p(scratch.data_ptr()),
                        scratch.numel(), s)
    if st != 0:
        raise RuntimeError(f"hotref_ewald failed ({st}): {L.hotref_last_error().decode()}")
    torch.cuda.current_stream(dev).synchronize()
    del scratch
    return acc, pot


PROBE_KINDS = {0: "fp32 fma", 1: "fp32 mul", 2: "fp32 add", 3: "fp32 fma/mul/add",
               4: "fp32 fma + rsq per 16", 5: "fp64 fma", 6: "fp32 fma accumulate"}


def valu_probe(repeats: int = 5) -> dict:
    """Wave instructions per second of each probe kind on the current GPU."""
    import torch
    L = lib()
    buf = torch.empty(L.hotref_valu_probe_scratch(), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    out = {}
    for kind, name in PROBE_KINDS.items():
        ms, wi = C.c_double(), C.c_double()
        st = L.hotref_valu_probe(kind, C.c_void_p(buf.data_ptr()), buf.numel(), int(repeats),
                                 C.byref(ms), C.byref(wi))
        if st != 0:
            raise RuntimeError(f"hotref_valu_probe({kind}) failed ({st})")
        out[name] = {"ms": ms.value, "wave_instructions": wi.value,
                     "wave_instr_per_s": wi.value / (ms.value * 1e-3)}
    return out
