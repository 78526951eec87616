"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/hot.h declares, rejects bad parameters before touching a GPU, and its
host-built far-field table (a separate derivation from the oracle's) agrees
with the oracle's table."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1407_2600_amd import hot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hot.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hot_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hot.lib()
    names = _declared()
    assert "hot_forces" in names and "hot_vjp" in names and "hot_kdk" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(hot.EXPORTED)


def test_reference_library_exports_every_declared_symbol():
    """libhotref (the FP64 Ewald reference, include/hotref.h) loads and
    exports what its header declares; its scratch size is a host query."""
    from paper_1407_2600_amd import hotref
    src = open(os.path.join(ROOT, "include", "hotref.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(hotref_[a-z_]+)\s*\(", src)))
    L = hotref.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(hotref.EXPORTED)
    small = L.hotref_scratch_size(4096, 100)
    big = L.hotref_scratch_size(1 << 30, 1000)
    assert 0 < small < big < (1 << 30)
    # no compute without a GPU: bad arguments are refused on the host
    assert L.hotref_ewald(0, None, None, 0, 1, None, 1.0, 1.0, 0.0, None, None, None, 0,
                          None) == 1


def test_version_and_error_strings():
    L = hot.lib()
    assert L.hot_version().startswith(b"libhot")
    assert isinstance(L.hot_last_error(), bytes)


@pytest.mark.parametrize("bad", [dict(box=0.0), dict(theta=1.0), dict(theta=-0.1), dict(order=5),
                                 dict(eps=-1.0), dict(leaf_max=0), dict(far_order=13),
                                 dict(periodic=2), dict(precision=7), dict(group_max=0),
                                 dict(err_tol=-1e-3), dict(err_tol=float("nan")),
                                 dict(err_tol=float("inf")), dict(kernel=2),
                                 dict(kernel="k1", eps=0.0), dict(local_order=3),
                                 dict(local_order=6), dict(local_order=-2),
                                 dict(local_order=4, local_tol=-1e-3),
                                 dict(local_order=4, local_tol=float("nan"))])
def test_create_rejects_bad_parameters(bad):
    L = hot.lib()
    prm = hot.make_params(**dict(dict(eps=0.01), **{k: v for k, v in bad.items()
                                                    if k not in ("precision", "kernel") or
                                                    v in hot.KERNELS}))
    if "precision" in bad:
        prm.precision = bad["precision"]
    if bad.get("kernel") not in (None, *hot.KERNELS):
        prm.kernel = bad["kernel"]
    h = C.c_void_p(123)
    st = L.hot_create(C.byref(prm), C.byref(h))
    assert st == hot.HOT_EINVAL
    assert h.value is None
    assert len(L.hot_last_error()) > 0


def test_null_arguments():
    L = hot.lib()
    assert L.hot_forces(None, 10, None, None, None, None, None, 0, None) == hot.HOT_EINVAL
    assert L.hot_workspace_size(None, 100) == 0
    assert L.hot_workspace_size_min(None, 100, 1) == 0
    assert L.hot_get_stats(None, None) == hot.HOT_EINVAL
    L.hot_destroy(None)


@pytest.mark.parametrize("pf", [2, 4, 8, 10])
def test_far_table_matches_oracle(pf):
    lib_tab = hot.far_table(pf, 1.0)
    ora = oracle.psi_table(2 * pf, 1.0)
    deg = np.array([sum(m) for m in oracle.mi_list(2 * pf)])
    for d in range(0, 2 * pf + 1):
        s = deg == d
        scale = np.max(np.abs(ora[s]))
        err = np.max(np.abs(lib_tab[s] - ora[s]))
        # the real/reciprocal split cancels more digits as the degree grows:
        # both tables are alpha-independent to ~1e-10 at degree 16
        rtol = 1e-11 if d <= 8 else (1e-8 if d <= 18 else 1e-6)
        if d % 2:  # odd degrees vanish: both sides are rounding noise
            scale = np.max(np.abs(ora[deg == d - 1]))
            rtol = 1e-11
        assert err <= rtol * max(scale, 1e-300) + 1e-14, (d, err, scale)


@pytest.mark.parametrize("offset", [0, 4, 12, 14, 22, 26])
def test_far_table_offsets_match_oracle(offset):
    pf = 6
    r0 = np.array([offset // 9 - 1, (offset // 3) % 3 - 1, offset % 3 - 1], float) * 0.5
    lib_tab = hot.far_table(pf, 1.0, offset)
    ora = oracle.psi_table_at(2 * pf, r0, 1.0)
    deg = np.array([sum(m) for m in oracle.mi_list(2 * pf)])
    for d in range(0, 2 * pf + 1, 2):
        s = deg == d
        scale = np.max(np.abs(ora[s]))
        # the Ewald split cancels more digits at high degree (both tables are
        # independent of the split parameter to ~1e-10 at degree 10-12)
        rtol = 1e-12 if d <= 2 else (2e-10 if d <= 8 else 2e-9)
        assert np.max(np.abs(lib_tab[s] - ora[s])) <= rtol * scale, (d,)


def test_far_table_box_scaling_and_rejects():
    t1 = hot.far_table(6, 1.0)
    t2 = hot.far_table(6, 2.0)
    deg = np.array([sum(m) for m in oracle.mi_list(12)])
    np.testing.assert_allclose(t2, t1 / 2.0 ** (deg + 1), rtol=1e-9, atol=1e-15)
    with pytest.raises(hot.HotError):
        hot.far_table(13, 1.0)
    with pytest.raises(hot.HotError):
        hot.far_table(4, 1.0, 27)
