"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/nmf.h declares, and validates configurations."""

import ctypes
import os
import re

import pytest

from paper_1510_05237_amd import nmf as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nmf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nmf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    names = _declared()
    assert "nmf_create" in names and "nmf_als_step" in names
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares the same set
    assert sorted(B.SIGNATURES) == names


def _cfg(**kw):
    c = dict(n=1000, m=2000, k=10, mode=B.NMF_MODE_COLUMN, t_u=50, t_v=60, dtype=B.NMF_F32, flags=0)
    c.update(kw)
    return B.nmf_config(**c)


def test_workspace_size_grows_with_problem():
    a = B.nmf_workspace_size(_cfg(), 20000)
    b = B.nmf_workspace_size(_cfg(), 40000)
    c = B.nmf_workspace_size(_cfg(dtype=B.NMF_F64), 20000)
    assert 0 < a < b and a < c
    assert a % 256 == 0


@pytest.mark.parametrize("kw,status", [
    (dict(k=0), B.NMF_ERR_INVALID_ARG),
    (dict(k=129), B.NMF_ERR_UNSUPPORTED),
    (dict(k=1001), B.NMF_ERR_UNSUPPORTED),
    (dict(n=5, m=3, k=4), B.NMF_ERR_INVALID_ARG),
    (dict(t_u=0), B.NMF_ERR_INVALID_ARG),
    (dict(t_v=-2), B.NMF_ERR_INVALID_ARG),
    (dict(mode=7), B.NMF_ERR_UNSUPPORTED),
    (dict(dtype=3), B.NMF_ERR_UNSUPPORTED),
    (dict(n=0), B.NMF_ERR_INVALID_ARG),
    (dict(n=1 << 29), B.NMF_ERR_UNSUPPORTED),
    (dict(m=1 << 29), B.NMF_ERR_UNSUPPORTED),
    (dict(m=(1 << 31) // 50, k=50), B.NMF_ERR_UNSUPPORTED),
])
def test_config_validation(kw, status):
    with pytest.raises(B.NMFError) as ei:
        B.nmf_workspace_size(_cfg(**kw), 100)
    assert ei.value.status == status


@pytest.mark.parametrize("k,dtype,row_bytes", [(52, B.NMF_F32, 64 * 4), (50, B.NMF_F64, 56 * 8),
                                                (5, B.NMF_F32, 16 * 4), (128, B.NMF_F32, 128 * 4)])
def test_dense_factor_limit(k, dtype, row_bytes):
    """A dense factor copy (rows x k, rows padded to 64 bytes) must stay below
    4 GiB: the largest accepted row count and the first refused one."""
    top = ((1 << 32) - 1) // row_bytes
    assert B.nmf_workspace_size(_cfg(m=top, k=k, dtype=dtype), 100) > 0
    with pytest.raises(B.NMFError) as ei:
        B.nmf_workspace_size(_cfg(m=top + 1, k=k, dtype=dtype), 100)
    assert ei.value.status == B.NMF_ERR_UNSUPPORTED


def test_create_rejects_null_arguments_without_a_device():
    lib = B.load_library()
    cfg = _cfg()
    h = ctypes.c_void_p()
    st = lib.nmf_create(ctypes.byref(cfg), None, None, None, 10, None, None, None, 0, None, ctypes.byref(h))
    assert st == B.NMF_ERR_INVALID_ARG
    assert h.value is None
    assert "NULL" in B.nmf_last_error(None)


def test_create_static_rejects_a_problem_beyond_its_workspace():
    """The static workspace holds NMF_STATIC_WORKSPACE_BYTES; a larger
    problem is refused before any device work (no GPU needed)."""
    lib = B.load_library()
    cfg = _cfg(n=100000, m=200000, k=50, t_u=1000, t_v=2000)
    assert B.nmf_workspace_size(cfg, 20_000_000) > 64 << 20
    h = ctypes.c_void_p()
    rp = (ctypes.c_int64 * 2)(0, 1)
    st = lib.nmf_create_static(ctypes.byref(cfg), rp, rp, rp, 20_000_000, rp, None, None, ctypes.byref(h))
    assert st == B.NMF_ERR_WORKSPACE
    assert h.value is None
    assert "static workspace holds 67108864" in B.nmf_last_error(None)
