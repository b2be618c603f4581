"""ctypes binding of the enforced-sparsity NMF C ABI (include/nmf.h).

Argument marshalling only: every step of the factorization runs in the HIP
kernels of ``libnmf.so``.  PyTorch provides device memory (the workspace,
caller tensors) and the HIP stream; nothing here computes on the data.

The low-level functions carry the C names (``nmf_create``, ``nmf_als_step``,
...).  ``NMF`` wraps one handle together with the workspace tensor that
backs it, and ``NMFLoss`` exposes the squared loss with its hand-written
gradient to ``torch.autograd``.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf.so")

# status codes
NMF_OK = 0
NMF_ERR_INVALID_ARG = -1
NMF_ERR_INVALID_INPUT = -2
NMF_ERR_UNSUPPORTED = -3
NMF_ERR_NOT_SPD = -4
NMF_ERR_NONFINITE = -5
NMF_ERR_DEVICE = -6
NMF_ERR_STATE = -7
NMF_ERR_WORKSPACE = -8

NMF_MODE_COLUMN = 0
NMF_MODE_NONE = 1
NMF_MODE_WHOLE = 2
NMF_F32 = 0
NMF_F64 = 1
NMF_FLAG_NO_METRICS = 1
NMF_FLAG_NO_HOT = 2

_STATUS_NAMES = {
    0: "NMF_OK", -1: "NMF_ERR_INVALID_ARG", -2: "NMF_ERR_INVALID_INPUT", -3: "NMF_ERR_UNSUPPORTED",
    -4: "NMF_ERR_NOT_SPD", -5: "NMF_ERR_NONFINITE", -6: "NMF_ERR_DEVICE", -7: "NMF_ERR_STATE",
    -8: "NMF_ERR_WORKSPACE",
}


class NMFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class nmf_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("k", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("t_u", ctypes.c_int64),
        ("t_v", ctypes.c_int64),
        ("dtype", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PD = ctypes.POINTER(ctypes.c_double)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)

# name -> (restype, argtypes); every function declared in include/nmf.h
SIGNATURES = {
    "nmf_workspace_size": (_I32, [ctypes.POINTER(nmf_config), _I64, ctypes.POINTER(ctypes.c_size_t)]),
    "nmf_create": (_I32, [ctypes.POINTER(nmf_config), _P, _P, _P, _I64, _P, _P, _P, ctypes.c_size_t, _P,
                          ctypes.POINTER(_P)]),
    "nmf_create_static": (_I32, [ctypes.POINTER(nmf_config), _P, _P, _P, _I64, _P, _P, _P, ctypes.POINTER(_P)]),
    "nmf_als_step": (_I32, [_P, _I32]),
    "nmf_half_step": (_I32, [_P, _I32]),
    "nmf_error": (_I32, [_P, _PD]),
    "nmf_residual": (_I32, [_P, _PD]),
    "nmf_history": (_I32, [_P, _P, _P, _P, _P, _I32, _PI32]),
    "nmf_max_nnz": (_I32, [_P, _PI64]),
    "nmf_get_factors": (_I32, [_P, _P, _P]),
    "nmf_get_sparse": (_I32, [_P, _I32, _P, _P, _P, _PI64]),
    "nmf_set_factors": (_I32, [_P, _P, _P, _P]),
    "nmf_get_pre": (_I32, [_P, _I32, _P]),
    "nmf_loss_fwd": (_I32, [_P, _P, _P, _P]),
    "nmf_loss_bwd": (_I32, [_P, _P, _P, _P, _P, _P]),
    "nmf_set_param": (_I32, [_P, _I32, _I64]),
    "nmf_profile": (_I32, [_P, _I32]),
    "nmf_profile_stages": (_I32, [_P, ctypes.c_uint32]),
    "nmf_profile_read": (_I32, [_P, _P, _P, _I32]),
    "nmf_last_error": (ctypes.c_char_p, [_P]),
    "nmf_destroy": (None, [_P]),
    "nmf_batch_workspace_size": (_I32, [_I32, ctypes.POINTER(nmf_config), _PI64, ctypes.POINTER(ctypes.c_size_t)]),
    "nmf_batch_create": (_I32, [_I32, ctypes.POINTER(nmf_config), _P, _P, _P, _PI64, _P, _P, ctypes.c_size_t, _P,
                                ctypes.POINTER(_P)]),
    "nmf_batch_step": (_I32, [_P, _I32, _I32]),
    "nmf_batch_set_param": (_I32, [_P, _I32, _I32, ctypes.c_int64]),
    "nmf_batch_tune": (_I32, [_P, _I32, _P]),
    "nmf_get_param": (_I32, [_P, _I32, _P]),
    "nmf_enforce": (_I32, [_P, _I32, _I64, _I64]),
    "nmf_sequential": (_I32, [_P, _I32, _I32]),
    "nmf_topic_counts": (_I32, [_P, _P, _I32, _P]),
    "nmf_topic_accuracy": (_I32, [_P, _P, _I32, _P]),
    "nmf_history_field": (_I32, [_P, _I32, _P, _I32, _P]),
    "nmf_accuracy_from_counts": (_I32, [_P, _I32, _I32, _P]),
    "nmf_batch_errors": (_I32, [_P, _P, _P]),
    "nmf_batch_problem": (_P, [_P, _I32]),
    "nmf_batch_last_error": (ctypes.c_char_p, [_P]),
    "nmf_batch_destroy": (None, [_P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnmf.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1510_05237_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int, handle=None):
    if st != NMF_OK:
        msg = load_library().nmf_last_error(handle)
        raise NMFError(st, msg.decode() if msg else "")


def _ptr(x) -> Optional[int]:
    """Raw address of a torch tensor or numpy array (or None)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return x.ctypes.data
    import torch

    if isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr()
    raise TypeError(f"unsupported array type {type(x)}")


def _shape_size(x):
    """(shape, bytes per element) of a numpy array or torch tensor."""
    if isinstance(x, np.ndarray):
        return tuple(x.shape), x.itemsize
    import torch

    if isinstance(x, torch.Tensor):
        return tuple(x.shape), x.element_size()
    raise TypeError(f"unsupported array type {type(x)}")


# The library receives bare pointers and cannot see an array's length or
# element type, so the binding refuses what the library would misread: a
# wrong element size with TypeError, a wrong length or shape with
# NMFError(NMF_ERR_INVALID_ARG), the status the library gives a bad size.


def _check_csr(n: int, elt: int, indptr, indices, data) -> int:
    """A as n + 1 int64 row offsets, then int32 column indices and values of
    `elt` bytes, at least as many as the offsets end at; returns nnz."""
    shape, size = _shape_size(indptr)
    if size != 8:
        raise TypeError("indptr must hold int64 row offsets")
    if shape != (n + 1,):
        raise NMFError(NMF_ERR_INVALID_ARG, f"indptr must have n + 1 = {n + 1} entries, got shape {shape}")
    nnz = int(indptr[-1])
    for name, x, want, what in (("indices", indices, 4, "int32 column indices"),
                                ("data", data, elt, f"{elt}-byte values")):
        shape, size = _shape_size(x)
        if size != want:
            raise TypeError(f"{name} must hold {what}")
        if len(shape) != 1 or shape[0] < nnz:
            raise NMFError(NMF_ERR_INVALID_ARG, f"{name} must hold the {nnz} entries indptr ends at, "
                                                f"got shape {shape}")
    return nnz


def _check_factor(x, name: str, rows: int, k: int, elt: int):
    """A factor (or initial guess) as a rows x k matrix of `elt`-byte values."""
    if x is None:
        return
    shape, size = _shape_size(x)
    if size != elt:
        raise TypeError(f"{name} must hold {elt}-byte values")
    if shape != (rows, k):
        raise NMFError(NMF_ERR_INVALID_ARG, f"{name} must be {rows} x {k}, got shape {shape}")


def _stream_ptr(stream) -> Optional[int]:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---------------------------------------------------------------- C names


def nmf_workspace_size(cfg: nmf_config, nnz: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().nmf_workspace_size(ctypes.byref(cfg), nnz, ctypes.byref(out)))
    return out.value


def nmf_create(cfg, a_rowptr, a_col, a_val, nnz, u0, v0, workspace, ws_bytes, stream) -> int:
    h = _P()
    st = load_library().nmf_create(ctypes.byref(cfg), _ptr(a_rowptr), _ptr(a_col), _ptr(a_val), nnz,
                                   _ptr(u0), _ptr(v0), _ptr(workspace), ws_bytes, stream, ctypes.byref(h))
    _check(st, None)
    return h.value


def nmf_create_static(cfg, a_rowptr, a_col, a_val, nnz, u0, v0, stream) -> int:
    """nmf_create on the library's static device workspace (no allocation)."""
    h = _P()
    st = load_library().nmf_create_static(ctypes.byref(cfg), _ptr(a_rowptr), _ptr(a_col), _ptr(a_val), nnz,
                                          _ptr(u0), _ptr(v0), stream, ctypes.byref(h))
    _check(st, None)
    return h.value


def nmf_als_step(h: int, iters: int):
    _check(load_library().nmf_als_step(h, iters), h)


def nmf_half_step(h: int, which: int):
    _check(load_library().nmf_half_step(h, which), h)


def nmf_error(h: int) -> float:
    e = ctypes.c_double(0)
    _check(load_library().nmf_error(h, ctypes.byref(e)), h)
    return e.value


def nmf_residual(h: int) -> float:
    r = ctypes.c_double(0)
    _check(load_library().nmf_residual(h, ctypes.byref(r)), h)
    return r.value


def nmf_history(h: int, cap: int = 4096):
    E = np.zeros(cap, np.float64)
    R = np.zeros(cap, np.float64)
    nu = np.zeros(cap, np.int64)
    nv = np.zeros(cap, np.int64)
    ln = ctypes.c_int32(0)
    _check(load_library().nmf_history(h, _ptr(E), _ptr(R), _ptr(nu), _ptr(nv), cap, ctypes.byref(ln)), h)
    n = ln.value
    return E[:n], R[:n], nu[:n], nv[:n]


def nmf_max_nnz(h: int) -> int:
    v = ctypes.c_int64(0)
    _check(load_library().nmf_max_nnz(h, ctypes.byref(v)), h)
    return v.value


def nmf_get_factors(h: int, u_dense, v_dense):
    _check(load_library().nmf_get_factors(h, _ptr(u_dense), _ptr(v_dense)), h)


def nmf_get_sparse(h: int, which: int, row_ptr=None, topic=None, val=None) -> int:
    nnz = ctypes.c_int64(0)
    _check(load_library().nmf_get_sparse(h, which, _ptr(row_ptr), _ptr(topic), _ptr(val), ctypes.byref(nnz)), h)
    return nnz.value


def nmf_set_factors(h: int, u, u_prev=None, v=None):
    _check(load_library().nmf_set_factors(h, _ptr(u), _ptr(u_prev), _ptr(v)), h)


def nmf_get_pre(h: int, which: int, dst):
    _check(load_library().nmf_get_pre(h, which, _ptr(dst)), h)


def nmf_loss_fwd(h: int, U, V, loss_dev):
    _check(load_library().nmf_loss_fwd(h, _ptr(U), _ptr(V), _ptr(loss_dev)), h)


def nmf_loss_bwd(h: int, U, V, g_scale, gU, gV):
    _check(load_library().nmf_loss_bwd(h, _ptr(U), _ptr(V), _ptr(g_scale), _ptr(gU), _ptr(gV)), h)


NMF_PARAM_SPARSE_ROW_V = 0
NMF_PARAM_SPARSE_ROW_U = 1
NMF_PARAM_WIDE_V = 2
NMF_PARAM_WIDE_U = 3
NMF_PARAM_WAVES_V = 4
NMF_PARAM_WAVES_U = 5


def nmf_set_param(h: int, param: int, value: int):
    _check(load_library().nmf_set_param(h, param, value), h)


def nmf_sequential(h: int, k2: int, iters: int):
    _check(load_library().nmf_sequential(h, k2, iters), h)


def nmf_enforce(h: int, mode: int, t_u: int, t_v: int):
    _check(load_library().nmf_enforce(h, mode, t_u, t_v), h)


def nmf_topic_counts(h: int, labels, n_labels: int, k: int) -> np.ndarray:
    lab = labels if not isinstance(labels, np.ndarray) else np.ascontiguousarray(labels, np.int32)
    out = np.zeros(k * n_labels, np.int64)
    _check(load_library().nmf_topic_counts(h, _ptr(lab), n_labels, _ptr(out)), h)
    return out.reshape(k, n_labels)


HIST_FIELDS = ("E", "R", "nnz_u", "nnz_v", "dead_u", "dead_v", "cond_u", "cond_v", "gathered_v", "gathered_u")


def nmf_history_field(h: int, field: str, cap: int = 4096) -> np.ndarray:
    out = np.zeros(cap, np.float64)
    n = ctypes.c_int32()
    _check(load_library().nmf_history_field(h, HIST_FIELDS.index(field), _ptr(out), cap, ctypes.byref(n)), h)
    return out[: n.value]


def nmf_topic_accuracy(h: int, labels, n_labels: int, k: int) -> np.ndarray:
    lab = labels if not isinstance(labels, np.ndarray) else np.ascontiguousarray(labels, np.int32)
    out = np.zeros(k, np.float64)
    _check(load_library().nmf_topic_accuracy(h, _ptr(lab), n_labels, _ptr(out)), h)
    return out


def accuracy_from_counts(counts, n_labels: int) -> np.ndarray:
    """Eq. (acc) of every topic from its k x n_labels label counts (the
    library's nmf_accuracy_from_counts; no device needed)."""
    cnt = np.ascontiguousarray(np.asarray(counts, dtype=np.int64).reshape(-1, n_labels))
    out = np.zeros(cnt.shape[0], np.float64)
    _check(load_library().nmf_accuracy_from_counts(_ptr(cnt), cnt.shape[0], n_labels, _ptr(out)), None)
    return out


def nmf_get_param(h: int, param: int) -> int:
    v = ctypes.c_int64()
    _check(load_library().nmf_get_param(h, param, ctypes.byref(v)), h)
    return v.value


NMF_NUM_STAGES = 9
STAGE_NAMES = ["spmm_v", "select_v", "repack_v", "gram_v", "spmm_u", "select_u", "repack_u", "gram_u",
               "metrics"]


def nmf_profile(h: int, enable: bool):
    _check(load_library().nmf_profile(h, 1 if enable else 0), h)


def nmf_profile_stages(h: int, stages):
    """Bracket only the named stages (names from STAGE_NAMES) with events."""
    mask = 0
    for s in stages:
        mask |= 1 << STAGE_NAMES.index(s)
    _check(load_library().nmf_profile_stages(h, mask), h)


def nmf_profile_read(h: int):
    ms = np.zeros(NMF_NUM_STAGES, np.float64)
    cnt = np.zeros(NMF_NUM_STAGES, np.int64)
    _check(load_library().nmf_profile_read(h, _ptr(ms), _ptr(cnt), NMF_NUM_STAGES), h)
    return {STAGE_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(NMF_NUM_STAGES)}


def nmf_last_error(h: Optional[int] = None) -> str:
    return load_library().nmf_last_error(h).decode()


def nmf_destroy(h: int):
    load_library().nmf_destroy(h)


NMF_BATCH_LOOP = 0
NMF_BATCH_LOOP_GRAPH = 1
NMF_BATCH_FUSED = 2
NMF_BATCH_FUSED_GRAPH = 3
BATCH_MODES = {"loop": NMF_BATCH_LOOP, "loop_graph": NMF_BATCH_LOOP_GRAPH, "fused": NMF_BATCH_FUSED,
               "fused_graph": NMF_BATCH_FUSED_GRAPH}


def _bcheck(st: int, b=None):
    if st != NMF_OK:
        msg = load_library().nmf_batch_last_error(b)
        raise NMFError(st, msg.decode() if msg else "")


def nmf_batch_workspace_size(cfgs, nnz) -> int:
    n = len(cfgs)
    arr = (nmf_config * n)(*cfgs)
    nz = np.ascontiguousarray(nnz, np.int64)
    out = ctypes.c_size_t()
    _bcheck(load_library().nmf_batch_workspace_size(n, arr, nz.ctypes.data_as(_PI64), ctypes.byref(out)))
    return out.value


def nmf_batch_create(cfgs, rowptrs, cols, vals, nnz, u0s, workspace, ws_bytes, stream) -> int:
    n = len(cfgs)
    arr = (nmf_config * n)(*cfgs)
    ptrs = [(_P * n)(*[_ptr(x) for x in xs]) for xs in (rowptrs, cols, vals, u0s)]
    nz = np.ascontiguousarray(nnz, np.int64)
    b = _P()
    _bcheck(load_library().nmf_batch_create(n, arr, ptrs[0], ptrs[1], ptrs[2], nz.ctypes.data_as(_PI64), ptrs[3],
                                            _ptr(workspace), ws_bytes, stream, ctypes.byref(b)))
    return b.value


def nmf_batch_step(b: int, iters: int, how: int):
    _bcheck(load_library().nmf_batch_step(b, iters, how), b)


def nmf_batch_set_param(b: int, i: int, param: int, value: int):
    _bcheck(load_library().nmf_batch_set_param(b, i, param, value), b)


def nmf_batch_tune(b: int, iters: int = 2):
    out = np.zeros(6, np.int32)
    _bcheck(load_library().nmf_batch_tune(b, iters, _ptr(out)), b)
    keys = ("wide", "sparse_row", "waves")
    return {"v": dict(zip(keys, map(int, out[:3]))), "u": dict(zip(keys, map(int, out[3:])))}


def nmf_batch_errors(b: int, count: int):
    E = np.zeros(count, np.float64)
    st = np.zeros(count, np.int32)
    load_library().nmf_batch_errors(b, _ptr(E), _ptr(st))
    return E, st


# ---------------------------------------------------------------- handle object

_MODES = {"column": NMF_MODE_COLUMN, "none": NMF_MODE_NONE, "whole": NMF_MODE_WHOLE}


class NMF:
    """One factorization problem on one GPU.

    ``indptr``/``indices``/``data``: A in CSR over term rows (numpy arrays or
    torch tensors, host or device).  ``u0``: initial U (n x k); ``v0``
    optional.  ``dtype``: "f32" or "f64" (the type of data/u0/v0).
    ``static_workspace``: run on the library's static per-device workspace
    (nmf_create_static: no device allocation; one such handle per device).
    """

    def __init__(self, n, m, indptr, indices, data, u0, *, t_u, t_v, v0=None, mode="column",
                 dtype="f32", flags=0, device="cuda:0", stream=None, static_workspace=False):
        import torch

        load_library()
        self.device = torch.device(device)
        self.dtype = dtype
        self.np_dtype = np.float32 if dtype == "f32" else np.float64
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64
        k = int(u0.shape[1])
        self.n, self.m, self.k = int(n), int(m), k
        self.cfg = nmf_config(n=int(n), m=int(m), k=k, mode=_MODES[mode], t_u=int(t_u), t_v=int(t_v),
                              dtype=NMF_F32 if dtype == "f32" else NMF_F64, flags=int(flags))
        elt = 4 if dtype == "f32" else 8
        nnz = _check_csr(self.n, elt, indptr, indices, data)
        _check_factor(u0, "u0", self.n, k, elt)
        _check_factor(v0, "v0", self.m, k, elt)
        self.nnz = nnz
        with torch.cuda.device(self.device):
            self.ws_bytes = nmf_workspace_size(self.cfg, nnz)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if static_workspace:
                # the library's own per-device workspace: nothing is allocated
                self.workspace = None
                self.h = nmf_create_static(self.cfg, indptr, indices, data, nnz, u0, v0, self.stream.cuda_stream)
            else:
                self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
                self.h = nmf_create(self.cfg, indptr, indices, data, nnz, u0, v0, self.workspace,
                                    self.ws_bytes, self.stream.cuda_stream)

    # -- iteration
    def step(self, iters: int = 1):
        nmf_als_step(self.h, iters)

    def half_step(self, which: int):
        nmf_half_step(self.h, which)

    # -- queries
    def error(self) -> float:
        return nmf_error(self.h)

    def residual(self) -> float:
        return nmf_residual(self.h)

    def history(self, cap: int = 4096):
        return nmf_history(self.h, cap)

    def max_nnz(self) -> int:
        return nmf_max_nnz(self.h)

    def factors(self):
        """Dense (U, V) as float arrays on the host."""
        U = np.zeros((self.n, self.k), self.np_dtype)
        V = np.zeros((self.m, self.k), self.np_dtype)
        nmf_get_factors(self.h, U, V)
        return U, V

    def factors_device(self):
        import torch

        U = torch.empty((self.n, self.k), dtype=self.torch_dtype, device=self.device)
        V = torch.empty((self.m, self.k), dtype=self.torch_dtype, device=self.device)
        nmf_get_factors(self.h, U, V)
        return U, V

    def sparse(self, which: int):
        rows = self.n if which == 0 else self.m
        nnz = nmf_get_sparse(self.h, which)
        rp = np.zeros(rows + 1, np.int32)
        tp = np.zeros(max(nnz, 1), np.uint8)
        vl = np.zeros(max(nnz, 1), self.np_dtype)
        nmf_get_sparse(self.h, which, rp, tp, vl)
        return rp, tp[:nnz], vl[:nnz]

    def pre(self, which: int):
        rows = self.m if which == 0 else self.n
        out = np.zeros((rows, self.k), self.np_dtype)
        nmf_get_pre(self.h, which, out)
        return out

    def set_factors(self, u, u_prev=None, v=None):
        elt = 4 if self.dtype == "f32" else 8
        _check_factor(u, "u", self.n, self.k, elt)
        _check_factor(u_prev, "u_prev", self.n, self.k, elt)
        _check_factor(v, "v", self.m, self.k, elt)
        nmf_set_factors(self.h, u, u_prev, v)

    def set_param(self, param: int, value: int):
        nmf_set_param(self.h, param, value)

    def get_param(self, param: int) -> int:
        return nmf_get_param(self.h, param)

    def history_field(self, field: str, cap: int = 4096) -> np.ndarray:
        """One field of the per-iteration record (see HIST_FIELDS), oldest first."""
        return nmf_history_field(self.h, field, cap)

    def topic_counts(self, labels, n_labels: int) -> np.ndarray:
        """k x n_labels: documents of each label with an entry in each column of V."""
        return nmf_topic_counts(self.h, labels, n_labels, self.k)

    def topic_accuracy(self, labels, n_journals: int) -> np.ndarray:
        """Eq. (acc) of every topic for documents labelled by journal."""
        return nmf_topic_accuracy(self.h, labels, n_journals, self.k)

    def sequential(self, k2: int, iters: int):
        """Algorithm 3: k / k2 blocks of k2 topics, ``iters`` iterations each."""
        nmf_sequential(self.h, k2, iters)

    def enforce(self, t_u: int, t_v: int, mode: str = "column"):
        """Apply the top-t rule once to the current U and V."""
        nmf_enforce(self.h, _MODES[mode], t_u, t_v)

    def profile(self, enable: bool, stages=None):
        """Bracket every stage (or only `stages`, a list of STAGE_NAMES) with
        HIP events while enabled."""
        if enable and stages is not None:
            nmf_profile_stages(self.h, stages)
        else:
            nmf_profile(self.h, enable)

    def profile_read(self):
        return nmf_profile_read(self.h)

    def close(self):
        if getattr(self, "h", None):
            nmf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _loss_operands(problem, U, V):
    """The loss entry points read U (n x k) and V (m x k) of the problem's
    dtype on the problem's device; anything else is refused before a kernel
    sees it."""
    import torch

    for name, X, rows in (("U", U, problem.n), ("V", V, problem.m)):
        if not isinstance(X, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if X.dtype != problem.torch_dtype:
            raise TypeError(f"{name} must have the problem's dtype {problem.torch_dtype}")
        if X.device != torch.device(problem.device):
            raise ValueError(f"{name} is on {X.device}, the problem on {problem.device}")
        if tuple(X.shape) != (rows, problem.k):
            raise ValueError(f"{name} has shape {tuple(X.shape)}, expected {(rows, problem.k)}")


class _on_problem_stream:
    """Orders the problem's stream after the caller's current stream on
    entry (the operands may still be in flight there) and the current
    stream after the problem's stream on exit."""

    def __init__(self, problem):
        self.problem = problem

    def __enter__(self):
        import torch

        self.cur = torch.cuda.current_stream(self.problem.device)
        # a batch member runs on the batch's own stream, which torch does not
        # know: wait for the caller's stream on the host instead
        self.own = getattr(self.problem, "stream", None)
        if self.own is None:
            self.cur.synchronize()
        elif self.own != self.cur:
            self.own.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        # the loss entry points synchronize their stream before returning;
        # the event wait keeps the order explicit all the same
        if self.own is not None and self.own != self.cur:
            self.cur.wait_stream(self.own)
        return False


class NMFLoss:
    """``NMFLoss.apply(problem, U, V)`` -> L = ||A - U V^T||_F^2 (float64 scalar
    tensor) with the hand-written gradient (-2 A V + 2 U V^T V, and the
    transpose), A being the matrix held by ``problem`` (an ``NMF``)."""

    _fn = None

    @classmethod
    def _function(cls):
        if cls._fn is None:
            import torch

            class _Loss(torch.autograd.Function):
                @staticmethod
                def forward(ctx, problem, U, V):
                    _loss_operands(problem, U, V)
                    U = U.contiguous()
                    V = V.contiguous()
                    out = torch.empty((), dtype=torch.float64, device=U.device)
                    with _on_problem_stream(problem):
                        nmf_loss_fwd(problem.h, U, V, out)
                    ctx.problem = problem
                    ctx.save_for_backward(U, V)
                    return out

                @staticmethod
                def backward(ctx, g):
                    U, V = ctx.saved_tensors
                    problem = ctx.problem
                    g = g.to(device=U.device, dtype=torch.float64).contiguous()
                    gU = torch.empty_like(U) if ctx.needs_input_grad[1] else None
                    gV = torch.empty_like(V) if ctx.needs_input_grad[2] else None
                    with _on_problem_stream(problem):
                        nmf_loss_bwd(problem.h, U, V, g, gU, gV)
                    return None, gU, gV

            cls._fn = _Loss
        return cls._fn

    @classmethod
    def apply(cls, problem, U, V):
        return cls._function().apply(problem, U, V)


class _BatchMember(NMF):
    """View of one problem of an ``NMFBatch`` (its handle belongs to the batch)."""

    def __init__(self, h, n, m, k, dtype, device):
        import torch

        self.h = h
        self.n, self.m, self.k = n, m, k
        self.dtype = dtype
        self.np_dtype = np.float32 if dtype == "f32" else np.float64
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64
        self.device = device

    def close(self):
        self.h = None


class NMFBatch:
    """Independent problems advanced together on one GPU.

    ``problems``: sequence of dicts with ``n, m, indptr, indices, data, u0,
    t_u, t_v`` (A in CSR over term rows; host or device arrays of ``dtype``).
    ``step(iters, how)`` runs ``iters`` iterations of every problem as
    ``how``: "loop" (each problem's own launches), "loop_graph" (that loop
    captured as a HIP graph), "fused" (one launch per stage for all problems)
    or "fused_graph" (the fused launches captured as a graph).
    """

    def __init__(self, problems, *, dtype="f32", mode="column", flags=0, device="cuda:0", stream=None):
        import torch

        load_library()
        self.device = torch.device(device)
        self.dtype = dtype
        cfgs, nnz = [], []
        elt = 4 if dtype == "f32" else 8
        for p in problems:
            k = int(p["u0"].shape[1])
            cfgs.append(nmf_config(n=int(p["n"]), m=int(p["m"]), k=k, mode=_MODES[mode], t_u=int(p["t_u"]),
                                   t_v=int(p["t_v"]), dtype=NMF_F32 if dtype == "f32" else NMF_F64,
                                   flags=int(flags)))
            nnz.append(_check_csr(int(p["n"]), elt, p["indptr"], p["indices"], p["data"]))
            _check_factor(p["u0"], "u0", int(p["n"]), k, elt)
        self.count = len(cfgs)
        with torch.cuda.device(self.device):
            self.ws_bytes = nmf_batch_workspace_size(cfgs, nnz)
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            torch.cuda.current_stream(self.device).synchronize()
            s = stream.cuda_stream if stream is not None else None
            self.b = nmf_batch_create(cfgs, [p["indptr"] for p in problems], [p["indices"] for p in problems],
                                      [p["data"] for p in problems], nnz, [p["u0"] for p in problems],
                                      self.workspace, self.ws_bytes, s)
        lib = load_library()
        self.members = [_BatchMember(lib.nmf_batch_problem(self.b, i), c.n, c.m, c.k, dtype, self.device)
                        for i, c in enumerate(cfgs)]

    def step(self, iters: int = 1, how: str = "fused_graph"):
        nmf_batch_step(self.b, iters, BATCH_MODES[how])

    def set_param(self, param: int, value: int, problem: int = -1):
        """Tuning parameter of one problem (or all, -1); re-records the fused launches."""
        nmf_batch_set_param(self.b, problem, param, value)

    def tune(self, iters: int = 2):
        """Pick each half-step's SpMM form by timing the fused batch (advances
        every problem 16 * (1 + iters) iterations); returns the choice."""
        return nmf_batch_tune(self.b, iters)

    def errors(self):
        """(E, status) per problem, after waiting for the batch."""
        return nmf_batch_errors(self.b, self.count)

    def problem(self, i: int) -> NMF:
        return self.members[i]

    def close(self):
        if getattr(self, "b", None):
            for mem in self.members:
                mem.close()
            load_library().nmf_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
