"""The Python binding refuses arrays the library would misread (no GPU
needed: the checks run before any device call).  The library receives bare
pointers, so a wrong element size or length cannot be seen behind the C ABI."""

import numpy as np
import pytest

import synth
from paper_1510_05237_amd import NMF, NMFError
from paper_1510_05237_amd import nmf as B


@pytest.fixture(scope="module")
def small():
    c = synth.make_corpus(50, 40, seed=36, alpha=1.1, nnz=300, dtype="f32")
    u0, v0 = synth.make_init(50, 40, 3, seed=36, dtype="f32")
    return c, u0, v0


def _make(c, u0, **kw):
    args = dict(indptr=c.indptr, indices=c.indices, data=c.data)
    args.update(kw)
    return NMF(c.n, c.m, args["indptr"], args["indices"], args["data"], u0, t_u=5, t_v=5, dtype="f32",
               v0=kw.get("v0"))


def test_element_sizes_are_checked(small):
    c, u0, _ = small
    with pytest.raises(TypeError, match="indptr"):
        _make(c, u0, indptr=c.indptr.astype(np.int32))
    with pytest.raises(TypeError, match="indices"):
        _make(c, u0, indices=c.indices.astype(np.int64))
    with pytest.raises(TypeError, match="data"):
        _make(c, u0, data=c.data.astype(np.float64))
    with pytest.raises(TypeError, match="u0"):
        _make(c, u0.astype(np.float64))


def test_lengths_and_shapes_are_checked(small):
    c, u0, v0 = small
    for kw, word in ((dict(indptr=c.indptr[:-1].copy()), "indptr"),
                     (dict(indices=c.indices[:-1].copy()), "indices"),
                     (dict(data=c.data[:-1].copy()), "data")):
        with pytest.raises(NMFError, match=word) as ei:
            _make(c, u0, **kw)
        assert ei.value.status == B.NMF_ERR_INVALID_ARG
    with pytest.raises(NMFError, match="u0") as ei:
        _make(c, np.ascontiguousarray(u0[:-1]))
    assert ei.value.status == B.NMF_ERR_INVALID_ARG
    with pytest.raises(NMFError, match="v0") as ei:
        _make(c, u0, v0=np.ascontiguousarray(v0[:, :2]))
    assert ei.value.status == B.NMF_ERR_INVALID_ARG
    # a row pointer ending past the stored entries is a length error too
    ip = c.indptr.copy()
    ip[-1] += 1
    with pytest.raises(NMFError) as ei:
        _make(c, u0, indptr=ip)
    assert ei.value.status == B.NMF_ERR_INVALID_ARG


def test_factor_check_accepts_the_right_forms():
    import torch

    B._check_factor(np.zeros((7, 3), np.float64), "u", 7, 3, 8)
    B._check_factor(torch.zeros(7, 3, dtype=torch.float32), "u", 7, 3, 4)
    B._check_factor(None, "v", 5, 3, 4)
    with pytest.raises(TypeError):
        B._check_factor(torch.zeros(7, 3, dtype=torch.float64), "u", 7, 3, 4)
    with pytest.raises(NMFError):
        B._check_factor(np.zeros((3, 7), np.float32), "u", 7, 3, 4)
    assert B._check_csr(2, 4, np.array([0, 1, 3], np.int64), np.zeros(3, np.int32), np.ones(3, np.float32)) == 3
