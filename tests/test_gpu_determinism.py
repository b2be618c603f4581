"""Reproducibility of the entry-by-entry adds of the sparse product (the U
half's gathers of V rows with few entries) under forced collisions: a
corpus whose few most frequent terms occur in almost every document, so the
lanes of one step mostly belong to one long term row and add into the same
(row, topic) places of the accumulator many times per instruction.  Two
handles on the same input must give bitwise equal factors, pre-selection
matrices and histories, and a teacher-forced U half must meet the FP64
oracle.  Every test prints its case before touching the GPU."""

import numpy as np
import pytest

import oracle
import synth
from tests.parity import check_pre

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_forced_collisions_are_reproducible(dtype):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF
    from paper_1510_05237_amd.nmf import NMF_PARAM_SPARSE_ROW_U

    n, m, k = 300, 8000, 8
    c = synth.make_corpus(n, m, seed=61, alpha=1.8, per_doc=30, dtype=dtype)
    lens = np.diff(c.indptr)
    u0, _ = synth.make_init(n, m, k, seed=61, dtype=dtype)
    _say(f"forced collisions {dtype} {n}x{m} nnz={c.nnz} k={k}, longest term row {lens.max()} "
         f"(the top 5 hold {np.sort(lens)[-5:].sum() / c.nnz:.0%}); V rows of <= 8 entries gathered entry by entry")
    runs = []
    for rep in range(2):
        p = NMF(n, m, c.indptr, c.indices, c.data, u0, t_u=60, t_v=2500, dtype=dtype, device="cuda:0")
        p.set_param(NMF_PARAM_SPARSE_ROW_U, 8)
        p.step(3)
        U, V = p.factors()
        E, R, nu, nv = p.history()
        runs.append((U, V, p.pre(0), p.pre(1), E, R))
        if rep == 0:
            # one more U half from the GPU's own V, against the oracle
            p.half_step(0)
            _, V1 = p.factors()
            p.half_step(1)
            upre = p.pre(1)
            _, info = oracle.half_step(c.scipy(), V1.astype(np.float64), 60)
            w = check_pre(upre, oracle.clamp(info["X_pre"]), 1e-4 if dtype == "f32" else 1e-9)
            nz = np.count_nonzero(V1, axis=1)
            _say(f"  V rows with 1..8 entries: {int(((nz > 0) & (nz <= 8)).sum())}; U_pre vs oracle {w:.2e}")
        p.close()
    for name, a, b in zip(("U", "V", "V_pre", "U_pre", "E", "R"), runs[0], runs[1]):
        assert np.array_equal(a, b, equal_nan=True), name
    _say("  two runs bitwise equal")
