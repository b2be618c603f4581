"""nmf_create_static (the handle on the library's static per-device
workspace, for callers that cannot allocate) against nmf_create on the same
inputs: two handles in a row on the static workspace, the second on a
smaller problem (the workspace then holds the first one's leftovers), each
compared with an ordinary handle run beside it.  The kernels are the same,
so factors, pre-selection matrices and the history must be bitwise equal.
Also: a second live handle on the same device is refused.  Every test
prints its case before touching the GPU."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _run(NMF, c, u0, k, t_u, t_v, dtype, iters, static):
    p = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype=dtype, device="cuda:0",
            static_workspace=static)
    p.step(iters)
    U, V = p.factors()
    E, R, nu, nv = p.history()
    vpre, upre = p.pre(0), p.pre(1)
    return p, (U, V, E, R, nu, nv, vpre, upre)


def test_static_workspace_matches_caller_workspace():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF, NMFError
    from paper_1510_05237_amd.nmf import NMF_ERR_STATE

    cases = [
        # (n, m, nnz, k, t_u, t_v, dtype, seed): the second is smaller
        (3000, 5000, 200000, 16, 300, 400, "f32", 31),
        (900, 700, 9000, 7, 60, 50, "f64", 32),
    ]
    for (n, m, nnz, k, t_u, t_v, dtype, seed) in cases:
        _say(f"static workspace {dtype} {n}x{m} nnz={nnz} k={k} t_u={t_u} t_v={t_v}: 4 iterations, "
             f"static vs caller workspace")
        c = synth.make_corpus(n, m, seed=seed, alpha=1.1, nnz=nnz, dtype=dtype)
        u0, _ = synth.make_init(n, m, k, seed=seed, dtype=dtype)
        ps, got = _run(NMF, c, u0, k, t_u, t_v, dtype, 4, True)
        if seed == 31:
            _say("  a second static handle on the same device while the first lives")
            with pytest.raises(NMFError) as ei:
                NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype=dtype,
                    device="cuda:0", static_workspace=True)
            assert ei.value.status == NMF_ERR_STATE
        pr, ref = _run(NMF, c, u0, k, t_u, t_v, dtype, 4, False)
        names = ("U", "V", "E", "R", "nnz_u", "nnz_v", "V_pre", "U_pre")
        for name, a, b in zip(names, got, ref):
            assert a.shape == b.shape, name
            assert np.array_equal(a, b, equal_nan=True), name
        _say(f"  identical: E {got[2][-1]:.8f}, nnz U {int(got[4][-1])} V {int(got[5][-1])}")
        ps.close()
        pr.close()
