"""GPU parity at the full 100k terms x 200k docs / 20M-nnz FP32 size, in the
launch configuration bench.py times (default parameters).  Each half-step
starts from the GPU's own state; the FP64 oracle recomputes the whole
pre-selection matrix from that state, and the top-t rule is re-applied on
the CPU to the GPU's own pre-selection values (which must then give the
GPU's factor exactly).  Every test prints its case before touching the GPU."""

import numpy as np
import pytest

import oracle
import synth
from tests.parity import rel_fro

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_fp32_100kx200k_half_steps():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF

    c, u0, _, p = synth.make_workload("plain_f32_100kx200k")
    A = c.scipy()
    At = A.T.tocsr()
    dev = torch.device("cuda:0")
    _say(f"fp32 full size {c.n}x{c.m} nnz={c.nnz} k={p['k']} t_u={p['t_u']} t_v={p['t_v']}: 2 iterations of half-steps")
    prob = NMF(c.n, c.m, torch.from_numpy(c.indptr).to(dev), torch.from_numpy(c.indices).to(dev),
               torch.from_numpy(c.data).to(dev), torch.from_numpy(u0).to(dev), t_u=p["t_u"], t_v=p["t_v"],
               dtype="f32", device=dev)
    for it in range(2):
        U_in = u0 if it == 0 else prob.factors()[0]
        prob.half_step(0)
        vpre = prob.pre(0)
        _, V = prob.factors()
        _, info = oracle.half_step(At, U_in.astype(np.float64), p["t_v"])
        rv = rel_fro(vpre, oracle.clamp(info["X_pre"]))
        np.testing.assert_array_equal(V, oracle.topt_per_column(vpre.astype(np.float64), p["t_v"]).astype(np.float32))
        assert int(np.count_nonzero(V)) == int(np.minimum((vpre > 0).sum(0), p["t_v"]).sum())
        prob.half_step(1)
        upre = prob.pre(1)
        U, _ = prob.factors()
        _, info = oracle.half_step(A, V.astype(np.float64), p["t_u"])
        ru = rel_fro(upre, oracle.clamp(info["X_pre"]))
        np.testing.assert_array_equal(U, oracle.topt_per_column(upre.astype(np.float64), p["t_u"]).astype(np.float32))
        _say(f"  iteration {it}: V_pre rel {rv:.2e}, U_pre rel {ru:.2e}, nnz U {np.count_nonzero(U)} V {np.count_nonzero(V)}")
        assert rv <= 1e-4 and ru <= 1e-4, (it, rv, ru)
    # a full iteration records E; it matches the oracle's E of the GPU's factors
    prob.step(1)
    U, V = prob.factors()
    E = prob.error()
    Eo = oracle.error(A, U.astype(np.float64), V.astype(np.float64))
    _say(f"  E gpu {E:.8f} oracle {Eo:.8f}")
    assert abs(E - Eo) <= 1e-6 * Eo
    prob.close()
