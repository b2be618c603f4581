"""GPU tests of the loss entry points' guards and of non-finite results:
* the autograd loss raises while a sticky numerical error is pending;
* central differences of NMFLoss itself (its own forward at perturbed
  points, FP64) agree with its backward;
* a k > 64 loss and gradient (two topics per lane) against the FP64 oracle;
* a float32 product that overflows raises NMF_ERR_NONFINITE instead of
  being clamped to zero.
Every test prints its case before touching the GPU."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests.parity import col_rel, rel_fro

pytestmark = pytest.mark.gpu


def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF, NMFError, NMFLoss

    return NMF, NMFError, NMFLoss


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_loss_raises_on_pending_status():
    """Exactly singular Gram of the current U (two equal columns): the V half
    raises NOT_SPD on the device; the loss then refuses to run."""
    NMF, NMFError, NMFLoss = _lib()
    import torch

    c = synth.make_corpus(60, 40, seed=91, alpha=1.1, nnz=500, dtype="f64")
    u0, _ = synth.make_init(60, 40, 3, seed=91, dtype="f64")
    _say("fp64 60x40: loss after a pending NOT_SPD")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=20, t_v=20, dtype="f64")
    # integer entries: the Gram matrix and its pivot 0 are exact
    bad = np.floor(u0 * 4.0) + 1.0
    bad[:, 1] = bad[:, 0]
    with pytest.raises(NMFError) as ei:
        prob.set_factors(bad)
    assert ei.value.status == -4
    U = torch.tensor(u0, device="cuda:0", requires_grad=True)
    V = torch.rand(40, 3, dtype=torch.float64, device="cuda:0", requires_grad=True)
    with pytest.raises(NMFError) as ei:
        NMFLoss.apply(prob, U, V)
    assert ei.value.status == -4
    prob.close()


def test_loss_finite_differences_of_the_function_itself():
    """FP64: L is exactly quadratic in each entry, so the central difference
    of NMFLoss's own forward at u +- h (h = 0.25) equals the derivative up to
    rounding; checked at 64 entries (32 of U, 32 of V, half in the support)."""
    _, _, NMFLoss = _lib()
    import torch
    from paper_1510_05237_amd import NMF

    c = synth.make_corpus(400, 300, seed=92, alpha=1.1, nnz=6000, dtype="f64")
    k = 6
    rng = np.random.Generator(np.random.PCG64(92))
    U = synth.sparse_factor_init(400, k, 60, rng=rng, dtype="f64")
    V = synth.sparse_factor_init(300, k, 50, rng=rng, dtype="f64")
    _say(f"fp64 NMFLoss central differences 400x300 nnz={c.nnz} k={k}")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, U, t_u=60, t_v=50, dtype="f64")
    dev = torch.device("cuda:0")
    Ut = torch.tensor(U, device=dev, requires_grad=True)
    Vt = torch.tensor(V, device=dev, requires_grad=True)
    L = NMFLoss.apply(prob, Ut, Vt)
    L.backward()
    gU, gV = Ut.grad.cpu().numpy(), Vt.grad.cpu().numpy()
    assert float(L) == pytest.approx(oracle.loss(c.scipy(), U, V), rel=1e-10)
    h = 0.25
    scale = max(np.abs(gU).max(), np.abs(gV).max())

    def pick(M, seed):
        r = np.random.default_rng(seed)
        ins = np.argwhere(M != 0)
        outs = np.argwhere(M == 0)
        return [tuple(x) for x in ins[r.choice(len(ins), 16, replace=False)]] + \
               [tuple(x) for x in outs[r.choice(len(outs), 16, replace=False)]]

    with torch.no_grad():
        for M, g, X, seed in ((U, gU, Ut, 1), (V, gV, Vt, 2)):
            for (i, j) in pick(M, seed):
                Xp = X.detach().clone()
                Xm = X.detach().clone()
                Xp[i, j] += h
                Xm[i, j] -= h
                if X is Ut:
                    Lp, Lm = NMFLoss.apply(prob, Xp, Vt.detach()), NMFLoss.apply(prob, Xm, Vt.detach())
                else:
                    Lp, Lm = NMFLoss.apply(prob, Ut.detach(), Xp), NMFLoss.apply(prob, Ut.detach(), Xm)
                fd = (float(Lp) - float(Lm)) / (2 * h)
                assert g[i, j] == pytest.approx(fd, rel=1e-7, abs=1e-9 * scale), (i, j)
    prob.close()


def test_loss_k_above_64_against_oracle():
    """k = 80 (two topics per lane in the products): L and both gradients
    against the FP64 oracle, per column too."""
    _, _, NMFLoss = _lib()
    import torch
    from paper_1510_05237_amd import NMF

    c = synth.make_corpus(1500, 2500, seed=93, alpha=1.1, per_doc=50, dtype="f32")
    k = 80
    rng = np.random.Generator(np.random.PCG64(93))
    U = synth.sparse_factor_init(1500, k, 60, rng=rng, dtype="f32")
    V = synth.sparse_factor_init(2500, k, 90, rng=rng, dtype="f32")
    _say(f"fp32 loss/gradient 1500x2500 nnz={c.nnz} k={k}")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, U, t_u=60, t_v=90, dtype="f32")
    Ut = torch.tensor(U, device="cuda:0", requires_grad=True)
    Vt = torch.tensor(V, device="cuda:0", requires_grad=True)
    L = NMFLoss.apply(prob, Ut, Vt)
    L.backward()
    A = c.scipy()
    gU_or, gV_or = oracle.loss_grad(A, U, V)
    gU, gV = Ut.grad.cpu().numpy(), Vt.grad.cpu().numpy()
    _say(f"  grad rel U {rel_fro(gU, gU_or):.2e} (worst column {col_rel(gU, gU_or):.2e}) "
         f"V {rel_fro(gV, gV_or):.2e} (worst column {col_rel(gV, gV_or):.2e})")
    assert float(L) == pytest.approx(oracle.loss(A, U, V), rel=1e-5)
    assert col_rel(gU, gU_or) <= 1e-4 and col_rel(gV, gV_or) <= 1e-4
    prob.close()


def test_float32_overflow_raises_nonfinite():
    """A float32 product past the float32 range (two entries of 3e38 in one
    document) becomes inf on the device; the epilogue raises the sticky
    NONFINITE status and the next synchronizing call reports it, instead of
    the clamp turning it into a zero."""
    NMF, NMFError, _ = _lib()
    n, m, k = 8, 6, 2
    Ad = np.zeros((n, m), np.float32)
    Ad[0, :] = 3.0e38
    Ad[1, :] = 3.0e38
    Ad[2:, :] = 1.0
    A = sp.csr_matrix(Ad)
    u0 = np.ones((n, k), np.float32)
    u0[:, 1] = np.arange(1, n + 1, dtype=np.float32)
    _say("fp32 8x6 with entries 3e38: overflow -> NMF_ERR_NONFINITE")
    prob = NMF(n, m, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, u0, t_u=4, t_v=4,
               dtype="f32", flags=0)
    prob.half_step(0)
    with pytest.raises(NMFError) as ei:
        prob.factors()
    assert ei.value.status == -5
    prob.close()
