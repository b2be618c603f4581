#!/usr/bin/env python3
"""Benchmark of the enforced-sparsity ALS hot path on one MI355X.

One step = one ALS iteration of Algorithm 2 with per-column top-t (V half:
A^T U, FP64 solve, clamp, top-t_v, sparse repack, Gram + FP64 inverse; U half
mirrored; then R and E), on the 100k terms x 200k docs / 20M-nnz FP32
workload with k = 50, t_u = 1000, t_v = 2000.  Inputs are synthetic (Zipf
terms, lognormal TF-IDF values) and resident in HBM before timing starts.

Prints one JSON line: iterations/s (timed with only the dominant product
stage bracketed by HIP events), plus that stage's roofline (algorithmic bytes
per launch / event-timed stage duration, with the HBM bytes of the counter
runs when they match the kernel sources), a per-stage breakdown from a
separate pass with every stage bracketed, the FP64 CPU oracle timed on a
bounded sample of the same workload, and the batched comparison: 256
independent corpora of uneven size (n in [500, 50k], m in [300, 20k],
density 0.1-2 %, k in 5..64) solved per problem, per problem under a HIP
graph, and with one launch per stage for all of them under a HIP graph.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --copy-calibration      # plain copy kernel for counter scaling
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmm_traffic_100kx200k.json")
# the product stages' kernels: the fused V half and the U half's stream
SPMM_SRCS = [os.path.join(ROOT, "paper_1510_05237_amd", "csrc", f) for f in ("k_vhalf.hip", "k_spmm.hip")]


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmm_algorithmic_bytes(rows_out: int, rows_f: int, nnz_a: int, nnz_f: float, k: int, elt: int,
                           keep_c: bool) -> float:
    """Bytes one fused SpMM launch must move: the A orientation it streams
    (value + int32 index per nonzero, int64 row offsets), the sparse fixed
    factor once (value + 1-byte topic per entry, int32 row offsets), and the
    dense k-wide output written once (twice in the U half, which also keeps
    the raw product for the error)."""
    a = nnz_a * (elt + 4) + (rows_out + 1) * 8
    f = nnz_f * (elt + 1) + (rows_f + 1) * 4
    out = rows_out * k * elt * (2 if keep_c else 1)
    return float(a + f + out)


def kernels_sha() -> str:
    h = hashlib.sha256()
    for path in SPMM_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(stage: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    absent or taken on a different version of the product kernels."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernels_sha():
        return None
    s = t.get("stages", {}).get(stage)
    if not s:
        return None
    return float(s["fetch_bytes"] + s["write_bytes"])


def host_info() -> dict:
    """CPU model, logical cores and RAM of the host the oracle runs on."""
    model, ram = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cores": os.cpu_count(), "ram_gib": ram}


def _blas_threads() -> int:
    from threadpoolctl import threadpool_info

    return max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])


def cpu_baseline(corpus, u0, p, iters: int):
    """The FP64 oracle as it stands, on all of the host's cores (its dense
    products and solves run in the multithreaded BLAS; scipy's sparse
    products are single-threaded), on a bounded sample: one untimed
    iteration from U0, then `iters` timed steady-state iterations of the same
    workload."""
    from threadpoolctl import threadpool_limits

    import oracle

    A = corpus.scipy()
    cores = os.cpu_count() or 1
    with threadpool_limits(limits=cores):
        st = oracle.als(A, u0, p["t_u"], p["t_v"], 1)
        times = []
        for _ in range(iters):
            t0 = time.perf_counter()
            st = oracle.als(A, u0, p["t_u"], p["t_v"], 1, state=st)
            times.append(time.perf_counter() - t0)
        threads = _blas_threads()
    med = statistics.median(times)
    return {
        "value": 1.0 / med,
        "unit": "it/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{iters} steady-state ALS iterations (after 1 untimed from U0) of the full "
                   f"{corpus.n}x{corpus.m} / {corpus.nnz}-nnz workload, FP64 numpy/scipy oracle, BLAS on "
                   f"{threads} threads (sparse products single-threaded), median {med:.2f} s/iteration"),
        "host": host_info(),
        "E_after": float(st.E[-1]),
    }


def cpu_loss_baseline():
    """The FP64 oracle's loss and gradient (Eq. (2) squared, both partial
    derivatives) once on the 100k x 200k matrix with sparse U, V (t = 1000
    and 2000 per column, seed 4): the same evaluation NMFLoss performs."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    import synth

    c, _, _, p = synth.make_workload("plain_f32_100kx200k", with_init=False)
    rng = np.random.Generator(np.random.PCG64(4))
    U = synth.sparse_factor_init(c.n, p["k"], p["t_u"], rng=rng, dtype="f32")
    V = synth.sparse_factor_init(c.m, p["k"], p["t_v"], rng=rng, dtype="f32")
    A = c.scipy()
    with threadpool_limits(limits=os.cpu_count() or 1):
        t0 = time.perf_counter()
        oracle.loss(A, U, V)
        oracle.loss_grad(A, U, V)
        dt = time.perf_counter() - t0
    return {"workload": "plain_f32_100kx200k sparse U,V (t_u=1000, t_v=2000, seed 4)", "ms_fwd_bwd": round(dt * 1e3, 1),
            "threads": _blas_threads()}


def cpu_batch_baseline(problems, sample: int = 16):
    """The FP64 oracle on a sample of the many-corpora batch: one ALS
    iteration (after one untimed) of `sample` corpora spread over the batch
    (the smallest and the largest included), extrapolated to one iteration
    of every corpus by the sample's time per nonzero."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    import oracle

    nnz = np.array([int(p["indptr"][-1]) for p in problems])
    order = np.argsort(nnz, kind="stable")
    pick = sorted(set(order[np.linspace(0, len(problems) - 1, sample).round().astype(int)].tolist()))
    t_tot, nnz_s = 0.0, 0
    with threadpool_limits(limits=os.cpu_count() or 1):
        for i in pick:
            p = problems[i]
            A = sp.csr_matrix((p["data"].astype(np.float64), p["indices"], p["indptr"]), shape=(p["n"], p["m"]))
            u0 = p["u0"].astype(np.float64)
            st = oracle.als(A, u0, p["t_u"], p["t_v"], 1)
            t0 = time.perf_counter()
            oracle.als(A, u0, p["t_u"], p["t_v"], 1, state=st)
            t_tot += time.perf_counter() - t0
            nnz_s += int(nnz[i])
    est = t_tot * nnz.sum() / nnz_s
    return {"corpora_timed": len(pick), "nnz_timed": nnz_s, "s_timed": round(t_tot, 2),
            "s_per_batch_iteration_extrapolated": round(float(est), 1), "threads": _blas_threads(),
            "note": "one ALS iteration of every corpus, extrapolated from the sample by nonzeros"}


def batch_bench(problems, iters: int, warmup: int):
    """The many-corpora workload solved three ways from the same start: (i) a
    per-problem loop of ALS iterations, (ii) that loop captured as a HIP
    graph, (iii) one launch per stage for all problems, captured as a graph
    (plus (iii) without the graph).  The SpMM forms are first picked by the
    batch autotuner; every variant then restarts each problem from its U0 and
    must end at bit-identical errors (equal accuracy)."""
    import numpy as np
    import torch

    from paper_1510_05237_amd import NMFBatch

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    b = NMFBatch(problems, dtype="f32", device=dev)
    u0d = [torch.from_numpy(p["u0"]).to(dev) for p in problems]
    torch.cuda.synchronize()
    log(f"batch: created {len(problems)} problems in {time.perf_counter() - t0:.1f}s "
        f"(workspace {b.ws_bytes / 2**30:.2f} GiB)")

    def restart():
        for i, u in enumerate(u0d):
            b.problem(i).set_factors(u)
        torch.cuda.synchronize()

    # the autotuner picks each half's SpMM form on the fused batch; every
    # variant below then runs with that choice
    b.step(2, "fused")
    t0 = time.perf_counter()
    tuned = b.tune(iters=1)
    torch.cuda.synchronize()
    log(f"batch: tuned in {time.perf_counter() - t0:.1f}s: {tuned}")

    res, errs = {}, {}
    for how in ("loop", "loop_graph", "fused", "fused_graph"):
        restart()
        b.step(warmup, how)  # graph modes capture here
        restart()
        t0 = time.perf_counter()
        b.step(iters, how)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        E, st = b.errors()
        errs[how] = E
        res[how] = dt * 1e3 / iters
        log(f"batch {how}: {res[how]:.3f} ms per batch iteration")
        if np.any(st != 0):
            raise RuntimeError(f"batch {how}: member status {st[st != 0][:4]}")
    equal = all(np.array_equal(errs["loop"], e) for e in errs.values())
    nnz = sum(int(p["indptr"][-1]) for p in problems)
    # algorithmic bytes of one batch iteration's two products, every problem
    # at its factors' final storage (the same count as the single-problem
    # roofline), over the fused and graph-captured iteration time
    prod_bytes = 0.0
    for i, p in enumerate(problems):
        _, _, nu, nv = b.problem(i).history()
        prod_bytes += spmm_algorithmic_bytes(p["m"], p["n"], int(p["indptr"][-1]), float(nu[-1]), p["k"], 4, False)
        prod_bytes += spmm_algorithmic_bytes(p["n"], p["m"], int(p["indptr"][-1]), float(nv[-1]), p["k"], 4, True)
    gbs = prod_bytes / (res["fused_graph"] * 1e-3) / 1e9
    b.close()
    del u0d
    torch.cuda.empty_cache()
    return {
        "workload": f"batch_{len(problems)}_corpora",
        "problems": len(problems),
        "nnz_total": nnz,
        "iters": iters,
        "warmup": warmup,
        "ms_per_batch_iteration": {h: round(v, 3) for h, v in res.items()},
        "problem_iters_per_s": {h: round(len(problems) * 1e3 / v, 1) for h, v in res.items()},
        "speedup_vs_loop": {h: round(res["loop"] / v, 2) for h, v in res.items()},
        "equal_accuracy": bool(equal),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(gbs / 8000.0, 4), "algorithmic_bytes_per_iteration": prod_bytes,
                     "note": "both products' algorithmic bytes of every problem over the whole fused, "
                             "graph-captured batch iteration"},
        "tuned_spmm": tuned,
        "E_mean": float(np.mean(errs["fused_graph"])),
    }


def sweep_maxnnz(iters: int = 50):
    """Storage of enforced sparsity against the dense baseline (Section 3.2):
    on a PubMed-sized stand-in (20 112 terms x 7 510 docs, 0.4 % density,
    k = 5), the largest number of nonzeros of U and V stored at any half-step
    end, and the final E, for column-wise enforcement at several t and initial
    guesses U0 with several numbers of nonzeros per column; and Algorithm 1
    (dense) with the rule applied once after its last iteration."""
    import numpy as np
    import torch

    import synth
    from paper_1510_05237_amd import NMF

    n, m, k = 20112, 7510, 5
    c = synth.make_corpus(n, m, seed=7, alpha=1.1, nnz=int(round(0.004 * n * m)), dtype="f32")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(c.indptr).to(dev)
    ci = torch.from_numpy(c.indices).to(dev)
    cv = torch.from_numpy(c.data).to(dev)
    ts = [10, 30, 100, 300, 1000, 3000]
    rows = []
    for p0 in [20, 200, 2000, n]:
        rng = np.random.Generator(np.random.PCG64(1000 + p0))
        u0 = synth.sparse_factor_init(n, k, p0, rng=rng, dtype="f32")
        for t in ts:
            h = NMF(n, m, rp, ci, cv, torch.from_numpy(u0).to(dev), t_u=t, t_v=t, dtype="f32", device=dev)
            h.step(iters)
            rows.append(dict(u0_nnz_per_col=p0, t=t, rule="during", max_nnz=h.max_nnz(), E=h.error()))
            h.close()
        log(f"sweep: U0 with {p0} nonzeros per column done")
    u0, _ = synth.make_init(n, m, k, seed=7, dtype="f32")
    dense = []
    for t in ts:
        h = NMF(n, m, rp, ci, cv, torch.from_numpy(u0).to(dev), t_u=1, t_v=1, dtype="f32", device=dev,
                mode="none")
        h.step(iters)
        E_dense, mx = h.error(), h.max_nnz()
        h.enforce(t, t)
        dense.append(dict(t=t, rule="after", max_nnz=mx, E_dense=E_dense, E=h.error()))
        h.close()
    return {"workload": f"pubmed_like_{n}x{m}", "nnz": c.nnz, "k": k, "iters": iters,
            "enforced_during": rows, "dense_then_enforced": dense}


def sweep_accuracy(iters: int = 50):
    """Clustering accuracy of Eq. (acc) against sparsity (Section 3.2) on a
    PubMed-shaped corpus with planted labels (20 112 terms x 7 510 docs,
    5 journals, 80 distinct terms per doc, k = 5): the mean over topics for
    t per column enforced on U and V, on U only, on V only, and for dense
    Algorithm 1 with the rule applied once afterwards."""
    import numpy as np
    import torch

    import synth
    from paper_1510_05237_amd import NMF

    n, m, k, n_j = 20112, 7510, 5, 5
    c, labels = synth.make_labeled_corpus(n, m, n_j, 80, seed=9, dtype="f32")
    u0, _ = synth.make_init(n, m, k, seed=9, dtype="f32")
    dev = torch.device("cuda:0")
    args = [torch.from_numpy(x).to(dev) for x in (c.indptr, c.indices, c.data, u0)]
    lab = torch.from_numpy(labels).to(dev)
    rows = []
    for t in [10, 30, 100, 300, 1000, 3000]:
        res = dict(t=t)
        for name, tu, tv, mode in (("both", t, t, "column"), ("u_only", t, m, "column"),
                                   ("v_only", n, t, "column"), ("after", 1, 1, "none")):
            h = NMF(n, m, *args, t_u=tu, t_v=tv, dtype="f32", device=dev, mode=mode)
            h.step(iters)
            if name == "after":
                h.enforce(t, t)
            res[name] = float(np.mean(h.topic_accuracy(lab, n_j)))
            h.close()
        rows.append(res)
        log(f"accuracy sweep: t={t} {res}")
    return {"workload": f"planted_{n}x{m}_{n_j}_journals", "nnz": c.nnz, "k": k, "iters": iters, "rows": rows}


def compare_rules(total_iters: int = 100):
    """Time of 100 ALS iterations for a 5-topic factorization of a
    PubMed-sized stand-in (20 112 x 7 510, 0.4 % density): the top-t rule over
    the whole factor (t = 500 entries), per column (t = 100), and sequential
    ALS (Algorithm 3) with one topic per block, 20 iterations per block (the
    comparison of the paper's Section 4 timing table, on synthetic data).
    Wall time around the enqueued iterations, HIP-synchronized."""
    import torch

    import synth
    from paper_1510_05237_amd import NMF

    n, m, k = 20112, 7510, 5
    c = synth.make_corpus(n, m, seed=7, alpha=1.1, nnz=int(round(0.004 * n * m)), dtype="f32")
    u0, _ = synth.make_init(n, m, k, seed=7, dtype="f32")
    dev = torch.device("cuda:0")
    args = [torch.from_numpy(x).to(dev) for x in (c.indptr, c.indices, c.data, u0)]
    out = {}
    for name, mode, t_u, t_v in (("whole", "whole", 500, 500), ("column", "column", 100, 100),
                                 ("sequential", "column", 100, 100)):
        times = []
        for rep in range(3):
            h = NMF(n, m, *args, t_u=t_u, t_v=t_v, dtype="f32", device=dev, mode=mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "sequential":
                h.sequential(1, total_iters // k)
            else:
                h.step(total_iters)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            E = h.error()
            h.close()
        out[name] = dict(ms=round(min(times), 3), E=E)
        log(f"rules: {name} {out[name]}")
    res = [{"workload": f"pubmed_like_{n}x{m}", "nnz": c.nnz, "k": k, "iters": total_iters, "rules": out}]
    res.append(compare_rules_wide(total_iters))
    return res


def compare_rules_wide(total_iters: int = 100):
    """Per-column ALS (Algorithm 2) against sequential ALS (Algorithm 3) with
    one topic per block at k = 50 on the 100k x 200k corpus (t = 1000 / 2000
    per column): 100 iterations each, the sequential run as 50 blocks of two.
    Sequential blocks gather and store only their own column of the fixed
    factor; every other stage still spans all k columns."""
    import torch

    import synth
    from paper_1510_05237_amd import NMF

    c, u0, _, p = synth.make_workload("plain_f32_100kx200k")
    k = p["k"]
    dev = torch.device("cuda:0")
    args = [torch.from_numpy(x).to(dev) for x in (c.indptr, c.indices, c.data, u0)]
    out = {}
    for name in ("column", "sequential"):
        times = []
        for rep in range(2):
            h = NMF(c.n, c.m, *args, t_u=p["t_u"], t_v=p["t_v"], dtype="f32", device=dev, mode="column")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "sequential":
                h.sequential(1, total_iters // k)
            else:
                h.step(total_iters)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            E = h.error()
            h.close()
        out[name] = dict(ms=round(min(times), 3), E=E)
        log(f"rules (k={k}): {name} {out[name]}")
    return {"workload": f"plain_{c.n}x{c.m}", "nnz": c.nnz, "k": k, "k2": 1, "iters": total_iters, "rules": out}


def scale_oracle_sample(docs=(25_000, 100_000), iters: int = 2):
    """The FP64 oracle beside the scale configuration (1M terms, 200 terms
    per document, k = 100, alpha = 1.05), on document samples of the same
    recipe drawn on the host: per sample one untimed iteration from U0, then
    `iters` timed ones; t_u = 5000 as in the configuration, t_v scaled with
    the documents (20000 per 5M).  An oracle iteration costs a part fixed by
    the 1M terms (U's dense pre-selection matrix, its solve and its select)
    plus a part linear in the documents, so the two samples give the
    5M-document figure on a straight line.  Host only: no GPU is touched."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    import oracle
    from synth.scale import make_scale_corpus, make_scale_init

    n, m_full, d, k, t_u, t_v_full = 1_000_000, 5_000_000, 200, 100, 5000, 20000
    u0 = make_scale_init(n, k, seed=3, device="cpu").double().numpy()
    pts = []
    with threadpool_limits(limits=os.cpu_count() or 1):
        for m in docs:
            c = make_scale_corpus(n, m, d, seed=3, alpha=1.05, device="cpu")
            A = sp.csr_matrix((c.data.double().numpy(), c.indices.numpy().astype(np.int64), c.indptr.numpy()),
                              shape=(n, m))
            del c
            t_v = max(1, t_v_full * m // m_full)
            st = oracle.als(A, u0, t_u, t_v, 1)
            times = []
            for _ in range(iters):
                t0 = time.perf_counter()
                st = oracle.als(A, u0, t_u, t_v, 1, state=st)
                times.append(time.perf_counter() - t0)
            med = statistics.median(times)
            pts.append({"docs": m, "nnz": m * d, "t_v": t_v, "s_per_iteration": round(med, 2)})
            log(f"scale oracle sample: {m} documents, {med:.2f} s per steady-state iteration")
        threads = _blas_threads()
    (m0, s0), (m1, s1) = [(q["docs"], q["s_per_iteration"]) for q in pts[:2]]
    est = s0 + (s1 - s0) / (m1 - m0) * (m_full - m0)
    return {"workload": f"scale_{n}x{m_full}_k{k}", "kind": "oracle", "samples": pts,
            "s_per_iteration_extrapolated": round(est, 1), "it_per_s_extrapolated": round(1.0 / est, 5),
            "cores": threads, "host": host_info(),
            "note": ("FP64 numpy/scipy oracle, BLAS on all host threads (sparse products single-threaded); "
                     "each sample: 1 untimed iteration from U0, then the median of the timed ones; "
                     "extrapolated linearly in the document count to 5M documents (1B nonzeros)")}


def scale_rate(warm: int = 2, iters: int = 3):
    """The scale configuration (1M terms x 5M documents, 200 terms per
    document, 1B nonzeros, k = 100, t = 5000 / 20000 per column, FP32 with
    FP64 solves; corpus drawn on the GPU by synth.scale): handle creation
    time, then `iters` iterations after `warm` untimed ones, wall time per
    iteration and the event-timed stage breakdown of the same iterations."""
    import torch

    from paper_1510_05237_amd import NMF
    from synth.scale import make_scale_corpus, make_scale_init

    n, m, d, k, t_u, t_v = 1_000_000, 5_000_000, 200, 100, 5000, 20000
    dev = torch.device("cuda:0")
    c = make_scale_corpus(n, m, d, seed=3, alpha=1.05, device=dev)
    u0 = make_scale_init(n, k, seed=3, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = NMF(n, m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype="f32", device=dev)
    torch.cuda.synchronize()
    created = time.perf_counter() - t0
    del c
    log(f"scale: handle created in {created:.1f}s (workspace {prob.ws_bytes / 2**30:.1f} GiB)")
    prob.step(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.step(iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / iters
    prob.profile(True)
    prob.step(iters)
    torch.cuda.synchronize()
    pr = prob.profile_read()
    prob.profile(False)
    E = prob.error()
    prob.close()
    return {"workload": f"scale_{n}x{m}_k{k}", "nnz": m * d, "create_s": round(created, 2),
            "ms_per_iteration": round(ms, 2), "it_per_s": round(1e3 / ms, 2),
            "stage_ms": {st: round(v[0] / max(v[1], 1), 3) for st, v in pr.items()}, "E": E}


def compare_autograd(reps: int = 20):
    """The autograd loss on the 100k x 200k matrix with sparse U, V (t = 1000
    and 2000 per column): NMFLoss forward + backward against the same two
    ABI calls made directly (nmf_loss_fwd, nmf_loss_bwd), same outputs."""
    import numpy as np
    import torch

    import synth
    from paper_1510_05237_amd import NMF, NMFLoss
    from paper_1510_05237_amd.nmf import nmf_loss_bwd, nmf_loss_fwd

    c, _, _, p = synth.make_workload("plain_f32_100kx200k", with_init=False)
    k = p["k"]
    rng = np.random.Generator(np.random.PCG64(4))
    U = synth.sparse_factor_init(c.n, k, p["t_u"], rng=rng, dtype="f32")
    V = synth.sparse_factor_init(c.m, k, p["t_v"], rng=rng, dtype="f32")
    dev = torch.device("cuda:0")
    prob = NMF(c.n, c.m, torch.from_numpy(c.indptr).to(dev), torch.from_numpy(c.indices).to(dev),
               torch.from_numpy(c.data).to(dev), torch.from_numpy(U).to(dev), t_u=p["t_u"], t_v=p["t_v"],
               dtype="f32", device=dev)
    Ut = torch.tensor(U, device=dev, requires_grad=True)
    Vt = torch.tensor(V, device=dev, requires_grad=True)

    def autograd_step():
        Ut.grad = None
        Vt.grad = None
        L = NMFLoss.apply(prob, Ut, Vt)
        L.backward()
        return L

    Ud, Vd = Ut.detach(), Vt.detach()
    Ld = torch.empty((), dtype=torch.float64, device=dev)
    one = torch.ones((), dtype=torch.float64, device=dev)
    gU, gV = torch.empty_like(Ud), torch.empty_like(Vd)

    def direct_step():
        nmf_loss_fwd(prob.h, Ud, Vd, Ld)
        nmf_loss_bwd(prob.h, Ud, Vd, one, gU, gV)
        return Ld

    res = {}
    for name, fn in (("autograd", autograd_step), ("direct", direct_step)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name] = round((time.perf_counter() - t0) * 1e3 / reps, 4)
    L = autograd_step()
    direct_step()
    torch.cuda.synchronize()
    same = bool(float(L.detach()) == float(Ld) and torch.equal(Ut.grad, gU) and torch.equal(Vt.grad, gV))
    prob.close()
    return {"workload": "plain_f32_100kx200k sparse U,V (t_u=1000, t_v=2000, seed 4)", "k": k,
            "ms_fwd_bwd": res, "identical_outputs": same, "loss": float(L.detach())}


def copy_calibration(gib: float = 1.0, reps: int = 5):
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch

    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_f32_100kx200k")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="corpora in the batched comparison (0: skip)")
    ap.add_argument("--batch-iters", type=int, default=30)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--sweep-maxnnz", action="store_true",
                    help="print the max-NNZ sweep (enforced sparsity against dense ALS) and exit")
    ap.add_argument("--sweep-accuracy", action="store_true",
                    help="print the clustering-accuracy sweep (Eq. (acc) against t) and exit")
    ap.add_argument("--compare-rules", action="store_true",
                    help="print the whole-matrix / per-column / sequential timing comparison and exit")
    ap.add_argument("--compare-rules-k50", action="store_true",
                    help="print only the k = 50 per-column / sequential comparison and exit")
    ap.add_argument("--scale", action="store_true",
                    help="print the 1M x 5M (1B nonzeros, k = 100) rate and stage breakdown and exit")
    ap.add_argument("--scale-oracle", action="store_true",
                    help="print the FP64 oracle's time per iteration at the 1M x 5M scale, extrapolated from "
                         "document samples timed on the host (no GPU), and exit")
    ap.add_argument("--compare-autograd", action="store_true",
                    help="print the autograd-loss timing against direct ABI calls and exit")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched comparison (for profiling it); prints its JSON object")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the ALS iteration on a single MI355X "
              "(there is no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.scale_oracle:
        print(json.dumps({"scale_oracle": scale_oracle_sample()}), flush=True)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.compare_autograd:
        print(json.dumps({"autograd_comparison": compare_autograd()}), flush=True)
        return
    if args.compare_rules:
        print(json.dumps({"rules_comparison": compare_rules()}), flush=True)
        return
    if args.compare_rules_k50:
        print(json.dumps({"rules_comparison": [compare_rules_wide()]}), flush=True)
        return
    if args.scale:
        print(json.dumps({"scale": scale_rate()}), flush=True)
        return
    if args.sweep_accuracy:
        print(json.dumps({"accuracy_sweep": sweep_accuracy()}), flush=True)
        return
    if args.sweep_maxnnz:
        print(json.dumps({"maxnnz_sweep": sweep_maxnnz()}), flush=True)
        return

    import numpy as np
    import torch

    import synth
    from paper_1510_05237_amd import NMF

    batch = None
    if args.batch > 0:
        # drawn before anything touches the GPU: the generator forks workers
        t0 = time.perf_counter()
        batch = synth.make_batch(synth.batched_params(args.batch), dtype="f32",
                                 workers=min(16, os.cpu_count() or 1))
        log(f"generated the {args.batch}-corpus batch ({sum(p['nnz'] for p in batch)} nnz) "
            f"in {time.perf_counter() - t0:.1f}s")
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batch_only:
        if not batch:
            sys.exit("--batch-only needs --batch > 0")
        print(json.dumps({"batched": batch_bench(batch, args.batch_iters, args.batch_warmup)}), flush=True)
        return
    dev = torch.device("cuda:0")
    log(f"generating {args.workload}")
    t0 = time.perf_counter()
    corpus, u0, _, p = synth.make_workload(args.workload)
    log(f"generated n={corpus.n} m={corpus.m} nnz={corpus.nnz} in {time.perf_counter() - t0:.1f}s")
    dtype = p["dtype"]
    elt = 4 if dtype == "f32" else 8
    # inputs resident in HBM before anything is timed
    rp = torch.from_numpy(corpus.indptr).to(dev)
    ci = torch.from_numpy(corpus.indices).to(dev)
    cv = torch.from_numpy(corpus.data).to(dev)
    u0d = torch.from_numpy(u0).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = NMF(corpus.n, corpus.m, rp, ci, cv, u0d, t_u=p["t_u"], t_v=p["t_v"], dtype=dtype, device=dev)
    torch.cuda.synchronize()
    log(f"created handle in {time.perf_counter() - t0:.1f}s (workspace {prob.ws_bytes / 2**30:.2f} GiB)")

    # iteration 1 starts from the dense U0; it is timed on its own
    t0 = time.perf_counter()
    prob.step(1)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    if args.warmup > 1:
        prob.step(args.warmup - 1)
    torch.cuda.synchronize()
    log(f"warm-up done (first iteration {first_ms:.2f} ms)")

    E, R, nu, nv = None, None, None, None
    k = p["k"]
    # stage breakdown: every stage bracketed by events (each recorded event
    # delays the next launch by a few microseconds, so this pass is not the
    # headline); it also names the dominant kernel
    prob.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.step(args.steps)
    torch.cuda.synchronize()
    ms_all_events = (time.perf_counter() - t0) * 1e3 / args.steps
    prof = prob.profile_read()
    prob.profile(False)
    stage_ms = {name: (ms / cnt if cnt else None) for name, (ms, cnt) in prof.items()}
    _, _, nu, nv = prob.history(args.steps)
    nnz_u = float(np.mean(nu))
    nnz_v = float(np.mean(nv))
    bytes_v = spmm_algorithmic_bytes(corpus.m, corpus.n, corpus.nnz, nnz_u, k, elt, keep_c=False)
    bytes_u = spmm_algorithmic_bytes(corpus.n, corpus.m, corpus.nnz, nnz_v, k, elt, keep_c=True)
    kern = {}
    for stage, nbytes in (("spmm_v", bytes_v), ("spmm_u", bytes_u)):
        ms = stage_ms[stage]
        kern[stage] = dict(ms=ms, algorithmic_bytes=nbytes, gbs=nbytes / (ms * 1e-3) / 1e9)
    dom = max(kern, key=lambda s: kern[s]["ms"])
    log(f"stage breakdown pass: {ms_all_events:.3f} ms/iteration with every stage bracketed; dominant {dom}")

    # the timed region: only the dominant kernel is bracketed by events
    prob.profile(True, stages=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = prob.profile_read()
    prob.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} iterations: {ms_per_step:.3f} ms/iteration")
    dms, dcnt = prof[dom]
    assert dcnt == args.steps, (dom, dcnt)
    kern[dom]["ms"] = dms / dcnt
    kern[dom]["gbs"] = kern[dom]["algorithmic_bytes"] / (kern[dom]["ms"] * 1e-3) / 1e9
    E, R, nu, nv = prob.history(args.steps)
    achieved = kern[dom]["gbs"]
    traffic = read_traffic(dom)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": ("V-half product stage: k_vhalf (A^T U: hot block on fp32 MFMA + streamed gathers, "
                   "float64 MFMA solve, clamp)"
                   if dom == "spmm_v" else "U-half product stage: k_spmm + k_spmm_heavy (A V, float64 solve)"),
        "algorithmic_bytes_per_launch": kern[dom]["algorithmic_bytes"],
        "launch_ms": round(kern[dom]["ms"], 4),
    }
    out = {
        "metric": "ALS iters/sec + SpMM HBM GB/s (20M nnz, k=50); batched vs per-problem loop",
        "value": round(1e3 / ms_per_step, 2),
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": corpus.n, "m": corpus.m, "nnz": corpus.nnz, "k": k,
                   "t_u": p["t_u"], "t_v": p["t_v"], "mode": "column", "solve": "f64"},
        "roofline": roofline,
        "spmm_gbs": {s: round(v["gbs"], 1) for s, v in kern.items()},
        "stage_ms": {s: (round(v, 4) if v is not None else None) for s, v in stage_ms.items()},
        "ms_per_step_every_stage_bracketed": round(ms_all_events, 4),
        "first_iteration_ms": round(first_ms, 3),
        "E_last": float(E[-1]),
        "nnz_u": nnz_u,
        "nnz_v": nnz_v,
    }
    prob.close()
    del rp, ci, cv, u0d
    torch.cuda.empty_cache()
    out["batched"] = batch_bench(batch, args.batch_iters, args.batch_warmup) if batch else None
    batch_problems = batch
    batch = None
    if not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(corpus, u0, p, args.cpu_iters)
        log("timing the oracle's loss and gradient, and a sample of the batch")
        out["cpu_baseline"]["loss_fwd_bwd"] = cpu_loss_baseline()
        if batch_problems:
            out["cpu_baseline"]["batched"] = cpu_batch_baseline(batch_problems)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
