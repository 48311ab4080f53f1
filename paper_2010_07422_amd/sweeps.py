"""Sweeps over the IRCUR library: size scaling, concurrent instances and the
recovery phase transition.

* ``scaling_sweep`` -- iterations/s, pass-kernel bandwidth and time to
  e <= eps as n grows (square planted instances, IRCUR-R and IRCUR-F); the
  per-iteration cost of Algorithm 1 is O(r^2 n log^2 n) (Section 3.3), so
  iterations/s should fall roughly like n log^2 n once the pass dominates.
* ``concurrent_throughput`` -- k independent instances, each on its own
  stream, stepped together: aggregate iterations/s.
* ``phase_transition`` -- the empirical recovery map of Section 4.1 /
  Fig. 1: for each rank r, sampling constant c (|I| = |J| = ceil(c r ln n))
  and outlier fraction alpha, the share of trials whose final L is within
  `tol` of the planted L in relative Frobenius norm.  Ranks above 16 take
  the wide SVD variant, which holds |J| up to about 70 in LDS, so the default
  map covers r = 5 and 10.

Every number here comes from the GPU library (``IRCUR``); instances are drawn
on the device by ``synth.planted_device``.
"""
from __future__ import annotations

import math
import time

from . import synth
from .ircur import IRCUR


def pass_bytes(n1, n2, sI, sJ, r, b_d, b_f):
    """Algorithmic HBM bytes of one pass launch: the sampled rows of D and of
    D^T, the factors read (B_k, A_k^T) and written (B_{k+1}, A_{k+1}^T)."""
    return b_d * (sI * n2 + sJ * n1) + 2 * b_f * r * (n1 + n2)


def _dtype(name):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[name]


def sampled_rel_err(At, B, W, V, nsamp=1 << 16, seed=0):
    """Relative error of L = A B against W V^T on `nsamp` random entries (both
    sides in float64 on the device)."""
    import torch
    n1, n2 = W.shape[0], V.shape[0]
    g = torch.Generator(device=W.device)
    g.manual_seed(seed)
    i = torch.randint(0, n1, (nsamp,), generator=g, device=W.device)
    j = torch.randint(0, n2, (nsamp,), generator=g, device=W.device)
    Lg = (At.double()[:, i] * B.double()[:, j]).sum(0)
    Lt = (W[i] * V[j]).sum(1)
    return float(torch.linalg.vector_norm(Lg - Lt) / torch.linalg.vector_norm(Lt))


def dense_rel_err(At, B, W, V):
    """||A B - W V^T||_F / ||W V^T||_F formed densely (small n)."""
    import torch
    L = W @ V.T
    return float(torch.linalg.matrix_norm(At.double().T @ B.double() - L) / torch.linalg.matrix_norm(L))


def scaling_sweep(ns=(1000, 3000, 10000, 30000), r=10, alpha=0.3, c=3.0, dtype="bf16",
                  modes=("R", "F"), steps=100, warmup=10, eps=1e-5, seed=0, pass_reps=200):
    """One planted instance per n (drawn on the device); for each mode the
    iteration rate over `steps` iterations after `warmup`, the pass kernel's
    mean duration and algorithmic bandwidth, and a solve to e <= eps with its
    time, iteration count and sampled error against the planted L."""
    import torch
    out = []
    b_d = {"f64": 8, "f32": 4, "bf16": 2}[dtype]
    b_f = 8 if dtype == "f64" else 4
    for n in ns:
        p = synth.planted_device(n, n, r, alpha, seed=seed + n, dtype=_dtype(dtype))
        s = min(n, synth.sample_size(c, r, n))
        for mode in modes:
            res = mode == "R"
            ctx = IRCUR(p.D, r, s, s, p.Lmax, gamma=0.7, eps=-1.0, max_iter=warmup + steps + 2, seed=1,
                        resample=res)
            ctx.enqueue(warmup)
            ctx.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.enqueue(steps)
            ctx.sync()
            t = time.perf_counter() - t0
            pass_us = ctx.time_pass(pass_reps)
            ctx.close()
            ctx = IRCUR(p.D, r, s, s, p.Lmax, gamma=0.7, eps=eps, max_iter=100, seed=1, resample=res)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, e, _ = ctx.solve()
            tt = time.perf_counter() - t0
            At, B = ctx.factors()
            ctx.close()
            out.append(dict(n=n, s=s, r=r, mode=mode, dtype=dtype, iters_per_s=steps / t,
                            pass_us=pass_us, pass_GBs=pass_bytes(n, n, s, s, r, b_d, b_f) / (pass_us * 1e3),
                            time_to_tol_ms=1e3 * tt, iters_to_tol=it, e_final=e,
                            rel_err_L_sampled=sampled_rel_err(At, B, p.W, p.V)))
        del p
        torch.cuda.empty_cache()
    return out


def concurrent_throughput(n=3000, r=5, alpha=0.2, c=4.0, dtype="f32", ks=(1, 2, 4, 8), steps=200,
                          warmup=10, seed=0):
    """Aggregate iterations/s of k independent IRCUR-R instances, each with
    its own stream (default priority), enqueued round-robin in chunks."""
    import torch
    out = []
    kmax = max(ks)
    inst = [synth.planted_device(n, n, r, alpha, seed=seed + b, dtype=_dtype(dtype)) for b in range(kmax)]
    s = min(n, synth.sample_size(c, r, n))
    streams = [torch.cuda.Stream() for _ in range(kmax)]
    for k in ks:
        ctxs = [IRCUR(inst[b].D, r, s, s, inst[b].Lmax, gamma=0.7, eps=-1.0, max_iter=warmup + steps + 2,
                      seed=10 + b, resample=True, stream=streams[b]) for b in range(k)]
        for cx in ctxs:
            cx.enqueue(warmup)
        for cx in ctxs:
            cx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chunk = 8
        for q in range(0, steps, chunk):
            for cx in ctxs:
                cx.enqueue(min(chunk, steps - q))
        for cx in ctxs:
            cx.sync()
        t = time.perf_counter() - t0
        for cx in ctxs:
            cx.close()
        out.append(dict(n=n, r=r, s=s, dtype=dtype, instances=k, iters_per_s=k * steps / t))
    return out


def phase_transition(n=1000, ranks=(5, 10), cs=(1.0, 2.0, 3.0, 4.0, 5.0, 6.0),
                     alphas=(0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.45, 0.5), trials=50,
                     tol=1e-3, gamma=0.7, eps=1e-5, max_iter=100, dtype="f64", seed=0):
    """Share of successful recoveries per (r, c, alpha): IRCUR-R from L_0 = 0
    with zeta_0 = max|L|, stopped at e <= eps or max_iter; a trial succeeds
    when ||L - L*||_F / ||L*||_F <= tol.  Returns the rows of the map and the
    number of trials per second."""
    import torch
    rows = []
    t0 = time.perf_counter()
    ntr = 0
    for r in ranks:
        for c in cs:
            s = min(n, synth.sample_size(c, r, n))
            if s < r:
                continue
            for a in alphas:
                ok = 0
                iters = 0
                for t in range(trials):
                    tseed = seed + 1000003 * r + 10007 * int(round(10 * c)) + 101 * int(round(1000 * a)) + t
                    p = synth.planted_device(n, n, r, a, seed=tseed, dtype=_dtype(dtype))
                    ctx = IRCUR(p.D, r, s, s, p.Lmax, gamma=gamma, eps=eps, max_iter=max_iter, seed=tseed,
                                resample=True)
                    it, _, _ = ctx.solve()
                    At, B = ctx.factors()
                    ctx.close()
                    err = dense_rel_err(At, B, p.W, p.V)
                    ok += 1 if err <= tol else 0
                    iters += it
                    ntr += 1
                rows.append(dict(r=r, c=c, s=s, alpha=a, trials=trials, success=ok / trials,
                                 mean_iters=iters / trials))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return rows, ntr / t
