"""GPU runs of the named workloads and edge cases, through the C ABI.

- n = 3000, r = 5, FP32: to e <= 1e-5 against the FP64 oracle on the same
  (float-rounded) D and index sets, <= 1e-5;
- (the n = 10^4 BF16/FP64 and video workloads are compared with the oracle
  in test_gpu_northstar.py)
- edge cases: |I| = n1 and |J| = n2 (CUR of the whole matrix), r = 1,
  zeta_0 = 0, exact low rank, a NaN in D, resume from a checkpoint, IRCUR-F,
  err_mode 1, bitwise repeatability.
"""
import numpy as np
import pytest

from oracle import ircur as O
from oracle import sampler
from paper_2010_07422_amd import synth
from tests.gpu_util import require_gpu, to_dev, factors_np

pytestmark = pytest.mark.gpu


def _ctx(torch, D, dtype, r, sI, sJ, zeta0, **kw):
    from paper_2010_07422_amd.ircur import IRCUR
    Dd = to_dev(torch, D, dtype) if not hasattr(D, "is_cuda") else D
    return IRCUR(Dd, r, sI, sJ, zeta0, **kw), Dd


def test_planted_n3000_r5_f32_against_oracle():
    torch = require_gpu()
    cfg = synth.CONFIGS["planted_n3000_r5_f32"]
    n, r = cfg["n"], cfg["r"]
    p = synth.planted(n, n, r, cfg["alpha"], seed=cfg["data_seed"])
    s = synth.sample_size(cfg["c"], r, n)
    D32 = p.D.astype(np.float32)
    print("case n=3000 r=5 f32", flush=True)
    ctx, _ = _ctx(torch, D32, torch.float32, r, s, s, p.Lmax, gamma=cfg["gamma"], eps=cfg["eps"],
                  max_iter=cfg["max_iter"], seed=cfg["index_seed"], resample=True)
    it, e, rc = ctx.solve()
    A, B = factors_np(ctx)
    ref = O.ircur(D32.astype(np.float64), r, s, s, p.Lmax, cfg["gamma"], 0.0, it, seed=cfg["index_seed"],
                  resample=True)
    d = O.factored_rel_diff(A, B, ref.A, ref.B)
    print("iters", it, "e", e, "diff vs oracle", d, "vs truth", O.factored_rel_diff(A, B, p.W, p.V.T), flush=True)
    assert e <= 1e-5 and d <= 1e-5
    ctx.close()


@pytest.mark.parametrize("case", ["full_sets", "rank1", "zeta0_zero", "exact_rank"])
def test_edge_cases_f64(case):
    torch = require_gpu()
    print("case edge", case, flush=True)
    if case == "full_sets":
        p = synth.planted(60, 50, 3, 0.05, seed=3)
        D, r, sI, sJ, z0, iters = p.D, 3, 60, 50, p.Lmax, 6
    elif case == "rank1":
        p = synth.planted(300, 280, 1, 0.1, seed=4)
        D, r, sI, sJ, z0, iters = p.D, 1, 40, 37, p.Lmax, 8
    elif case == "zeta0_zero":
        p = synth.planted(200, 200, 2, 0.1, seed=5)
        D, r, sI, sJ, z0, iters = p.D, 2, 30, 30, 0.0, 3
    else:
        D, _, _ = synth.exact_lowrank(250, 240, 4, seed=6)
        r, sI, sJ, z0, iters = 4, 40, 40, float(np.abs(D).max()), 3
    ctx, _ = _ctx(torch, D, torch.float64, r, sI, sJ, z0, eps=-1.0, max_iter=iters, seed=9, resample=True)
    ctx.solve()
    A, B = factors_np(ctx)
    ref = O.ircur(D, r, sI, sJ, z0, 0.7, -1.0, iters, seed=9, resample=True)
    if case == "zeta0_zero":
        assert np.all(A == 0.0) and np.all(B == 0.0)      # S = D on the blocks: M = 0, U^+ = 0
        assert np.abs(ref.A @ ref.B).max() == 0.0
    else:
        d = O.factored_rel_diff(A, B, ref.A, ref.B)
        print("diff", d, flush=True)
        assert d <= 1e-10
    if case == "exact_rank":
        assert O.factored_rel_diff(A, B, D, np.eye(D.shape[1])) <= 1e-13    # Theorem 1
    ctx.close()


def test_nonfinite_input_is_reported():
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IrcurError, ERR_NONFINITE
    p = synth.planted(200, 200, 2, 0.1, seed=5)
    D = p.D.copy()
    I, J = sampler.draw_IJ(1, 0, 200, 200, 30, 30)
    D[I[3], 17] = np.nan
    ctx, _ = _ctx(torch, D, torch.float64, 2, 30, 30, p.Lmax, eps=-1.0, max_iter=5, seed=1)
    with pytest.raises(IrcurError) as ei:
        ctx.solve()
    assert ei.value.code == ERR_NONFINITE
    ctx.close()


def test_checkpoint_resume_is_bitwise():
    torch = require_gpu()
    p = synth.planted(800, 700, 4, 0.1, seed=8)
    kw = dict(eps=-1.0, max_iter=20, seed=3, resample=True)
    ctx, Dd = _ctx(torch, p.D, torch.float32, 4, 90, 80, p.Lmax, **kw)
    ctx.enqueue(8)
    ctx.sync()
    blob = ctx.get_state()
    ctx.enqueue(12)
    ctx.sync()
    A1, B1 = factors_np(ctx)
    h1 = ctx.history()
    ctx2, _ = _ctx(torch, Dd, None, 4, 90, 80, p.Lmax, **kw)
    ctx2.set_state(blob)
    ctx2.enqueue(12)
    ctx2.sync()
    A2, B2 = factors_np(ctx2)
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2)
    assert h1 == ctx2.history()
    ctx.close()
    ctx2.close()


def test_repeat_is_bitwise_and_modes():
    torch = require_gpu()
    p = synth.planted(600, 650, 3, 0.1, seed=12)
    res = []
    for rep in range(2):
        ctx, _ = _ctx(torch, p.D, torch.float64, 3, 70, 75, p.Lmax, eps=-1.0, max_iter=12, seed=4, resample=False)
        ctx.solve()
        res.append(factors_np(ctx) + (ctx.history(),))
        ctx.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]
    # IRCUR-F against the oracle
    ref = O.ircur(p.D, 3, 70, 75, p.Lmax, 0.7, -1.0, 12, seed=4, resample=False)
    assert O.factored_rel_diff(res[0][0], res[0][1], ref.A, ref.B) <= 1e-10
    assert np.allclose(res[0][2], ref.e_hist, rtol=1e-6)
    # err_mode 1 (the below-threshold part of D - L_k) against the oracle
    ctx, _ = _ctx(torch, p.D, torch.float64, 3, 70, 75, p.Lmax, eps=-1.0, max_iter=6, seed=4, resample=True,
                  err_mode=1)
    ctx.solve()
    ref = O.ircur(p.D, 3, 70, 75, p.Lmax, 0.7, -1.0, 6, seed=4, resample=True, err_mode=1)
    assert np.allclose(ctx.history(), ref.e_hist, rtol=1e-6)
    ctx.close()


def test_time_pass_leaves_the_run_unchanged():
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IrcurError, ERR_STATE
    p = synth.planted(700, 650, 3, 0.1, seed=21)
    kw = dict(eps=-1.0, max_iter=20, seed=2, resample=True)
    print("case time_pass", flush=True)
    ctx, Dd = _ctx(torch, p.D, torch.float32, 3, 80, 75, p.Lmax, **kw)
    with pytest.raises(IrcurError) as ei:
        ctx.time_pass(3)
    assert ei.value.code == ERR_STATE
    ctx.enqueue(6)
    ctx.sync()
    A0, B0 = factors_np(ctx)
    us = ctx.time_pass(20)
    A1, B1 = factors_np(ctx)
    assert us > 0.0 and np.array_equal(A0, A1) and np.array_equal(B0, B1)
    ctx.enqueue(6)
    ctx.sync()
    A1, B1 = factors_np(ctx)
    ctx2, _ = _ctx(torch, Dd, None, 3, 80, 75, p.Lmax, **kw)
    ctx2.enqueue(12)
    ctx2.sync()
    A2, B2 = factors_np(ctx2)
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2)
    assert ctx.history() == ctx2.history()
    ctx.close()
    ctx2.close()


@pytest.mark.parametrize("eps,max_iter", [(1e-5, 100), (1e-3, 100), (0.0, 3), (0.0, 11), (1e-5, 1)])
def test_solve_stops_where_single_steps_stop(eps, max_iter):
    """ircur_solve (chunks enqueued two at a time, iterations past the device
    stop are no-ops) ends at the same iteration, with the same e history and
    the same factors bit for bit, as single steps stopped by the host."""
    torch = require_gpu()
    n, r = 1000, 5
    p = synth.planted(n, n, r, 0.1, seed=31)
    s = synth.sample_size(4, r, n)
    print(f"case solve vs steps eps={eps} max_iter={max_iter}", flush=True)
    a, Dd = _ctx(torch, p.D.astype(np.float32), torch.float32, r, s, s, p.Lmax, gamma=0.7, eps=eps,
                 max_iter=max_iter, seed=5, resample=True)
    it, e, rc = a.solve()
    b, _ = _ctx(torch, Dd, None, r, s, s, p.Lmax, gamma=0.7, eps=eps, max_iter=max_iter, seed=5, resample=True)
    k = 0
    while k < max_iter:
        eb = b.step()
        k += 1
        if eb <= eps:
            break
    assert it == k
    assert a.history() == b.history()
    Aa, Ba = factors_np(a)
    Ab, Bb = factors_np(b)
    assert np.array_equal(Aa, Ab) and np.array_equal(Ba, Bb)
    a.close()
    b.close()
