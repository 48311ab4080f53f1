"""GPU parity at the headline shape and on the full named workloads, against
the FP64 oracle on the same D and the same index sets.

- n = 10^4, r = 10, alpha = 0.3, |I| = |J| = ceil(3 r ln n) = 277, IRCUR-R:
  * FP64 storage: the GPU solve to e <= 1e-5 stops at the oracle's iteration,
    with the oracle's e history, L within 1e-10 and the sparse blocks
    [S_k]_{I,:}, [S_k]_{:,J} of the last iteration entry by entry;
  * BF16 storage (FP32 arithmetic, FP64 SVD): L and both sparse blocks within
    1e-2 of the oracle run on the bf16-rounded D (the arithmetic error) and of
    the oracle run on the original D (arithmetic plus the rounding of D);
- the 76800 x 1200 video stand-in in FP32: the whole IRCUR-R trajectory (the
  e history, the stopping iteration, L at the end and the last sparse blocks);
- n = 3 * 10^4 FP64 (the size sweep's largest point): the first five
  iterations against the oracle.
"""
import math

import numpy as np
import pytest

from oracle import ircur as O
from paper_2010_07422_amd import synth
from tests.gpu_util import require_gpu, to_dev, factors_np

pytestmark = pytest.mark.gpu


def _blocks(ctx):
    cur = ctx.cur()
    return (cur["S_I"].double().cpu().numpy(), cur["S_J"].double().cpu().numpy(), cur["I"], cur["J"])


def _mask_agrees(S_gpu, ref_S, ref_X, zeta, band):
    """Support of the sparse block: identical except where the oracle's |x| is
    within `band` of zeta (a decision that rounding may take either way)."""
    diff = (S_gpu != 0) != (ref_S != 0)
    near = np.abs(np.abs(ref_X) - zeta) <= band
    return int(np.count_nonzero(diff & ~near)), int(np.count_nonzero(diff))


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


@pytest.fixture(scope="module")
def planted_1e4():
    n, r = 10000, 10
    p = synth.planted(n, n, r, 0.3, seed=0)
    return p, r, synth.sample_size(3, r, n)


def test_f64_n10000_r10_full_solve_against_oracle(planted_1e4):
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IRCUR
    p, r, s = planted_1e4
    print(f"case n=10000 r=10 s={s} f64 solve vs oracle", flush=True)
    D = to_dev(torch, p.D, torch.float64)
    ctx = IRCUR(D, r, s, s, p.Lmax, gamma=0.7, eps=1e-5, max_iter=100, seed=1, resample=True)
    it, e, rc = ctx.solve()
    A, B = factors_np(ctx)
    SI, SJ, I, J = _blocks(ctx)
    h = np.array(ctx.history())
    ctx.close()
    del D
    ref = O.ircur(p.D, r, s, s, p.Lmax, 0.7, 1e-5, 100, seed=1, resample=True)
    print("gpu iters", it, "e", e, "oracle iters", ref.k, "e", ref.e_hist[-1], flush=True)
    assert it == ref.k and e <= 1e-5
    assert np.array_equal(I, ref.I) and np.array_equal(J, ref.J)
    # e history: relative 1e-9, or absolute 1e-14 where e is at rounding level
    assert np.all(np.abs(h - ref.e_hist) <= 1e-9 * np.array(ref.e_hist) + 1e-14)
    dL = O.factored_rel_diff(A, B, ref.A, ref.B)
    print("L rel diff", dL, "vs planted L", O.factored_rel_diff(A, B, p.W, p.V.T), flush=True)
    assert dL <= 1e-10
    zeta = p.Lmax * 0.7 ** (it - 1)
    last = ref.last
    for S_g, S_o, X_o in ((SI, last["S_I"], last["X_I"]), (SJ, last["S_J"], last["X_J"])):
        bad, flips = _mask_agrees(S_g, S_o, X_o, zeta, 1e-9 * zeta)
        assert bad == 0, flips
        both = (S_g != 0) & (S_o != 0)
        assert np.max(np.abs(S_g - S_o)[both]) <= 1e-10 * np.abs(S_o).max()
        assert _rel(S_g, S_o) <= 1e-10


def test_bf16_n10000_r10_against_oracle(planted_1e4):
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IRCUR
    p, r, s = planted_1e4
    print(f"case n=10000 r=10 s={s} bf16 solve vs oracle (rounded D and original D)", flush=True)
    Dbf = to_dev(torch, p.D, torch.float64).to(torch.bfloat16)
    Dr = Dbf.double().cpu().numpy()
    ctx = IRCUR(Dbf, r, s, s, p.Lmax, gamma=0.7, eps=1e-5, max_iter=100, seed=1, resample=True)
    it, e, rc = ctx.solve()
    A, B = factors_np(ctx)
    SI, SJ, I, J = _blocks(ctx)
    ctx.close()
    del Dbf
    assert e <= 1e-5
    for name, Dref in (("bf16-rounded D", Dr), ("original D", p.D)):
        ref = O.ircur(Dref, r, s, s, p.Lmax, 0.7, -1.0, it, seed=1, resample=True)
        assert np.array_equal(I, ref.I) and np.array_equal(J, ref.J)
        dL = O.factored_rel_diff(A, B, ref.A, ref.B)
        dSI = _rel(SI, ref.last["S_I"])
        dSJ = _rel(SJ, ref.last["S_J"])
        print(f"vs oracle on {name}: L {dL:.3e}  S_I {dSI:.3e}  S_J {dSJ:.3e}", flush=True)
        assert dL <= 1e-2 and dSI <= 1e-2 and dSJ <= 1e-2


def test_video_76800x1200_f32_full_trajectory():
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IRCUR
    cfg = synth.CONFIGS["video_76800x1200_r2_f32"]
    v = synth.video(cfg["h"], cfg["w"], cfg["frames"], seed=cfg["data_seed"])
    Lmax = float(np.abs(v.F @ v.G.T).max())
    r, sI, sJ = cfg["r"], cfg["sI"], cfg["sJ"]
    print("case video 76800x1200 f32 full trajectory", flush=True)
    D = to_dev(torch, v.D, torch.float32)
    ctx = IRCUR(D, r, sI, sJ, Lmax, gamma=cfg["gamma"], eps=cfg["eps"], max_iter=cfg["max_iter"],
                seed=cfg["index_seed"], resample=True)
    it, e, rc = ctx.solve()
    A, B = factors_np(ctx)
    SI, SJ, I, J = _blocks(ctx)
    h = np.array(ctx.history())
    ctx.close()
    del D
    ref = O.ircur(v.D.astype(np.float64), r, sI, sJ, Lmax, cfg["gamma"], cfg["eps"], cfg["max_iter"],
                  seed=cfg["index_seed"], resample=True)
    print("gpu iters", it, "e", e, "oracle iters", ref.k, "e", ref.e_hist[-1], flush=True)
    assert it == ref.k and e <= 1e-5
    assert np.array_equal(I, ref.I) and np.array_equal(J, ref.J)
    # e history: 1e-3 relative, plus an absolute floor for the FP32 rounding of
    # the entries of D - L that make up its numerator (~ 2 eps_32 max|D|)
    eps32 = 2.0 ** -23
    dmax = float(np.abs(v.D).max())
    hdiff = np.abs(h - ref.e_hist)
    print("e history max rel diff", (hdiff / np.array(ref.e_hist)).max(), flush=True)
    assert np.all(hdiff <= 1e-3 * np.array(ref.e_hist) + 2 * eps32 * dmax)
    dL = O.factored_rel_diff(A, B, ref.A, ref.B)
    print("L rel diff", dL, "vs background", O.factored_rel_diff(A, B, v.F, v.G.T), flush=True)
    assert dL <= 1e-5
    zeta = Lmax * cfg["gamma"] ** (it - 1)
    # a threshold decision is pinned only where |x| stays clear of zeta by more
    # than the two runs' entrywise difference in L on the sampled blocks (taken
    # from their final factors) plus the FP32 rounding of x
    dLI = np.abs(A[I] @ B - ref.A[I] @ ref.B).max()
    dLJ = np.abs(A @ B[:, J] - ref.A @ ref.B[:, J]).max()
    band = 2.0 * max(dLI, dLJ) + 4 * eps32 * dmax
    print("entrywise L difference on the blocks", dLI, dLJ, "band", band, flush=True)
    for S_g, S_o, X_o in ((SI, ref.last["S_I"], ref.last["X_I"]), (SJ, ref.last["S_J"], ref.last["X_J"])):
        bad, flips = _mask_agrees(S_g, S_o, X_o, zeta, band)
        print("support flips", flips, "outside the band", bad, "of", S_o.size, flush=True)
        assert bad == 0, flips
        assert _rel(S_g, S_o) <= 1e-5


def test_f64_n30000_first_iterations_against_oracle():
    """The largest size of the scaling sweep, FP64, drawn on the device with
    the planted recipe; five IRCUR-R iterations against the oracle on the
    same D (copied to the host) and index sets."""
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IRCUR
    n, r = 30000, 10
    s = synth.sample_size(3, r, n)
    print(f"case n=30000 r=10 s={s} f64, 5 iterations vs oracle", flush=True)
    pd = synth.planted_device(n, n, r, 0.3, seed=5, dtype=torch.float64)
    Lmax = pd.Lmax
    ctx = IRCUR(pd.D, r, s, s, Lmax, gamma=0.7, eps=-1.0, max_iter=5, seed=2, resample=True)
    it, e, rc = ctx.solve()
    A, B = factors_np(ctx)
    h = np.array(ctx.history())
    ctx.close()
    Dh = pd.D.cpu().numpy()
    del pd
    torch.cuda.empty_cache()
    ref = O.ircur(Dh, r, s, s, Lmax, 0.7, -1.0, 5, seed=2, resample=True)
    dL = O.factored_rel_diff(A, B, ref.A, ref.B)
    print("iters", it, "L rel diff", dL, "e", h, ref.e_hist, flush=True)
    assert it == 5 and dL <= 1e-10
    assert np.all(np.abs(h - ref.e_hist) <= 1e-9 * np.array(ref.e_hist) + 1e-14)
