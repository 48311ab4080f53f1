"""ircur_to_svd_noalloc (Algorithm 2 on the current factors with the
library's fixed device workspace) against ircur_to_svd, which allocates its
workspace: two calls in a row, the second on a smaller problem, both checked
bit for bit against the allocating entry point on the same context and
against the oracle's Algorithm 2 on the same factors."""
import numpy as np
import pytest

from oracle import ircur as O
from paper_2010_07422_amd import synth
from tests.gpu_util import require_gpu, to_dev, factors_np

pytestmark = pytest.mark.gpu


def _ctx(torch, n1, n2, r, s, seed, dtype):
    from paper_2010_07422_amd.ircur import IRCUR
    p = synth.planted(n1, n2, r, 0.1, seed=seed)
    ctx = IRCUR(to_dev(torch, p.D, dtype), r, s, s, p.Lmax, gamma=0.7, eps=-1.0, max_iter=12, seed=seed,
                resample=True)
    ctx.solve()
    return ctx


@pytest.mark.parametrize("dtname", ["f64", "f32"])
def test_noalloc_matches_allocating_entry_point(dtname):
    torch = require_gpu()
    dtype = {"f64": torch.float64, "f32": torch.float32}[dtname]
    # second call smaller in every size (n1, n2, r and the Gram workgroups)
    for n1, n2, r, s, seed in ((2500, 1900, 8, 180, 21), (640, 520, 3, 70, 22)):
        print(f"case noalloc {dtname} n1={n1} n2={n2} r={r}", flush=True)
        ctx = _ctx(torch, n1, n2, r, s, seed, dtype)
        Wn, sn, Vn = (t.cpu().numpy() for t in ctx.to_svd(noalloc=True))
        Wa, sa, Va = (t.cpu().numpy() for t in ctx.to_svd())
        # same kernels, same launch shape: identical bits
        assert np.array_equal(Wn, Wa) and np.array_equal(sn, sa) and np.array_equal(Vn, Va)
        A, B = factors_np(ctx)
        Wo, so, Vo = O.factors_to_svd(A, B)
        assert np.allclose(sn, so, rtol=1e-12, atol=0)
        L = (Wo * so) @ Vo.T
        assert np.linalg.norm((Wn * sn) @ Vn.T - L) <= 1e-12 * np.linalg.norm(L)
        ctx.close()


def test_noalloc_repeated_calls_keep_no_state():
    """The workspace keeps the previous call's contents; a call on another
    context right after must not depend on them."""
    torch = require_gpu()
    big = _ctx(torch, 3000, 2800, 12, 200, 31, torch.float64)
    small = _ctx(torch, 300, 260, 2, 40, 32, torch.float64)
    print("case noalloc interleaved big/small contexts", flush=True)
    ref_small = [t.cpu().numpy() for t in small.to_svd()]
    big.to_svd(noalloc=True)
    got_small = [t.cpu().numpy() for t in small.to_svd(noalloc=True)]
    for a, b in zip(got_small, ref_small):
        assert np.array_equal(a, b)
    big.close()
    small.close()
