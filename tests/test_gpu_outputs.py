"""GPU outputs outside the iteration loop, through the C ABI, against the oracle:

- ircur_get_cur: C_k, U_k^+, R_k and the sparse blocks of the last iteration
  (Algorithm 1's output), recomputed from that iteration's inputs;
- ircur_sparse_full: T_zeta(D - A_k B_k) over all of D;
- ircur_to_svd: Algorithm 2 on the factored estimate.
"""
import numpy as np
import pytest

from oracle import ircur as O
from oracle import sampler
from paper_2010_07422_amd import synth
from tests.gpu_util import require_gpu, to_dev, factors_np

pytestmark = pytest.mark.gpu


def _run(torch, p, r, s1, s2, iters, dtype, resample=True, seed=3, eps=0.0):
    from paper_2010_07422_amd.ircur import IRCUR
    Dd = to_dev(torch, p.D, dtype)
    ctx = IRCUR(Dd, r, s1, s2, p.Lmax, gamma=0.7, eps=eps, max_iter=iters, seed=seed, resample=resample)
    ctx.solve()
    return ctx, Dd


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("dtname,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_get_cur_matches_oracle(dtname, tol):
    torch = require_gpu()
    dtype = {"f64": torch.float64, "f32": torch.float32}[dtname]
    n1, n2, r, s1, s2, iters = 700, 650, 4, 60, 55, 4
    p = synth.planted(n1, n2, r, 0.1, seed=11)
    D = p.D if dtname == "f64" else p.D.astype(np.float32).astype(np.float64)
    print(f"case get_cur {dtname} n1={n1} n2={n2} r={r}", flush=True)
    ctx, Dd = _run(torch, p, r, s1, s2, iters, dtype)
    cur = {k: (v.double().cpu().numpy() if hasattr(v, "cpu") else v) for k, v in ctx.cur().items()}
    ref = O.ircur(D, r, s1, s2, p.Lmax, 0.7, 0.0, iters, seed=3, resample=True, keep_states=True)
    A_prev, B_prev = ref.state_hist[-2]
    I, J = ref.IJ_hist[-1]
    assert np.array_equal(cur["I"], I) and np.array_equal(cur["J"], J)
    C, Up, R, SI, SJ = O.cur_components(D, A_prev, B_prev, I, J, p.Lmax * 0.7 ** (iters - 1), r)
    for name, got, want in (("C", cur["C"], C), ("R", cur["R"], R), ("U+", cur["Upinv"], Up)):
        d = _rel(got, want)
        print(name, d, flush=True)
        assert d <= tol, name
    # sparse blocks: same support, same values
    assert np.array_equal(cur["S_I"] != 0, SI != 0) and np.array_equal(cur["S_J"] != 0, SJ != 0)
    assert _rel(cur["S_I"], SI) <= tol and _rel(cur["S_J"], SJ) <= tol
    # the output reproduces the estimate: C U^+ R = A_k B_k
    A, B = factors_np(ctx)
    Lcur = cur["C"] @ cur["Upinv"] @ cur["R"]
    assert _rel(Lcur, A @ B) <= (1e-11 if dtname == "f64" else 1e-5)
    # [S]_{I,J} is the same in both blocks, and R + S_I = D[I, :]
    assert np.array_equal(cur["S_I"][:, J], cur["S_J"][I, :])
    Dh = Dd.double().cpu().numpy()
    ulp = 2.0 ** -52 if dtname == "f64" else 2.0 ** -23
    assert np.allclose(cur["R"] + cur["S_I"], Dh[I, :], rtol=0, atol=4 * ulp * np.abs(Dh).max())
    ctx.close()


def test_get_cur_requires_an_iteration():
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IRCUR, IrcurError
    p = synth.planted(200, 180, 2, 0.1, seed=1)
    ctx = IRCUR(to_dev(torch, p.D, torch.float64), 2, 30, 30, p.Lmax, max_iter=5)
    with pytest.raises(IrcurError):
        ctx.cur()
    ctx.step()
    ctx.cur()
    ctx.reset()
    with pytest.raises(IrcurError):
        ctx.cur()
    ctx.close()


@pytest.mark.parametrize("dtname", ["f64", "f32", "bf16"])
def test_sparse_full_matches_threshold_of_factors(dtname):
    torch = require_gpu()
    dtype = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtname]
    n, r = 1000, 5
    p = synth.planted(n, n, r, 0.1, seed=0)
    s = synth.sample_size(4, r, n)
    print(f"case sparse_full {dtname}", flush=True)
    ctx, Dd = _run(torch, p, r, s, s, 40, dtype)
    A, B = factors_np(ctx)
    Dh = Dd.double().cpu().numpy()
    X = Dh - A @ B
    for zeta in (-1.0, 1e-3 * p.Lmax, 0.0):
        S, nnz = ctx.sparse_full(zeta)
        Sh = S.double().cpu().numpy()
        z = p.Lmax * 0.7 ** 40 if zeta < 0 else zeta
        ref = O.hard_threshold(X, z)
        # decisions compared away from a rounding band around zeta
        band = np.abs(np.abs(X) - z) <= (1e-12 if dtname == "f64" else 1e-4) * np.abs(Dh).max()
        assert np.array_equal((Sh != 0)[~band], (ref != 0)[~band])
        assert nnz == int(np.count_nonzero(Sh))
        keep = (Sh != 0) & (ref != 0)
        rt = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}[dtname]
        assert np.allclose(Sh[keep], ref[keep], rtol=rt, atol=rt * np.abs(Dh).max() * 1e-2)
    # recovered foreground: the planted support, at a threshold between the
    # residual's noise level and the smallest planted outliers
    if dtname == "f64":
        S, nnz = ctx.sparse_full(1e-6 * p.Lmax)
        Sh = S.cpu().numpy().reshape(-1)
        truth = np.zeros(n * n, bool)
        truth[p.support] = np.abs(p.values) > 1e-6 * p.Lmax
        assert np.array_equal(Sh != 0, truth)
    ctx.close()


@pytest.mark.parametrize("dtname", ["f64", "f32", "bf16"])
def test_sparse_full_strided_and_ragged(dtname):
    """Rows of D and S with a padded stride (16-byte aligned rows, a last
    vector of the row cut short: the vector kernel with its ragged tail) and
    with an unpadded odd stride (rows off 16-byte boundaries: the per-element
    kernel); both against the threshold of D - A_k B_k."""
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import IRCUR
    dtype = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtname]
    n1, n2, ld, r = 300, 1003, 1008, 4
    p = synth.planted(n1, n2, r, 0.1, seed=21)
    print(f"case sparse_full strided {dtname} n1={n1} n2={n2} ld={ld}", flush=True)
    big = torch.zeros((n1, ld), dtype=torch.float64, device="cuda")
    big[:, :n2] = torch.tensor(p.D, dtype=torch.float64, device="cuda")
    Dpad = big.to(dtype)[:, :n2]
    assert Dpad.stride(0) == ld
    ctx = IRCUR(Dpad, r, 60, 60, p.Lmax, gamma=0.7, eps=0.0, max_iter=12, seed=3, resample=True)
    ctx.solve()
    A, B = factors_np(ctx)
    Dh = Dpad.double().cpu().numpy()
    X = Dh - A @ B
    z = 1e-3 * p.Lmax
    ref = O.hard_threshold(X, z)
    band = np.abs(np.abs(X) - z) <= (1e-12 if dtname == "f64" else 1e-4) * np.abs(Dh).max()
    rt = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}[dtname]
    Spad = torch.full((n1, ld), 7.0, dtype=dtype, device="cuda")
    for out in (Spad[:, :n2], None):
        S, nnz = ctx.sparse_full(z, out=out)
        Sh = S.double().cpu().numpy()
        assert np.array_equal((Sh != 0)[~band], (ref != 0)[~band])
        assert nnz == int(np.count_nonzero(Sh))
        keep = (Sh != 0) & (ref != 0)
        assert np.allclose(Sh[keep], ref[keep], rtol=rt, atol=rt * np.abs(Dh).max() * 1e-2)
    # the padding columns of the output rows are left untouched
    assert bool((Spad[:, n2:] == 7.0).all())
    # timed relaunches (no count) rewrite the same values
    S0 = Spad[:, :n2].clone()
    us = ctx.time_sparse(Spad[:, :n2], z, reps=3)
    assert us > 0.0
    assert torch.equal(Spad[:, :n2], S0)
    ctx.close()


@pytest.mark.parametrize("dtname", ["f64", "f32"])
def test_to_svd_matches_dense_svd(dtname):
    torch = require_gpu()
    dtype = {"f64": torch.float64, "f32": torch.float32}[dtname]
    n1, n2, r = 900, 700, 6
    p = synth.planted(n1, n2, r, 0.1, seed=5)
    print(f"case to_svd {dtname}", flush=True)
    ctx, _ = _run(torch, p, r, 100, 100, 30, dtype)
    A, B = factors_np(ctx)
    W, sig, V = (t.cpu().numpy() for t in ctx.to_svd())
    L = A @ B
    s_ref = np.linalg.svd(L, compute_uv=False)[:r]
    assert np.allclose(sig, s_ref, rtol=1e-12, atol=0)
    assert np.all(np.diff(sig) <= 0)
    assert np.allclose(W.T @ W, np.eye(r), atol=1e-13)
    assert np.allclose(V.T @ V, np.eye(r), atol=1e-13)
    assert _rel((W * sig) @ V.T, L) <= 1e-13
    ctx.close()


def test_to_svd_rank_deficient_estimate():
    """Exact rank 2 with r = 4: the pinv rule drops two directions, and
    Algorithm 2 returns two zero singular values with zero vectors."""
    torch = require_gpu()
    D, Wt, Vt = synth.exact_lowrank(400, 350, 2, seed=2)
    from paper_2010_07422_amd.ircur import IRCUR
    ctx = IRCUR(to_dev(torch, D, torch.float64), 4, 60, 60, float(np.abs(D).max()), eps=-1.0, max_iter=3)
    ctx.solve()
    W, sig, V = (t.cpu().numpy() for t in ctx.to_svd())
    s_ref = np.linalg.svd(D, compute_uv=False)
    assert np.allclose(sig[:2], s_ref[:2], rtol=1e-12)
    assert np.all(sig[2:] == 0.0)
    assert np.all(W[:, 2:] == 0.0) and np.all(V[:, 2:] == 0.0)
    assert _rel((W * sig) @ V.T, D) <= 1e-12
    ctx.close()
