"""GPU parity of the unrolled, differentiable mode against the FP64 oracle.

- forward: per-instance losses and final factors equal the oracle's
  (hard threshold, tau_rel = 0, and gated) on a ragged batch;
- backward: d loss / d zeta_k equals the oracle's adjoint (G3: <= 1e-9 in
  FP64, <= 1e-4 in FP32);
- G2 on the device: central finite differences of the GPU forward in zeta_k
  agree with the GPU adjoint at n = 200 (FP64, gated);
- the torch.autograd.Function wrapper returns the same gradient.
"""
import numpy as np
import pytest

from oracle import ircur as O
from oracle import sampler
from oracle import unrolled as U
from paper_2010_07422_amd import synth
from tests.gpu_util import require_gpu, to_dev, factors_np

pytestmark = pytest.mark.gpu


def _batch(ns=(200, 257, 300), r=5, alpha=0.1, seed0=11):
    out = []
    for q, n in enumerate(ns):
        p = synth.planted(n, n, r, alpha, seed=seed0 + q)
        s = synth.sample_size(4, r, n)
        out.append((p, s, 100 + q))
    return out


def _gpu_batch(torch, items, r, K, tau, dtype):
    from paper_2010_07422_amd.ircur import IRCURUnrolled
    inst = []
    for p, s, seed in items:
        inst.append((to_dev(torch, p.D, dtype), to_dev(torch, p.W, dtype), to_dev(torch, p.V, dtype), s, s, seed))
    return IRCURUnrolled(inst, r, K, tau_rel=tau)


def _oracle(items, r, zetas, tau, f32=False):
    losses, grads = [], []
    for p, s, seed in items:
        n1, n2 = p.D.shape
        D = p.D.astype(np.float32).astype(np.float64) if f32 else p.D
        W = p.W.astype(np.float32).astype(np.float64) if f32 else p.W
        V = p.V.astype(np.float32).astype(np.float64) if f32 else p.V
        IJ = [sampler.draw_IJ(seed, k, n1, n2, s, s) for k in range(len(zetas))]
        ell, g, tape = U.loss_and_grad(D, IJ, zetas, r, tau, W, V)
        losses.append(ell)
        grads.append(g.zeta)
    return np.array(losses), np.sum(grads, axis=0), tape


@pytest.mark.parametrize("tau", [0.0, 0.05])
def test_forward_matches_oracle_f64(tau):
    torch = require_gpu()
    items = _batch()
    r, K = 5, 6
    zetas = 0.7 ** np.arange(K) * np.mean([p.Lmax for p, _, _ in items])
    print(f"case unrolled forward f64 tau={tau}", flush=True)
    ub = _gpu_batch(torch, items, r, K, tau, torch.float64)
    loss = ub.forward(torch.tensor(zetas)).cpu().numpy()
    ref, _, _ = _oracle(items, r, zetas, tau)
    print("loss", loss, ref, flush=True)
    assert np.allclose(loss, ref, rtol=1e-9, atol=0)
    # final factors of every instance
    for b, (p, s, seed) in enumerate(items):
        n1, n2 = p.D.shape
        IJ = [sampler.draw_IJ(seed, k, n1, n2, s, s) for k in range(K)]
        I0, J0 = ub.sets(b, 0)
        assert np.array_equal(I0, IJ[0][0]) and np.array_equal(J0, IJ[0][1])
        tape = U.forward(p.D, IJ, zetas, r, tau)
        At, B = ub.factors(b, K)
        A = At.cpu().numpy().T
        d = O.factored_rel_diff(A, B.cpu().numpy(), tape.A[-1], tape.B[-1])
        assert d <= 1e-10, (b, d)
    assert not np.any(ub.status() & 16)
    ub.close()


def test_backward_matches_oracle_f64():
    torch = require_gpu()
    items = _batch()
    r, K, tau = 5, 6, 0.05
    zetas = 0.7 ** np.arange(K) * np.mean([p.Lmax for p, _, _ in items])
    print("case unrolled backward f64", flush=True)
    ub = _gpu_batch(torch, items, r, K, tau, torch.float64)
    ub.forward(torch.tensor(zetas))
    dz = ub.backward().cpu().numpy()
    flags = ub.status()
    _, ref, _ = _oracle(items, r, zetas, tau)
    err = np.abs(dz - ref) / np.abs(ref)
    print("dzeta", dz, ref, "per-component rel err", err, "flags", flags, flush=True)
    # every component on its own scale (d zeta_k spans several decades)
    assert np.all(np.abs(dz - ref) <= 1e-9 * np.abs(ref) + 1e-14 * np.abs(ref).max())
    assert not np.any(flags & 1)
    ub.close()


def test_backward_hard_threshold_has_no_zeta_gradient():
    torch = require_gpu()
    items = _batch(ns=(200,))
    r, K = 5, 4
    zetas = 0.7 ** np.arange(K) * items[0][0].Lmax
    ub = _gpu_batch(torch, items, r, K, 0.0, torch.float64)
    ub.forward(torch.tensor(zetas))
    dz = ub.backward().cpu().numpy()
    assert np.all(dz == 0.0)
    ub.close()


def test_G2_central_differences_on_device():
    torch = require_gpu()
    items = _batch(ns=(200,))
    r, K, tau = 5, 8, 0.05
    zetas = 0.7 ** np.arange(K) * items[0][0].Lmax
    print("case unrolled FD n=200", flush=True)
    ub = _gpu_batch(torch, items, r, K, tau, torch.float64)
    ub.forward(torch.tensor(zetas))
    dz = ub.backward().cpu().numpy()
    fd = np.zeros(K)
    floor = np.zeros(K)

    def quotient(k, h):
        zp, zm = zetas.copy(), zetas.copy()
        zp[k] += h
        zm[k] -= h
        lp = float(ub.forward(torch.tensor(zp)).sum())
        l0a = float(ub.forward(torch.tensor(zetas)).sum())
        lm = float(ub.forward(torch.tensor(zm)).sum())
        l0b = float(ub.forward(torch.tensor(zetas)).sum())
        # noise of the difference: each forward's SVDs stop at their tolerance
        # from the subspace the previous forward left, so the loss at the same
        # zeta moves with the warm start; measured as the spread of two
        # evaluations at zeta (after the + and after the - step), plus round-off
        noise = abs(l0a - l0b) + 1e3 * 2.0 ** -52 * (abs(lp) + abs(lm))
        return (lp - lm) / (zp[k] - zm[k]), 2.0 * noise / (zp[k] - zm[k])

    for k in range(K):
        # central differences at h and h/2 combined by Richardson extrapolation
        # (the h^2 term of the truncation error cancels)
        h = 1e-4 * zetas[k]
        d1, n1 = quotient(k, h)
        d2, n2 = quotient(k, 0.5 * h)
        fd[k] = (4.0 * d2 - d1) / 3.0
        floor[k] = (4.0 * n2 + n1) / 3.0
    err = np.abs(fd - dz) / np.abs(dz)
    print("fd", fd, "adjoint", dz, "per-component rel err", err, "floor", floor, flush=True)
    # each component on its own scale: |fd_k - dz_k| <= 1e-6 |dz_k| + round-off floor
    assert np.all(np.abs(fd - dz) <= 1e-6 * np.abs(dz) + floor)
    ub.close()


def test_f32_against_f64_oracle():
    torch = require_gpu()
    items = _batch(ns=(1000, 1500))
    r, K, tau = 5, 10, 0.05
    zetas = 0.7 ** np.arange(K) * np.mean([p.Lmax for p, _, _ in items])
    print("case unrolled f32", flush=True)
    ub = _gpu_batch(torch, items, r, K, tau, torch.float32)
    loss = ub.forward(torch.tensor(zetas)).cpu().numpy()
    dz = ub.backward().cpu().numpy()
    ref_l, ref_g, _ = _oracle(items, r, zetas, tau, f32=True)
    lerr = np.abs(loss - ref_l).max() / np.abs(ref_l).max()
    gerr = np.abs(dz - ref_g) / np.abs(ref_g)
    print("f32 loss err", lerr, "grad per-component rel err", gerr, flush=True)
    assert lerr <= 1e-4
    assert np.all(np.abs(dz - ref_g) <= 1e-4 * np.abs(ref_g) + 1e-6 * np.abs(ref_g).max())
    ub.close()


def test_f32_full_batch_against_f64_oracle():
    """The unrolled workload as the benchmark runs it: 32 planted instances,
    n ~ U{1000..3000}, alpha ~ U[0.1, 0.3], r = 5, |I| = |J| = ceil(20 ln n),
    K = 10, tau_rel = 0.05, FP32 data and factors; every instance's loss and
    the batch's d loss / d zeta against the FP64 oracle on the float-rounded
    data."""
    torch = require_gpu()
    batch = synth.unrolled_batch(nb=32, r=5, seed=7)
    r, K, tau = 5, 10, 0.05
    zetas = 0.7 ** np.arange(K) * float(np.mean([it.inst.Lmax for it in batch]))
    items = [(it.inst, it.s, 1000 + b) for b, it in enumerate(batch)]
    print("case unrolled f32 full batch (32 instances)", flush=True)
    ub = _gpu_batch(torch, items, r, K, tau, torch.float32)
    loss = ub.forward(torch.tensor(zetas)).cpu().numpy()
    dz = ub.backward().cpu().numpy()
    flags = ub.status()
    ub.close()
    ref_l, ref_g, _ = _oracle(items, r, zetas, tau, f32=True)
    lerr = np.abs(loss - ref_l) / np.abs(ref_l)
    gerr = np.abs(dz - ref_g) / np.abs(ref_g)
    print("loss per-instance rel err max", lerr.max(), "grad per-component rel err", gerr, "flags",
          np.bitwise_or.reduce(flags), flush=True)
    assert lerr.max() <= 1e-4
    assert np.all(np.abs(dz - ref_g) <= 1e-4 * np.abs(ref_g) + 1e-6 * np.abs(ref_g).max())
    assert not np.any(flags & 16)


def test_autograd_function():
    torch = require_gpu()
    from paper_2010_07422_amd.ircur import unrolled_loss
    items = _batch(ns=(200, 220))
    r, K, tau = 5, 5, 0.05
    z0 = 0.7 ** np.arange(K) * np.mean([p.Lmax for p, _, _ in items])
    ub = _gpu_batch(torch, items, r, K, tau, torch.float64)
    zeta = torch.tensor(z0, dtype=torch.float32, requires_grad=True)
    loss = unrolled_loss(zeta, ub)
    loss.backward()
    ub2 = _gpu_batch(torch, items, r, K, tau, torch.float64)
    ub2.forward(zeta.detach())
    dz = ub2.backward().cpu().numpy()
    assert np.allclose(zeta.grad.numpy(), dz.astype(np.float32), rtol=1e-6, atol=0)
    ub.close()
    ub2.close()
