"""Pins of the unrolled-IRCUR oracle (CPU, FP64).

- G1: with tau_rel = 0 the unrolled forward is plain IRCUR over K steps.
- G2: the adjoint in zeta_k agrees with central finite differences (gated).
- G4: the adjoint in D agrees with directional finite differences (hard mask,
  with draws whose masks flip between the +h and -h runs rejected; and gated).
- The SVD adjoint alone agrees with finite differences of
  <G, pinv(H_r(M))> computed by LAPACK's pinv, for tall and wide cores.
"""
import numpy as np
import pytest

from oracle import ircur as O
from oracle import sampler
from oracle import unrolled as U
from paper_2010_07422_amd import synth


def _instance(n=200, r=5, alpha=0.1, K=10, seed=4, index_seed=9):
    p = synth.planted(n, n, r, alpha, seed=seed)
    s = synth.sample_size(4, r, n)
    IJ = [sampler.draw_IJ(index_seed, k, n, n, s, s) for k in range(K)]
    zetas = p.Lmax * 0.7 ** np.arange(K)
    return p, IJ, zetas, r


def test_G1_hard_gate_equals_plain_ircur():
    p, IJ, zetas, r = _instance()
    tape = U.forward(p.D, IJ, zetas, r, 0.0)
    ref = O.ircur(p.D, r, len(IJ[0][0]), len(IJ[0][1]), zetas[0], 0.7, -1.0, len(zetas), IJ=IJ,
                  zeta_sched=zetas, keep_states=True)
    for k in range(len(zetas)):
        Ao, Bo = ref.state_hist[k]
        d = O.factored_rel_diff(tape.A[k + 1], tape.B[k + 1], Ao, Bo)
        assert d <= 1e-12, (k, d)


def test_G2_zeta_gradient_matches_central_differences():
    p, IJ, zetas, r = _instance()
    tau = 0.05
    ell, g, tape = U.loss_and_grad(p.D, IJ, zetas, r, tau, p.W, p.V)
    assert min(tape.gaps) < 1.0
    fd = np.zeros_like(zetas)
    for k in range(len(zetas)):
        h = 1e-5 * zetas[k]
        zp, zm = zetas.copy(), zetas.copy()
        zp[k] += h
        zm[k] -= h
        lp = U.loss(*_final(p, IJ, zp, r, tau), p.W, p.V)
        lm = U.loss(*_final(p, IJ, zm, r, tau), p.W, p.V)
        fd[k] = (lp - lm) / (zp[k] - zm[k])
    err = np.abs(fd - g.zeta) / np.abs(g.zeta).max()
    assert np.abs(g.zeta).max() > 0
    assert err.max() <= 1e-6, (fd, g.zeta)


def _final(p, IJ, zetas, r, tau):
    t = U.forward(p.D, IJ, zetas, r, tau)
    return t.A[-1], t.B[-1]


def _masks(p, IJ, zetas, r, D):
    t = U.forward(D, IJ, zetas, r, 0.0)
    out = []
    for k, (I, J) in enumerate(IJ):
        A, B = t.A[k], t.B[k]
        out.append(np.abs(D[I, :] - A[I, :] @ B) > zetas[k])
        out.append(np.abs(D[:, J] - A @ B[:, J]) > zetas[k])
    return out, t


@pytest.mark.parametrize("tau", [0.0, 0.05])
def test_G4_D_gradient_matches_directional_differences(tau):
    p, IJ, zetas, r = _instance(K=6)
    zetas = 1.01 * zetas      # zeta_0 = max|L| is attained exactly by an uncorrupted entry
    ell, g, tape = U.loss_and_grad(p.D, IJ, zetas, r, tau, p.W, p.V, want_D=True)
    rng = np.random.default_rng(1)
    checked = 0
    for trial in range(6):
        Dir = rng.standard_normal(p.D.shape)
        h = 1e-7
        Dp, Dm = p.D + h * Dir, p.D - h * Dir
        if tau == 0.0:
            mp, _ = _masks(p, IJ, zetas, r, Dp)
            mm, _ = _masks(p, IJ, zetas, r, Dm)
            if any(not np.array_equal(a, b) for a, b in zip(mp, mm)):
                continue                         # a mask flips inside [-h, h]: derivative undefined
        lp = U.loss(*_final_D(Dp, IJ, zetas, r, tau), p.W, p.V)
        lm = U.loss(*_final_D(Dm, IJ, zetas, r, tau), p.W, p.V)
        fd = (lp - lm) / (2 * h)
        ad = float(np.sum(g.D * Dir))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
        checked += 1
    assert checked >= 3


def _final_D(D, IJ, zetas, r, tau):
    t = U.forward(D, IJ, zetas, r, tau)
    return t.A[-1], t.B[-1]


@pytest.mark.parametrize("sI,sJ,r", [(9, 7, 3), (6, 8, 2), (7, 7, 4)])
def test_svd_adjoint_matches_pinv_differences(sI, sJ, r):
    rng = np.random.default_rng(sI * 100 + sJ)
    M = rng.standard_normal((sI, sJ))
    G = rng.standard_normal((sJ, sI))

    def f(Mx):
        Wf, sf, Vtf = np.linalg.svd(Mx, full_matrices=False)
        Hr = (Wf[:, :r] * sf[:r]) @ Vtf[:r, :]
        return float(np.sum(G * np.linalg.pinv(Hr, rcond=1e-12)))

    W, s, Vt = np.linalg.svd(M, full_matrices=True)
    V = Vt.T
    Wr, Vr, sr = W[:, :r], V[:, :r], s[:r]
    T = Vr / sr                       # U^+ = T W_r^T
    Tb = G @ Wr
    Wb = G.T @ T
    Vb = Tb / sr
    sb = -np.sum(Tb * Vr, axis=0) / (sr * sr)
    Mb = U.svd_adjoint(W, s, V, r, Wb, Vb, sb)
    for trial in range(3):
        Dir = rng.standard_normal(M.shape)
        h = 1e-6
        fd = (f(M + h * Dir) - f(M - h * Dir)) / (2 * h)
        ad = float(np.sum(Mb * Dir))
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3), (fd, ad)


def test_gate_limits():
    x = np.array([-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 3.0])
    g, dS, dz = U.gate(x, 1.0, 0.0)
    assert np.array_equal(g, [1, 0, 0, 0, 0, 0, 1])
    g, dS, dz = U.gate(x, 1.0, 1e-9)
    assert np.allclose(g[[0, 2, 3, 4, 6]], [1, 0, 0, 0, 1])
    g, dS, dz = U.gate(np.array([1.0]), 1.0, 0.05)
    assert g[0] == 0.5
