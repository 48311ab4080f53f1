"""Unrolled K-step IRCUR with learnable thresholds, and its reverse-mode
adjoint, in FP64 NumPy.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.

The paper defines IRCUR with the hard threshold T_zeta of eq. (4) and the
geometric schedule of Algorithm 1; it does not define a differentiable form.
This module runs the same K iterations (Phase I, then Phase II, factored as in
``ircur.step``) with these readings:

* one learnable threshold zeta_k per iteration (k = 0 .. K-1; iteration k+1 of
  Algorithm 1 uses zeta_k);
* the hard threshold x * 1[|x| > zeta] is replaced by the gate
      S(x) = x g,   g = sigmoid((|x| - zeta) / (tau_rel zeta)),
  which tends to eq. (4) as tau_rel -> 0; tau_rel = 0 is eq. (4) exactly;
* per instance, loss = ||A_K B_K - L*||_F / ||L*||_F, summed over the batch;
* the index sets are fixed inputs (recorded draws), so the loss is a function
  of (zeta_0 .. zeta_{K-1}) and D only.

The adjoint is the chain rule through each step, written out:

  A_{k+1} = C T,  T = V_r Sigma_r^-1        B_{k+1} = W_r^T R
  C = D[:, J] - S(X_J), X_J = D[:, J] - A_k B_k[:, J]
  R = D[I, :] - S(X_I), X_I = D[I, :] - A_k[I, :] B_k,  M = R[:, J]
  (W, Sigma, V) = full SVD of M.

For the SVD it uses the first-order perturbation of the singular triplets
(textbook; e.g. Townsend, "Differentiating the singular value decomposition",
2016): with E = W^T dM V,
  d sigma_i = E_ii,
  d w_i = sum_{j != i} w_j (sigma_i E_ji + sigma_j E_ij) / (sigma_i^2 - sigma_j^2),
  d v_i = sum_{j != i} v_j (sigma_i E_ij + sigma_j E_ji) / (sigma_i^2 - sigma_j^2),
where j runs over the full bases (sigma_j = 0 and the missing entry of E taken
as 0 beyond min(|I|, |J|)).  This needs distinct leading singular values and
sigma_r > sigma_{r+1}; the routines report the gap.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EPS64 = 2.0 ** -52


# --------------------------------------------------------------------------
# Gate
# --------------------------------------------------------------------------

def _sigmoid(u):
    out = np.empty_like(u)
    pos = u >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-u[pos]))
    e = np.exp(u[~pos])
    out[~pos] = e / (1.0 + e)
    return out


def gate(X, zeta, tau_rel):
    """g, dS/dx and dS/dzeta for S = x g(x; zeta).

    tau_rel = 0: g = 1[|x| > zeta] (eq. (4)), dS/dx = g, dS/dzeta = 0.
    """
    ax = np.abs(X)
    if tau_rel == 0.0:
        g = (ax > zeta).astype(np.float64)
        return g, g.copy(), np.zeros_like(X)
    t = tau_rel * zeta
    g = _sigmoid((ax - zeta) / t)
    gg = g * (1.0 - g)
    dSdx = g + ax * gg / t
    # u = (|x| - zeta) / (tau_rel zeta) = |x| / (tau_rel zeta) - 1 / tau_rel
    dSdz = -X * ax * gg / (tau_rel * zeta * zeta)
    return g, dSdx, dSdz


# --------------------------------------------------------------------------
# Forward with a tape
# --------------------------------------------------------------------------

@dataclass
class Tape:
    D: np.ndarray
    r: int
    tau_rel: float
    IJ: list
    zetas: np.ndarray
    A: list = field(default_factory=list)     # A_0 .. A_K   (n1 x r)
    B: list = field(default_factory=list)     # B_0 .. B_K   (r x n2)
    svd: list = field(default_factory=list)   # per step: (W full, s, V full)
    gaps: list = field(default_factory=list)  # sigma_{r+1} / sigma_r per step


def _step(D, A, B, I, J, zeta, r, tau_rel):
    XI = D[I, :] - A[I, :] @ B
    gI, _, _ = gate(XI, zeta, tau_rel)
    R = D[I, :] - XI * gI
    XJ = D[:, J] - A @ B[:, J]
    gJ, _, _ = gate(XJ, zeta, tau_rel)
    C = D[:, J] - XJ * gJ
    M = R[:, J]
    W, s, Vt = np.linalg.svd(M, full_matrices=True)
    V = Vt.T
    if s[r - 1] <= max(M.shape) * EPS64 * s[0]:
        raise ValueError("core of rank < r: the unrolled adjoint needs sigma_r > 0")
    T = V[:, :r] / s[:r]
    A1 = C @ T
    B1 = W[:, :r].T @ R
    gap = s[r] / s[r - 1] if len(s) > r else 0.0
    return A1, B1, (W, s, V), gap


def forward(D, IJ, zetas, r, tau_rel, A0=None, B0=None):
    """K = len(zetas) unrolled iterations from (A0, B0) (default L_0 = 0)."""
    D = np.asarray(D, dtype=np.float64)
    n1, n2 = D.shape
    A = np.zeros((n1, r)) if A0 is None else np.asarray(A0, np.float64)
    B = np.zeros((r, n2)) if B0 is None else np.asarray(B0, np.float64)
    tape = Tape(D=D, r=r, tau_rel=float(tau_rel), IJ=list(IJ), zetas=np.asarray(zetas, np.float64))
    tape.A.append(A)
    tape.B.append(B)
    for k, zeta in enumerate(tape.zetas):
        I, J = IJ[k]
        A, B, svd, gap = _step(D, A, B, I, J, zeta, r, tau_rel)
        tape.A.append(A)
        tape.B.append(B)
        tape.svd.append(svd)
        tape.gaps.append(gap)
    return tape


def loss(A, B, Wstar, Vstar):
    """||A B - W* V*^T||_F / ||W* V*^T||_F (dense; the definition)."""
    Ls = Wstar @ Vstar.T
    return float(np.linalg.norm(A @ B - Ls) / np.linalg.norm(Ls))


def loss_adjoint(A, B, Wstar, Vstar):
    """d loss / dA, d loss / dB."""
    Ls = Wstar @ Vstar.T
    E = A @ B - Ls
    ne, nl = np.linalg.norm(E), np.linalg.norm(Ls)
    G = E / (ne * nl)
    return G @ B.T, A.T @ G


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------

def svd_adjoint(W, s, V, r, Wbar_r, Vbar_r, sbar_r):
    """M_bar from the adjoints of the top-r triplets (W_r, sigma_r, V_r).

    W: sI x sI, V: sJ x sJ full orthogonal bases, s: min(sI, sJ) values.
    """
    sI, sJ = W.shape[0], V.shape[0]
    m = len(s)
    sig_w = np.zeros(sI)
    sig_w[:m] = s
    sig_v = np.zeros(sJ)
    sig_v[:m] = s
    Eb = np.zeros((sI, sJ))
    aW = W.T @ Wbar_r          # aW[j, i] = w_j . Wbar_i
    aV = V.T @ Vbar_r          # aV[j, i] = v_j . Vbar_i
    for i in range(r):
        si = s[i]
        for j in range(sI):                      # d w_i = sum_j w_j (si E_ji + sj E_ij) / (si^2 - sj^2)
            if j == i:
                continue
            sj = sig_w[j]
            den = si * si - sj * sj
            Eb[j, i] += aW[j, i] * si / den
            if j < sJ:
                Eb[i, j] += aW[j, i] * sj / den
        for j in range(sJ):                      # d v_i = sum_j v_j (si E_ij + sj E_ji) / (si^2 - sj^2)
            if j == i:
                continue
            sj = sig_v[j]
            den = si * si - sj * sj
            Eb[i, j] += aV[j, i] * si / den
            if j < sI:
                Eb[j, i] += aV[j, i] * sj / den
        Eb[i, i] += sbar_r[i]
    return W @ Eb @ V.T


@dataclass
class Grads:
    zeta: np.ndarray            # d loss / d zeta_k
    D: np.ndarray | None        # d loss / dD (if requested)
    A0: np.ndarray
    B0: np.ndarray


def backward(tape: Tape, Abar, Bbar, want_D=False):
    """Reverse sweep from (d loss/dA_K, d loss/dB_K)."""
    D, r, tau = tape.D, tape.r, tape.tau_rel
    K = len(tape.zetas)
    dz = np.zeros(K)
    dD = np.zeros_like(D) if want_D else None
    for k in range(K - 1, -1, -1):
        A, B = tape.A[k], tape.B[k]
        I, J = tape.IJ[k]
        zeta = tape.zetas[k]
        W, s, V = tape.svd[k]
        # recompute the gathered slices of this step
        XI = D[I, :] - A[I, :] @ B
        gI, dSI, dzI = gate(XI, zeta, tau)
        R = D[I, :] - XI * gI
        XJ = D[:, J] - A @ B[:, J]
        gJ, dSJ, dzJ = gate(XJ, zeta, tau)
        C = D[:, J] - XJ * gJ
        Wr, Vr, sr = W[:, :r], V[:, :r], s[:r]
        T = Vr / sr
        # A_{k+1} = C T,  B_{k+1} = W_r^T R
        Cb = Abar @ T.T
        Tb = C.T @ Abar
        Rb = Wr @ Bbar
        Wb = R @ Bbar.T
        # T = V_r Sigma^-1
        Vb = Tb / sr
        sb = -np.sum(Tb * Vr, axis=0) / (sr * sr)
        Mb = svd_adjoint(W, s, V, r, Wb, Vb, sb)
        # M = R[:, J]
        Rb = Rb.copy()
        Rb[:, J] += Mb
        # R = D_I - S(X_I),  C = D_J - S(X_J)
        XIb = -Rb * dSI
        XJb = -Cb * dSJ
        dz[k] = -np.sum(Rb * dzI) - np.sum(Cb * dzJ)
        if want_D:
            dD[I, :] += Rb + XIb
            dD[:, J] += Cb + XJb
        # X_I = D_I - A[I, :] B,  X_J = D_J - A B[:, J]
        Abar_new = np.zeros_like(A)
        Bbar_new = np.zeros_like(B)
        Abar_new[I, :] -= XIb @ B.T
        Bbar_new -= A[I, :].T @ XIb
        Abar_new -= XJb @ B[:, J].T
        Bbar_new[:, J] -= A.T @ XJb
        Abar, Bbar = Abar_new, Bbar_new
    return Grads(zeta=dz, D=dD, A0=Abar, B0=Bbar)


def loss_and_grad(D, IJ, zetas, r, tau_rel, Wstar, Vstar, want_D=False):
    """One instance: loss and its gradients (zeta, optionally D)."""
    tape = forward(D, IJ, zetas, r, tau_rel)
    A, B = tape.A[-1], tape.B[-1]
    ell = loss(A, B, Wstar, Vstar)
    Ab, Bb = loss_adjoint(A, B, Wstar, Vstar)
    g = backward(tape, Ab, Bb, want_D=want_D)
    return ell, g, tape
