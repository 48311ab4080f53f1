"""FP64 CPU oracle of IRCUR, written step by step from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

Notation follows the paper.  D is n1 x n2; L_k is never formed: it is held as
L_k = A_k B_k with A_k (n1 x r) and B_k (r x n2).  With C, U, R the CUR
components of eq. (2) and U^+ = V_r Sigma_r^{-1} W_r^T the pseudo-inverse of
U = H_r([D - S]_{I,J}) = W_r Sigma_r V_r^T, eq. (3) gives

    L_{k+1} = C U^+ R = (C V_r Sigma_r^{-1}) (W_r^T R) =: A_{k+1} B_{k+1},

which is how the final product of Algorithm 1 ("do not compute this step") is
kept without forming an n1 x n2 matrix.  Every matrix op here is a plain NumPy
/ LAPACK call in float64.

Readings of the paper where it is silent or ambiguous (each is also listed in the
design notes of the repository):

* zeta schedule: Algorithm 1 sets zeta_{k+1} = gamma^k zeta_0, so the first
  iteration (k = 0) thresholds at zeta_0 itself.
* T_zeta keeps X_ij only when |X_ij| > zeta (strict, eq. (4)).
* The I x J block is written twice by Phase I (column pass and row pass); in
  exact arithmetic both agree.  Here M = R[:, J] (the row side).
* H_r is the truncated SVD; U^+ is Moore-Penrose: sigma_i (i <= r) is inverted
  only if sigma_i > max(|I|, |J|) * 2^-52 * sigma_1, otherwise that component
  is dropped (its column of A and row of B are zero).  M = 0 gives U^+ = 0.
* e_k (eq. (6)) is read literally ("R1"): the residual of L_{k+1} and S_{k+1}
  on the iteration's own I and J.  err_mode = 1 ("R2") instead uses the
  below-threshold part of D - L_k on the new I, J, i.e. [D - L_k - S_{k+1}].
* e_0 = 1, so at least one iteration runs.  A zero denominator gives e = 0.
* IRCUR-R evaluates L_k on newly drawn rows and columns through its factors,
  A_k[I_new, :] B_k and A_k B_k[:, J_new].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import sampler

EPS64 = 2.0 ** -52


# --------------------------------------------------------------------------
# Basic operators
# --------------------------------------------------------------------------

def hard_threshold(X: np.ndarray, zeta: float) -> np.ndarray:
    """T_zeta of eq. (4), section 3.2: keep X_ij where |X_ij| > zeta, else 0."""
    return np.where(np.abs(X) > zeta, X, 0.0)


def sample_size(c: float, r: int, n: int) -> int:
    """|I| = ceil(c r log n) (section 3.5, natural log)."""
    return int(math.ceil(c * r * math.log(n)))


def zeta_at(k: int, zeta0: float, gamma: float, sched=None) -> float:
    """zeta_{k+1} = gamma^k zeta_0 (Algorithm 1, Phase I); sched[k] overrides."""
    if sched is not None:
        return float(sched[k])
    return float(zeta0 * gamma ** k)


def truncated_svd_pinv(M: np.ndarray, r: int):
    """H_r of M by LAPACK SVD and the pseudo-inverse rule (section 3.1).

    Returns (W_r, sigma_r, V_r, keep) with W_r (|I| x r), V_r (|J| x r);
    columns of dropped components are set to zero and keep[i] is False.
    """
    W, s, Vt = np.linalg.svd(M, full_matrices=False)
    r_eff = min(r, s.size)
    Wr = np.zeros((M.shape[0], r))
    Vr = np.zeros((M.shape[1], r))
    sr = np.zeros(r)
    keep = np.zeros(r, dtype=bool)
    if s.size == 0:
        return Wr, sr, Vr, keep
    tol = max(M.shape) * EPS64 * s[0]
    for i in range(r_eff):
        if s[i] > tol:
            keep[i] = True
            Wr[:, i] = W[:, i]
            Vr[:, i] = Vt[i, :]
            sr[i] = s[i]
    return Wr, sr, Vr, keep


# --------------------------------------------------------------------------
# One iteration of Algorithm 1 (factored form)
# --------------------------------------------------------------------------

def step(D, A, B, I, J, zeta, r, err_mode=0):
    """Iteration k -> k+1 of Algorithm 1 on row set I and column set J.

    D: (n1, n2) float64.  A: (n1, r), B: (r, n2) factors of L_k = A B.
    Returns a dict with the new factors A1, B1 (L_{k+1} = A1 B1), the CUR
    pieces C, R, M (= [D - S_{k+1}]_{I,J}), the SVD (W_r, sigma, V_r, keep),
    the sparse blocks S_I = [S_{k+1}]_{I,:}, S_J = [S_{k+1}]_{:,J}, their masks,
    and e (eq. (6)).
    """
    D = np.asarray(D, dtype=np.float64)
    I = np.asarray(I)
    J = np.asarray(J)
    # Phase I: sampled rows and columns of L_k (eq. (5)), then T_zeta (eq. (4)).
    L_I = A[I, :] @ B                 # [L_k]_{I,:}
    L_J = A @ B[:, J]                 # [L_k]_{:,J}
    X_I = D[I, :] - L_I
    X_J = D[:, J] - L_J
    S_I = hard_threshold(X_I, zeta)   # [S_{k+1}]_{I,:}
    S_J = hard_threshold(X_J, zeta)   # [S_{k+1}]_{:,J}
    # Phase II: CUR components (eq. (2)).
    R = D[I, :] - S_I                 # R_{k+1} = [D - S_{k+1}]_{I,:}
    C = D[:, J] - S_J                 # C_{k+1} = [D - S_{k+1}]_{:,J}
    M = R[:, J]                       # [D - S_{k+1}]_{I,J}
    Wr, sr, Vr, keep = truncated_svd_pinv(M, r)
    inv = np.where(keep, 1.0 / np.where(keep, sr, 1.0), 0.0)
    # L_{k+1} = C U^+ R with U^+ = V_r Sigma_r^+ W_r^T (eq. (3)), kept factored.
    A1 = (C @ Vr) * inv[None, :]
    B1 = Wr.T @ R
    # Stopping criterion, eq. (6).
    den = np.linalg.norm(D[I, :]) + np.linalg.norm(D[:, J])
    if err_mode == 0:
        num = (np.linalg.norm(R - A1[I, :] @ B1)
               + np.linalg.norm(C - A1 @ B1[:, J]))
    elif err_mode == 1:
        num = np.linalg.norm(X_I - S_I) + np.linalg.norm(X_J - S_J)
    else:
        raise ValueError("err_mode must be 0 or 1")
    e = 0.0 if den == 0.0 else float(num / den)
    return dict(A1=A1, B1=B1, C=C, R=R, M=M, W_r=Wr, sigma=sr, V_r=Vr,
                keep=keep, S_I=S_I, S_J=S_J, mask_I=np.abs(X_I) > zeta,
                mask_J=np.abs(X_J) > zeta, X_I=X_I, X_J=X_J, e=e,
                den=float(den), num=float(num))


# --------------------------------------------------------------------------
# Algorithm 1 driver
# --------------------------------------------------------------------------

@dataclass
class Result:
    A: np.ndarray
    B: np.ndarray
    k: int
    e_hist: list
    I: np.ndarray | None = None
    J: np.ndarray | None = None
    last: dict | None = None
    IJ_hist: list = field(default_factory=list)
    state_hist: list = field(default_factory=list)


def ircur(D, r, sI, sJ, zeta0, gamma, eps, max_iter, seed=0, resample=True,
          err_mode=0, IJ=None, zeta_sched=None, init=None, k0=0,
          keep_states=False):
    """Algorithm 1 (IRCUR) in FP64.

    IJ: optional callable k -> (I, J) or list of (I, J) overriding the sampler
    (the GPU parity tests feed both sides the same sets).  init=(A, B, k0)
    resumes from a checkpoint taken after k0 iterations.
    """
    D = np.asarray(D, dtype=np.float64)
    n1, n2 = D.shape
    if init is None:
        A = np.zeros((n1, r))                  # L_0 = 0
        B = np.zeros((r, n2))
        k = 0
    else:
        A, B = np.array(init[0], dtype=np.float64), np.array(init[1], dtype=np.float64)
        k = k0
    e = 1.0                                    # e_0 := 1
    res = Result(A=A, B=B, k=k, e_hist=[])
    while e > eps and k < max_iter:
        if IJ is None:
            I, J = sampler.draw_IJ(seed, sampler.stream_id(k, resample), n1, n2, sI, sJ)
        elif callable(IJ):
            I, J = IJ(k)
        else:
            I, J = IJ[k]
        zeta = zeta_at(k, zeta0, gamma, zeta_sched)
        out = step(D, A, B, I, J, zeta, r, err_mode)
        A, B, e = out["A1"], out["B1"], out["e"]
        k += 1
        res.e_hist.append(e)
        res.IJ_hist.append((np.asarray(I), np.asarray(J)))
        res.last = out
        if keep_states:
            res.state_hist.append((A.copy(), B.copy()))
    res.A, res.B, res.k = A, B, k
    if res.last is not None:
        res.I, res.J = res.IJ_hist[-1]
    return res


def cur_components(D, A_prev, B_prev, I, J, zeta, r):
    """Output of Algorithm 1: C_k, U_k^+ and R_k of the last iteration.

    Recomputed from the factors entering that iteration; U^+ = V_r Sigma_r^+ W_r^T.
    """
    out = step(D, A_prev, B_prev, I, J, zeta, r)
    inv = np.where(out["keep"], 1.0 / np.where(out["keep"], out["sigma"], 1.0), 0.0)
    Upinv = (out["V_r"] * inv[None, :]) @ out["W_r"].T
    return out["C"], Upinv, out["R"], out["S_I"], out["S_J"]


# --------------------------------------------------------------------------
# Literal dense form (tiny inputs only)
# --------------------------------------------------------------------------

def ircur_dense(D, r, zeta0, gamma, IJ, iters):
    """Algorithm 1 with L_{k+1} = C U^+ R formed as a full matrix every step.

    Thresholds the full D - L_k and restricts to the sampled blocks afterwards;
    U^+ is numpy's pinv of H_r([D - S]_{I,J}).  For n <= 64 only.
    """
    D = np.asarray(D, dtype=np.float64)
    L = np.zeros_like(D)
    Ls, es = [], []
    for k in range(iters):
        I, J = IJ[k]
        zeta = zeta0 * gamma ** k
        T = hard_threshold(D - L, zeta)          # T_zeta[D - L_k], full
        S = np.zeros_like(D)
        S[:, J] = T[:, J]
        S[I, :] = T[I, :]
        C = (D - S)[:, J]
        R = (D - S)[I, :]
        Mw, Ms, Mvt = np.linalg.svd((D - S)[np.ix_(I, J)], full_matrices=False)
        U = (Mw[:, :r] * Ms[:r]) @ Mvt[:r, :]    # H_r
        L = C @ np.linalg.pinv(U) @ R
        E = D - L - S
        es.append((np.linalg.norm(E[I, :]) + np.linalg.norm(E[:, J]))
                  / (np.linalg.norm(D[I, :]) + np.linalg.norm(D[:, J])))
        Ls.append(L.copy())
    return Ls, es


# --------------------------------------------------------------------------
# Algorithm 2: CUR to SVD
# --------------------------------------------------------------------------

def cur_to_svd(C, Upinv, R):
    """Algorithm 2: two thin QRs and an SVD of the small middle factor.

    Returns W, Sigma (vector), V with C U^+ R = W diag(Sigma) V^T.
    """
    Qc, Rc = np.linalg.qr(C)
    Qr, Rr = np.linalg.qr(R.T)
    Wu, s, Vut = np.linalg.svd(Rc @ Upinv @ Rr.T)
    return Qc @ Wu, s, Qr @ Vut.T


def factors_to_svd(A, B):
    """Algorithm 2 applied to the factored estimate L = A B.

    Here C U^+ = A (n1 x r) and R is replaced by the r x n2 factor B, so the
    middle factor is R_A R_B^T (r x r) and both QRs are n x r.
    """
    Qa, Ra = np.linalg.qr(A)
    Qb, Rb = np.linalg.qr(B.T)
    Wu, s, Vut = np.linalg.svd(Ra @ Rb.T)
    return Qa @ Wu, s, Qb @ Vut.T


# --------------------------------------------------------------------------
# Error metric between two factored estimates
# --------------------------------------------------------------------------

def factored_rel_diff(A1, B1, A0, B0):
    """||A1 B1 - A0 B0||_F / ||A0 B0||_F without forming n1 x n2 matrices.

    A1 B1 - A0 B0 = [A1, -A0] [B1; B0]; with thin QRs P = Q_a R_a and
    Q^T = Q_b R_b^T the Frobenius norm equals ||R_a R_b^T||_F.
    """
    Pa = np.hstack([A1, -A0])
    Pb = np.vstack([B1, B0]).T
    _, Ra = np.linalg.qr(Pa)
    _, Rb = np.linalg.qr(Pb)
    num = np.linalg.norm(Ra @ Rb.T)
    _, Ra0 = np.linalg.qr(A0)
    _, Rb0 = np.linalg.qr(B0.T)
    den = np.linalg.norm(Ra0 @ Rb0.T)
    return float(num / den) if den > 0 else float(num)
