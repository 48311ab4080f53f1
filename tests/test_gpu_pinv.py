"""GPU parity of the rank-r pseudo-inverse of the core on graded spectra
(section 3.1: U^+ of H_r, Moore-Penrose).

D is an exact rank-5 matrix L = W diag(sigma) V^T (W, V with orthonormal
columns) whose singular values fall geometrically from 1 to 1/kappa, so the
core M = L[I, J] is graded the same way; with zeta_0 above max|L| nothing is
thresholded and one IRCUR iteration returns C U^+ R = L (Theorem 1).

- kappa = 1e2, 1e4: the GPU iteration equals the oracle's to 1e-10 and both
  reproduce L.
- kappa = 1e6: the Gram matrix Y^T Y of the GPU method has condition 1e12, so
  its sigma_r carries a relative error of order eps kappa^2; the component it
  scales has relative size 1/kappa in L, hence an error of order eps kappa in
  L.  The bound used is 100 eps kappa (2.2e-8).
- sigma_r / sigma_1 = 1e-9: inside the band where the rules differ.  The
  oracle keeps the component (1e-9 > max(|I|,|J|) eps = 2.2e-14); the GPU
  drops it (a Cholesky pivot of Y^T Y at 1e-18 of the largest is below
  max(|I|,|J|) eps: squared singular values under that are not resolved by
  the Gram matrix), warns, and equals the oracle run at rank r - 1 to 1e-10.
"""
import numpy as np
import pytest

from oracle import ircur as O
from oracle import sampler
from tests.gpu_util import require_gpu, to_dev, factors_np

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


def _graded(n1, n2, r, smin, seed):
    rng = np.random.default_rng(seed)
    W, _ = np.linalg.qr(rng.standard_normal((n1, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n2, r)))
    sig = smin ** (np.arange(r) / (r - 1)) * 100.0
    return (W * sig) @ V.T, W * sig, V


def _gpu_step(torch, D, r, s, z0):
    from paper_2010_07422_amd.ircur import IRCUR
    n1, n2 = D.shape
    I, J = sampler.draw_IJ(9, 0, n1, n2, s, s)
    ctx = IRCUR(to_dev(torch, D, torch.float64), r, s, s, z0, eps=-1.0, max_iter=1, seed=9, resample=False)
    ctx.step(I, J)
    A, B = factors_np(ctx)
    info = ctx.info()
    ctx.close()
    return A, B, I, J, info


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_graded_core_matches_oracle(kappa):
    torch = require_gpu()
    n, r, s = 500, 5, 100
    L, Wt, V = _graded(n, n, r, 1.0 / kappa, seed=int(np.log10(kappa)))
    z0 = 1.01 * float(np.abs(L).max())
    print(f"case graded kappa={kappa:g}", flush=True)
    A, B, I, J, info = _gpu_step(torch, L, r, s, z0)
    ref = O.step(L, np.zeros((n, r)), np.zeros((r, n)), I, J, z0, r)
    assert ref["keep"].all() and info.kept == r
    tol = 1e-10 if kappa <= 1e4 else 100 * EPS * kappa
    d_or = O.factored_rel_diff(A, B, ref["A1"], ref["B1"])
    d_tr = O.factored_rel_diff(A, B, Wt, V.T)
    print(f"vs oracle {d_or:.2e}  vs L {d_tr:.2e}  (tol {tol:.1e})", flush=True)
    assert d_or <= tol and d_tr <= tol


def test_core_inside_the_drop_band():
    torch = require_gpu()
    n, r, s = 500, 5, 100
    rng = np.random.default_rng(7)
    W, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    sig = np.array([100.0, 60.0, 30.0, 10.0, 1e-7])          # sigma_r / sigma_1 = 1e-9
    L = (W * sig) @ V.T
    z0 = 1.01 * float(np.abs(L).max())
    print("case graded core inside the drop band", flush=True)
    A, B, I, J, info = _gpu_step(torch, L, r, s, z0)
    ref = O.step(L, np.zeros((n, r)), np.zeros((r, n)), I, J, z0, r)
    ref4 = O.step(L, np.zeros((n, r - 1)), np.zeros((r - 1, n)), I, J, z0, r - 1)
    assert ref["keep"].all()                                 # the oracle keeps sigma_r
    assert info.kept == r - 1                                # the GPU drops it
    d4 = O.factored_rel_diff(A, B, ref4["A1"], ref4["B1"])
    d5 = O.factored_rel_diff(A, B, ref["A1"], ref["B1"])
    print(f"vs oracle at rank r-1 {d4:.2e}, at rank r {d5:.2e}", flush=True)
    assert d4 <= 1e-10
    assert d5 <= 2e-9                                         # the dropped component's size, 1e-9 of L
