"""The device-side planted generator (drawn here with torch on the CPU)
follows the planted recipe: rank-r L = W V^T, exactly round(alpha n1 n2)
outliers, values within +-10 mean|L|, and a seed that fixes the draw."""
import numpy as np
import pytest

from paper_2010_07422_amd import synth


@pytest.mark.parametrize("n1,n2,r,alpha", [(300, 200, 3, 0.1), (128, 257, 5, 0.3), (64, 64, 2, 0.0)])
def test_planted_device_recipe(n1, n2, r, alpha):
    torch = pytest.importorskip("torch")
    p = synth.planted_device(n1, n2, r, alpha, seed=9, device="cpu")
    L = (p.W @ p.V.T).numpy()
    D = p.D.numpy()
    S = D - L
    nz = np.abs(S) > 1e-9 * np.abs(L).max()
    assert nz.sum() == round(alpha * n1 * n2) == p.nnz
    assert np.abs(S).max() <= 10.0 * p.mean_abs * (1 + 1e-12)
    assert abs(p.mean_abs - np.abs(L).mean()) <= 1e-12 * p.mean_abs
    assert abs(p.Lmax - np.abs(L).max()) <= 1e-12 * p.Lmax
    assert np.linalg.matrix_rank(L) == r
    q = synth.planted_device(n1, n2, r, alpha, seed=9, device="cpu")
    assert torch.equal(p.D, q.D)


def test_planted_device_bf16_storage():
    torch = pytest.importorskip("torch")
    p = synth.planted_device(100, 90, 2, 0.2, seed=4, device="cpu", dtype=torch.bfloat16)
    q = synth.planted_device(100, 90, 2, 0.2, seed=4, device="cpu")
    assert p.D.dtype == torch.bfloat16
    assert torch.equal(p.D, q.D.to(torch.bfloat16))
