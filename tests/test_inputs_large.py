"""The device UΣV^T generator above the size where the device QR stops
returning an orthogonal factor builds U and V from half-size Haar blocks and
a permutation.  Checked on the CPU with the threshold lowered: U, V must be
orthogonal and the singular values exactly the requested log-spaced ones."""
import numpy as np

from paper_1401_5522_amd import inputs


def test_block_orthogonal_usv_keeps_the_spectrum(monkeypatch):
    monkeypatch.setattr(inputs, "HAAR_MAX_ELEMENTS", 10)
    N, kappa = 96, 1e4
    A = inputs.usv_torch(N, kappa, seed=(9,), device="cpu").numpy()
    s = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(np.sort(s)[::-1], inputs.sigmas(N, kappa), rtol=1e-12, atol=0)
    # no block structure left: every column has mass in both halves
    h = N // 2
    top = np.linalg.norm(A[:h], axis=0)
    bot = np.linalg.norm(A[h:], axis=0)
    assert (top > 0.05 * np.linalg.norm(A, axis=0)).all() and (bot > 0.05 * np.linalg.norm(A, axis=0)).all()
