"""The FGCR cycle with a BF16 basis keeps the preconditioned directions z_k as
the preconditioner made them and projects only their images q_k = M z_k
(classical Gram-Schmidt: b_jk = <qt_j, q_k> / |qt_j|^2, qt_k = q_k - sum_j
b_jk qt_j).  The projected directions zt_k = z_k - sum_j b_jk zt_j are never
formed: with Z = Zt (1 + B), B strictly upper triangular, the cycle's update
sum_k a_k zt_k equals Z c with (1 + B) c = a, solved by back substitution.

This checks that identity, and that the update leaves the residual the cycle
tracked (r - sum_k a_k qt_k = b - M (x + Z c)), in FP64 on random complex
data, with the recurrence written the way the device kernels order it (the
coefficients of step k indexed by j < k, the back substitution from the last
direction).  The transposed triangle gives another update and fails it."""
import numpy as np
import pytest


def _cycle(M, Z, r0):
    """One GCR cycle on the columns of Z: projected images, step coefficients
    (dots[k][j] = <qt_j, q_k>, |qt_j|^2, a_k) as the library keeps them."""
    n, m = Z.shape
    Qt = np.zeros((n, m), complex)
    Zt = np.zeros((n, m), complex)
    dots = np.zeros((m, m), complex)
    nq = np.zeros(m)
    a = np.zeros(m, complex)
    r = r0.copy()
    for k in range(m):
        q = M @ Z[:, k]
        dots[k, :k] = Qt[:, :k].conj().T @ q
        b = dots[k, :k] / nq[:k]
        Qt[:, k] = q - Qt[:, :k] @ b
        Zt[:, k] = Z[:, k] - Zt[:, :k] @ b
        nq[k] = np.vdot(Qt[:, k], Qt[:, k]).real
        a[k] = np.vdot(Qt[:, k], r) / nq[k]
        r = r - a[k] * Qt[:, k]
    return Qt, Zt, dots, nq, a, r


def _raw_coefficients(dots, nq, a):
    """(1 + B) c = a by back substitution, B[k, j] = dots[j][k] / nq[k] (j > k)."""
    m = len(a)
    c = np.zeros(m, complex)
    for k in range(m - 1, -1, -1):
        c[k] = a[k] - sum(dots[j, k] / nq[k] * c[j] for j in range(k + 1, m))
    return c


@pytest.mark.parametrize("m", [1, 2, 5, 16])
def test_raw_direction_combination(m):
    rng = np.random.default_rng(100 + m)
    n = 64
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    Z = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    x0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    bvec = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r0 = bvec - M @ x0
    Qt, Zt, dots, nq, a, r = _cycle(M, Z, r0)
    # the images of the projected directions are the projected images, and
    # they are orthogonal (conjugated dots)
    assert np.abs(M @ Zt - Qt).max() < 1e-10 * np.abs(Qt).max()
    G = Qt.conj().T @ Qt
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-10 * np.abs(G).max()
    c = _raw_coefficients(dots, nq, a)
    upd = Z @ c
    assert np.linalg.norm(upd - Zt @ a) < 1e-12 * np.linalg.norm(Zt @ a)
    # the residual the cycle tracked is the true residual of the combined solution
    assert np.linalg.norm(bvec - M @ (x0 + upd) - r) < 1e-10 * np.linalg.norm(r0)
    if m > 1:
        # the transposed triangle or a forward recurrence give another update
        B = np.zeros((m, m), complex)
        for j in range(m):
            B[:j, j] = dots[j, :j] / nq[:j]
        assert np.linalg.norm(np.linalg.solve(np.eye(m) + B, a) - c) < 1e-12 * np.linalg.norm(c)
        wrong = np.linalg.solve(np.eye(m) + B.T, a)
        assert np.linalg.norm(Z @ wrong - upd) > 1e-3 * np.linalg.norm(upd)
