"""Small numpy helpers shared by the tests (no operator arithmetic)."""
import numpy as np


def dense_matrix(apply, shape):
    """Dense matrix of a linear map on arrays of ``shape``, built column by column."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = apply(e.reshape(shape)).ravel()
    return M


def coords(L):
    """Integer coordinates (V, 4) of the lexicographic sites n = x + Lx(y + Ly(z + Lz t))."""
    V = int(np.prod(L))
    n = np.arange(V)
    out = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        out[:, mu] = n % L[mu]
        n = n // L[mu]
    return out


def site_index(L, x):
    return x[..., 0] + L[0] * (x[..., 1] + L[1] * (x[..., 2] + L[2] * x[..., 3]))


def neighbour(L, mu, step):
    """Index of x + step*mu for every site."""
    x = coords(L)
    x[:, mu] = (x[:, mu] + step) % L[mu]
    return site_index(L, x)


def gauge_rotate(L, U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^+."""
    out = np.empty_like(U)
    for mu in range(4):
        nf = neighbour(L, mu, +1)
        out[:, mu] = g @ U[:, mu] @ g[nf].conj().transpose(0, 2, 1)
    return out


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def parity_sites(L, p):
    """Lexicographic index of the site with checkerboard index cb = n >> 1 and parity p, for every cb."""
    x = coords(L)
    par = x.sum(axis=1) % 2
    n = np.arange(0, len(par), 2)
    return np.where(par[n] == p, n, n + 1)
