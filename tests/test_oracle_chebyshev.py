"""Pins of the oracle's Chebyshev filter (the recursively generated filter
functions for multigrid subspace set-up, Sec. 2.4).

The oracle runs the three-term recurrence with its matrix-free Mpc.  The pin is
independent of both: the dense normal matrix A = Mpc^+ Mpc is diagonalised
(numpy LAPACK) and T_k evaluated on its eigenvalues from the closed forms
T_k(cos t) = cos(k t) and T_k(+-cosh t) = (+-1)^k cosh(k t).
"""
import numpy as np
import pytest

import oracle
from oracle import Params
from paper_2203_17119_amd import synth
from helpers import dense_matrix, relerr

MOB = dict(b=1.5, c=0.5, M5=1.8)


def cheb_closed(k, x):
    """T_k(x) for real x from the trigonometric / hyperbolic closed forms."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(k * np.arccos(x[inside]))
    big = ~inside
    out[big] = np.sign(x[big]) ** k * np.cosh(k * np.arccosh(np.abs(x[big])))
    return out


@pytest.fixture(scope="module")
def small():
    L, Ls = (2, 2, 4, 2), 4
    P = Params(L, Ls, **MOB, mf=0.05)
    U = oracle.dirichlet(L, synth.gauge_field(L, 0.6, 121), (0, 0, 1, 0))
    v = synth.gaussian_fermion(L, Ls, 122, nsites=P.V // 2)
    Mpc = dense_matrix(lambda e: oracle.mpc(P, U, e), P.half_shape())
    lam, V = np.linalg.eigh(Mpc.conj().T @ Mpc)
    return P, U, v, lam, V


@pytest.mark.parametrize("frac", [0.0, 0.05, 0.3])
def test_chebyshev_matches_eigendecomposition(small, frac):
    """lo at the bottom of the spectrum (frac 0) or inside it, hi above the top:
    the filters must agree with T_k on every eigenvalue, including the ones
    below lo where T_k grows."""
    P, U, v, lam, V = small
    lo, hi = frac * lam[-1], 1.05 * lam[-1]
    orders = [0, 1, 2, 3, 7, 16]
    ws = oracle.chebyshev(P, U, v, lo, hi, orders)
    c = V.conj().T @ v.ravel()
    x = (2.0 * lam - (hi + lo)) / (hi - lo)
    for k, w in zip(orders, ws):
        expect = V @ (cheb_closed(k, x) * c)
        assert relerr(w.ravel(), expect) < 1e-11, k


def test_chebyshev_degenerate_orders_and_bounds(small):
    """T_0 = identity; on [lo, hi] containing the whole spectrum every filter is a
    contraction of the eigencomponents (|T_k| <= 1), so |w_k| <= |v|."""
    P, U, v, lam, V = small
    lo, hi = 0.0, 1.01 * lam[-1]
    ws = oracle.chebyshev(P, U, v, lo, hi, [0, 5, 20, 40])
    assert np.array_equal(ws[0], v)
    for w in ws[1:]:
        assert np.linalg.norm(w) <= np.linalg.norm(v) * (1 + 1e-12)


def test_chebyshev_amplifies_the_low_modes(small):
    """With lo above the lowest eigenvalues the filter output concentrates on the
    eigenvectors below lo: their share of |w_k|^2 grows with k."""
    P, U, v, lam, V = small
    lo, hi = lam[len(lam) // 8], 1.05 * lam[-1]
    low = lam < lo
    shares = []
    for w in oracle.chebyshev(P, U, v, lo, hi, [1, 4, 12]):
        c = V.conj().T @ w.ravel()
        shares.append(np.sum(np.abs(c[low]) ** 2) / np.sum(np.abs(c) ** 2))
    assert shares[0] < shares[1] < shares[2] and shares[2] > 0.9
