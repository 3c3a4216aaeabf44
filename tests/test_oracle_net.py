"""Pins of the oracle's network preconditioner and of its Adam reference.

Network (or_net_apply): the preconditioner is the composition
    restrict_odd o layer_{L-1} o ... o layer_0 o embed_odd
and each path of a layer is the transport its definition states.  Both are
checked here against code written in the test from the definitions alone:
  * every path pi of one layer, with W = delta_pi (x) identity, equals the
    transport written out with numpy neighbour tables: U_mu(x) phi(x+mu),
    U_mu(x-mu)^+ phi(x-mu), phi(x, s+-1) with zeros outside 0..Ls-1;
  * the network equals the explicit composition with the odd embedding and
    restriction done by numpy index arrays, for distinct channel counts per
    layer (a wrong layer offset reads another layer's block) on asymmetric
    lattices; an embedding on the wrong parity is shown to change the result.

Adam (oracle.adam_step) against closed forms that a dropped bias correction,
swapped moments or a misplaced epsilon would each break:
  * first step: w - lr g / (|g| + eps);
  * a constant gradient for t steps: the bias-corrected moments are exactly g
    and g^2, so w_t = w_0 - t lr g / (|g| + eps);
  * a gradient g then 0: m^ = beta1 g / (1 + beta1), v^ = beta2 g^2 / (1 + beta2).
"""
import numpy as np
import pytest

import oracle
from oracle import Params
from paper_2203_17119_amd import synth
from helpers import neighbour, parity_sites, relerr


def _transport_by_definition(L, Ls, U, phi, pi):
    """(T_pi phi)(x, s) for phi[n][s][chan][colour], from the path definitions."""
    if pi == 0:
        return phi.copy()
    if 1 <= pi <= 4:
        mu = pi - 1
        nf = neighbour(L, mu, +1)
        return np.einsum("nab,nscb->nsca", U[:, mu], phi[nf])
    if 5 <= pi <= 8:
        mu = pi - 5
        nb = neighbour(L, mu, -1)
        return np.einsum("nba,nscb->nsca", U[nb, mu].conj(), phi[nb])
    out = np.zeros_like(phi)
    if pi == 9:
        out[:, :-1] = phi[:, 1:]
    else:
        out[:, 1:] = phi[:, :-1]
    return out


@pytest.mark.parametrize("L", [(2, 4, 2, 4), (4, 2, 2, 2)])
def test_each_path_is_its_transport(L):
    Ls, C = 3, 2
    U = synth.gauge_field(L, 0.8, 11)
    rng = np.random.default_rng(12)
    V = int(np.prod(L))
    phi = rng.standard_normal((V, Ls, C, 3)) + 1j * rng.standard_normal((V, Ls, C, 3))
    for pi in range(11):
        W = np.zeros((11, C, C), dtype=np.complex128)
        W[pi] = np.eye(C)
        got = oracle.ptc_layer(L, Ls, U, W, phi)
        assert relerr(got, _transport_by_definition(L, Ls, U, phi, pi)) < 1e-14, pi


def _weights(chans, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((11, co, ci)) + 1j * rng.standard_normal((11, co, ci))
            for ci, co in zip(chans[:-1], chans[1:])]


@pytest.mark.parametrize("L,Ls,chans", [((2, 4, 2, 4), 3, [4, 6, 8, 4]), ((4, 2, 4, 2), 2, [4, 12, 4])])
def test_network_is_the_composition(L, Ls, chans):
    P = Params(L, Ls, 1.5, 0.5, 1.8, 0.1)
    U = synth.gauge_field(L, 0.7, 21)
    Ws = _weights(chans, 22)
    odd = synth.gaussian_fermion(L, Ls, 23, nsites=P.V // 2)
    got = oracle.net_apply(P, U, Ws, odd)

    def compose(parity):
        sites = parity_sites(L, parity)
        phi = np.zeros(P.full_shape(), dtype=np.complex128)  # [n][s][spin = channel][colour]
        phi[sites] = odd
        for W in Ws:
            phi = oracle.ptc_layer(L, Ls, U, W, phi)
        return phi[parity_sites(L, 1)]

    assert relerr(got, compose(1)) < 1e-13
    # the test can tell the embedding parity apart
    assert relerr(compose(0), compose(1)) > 1e-2


def test_network_is_linear_and_covariant():
    L, Ls, chans = (2, 2, 4, 2), 2, [4, 8, 4]
    P = Params(L, Ls, 1.5, 0.5, 1.8, 0.1)
    U = synth.gauge_field(L, 0.7, 31)
    Ws = _weights(chans, 32)
    a = synth.gaussian_fermion(L, Ls, 33, nsites=P.V // 2)
    b = synth.gaussian_fermion(L, Ls, 34, nsites=P.V // 2)
    lhs = oracle.net_apply(P, U, Ws, a + (0.5 - 2j) * b)
    rhs = oracle.net_apply(P, U, Ws, a) + (0.5 - 2j) * oracle.net_apply(P, U, Ws, b)
    assert relerr(lhs, rhs) < 1e-13


LR, B1, B2 = 1e-3, 0.9, 0.999


def test_adam_first_step():
    rng = np.random.default_rng(41)
    w, g = rng.standard_normal(50), rng.standard_normal(50)
    eps = 0.3
    w1, m, v = oracle.adam_step(w, g, np.zeros(50), np.zeros(50), 1, LR, B1, B2, eps)
    assert np.allclose(w1, w - LR * g / (np.abs(g) + eps), rtol=0, atol=1e-15)


def test_adam_constant_gradient_is_bias_corrected():
    rng = np.random.default_rng(42)
    w0, g = rng.standard_normal(30), rng.standard_normal(30)
    eps = 0.05
    w, m, v = w0, np.zeros(30), np.zeros(30)
    for t in range(1, 8):
        w, m, v = oracle.adam_step(w, g, m, v, t, LR, B1, B2, eps)
        assert np.allclose(w, w0 - t * LR * g / (np.abs(g) + eps), rtol=0, atol=1e-14), t


def test_adam_moments_after_a_zero_gradient():
    rng = np.random.default_rng(43)
    w0, g = rng.standard_normal(20), rng.standard_normal(20)
    eps = 0.2
    w1, m, v = oracle.adam_step(w0, g, np.zeros(20), np.zeros(20), 1, LR, B1, B2, eps)
    w2, m, v = oracle.adam_step(w1, np.zeros(20), m, v, 2, LR, B1, B2, eps)
    mhat = B1 * g / (1 + B1)
    vhat = B2 * g * g / (1 + B2)
    assert np.allclose(w2, w1 - LR * mhat / (np.sqrt(vhat) + eps), rtol=0, atol=1e-15)
