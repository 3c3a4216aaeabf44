"""Pins of the oracle's domain-boundary operators (Sec. 2.1, the construction
after eq. (schur)).

The lattice splits into a domain Omega (mask 1) and its complement; D_cut is
D5 on the gauge field whose links between the domains are zero.  The oracle's
projector is P = A^-1 Pi A, Pi the spin-space mask of the boundary sites, and

    R    = P - P D_Omega^-1 D_d D_Omegabar^-1 D_dbar,
    R^-1 = P - P D^-1 D_dbar.

What the paper states, checked here with dense matrices on small lattices:
* D_dbar P = D_dbar (P keeps exactly what the boundary hop sees), and P is a
  projector of the expected rank; dropping the A conjugation (for c != 0) or
  swapping the spin projectors breaks the first identity, so it pins them;
* eq. (schur): det D = det D_Omega det D_Omegabar det chi, with
  chi = 1 - D_Omega^-1 D_d D_Omegabar^-1 D_dbar (dense LU determinants);
* det chi = det R, R taken on the range of P;
* R R^-1 = P;
* for Shamir (c = 0) P is the Hermitian spin-space mask itself;
* the cut gauge field makes D_cut block diagonal with D's diagonal blocks.
"""
import numpy as np
import pytest

import oracle
from oracle import Params
from paper_2203_17119_amd import synth
from helpers import coords


def _mask_t(L, t_hi):
    """Omega = sites with t < t_hi."""
    return (coords(L)[:, 3] < t_hi).astype(np.int32)


def _mask_box(L, x_hi, t_hi):
    x = coords(L)
    return ((x[:, 0] < x_hi) & (x[:, 3] < t_hi)).astype(np.int32)


CASES = {
    # one boundary direction: every boundary site has one neighbour outside
    "t_split": dict(L=(2, 2, 2, 4), Ls=4, mask=lambda L: _mask_t(L, 2)),
    # a box in x and t: edge sites with one neighbour outside, corners with two
    "xt_box": dict(L=(4, 2, 2, 6), Ls=2, mask=lambda L: _mask_box(L, 2, 3)),
}


def _setup(name, c=0.5, seed=17):
    cfg = CASES[name]
    L, Ls = cfg["L"], cfg["Ls"]
    P = Params(L, Ls, 1.5, c, 1.8, 0.1)
    U = synth.gauge_field(L, 0.5, seed)
    mask = cfg["mask"](L)
    Uc = oracle.mask_cut(L, U, mask)
    return P, U, Uc, mask


def _omega_components(P, mask):
    return np.repeat(np.asarray(mask).ravel() == 1, 12 * P.Ls)


def _random_on_omega(P, mask, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(P.full_shape()) + 1j * rng.standard_normal(P.full_shape())
    return oracle.restrict(P, mask, psi)


@pytest.fixture(scope="module", params=list(CASES))
def dense(request):
    P, U, Uc, mask = _setup(request.param)
    D, Dc = oracle.dense_d5(P, U), oracle.dense_d5(P, Uc)
    Pm = oracle.dense_boundary_projector(P, mask)
    return request.param, P, U, Uc, mask, D, Dc, Pm


def test_cut_gauge_gives_the_diagonal_blocks(dense):
    name, P, U, Uc, mask, D, Dc, Pm = dense
    om = _omega_components(P, mask)
    ob = ~om
    assert np.array_equal(Dc[np.ix_(om, om)], D[np.ix_(om, om)])
    assert np.array_equal(Dc[np.ix_(ob, ob)], D[np.ix_(ob, ob)])
    assert np.abs(Dc[np.ix_(om, ob)]).max() == 0 and np.abs(Dc[np.ix_(ob, om)]).max() == 0
    assert np.abs(D[np.ix_(ob, om)]).max() > 0.1  # the domains do couple


def test_projector_keeps_what_the_boundary_hop_sees(dense):
    name, P, U, Uc, mask, D, Dc, Pm = dense
    off = D - Dc
    om = _omega_components(P, mask)
    # D_dbar P = D_dbar on fields of Omega, P^2 = P, nothing outside Omega
    assert np.abs(off[:, om] @ Pm[np.ix_(om, om)] - off[:, om]).max() < 1e-12
    assert np.abs(Pm @ Pm - Pm).max() < 1e-12
    assert np.abs(Pm[~om, :]).max() == 0 and np.abs(Pm[:, ~om]).max() == 0
    # rank: 2 spins at a site with one outside neighbour, 4 with more, times colours and Ls
    Pi = oracle.boundary_spin_mask(P.L, mask)
    ranks = np.rint(np.real(np.einsum("naa->n", Pi))).astype(int)
    assert set(ranks[np.asarray(mask) == 0]) <= {0}
    expect = int(ranks.sum()) * 3 * P.Ls
    assert np.linalg.matrix_rank(Pm) == expect
    if name == "t_split":
        assert set(ranks) == {0, 2}
    else:
        assert set(ranks) == {0, 2, 4}


def test_projector_pins_fail_for_wrong_variants(dense):
    """The identity D_dbar P = D_dbar fails without the A conjugation (c != 0)
    and with the spin projectors swapped: it pins both."""
    name, P, U, Uc, mask, D, Dc, Pm = dense
    off = D - Dc
    psi = _random_on_omega(P, mask, 5)
    want = off @ psi.ravel()
    Pi = oracle.boundary_spin_mask(P.L, mask)
    no_a = np.einsum("nab,nsbc->nsac", Pi, psi)
    swapped = np.einsum("nab,nsbc->nsac", np.where(np.abs(Pi) > 0, np.eye(4)[None] - Pi, 0.0), psi)
    a = oracle.a_site_matrix(P)
    ai = oracle.a_site_matrix(P, inverse=True)
    v = (psi.reshape(P.V, -1) @ a.T).reshape(psi.shape)
    v = np.einsum("nab,nsbc->nsac", np.where(np.abs(Pi) > 0, np.eye(4)[None] - Pi, 0.0), v)
    swapped_a = (v.reshape(P.V, -1) @ ai.T).reshape(psi.shape)
    for bad in (no_a, swapped, swapped_a):
        assert np.linalg.norm(off @ bad.ravel() - want) > 1e-3 * np.linalg.norm(want)
    good = oracle.boundary_projector(P, mask, psi)
    assert np.linalg.norm(off @ good.ravel() - want) < 1e-12 * np.linalg.norm(want)


def test_schur_determinant(dense):
    """eq. (schur): det D = det D_Omega det D_Omegabar det chi."""
    name, P, U, Uc, mask, D, Dc, Pm = dense
    om = _omega_components(P, mask)
    off = D - Dc
    chi = np.eye(D.shape[0]) - np.linalg.solve(Dc, off @ np.linalg.solve(Dc, off))
    s_d, l_d = np.linalg.slogdet(D)
    s_c, l_c = np.linalg.slogdet(Dc)
    s_x, l_x = np.linalg.slogdet(chi[np.ix_(om, om)])
    assert abs(l_d - (l_c + l_x)) < 1e-8 * max(1.0, abs(l_d))
    assert abs(s_d - s_c * s_x) < 1e-8


def test_det_chi_equals_det_r(dense):
    name, P, U, Uc, mask, D, Dc, Pm = dense
    om = _omega_components(P, mask)
    off = D - Dc
    K = np.linalg.solve(Dc, off @ np.linalg.solve(Dc, off))
    chi = np.eye(D.shape[0]) - K
    R = Pm - Pm @ K
    # R on the range of P, in an orthonormal basis Q of that range
    u, sv, _ = np.linalg.svd(Pm)
    r = int((sv > 1e-8 * sv[0]).sum())
    Q = u[:, :r]
    assert np.abs(Q @ (Q.conj().T @ R) - R).max() < 1e-10  # R maps into the range of P
    M = Q.conj().T @ R @ Q
    s_r, l_r = np.linalg.slogdet(M)
    s_x, l_x = np.linalg.slogdet(chi[np.ix_(om, om)])
    print(f"{name}: rank {r}, log|det chi| = {l_x:.12f}, log|det R| = {l_r:.12f}")
    assert abs(l_r - l_x) < 1e-8 * max(1.0, abs(l_x))
    assert abs(s_r - s_x) < 1e-8


def test_r_times_r_inverse_is_the_projector(dense):
    name, P, U, Uc, mask, D, Dc, Pm = dense
    psi = _random_on_omega(P, mask, 11)
    rinv = oracle.boundary_r(P, U, Uc, mask, psi, inverse=True)
    back = oracle.boundary_r(P, U, Uc, mask, rinv)
    want = oracle.boundary_projector(P, mask, psi)
    assert np.linalg.norm(back - want) < 1e-10 * np.linalg.norm(want)
    # and R^-1 R = P on the range of P
    back2 = oracle.boundary_r(P, U, Uc, mask, oracle.boundary_r(P, U, Uc, mask, want), inverse=True)
    assert np.linalg.norm(back2 - want) < 1e-10 * np.linalg.norm(want)


def test_shamir_projector_is_the_spin_mask():
    P, U, Uc, mask = _setup("xt_box", c=0.0)
    Pm = oracle.dense_boundary_projector(P, mask)
    assert np.abs(Pm - Pm.conj().T).max() < 1e-14
    psi = _random_on_omega(P, mask, 3)
    Pi = oracle.boundary_spin_mask(P.L, mask)
    assert np.abs(oracle.boundary_projector(P, mask, psi) - np.einsum("nab,nsbc->nsac", Pi, psi)).max() < 1e-14
