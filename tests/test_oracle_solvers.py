"""Pins of the oracle's Krylov solvers: exact results within their bounds.

Multi-shift CG (Jegerlehner's shifted recurrences) and flexible GCR are
checked against dense solves (numpy LAPACK) of the same systems on small
lattices, and against their own recomputed true residuals.
"""
import numpy as np
import pytest

import oracle
from oracle import Params
from paper_2203_17119_amd import synth
from helpers import dense_matrix, relerr

MOB = dict(b=1.5, c=0.5, M5=1.8)


def test_multishift_matches_dense_solves():
    L, Ls = (2, 4, 2, 2), 4
    P = Params(L, Ls, **MOB, mf=0.05)
    U = synth.gauge_field(L, 0.6, 101)
    b = synth.gaussian_fermion(L, Ls, 102, nsites=P.V // 2)
    shifts = synth.rational_shifts()
    tol = 1e-11
    x, it, iters, res = oracle.multishift(P, U, b, shifts, tol)
    assert it > 0 and np.all(iters > 0)
    Mpc = dense_matrix(lambda e: oracle.mpc(P, U, e), P.half_shape())
    A = Mpc.conj().T @ Mpc
    for k, s in enumerate(shifts):
        xd = np.linalg.solve(A + s * np.eye(len(A)), b.ravel())
        kappa = np.linalg.cond(A + s * np.eye(len(A)))
        assert relerr(x[k].ravel(), xd) < 10 * kappa * tol
        assert res[k] < 10 * tol
    # larger shifts converge no later than smaller ones
    order = np.argsort(shifts)
    assert np.all(np.diff(iters[order]) <= 0)


def test_multishift_4x4x4x4_ls8():
    w = synth.WORKLOADS["4^4x8_periodic"]
    P = Params(w.dims, w.Ls, w.b, w.c, w.M5, w.mf)
    U = synth.gauge_field(w.dims, w.eps, w.gauge_seed)
    b = synth.gaussian_fermion(w.dims, w.Ls, 103, nsites=P.V // 2)
    shifts = synth.rational_shifts()
    x, it, iters, res = oracle.multishift(P, U, b, shifts, 1e-8)
    assert it > 0
    assert np.all(res < 3e-8)


@pytest.mark.parametrize("m,normal", [(8, False), (16, False), (16, True)])
def test_gcr_matches_dense_solve(m, normal):
    L, Ls = (2, 2, 4, 2), 4
    P = Params(L, Ls, **MOB, mf=0.05)
    U = synth.gauge_field(L, 0.6, 111)
    b = synth.gaussian_fermion(L, Ls, 112, nsites=P.V // 2)
    x, it, res = oracle.fgcr(P, U, b, 1e-11, maxit=5000, m=m, normal=normal)
    assert it > 0 and res < 1e-11
    Mpc = dense_matrix(lambda e: oracle.mpc(P, U, e), P.half_shape())
    A = Mpc.conj().T @ Mpc if normal else Mpc
    xd = np.linalg.solve(A, b.ravel())
    assert relerr(x.ravel(), xd) < 1e-6


def test_fgcr_with_network_preconditioner_converges():
    L, Ls = (2, 2, 4, 2), 4
    P = Params(L, Ls, **MOB, mf=0.05)
    U = synth.gauge_field(L, 0.6, 121)
    b = synth.gaussian_fermion(L, Ls, 122, nsites=P.V // 2)
    rng = np.random.default_rng(5)
    chans = [4, 6, 4]
    # identity plus a perturbation on every path: a fixed, non-trivial linear preconditioner
    W = [0.01 * (rng.standard_normal((11, co, ci)) + 1j * rng.standard_normal((11, co, ci)))
         for ci, co in zip(chans[:-1], chans[1:])]
    W[0][0, :4, :4] += np.eye(4)
    W[1][0, :4, :4] += np.eye(4)
    x, it, res = oracle.fgcr(P, U, b, 1e-10, maxit=5000, m=16, weights=W)
    assert it > 0 and res < 1e-10
    r = b - oracle.mpc(P, U, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-10
