"""GPU parity of the DD-RHMC one-flavour boundary action (Sec. 2.3.1, eq. (ddrhmc))
and of the rational-function application it is built from.

    r(A) v = a0 v + sum_k alpha_k (A + beta_k)^-1 v,   A = Mpc^+ Mpc
    S = phi^+ r_q(A_d) r_m(A) r_q(A_d) phi,   r_q ~ x^{1/4},  r_m ~ x^{-1/2}

The oracle evaluates both with dense matrices on 2^4 and 2x2x2x4 lattices:
the rational functions exactly (dense inverses of A + beta_k), the exact
fractional powers by eigendecomposition; its CPU tests pin the action's
log det to the determinant ratio of eq. (ddrhmc).

Tolerances, from the solver's guarantee: every shifted system meets
|v - (A + beta_k) x_k| <= tol |v|, so |x_k - x_k*| <= tol |v| / (lmin + beta_k),
and the absolute error of r(A) v is at most e = tol |v| sum_k |alpha_k| / (lmin + beta_k).
The action's error follows from the two errors e_q (of psi) and e_m (of chi):
|dS| <= e_q |r_m(A)| (2 |psi| + e_q) + (|psi| + e_q) e_m.

Beyond the dense oracle's reach (8^4 x 8, and the benchmark's 16^4 x 12 field
with both operators) the inverse square root is checked by A r_m(A)^2 v = v.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf
from gpu_helpers import Case, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

RATIONAL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2203_17119_amd",
                        "rational")


def load_rational(name):
    with open(os.path.join(RATIONAL, name)) as fh:
        return json.load(fh)


RQ = load_rational("x0.25_0.01_100_n12.json")
RM = load_rational("x-0.5_0.01_100_n12.json")


def coeffs(r):
    return r["a0"], r["alpha"], r["beta"]


def err_bound(r, lmin, vnorm, tol):
    return tol * vnorm * sum(abs(a) / (lmin + b) for a, b in zip(r["alpha"], r["beta"]))


CASES = {
    # dims, Ls, mf, Dirichlet mask, eps, seed
    "2x2x2x2_ls4": ((2, 2, 2, 2), 4, 0.1, (1, 1, 1, 1), 0.5, 7),
    "2x2x2x4_ls4_tcut": ((2, 2, 2, 4), 4, 0.1, (0, 0, 0, 1), 0.5, 11),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    """The periodic context and the Dirichlet context of one field, with the
    oracle's dense normal operators."""
    dims, Ls, mf, mask, eps, seed = CASES[request.param]
    print(f"\n[ddrhmc case {request.param}]", flush=True)
    full = Case(dims, Ls, mf=mf, eps=eps, seed=seed)
    cut = Case(dims, Ls, mf=mf, dirichlet=mask, eps=eps, seed=seed)
    A = oracle.dense_normal(full.P, full.U)
    Ad = oracle.dense_normal(cut.P, cut.Ud)
    for M in (A, Ad):  # the committed approximations cover the spectrum
        lam = np.linalg.eigvalsh(M)
        assert RQ["lo"] <= lam[0] and lam[-1] <= RQ["hi"]
    yield full, cut, A, Ad
    full.close()
    cut.close()


@pytest.mark.parametrize("mode", [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F32])
@pytest.mark.parametrize("which", ["quarter", "minus_half"])
def test_rational_apply_matches_oracle(pair, mode, which):
    full, cut, A, Ad = pair
    r = RQ if which == "quarter" else RM
    tol = 1e-10
    v = full.half(31)
    expect = oracle.rational_dense(A, *coeffs(r)) @ v.ravel()
    out = torch().empty_like(to_gpu(v))
    s, st = dwf.dwf_rational_apply(full.ctx, dwf.make_rational(*coeffs(r)), to_gpu(v), out, tol=tol, mode=mode)
    assert s == dwf.DWF_OK and st["converged"] == 1, st
    lmin = np.linalg.eigvalsh(A)[0]
    bound = err_bound(r, lmin, np.linalg.norm(v), tol)
    err = np.linalg.norm(to_host(out).ravel() - expect)
    print(f"{which} mode {mode}: |r(A)v - oracle| = {err:.2e} (bound {bound:.2e}), worst shift {st['iters']} iters",
          flush=True)
    assert err <= bound


def test_rational_apply_in_place_and_repeat(pair):
    full, cut, A, Ad = pair
    v = full.half(32)
    r = dwf.make_rational(*coeffs(RM))
    a = to_gpu(v)
    b = torch().empty_like(a)
    dwf.dwf_rational_apply(full.ctx, r, a, b, tol=1e-10)
    dwf.dwf_rational_apply(full.ctx, r, a, a, tol=1e-10)  # in and out the same buffer
    assert np.array_equal(to_host(a), to_host(b))


@pytest.mark.parametrize("mode", [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F32])
def test_action_matches_oracle(pair, mode):
    full, cut, A, Ad = pair
    tol = 1e-10
    phi = full.half(33)
    S_rat = oracle.ddrhmc_action(full.P, full.U, cut.Ud, phi, quarter=coeffs(RQ), minus_half=coeffs(RM))
    S_exact = oracle.ddrhmc_action(full.P, full.U, cut.Ud, phi)
    s, S, sts = dwf.dwf_ddrhmc_action(full.ctx, cut.ctx, dwf.make_rational(*coeffs(RQ)),
                                      dwf.make_rational(*coeffs(RM)), to_gpu(phi), tol=tol, mode=mode)
    assert s == dwf.DWF_OK and all(x["converged"] for x in sts), sts
    lam, lam_d = np.linalg.eigvalsh(A), np.linalg.eigvalsh(Ad)
    psi = oracle.rational_dense(Ad, *coeffs(RQ)) @ phi.ravel()
    e_q = err_bound(RQ, lam_d[0], np.linalg.norm(phi), tol)
    e_m = err_bound(RM, lam[0], np.linalg.norm(psi) + e_q, tol)
    g_norm = lam[0] ** -0.5 * (1 + RM["max_rel_error"])
    pn = np.linalg.norm(psi)
    bound = e_q * g_norm * (2 * pn + e_q) + (pn + e_q) * e_m
    print(f"mode {mode}: S = {S:.12e}, oracle (rational) {S_rat:.12e}, exact {S_exact:.12e}, "
          f"|dS| = {abs(S - S_rat):.2e} (bound {bound:.2e})", flush=True)
    assert abs(S - S_rat) <= bound
    # the rational action is within the approximation's own bound of the exact one
    eq, em = RQ["max_rel_error"], RM["max_rel_error"]
    assert abs(S - S_exact) <= ((1 + eq) ** 2 * (1 + em) - 1) * lam[0] ** -0.5 * np.linalg.norm(
        oracle.herm_power(Ad, 0.25) @ phi.ravel()) ** 2 + bound


def test_action_argument_errors(pair):
    full, cut, A, Ad = pair
    phi = to_gpu(full.half(34))
    rq = dwf.make_rational(*coeffs(RQ))
    bad = dwf.make_rational(1.0, [1.0], [-0.5])
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_ddrhmc_action(full.ctx, cut.ctx, bad, rq, phi)
    assert e.value.status == dwf.DWF_EINVAL
    other = Case(full.dims, full.Ls + 1, mf=0.1, eps=0.5, seed=3)
    try:
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_ddrhmc_action(full.ctx, other.ctx, rq, rq, phi)
        assert e.value.status == dwf.DWF_EINVAL
    finally:
        other.close()
    empty = dwf.make_rational(0.0, [], [])
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_rational_apply(full.ctx, empty, phi, phi)
    assert e.value.status == dwf.DWF_EINVAL


def test_inverse_square_root_squared_at_8x8x8x8_ls8():
    """At a size the dense oracle cannot reach: A r_m(A)^2 v = v.  With
    r_m(l) = l^{-1/2} (1 + d), |d| <= eps on the spectrum (the n = 20
    approximation on [1e-5, 1000]), y = r_m(A) v + d1 and z = r_m(A) y + d2,
        A z - v = (A r_m(A)^2 - 1) v + A r_m(A) d1 + A d2,
    so |A z - v| <= (2 eps + eps^2) |v| + tol S0 (sqrt(top) (1 + eps) |v| + top |y|)
    with S0 = sum_k |alpha_k| / beta_k and top the spectrum's upper end
    (estimated by oracle power steps, with a margin of 1.5; the
    approximation's interval reaches ten times further)."""
    r = load_rational("x-0.5_1e-05_1000_n20.json")
    c = Case((8, 8, 8, 8), 8, mf=0.02, dirichlet=(1, 1, 1, 1), eps=0.7, seed=41)
    print("\n[ddrhmc 8x8x8x8_ls8 dirichlet]", flush=True)
    try:
        v = c.half(35)
        w = v / np.linalg.norm(v)
        for _ in range(20):
            w = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, w), True)
            top = np.linalg.norm(w)
            w = w / top
        top *= 1.5
        assert top < r["hi"]
        tol = 1e-11
        rm = dwf.make_rational(*coeffs(r))
        a = to_gpu(v)
        y = torch().empty_like(a)
        s1, st1 = dwf.dwf_rational_apply(c.ctx, rm, a, y, tol=tol)
        yn = np.linalg.norm(to_host(y))
        s2, st2 = dwf.dwf_rational_apply(c.ctx, rm, y, y, tol=tol)
        assert s1 == s2 == dwf.DWF_OK, (st1, st2)
        z = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, to_host(y)), True)
        eps = r["max_rel_error"]
        vn = np.linalg.norm(v)
        s0 = sum(abs(al) / be for al, be in zip(r["alpha"], r["beta"]))
        bound = 2 * eps + eps ** 2 + tol * s0 * (np.sqrt(top) * (1 + eps) + top * yn / vn)
        err = np.linalg.norm(z - v) / vn
        print(f"|A r(A)^2 v - v| / |v| = {err:.2e} (bound {bound:.2e}), worst shift {st1['iters']} iters",
              flush=True)
        assert err <= bound
    finally:
        c.close()


@pytest.mark.parametrize("which", ["periodic", "cut"])
def test_inverse_square_root_squared_16x16x16x16_ls12(which):
    """The benchmark's DD-RHMC field (16^4 x 12, mf 0.01, eps 0.7): the
    whole-lattice operator A and the block operator A_d with every face cut,
    each through the degree-20 approximation of x^{-1/2} on [1e-5, 1000]
    that the benchmark applies: A r_m(A)^2 v = v within the bound of the
    8^4 x 8 test (the spectrum's top from eight oracle power steps, margin
    1.5), the last A applied by the oracle on the whole lattice."""
    from paper_2203_17119_amd import synth
    w = synth.WORKLOADS["16^4x12_multishift"]
    r = load_rational("x-0.5_1e-05_1000_n20.json")
    mask = (0, 0, 0, 0) if which == "periodic" else (1, 1, 1, 1)
    print(f"\n[ddrhmc 16x16x16x16_ls12 {which}: A r_m(A)^2 v = v]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=mask, eps=w.eps, seed=w.gauge_seed)
    try:
        v = c.half(w.source_seeds[0])
        u = v / np.linalg.norm(v)
        for _ in range(8):
            u = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, u), True)
            top = np.linalg.norm(u)
            u = u / top
        del u
        top *= 1.5
        assert top < r["hi"]
        tol = 1e-11
        rm = dwf.make_rational(*coeffs(r))
        a = to_gpu(v)
        y = torch().empty_like(a)
        s1, st1 = dwf.dwf_rational_apply(c.ctx, rm, a, y, tol=tol)
        yn = float(y.norm())
        s2, st2 = dwf.dwf_rational_apply(c.ctx, rm, y, y, tol=tol)
        assert s1 == s2 == dwf.DWF_OK, (st1, st2)
        z = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, to_host(y)), True)
        eps = r["max_rel_error"]
        vn = np.linalg.norm(v)
        s0 = sum(abs(al) / be for al, be in zip(r["alpha"], r["beta"]))
        bound = 2 * eps + eps ** 2 + tol * s0 * (np.sqrt(top) * (1 + eps) + top * yn / vn)
        err = np.linalg.norm(z - v) / vn
        print(f"spectrum top {top / 1.5:.1f}: |A r(A)^2 v - v| / |v| = {err:.2e} (bound {bound:.2e}), "
              f"worst shift {st1['iters']} iterations, {st1['seconds']:.2f} s", flush=True)
        assert err <= bound
    finally:
        c.close()
