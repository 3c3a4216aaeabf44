"""GPU parity of the operator entry points against the FP64 oracle.

Every call goes through the C ABI (libdwf.so via ctypes).  FP64 results must
agree with the oracle to 1e-12 relative; lower storage precisions to the
rounding level of their format (FP32 1e-6, FP16 with per-site scale 2e-3,
BF16 1.5e-2).  Lattices include ragged workgroup tails, asymmetric extents
and Dirichlet faces.
"""
import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf
from gpu_helpers import SITE_TOL, TOL, Case, relerr, site_relerr, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

# Ls = 8, 12 and 16 run the Toeplitz (twisted-circulant) form of the dense
# fifth-dimension epilogue, the others the general dense form.  The Toeplitz
# form is applied as the recurrence of (b + c S)(d + e S)^-1 when |e/d| <= 1/2
# (d = b (4 - M5) + 1, e = c (4 - M5) - 1): the default Moebius parameters
# give |e/d| = 0.02, the r027 case 0.27; the Shamir case at M5 = 3.6 (0.71)
# keeps the explicit Ls x Ls product.
CASES = {
    "2x2x4x2_ls8_r027": dict(dims=(2, 2, 4, 2), Ls=8, b=2.0, c=1.0, M5=1.2, mf=0.1, dirichlet=(0, 0, 1, 0), seed=35),
    "2x2x2x4_ls12_shamir_dense": dict(dims=(2, 2, 2, 4), Ls=12, b=1.0, c=0.0, M5=3.6, mf=0.1, seed=36),
    "4^4x8_periodic": dict(dims=(4, 4, 4, 4), Ls=8, eps=0.4, seed=1001),
    "2x4x2x4_ls16_dirichlet": dict(dims=(2, 4, 2, 4), Ls=16, dirichlet=(0, 1, 0, 1), mf=0.03, seed=33),
    "4x2x2x2_ls12": dict(dims=(4, 2, 2, 2), Ls=12, mf=0.2, seed=34),
    "4x6x2x8_ls5_dirichlet": dict(dims=(4, 6, 2, 8), Ls=5, dirichlet=(1, 0, 1, 1), mf=0.07, seed=31),
    "2x2x2x2_ls3": dict(dims=(2, 2, 2, 2), Ls=3, dirichlet=(0, 0, 0, 1), seed=32),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    c = Case(**CASES[request.param])
    yield c
    c.close()


@pytest.mark.parametrize("out_parity,dagger", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_dhop_matches_oracle(case, out_parity, dagger):
    x = case.half(7)
    out = torch().empty_like(to_gpu(x))
    dwf.dwf_dhop(case.ctx, out_parity, dagger, to_gpu(x), out)
    expect = case.oracle_dhop(x, out_parity, bool(dagger))
    got = to_host(out)
    assert relerr(got, expect) < 1e-12
    assert np.abs(got - expect).max() < 1e-12 * np.abs(expect).max()


@pytest.mark.parametrize("dagger", [0, 1])
def test_mooee_and_inverse_match_oracle(case, dagger):
    x = case.half(8)
    out = torch().empty_like(to_gpu(x))
    dwf.dwf_mooee(case.ctx, dagger, to_gpu(x), out)
    assert relerr(to_host(out), oracle.mooee(case.P, x, bool(dagger))) < 1e-13
    dwf.dwf_mooeeinv(case.ctx, dagger, to_gpu(x), out)
    assert relerr(to_host(out), oracle.mooeeinv(case.P, x, bool(dagger))) < 1e-12


@pytest.mark.parametrize("dagger", [0, 1])
def test_schur_apply_matches_oracle(case, dagger):
    x = case.half(9)
    out = torch().empty_like(to_gpu(x))
    dwf.dwf_schur_apply(case.ctx, dagger, to_gpu(x), out)
    expect = oracle.mpc(case.P, case.Ud, x, bool(dagger))
    assert relerr(to_host(out), expect) < 1e-12


@pytest.mark.parametrize("prec", [dwf.DWF_F64, dwf.DWF_F32, dwf.DWF_F16, dwf.DWF_BF16])
def test_internal_precisions(case, prec):
    T = torch()
    x = case.half(10)
    xin = case.lat.internal(prec)
    xout = case.lat.internal(prec)
    dwf.dwf_import(case.ctx, 0, prec, to_gpu(x), xin)
    # round trip is exact in FP64 and at format precision otherwise
    back = T.empty_like(to_gpu(x))
    dwf.dwf_export(case.ctx, 0, prec, xin, back)
    assert relerr(to_host(back), x) < (1e-16 if prec == dwf.DWF_F64 else TOL[prec] / 2)
    for out_parity, dagger in [(0, 0), (1, 1)]:
        dwf.dwf_dhop_internal(case.ctx, prec, out_parity, dagger, xin, xout)
        dwf.dwf_export(case.ctx, 0, prec, xout, back)
        expect = case.oracle_dhop(x, out_parity, bool(dagger))
        got = to_host(back)
        print(f"prec {prec} dhop: global {relerr(got, expect):.2e}, worst site {site_relerr(got, expect):.2e}",
              flush=True)
        assert relerr(got, expect) < TOL[prec]
        assert site_relerr(got, expect) < SITE_TOL[prec]
    for dagger in (0, 1):
        dwf.dwf_schur_apply_internal(case.ctx, prec, dagger, xin, xout)
        dwf.dwf_export(case.ctx, 0, prec, xout, back)
        expect = oracle.mpc(case.P, case.Ud, x, bool(dagger))
        got = to_host(back)
        print(f"prec {prec} Mpc dagger {dagger}: global {relerr(got, expect):.2e}, "
              f"worst site {site_relerr(got, expect):.2e}", flush=True)
        assert relerr(got, expect) < TOL[prec]
        assert site_relerr(got, expect) < SITE_TOL[prec]


def test_dhop_16x16x16x16_ls12_dirichlet():
    print("\n[16^4x12 dirichlet dhop]", flush=True)
    c = Case((16, 16, 16, 16), 12, mf=0.01, dirichlet=(1, 1, 1, 1), eps=0.7, seed=1002)
    try:
        x = c.half(2002)
        out = torch().empty_like(to_gpu(x))
        for out_parity, dagger in [(1, 0), (0, 1)]:
            dwf.dwf_dhop(c.ctx, out_parity, dagger, to_gpu(x), out)
            assert relerr(to_host(out), c.oracle_dhop(x, out_parity, bool(dagger))) < 1e-12
        dwf.dwf_schur_apply(c.ctx, 0, to_gpu(x), out)
        assert relerr(to_host(out), oracle.mpc(c.P, c.Ud, x, False)) < 1e-12
    finally:
        c.close()


@pytest.mark.parametrize("order", [(2, 2, 2), (4, 4, 2), (2, 1, 4), (8, 4, 4), (0, 0, 0)])
def test_site_orders(order):
    """Results do not depend on the internal (cache-blocked) site order or schedule."""
    print(f"\n[site order {order}]", flush=True)
    c = Case((8, 4, 4, 6), 4, mf=0.05, dirichlet=(1, 0, 0, 1), seed=41)
    try:
        dwf.dwf_set_site_order(c.ctx, *order)
        got = dwf.dwf_get_site_order(c.ctx)
        if order != (0, 0, 0):
            assert got == order
        x = c.half(12)
        xg = to_gpu(x)
        out = torch().empty_like(xg)
        for out_parity, dagger in [(0, 0), (1, 1)]:
            dwf.dwf_dhop(c.ctx, out_parity, dagger, xg, out)
            assert relerr(to_host(out), c.oracle_dhop(x, out_parity, bool(dagger))) < 1e-12
        for sb, run in [(3, 1), (5, 2), (8, 1)]:
            dwf.dwf_set_tile_schedule(c.ctx, dwf.DWF_K_STENCIL, sb, run)
            dwf.dwf_schur_apply(c.ctx, 1, xg, out)
            assert relerr(to_host(out), oracle.mpc(c.P, c.Ud, x, True)) < 1e-12
        # internal-layout round trip in every precision
        for prec in (dwf.DWF_F64, dwf.DWF_F16):
            buf = c.lat.internal(prec)
            dwf.dwf_import(c.ctx, 0, prec, xg, buf)
            dwf.dwf_dhop_internal(c.ctx, prec, 1, 0, buf, c.lat.internal(prec))
            dwf.dwf_export(c.ctx, 0, prec, buf, out)
            assert relerr(to_host(out), x) < (1e-16 if prec == dwf.DWF_F64 else 1e-3)
        b = c.full(13)
        xs = torch().zeros_like(to_gpu(b))
        status, st = dwf.dwf_cg(c.ctx, to_gpu(b), xs, tol=1e-10, mode=dwf.DWF_SOLVE_MIXED_F16)
        assert status == dwf.DWF_OK
        r = b - oracle.d5(c.P, c.Ud, to_host(xs))
        assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-8
    finally:
        c.close()


def test_repeated_calls_are_bitwise_identical(case):
    x = to_gpu(case.half(11))
    a = torch().empty_like(x)
    b = torch().empty_like(x)
    dwf.dwf_schur_apply(case.ctx, 1, x, a)
    dwf.dwf_schur_apply(case.ctx, 1, x, b)
    assert torch().equal(a, b)
