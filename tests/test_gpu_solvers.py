"""GPU parity of the solvers: CGNE (FP64 and mixed precision) and multi-shift CG.

Solutions are judged by their FP64 residuals (recomputed by the oracle where it
is affordable) and by their distance to the oracle's own solution, which is
bounded by roughly kappa * tol.
"""
import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf, synth
from gpu_helpers import Case, relerr, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

MODES = [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F32, dwf.DWF_SOLVE_MIXED_F16, dwf.DWF_SOLVE_MIXED_BF16]


@pytest.fixture(scope="module")
def c1():
    w = synth.WORKLOADS["4^4x8_periodic"]
    print("\n[case 4^4x8 periodic]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    b = c.full(w.source_seeds[0])
    xo, it, res = oracle.cgne(c.P, c.Ud, b, w.tol)
    yield c, b, xo, it, w.tol
    c.close()


@pytest.mark.parametrize("mode", MODES)
def test_cg_4x4x4x4_ls8(c1, mode):
    c, b, x_or, it_or, tol = c1
    x = torch().zeros_like(to_gpu(b))
    status, st = dwf.dwf_cg(c.ctx, to_gpu(b), x, tol=tol, mode=mode)
    assert status == dwf.DWF_OK and st["converged"] == 1
    assert st["res_normal"] <= tol * 1.0000001
    xg = to_host(x)
    # the true residual of the full system, recomputed by the oracle
    r = b - oracle.d5(c.P, c.Ud, xg)
    res_full = np.linalg.norm(r) / np.linalg.norm(b)
    assert abs(res_full - st["res_full"]) < 1e-3 * res_full + 1e-14
    assert relerr(xg, x_or) < 1e-6
    if mode == dwf.DWF_SOLVE_F64:
        assert abs(st["iters"] - it_or) <= 2
    else:
        assert st["reliable_updates"] >= 1


def test_cg_guess_is_used(c1):
    c, b, x_or, it_or, tol = c1
    x = to_gpu(x_or)
    status, st = dwf.dwf_cg(c.ctx, to_gpu(b), x, tol=1e-9, x0_is_guess=True)
    assert status == dwf.DWF_OK and st["iters"] <= 2


def test_cg_maxit_reports_noconv(c1):
    c, b, x_or, it_or, tol = c1
    x = torch().zeros_like(to_gpu(b))
    status, st = dwf.dwf_cg(c.ctx, to_gpu(b), x, tol=tol, maxit=5)
    assert status == dwf.DWF_ENOCONV and st["converged"] == 0 and st["iters"] == 5


@pytest.mark.parametrize("mode", [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F16])
def test_cg_16x16x16x16_ls12_dirichlet(mode):
    w = synth.WORKLOADS["16^4x12_dirichlet"]
    print(f"\n[16^4x12 dirichlet cg mode {mode}]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    try:
        b = c.full(w.source_seeds[0])
        x = torch().zeros_like(to_gpu(b))
        status, st = dwf.dwf_cg(c.ctx, to_gpu(b), x, tol=w.tol, mode=mode)
        print(st, flush=True)
        assert status == dwf.DWF_OK and st["res_normal"] <= w.tol * 1.0000001
        r = b - oracle.d5(c.P, c.Ud, to_host(x))
        res_full = np.linalg.norm(r) / np.linalg.norm(b)
        assert abs(res_full - st["res_full"]) < 1e-3 * res_full
        assert res_full < 1e-6
    finally:
        c.close()


@pytest.mark.parametrize("mode", [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F32])
def test_multishift_matches_oracle(c1, mode):
    c, b, x_or, it_or, tol = c1
    shifts = synth.rational_shifts()
    bs = [c.half(2010 + j) for j in range(2)]
    xs = [torch().zeros_like(to_gpu(bs[0])) for _ in range(len(bs) * len(shifts))]
    status, st = dwf.dwf_multishift_cg(c.ctx, [to_gpu(v) for v in bs], shifts, xs, tol=1e-8, mode=mode)
    assert status == dwf.DWF_OK
    for j, bj in enumerate(bs):
        xo, it, iters, res = oracle.multishift(c.P, c.Ud, bj, shifts, 1e-10)
        for k, s in enumerate(shifts):
            xg = to_host(xs[j * len(shifts) + k])
            ap = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, xg), True) + s * xg
            assert np.linalg.norm(bj - ap) / np.linalg.norm(bj) < 1.5e-8
            assert st[j * len(shifts) + k]["converged"] == 1
            assert relerr(xg, xo[k]) < 1e-5
