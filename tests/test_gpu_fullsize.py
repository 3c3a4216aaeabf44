"""GPU parity at the full workload sizes, on outputs the oracle computes site by site.

* 32^4 x Ls=12 Dirichlet block (the benchmark lattice): the hop in FP64 and in
  the FP16 internal path with the autotuned schedule the benchmark uses,
  compared with the oracle at sampled sites; the mixed-precision CGNE solution
  checked by the oracle's D5 residual at sampled sites.
* 16^4 x Ls=12, 8 right-hand sides x 12 shifts: batched multi-shift CG, every
  (rhs, shift) converged, sampled pairs re-checked with the oracle's Mpc.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf, synth
from gpu_helpers import Case, relerr, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

NSAMPLE = 64
# the autotuner's recorded choices, which the benchmark applies
TUNE_CACHE = os.path.join(os.path.dirname(dwf.__file__), "tune_cache.jsonl")


def tuned_cache():
    return TUNE_CACHE if os.path.exists(TUNE_CACHE) else None


@pytest.fixture(scope="module")
def c3():
    w = synth.WORKLOADS["32^4x12_dirichlet"]
    print("\n[32^4x12 dirichlet context]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    yield c, w
    c.close()


def _sample_sites(c, parity, seed):
    rng = np.random.default_rng(seed)
    cbs = rng.choice(c.P.V // 2, NSAMPLE, replace=False)
    n = 2 * cbs
    x = np.stack([(n // np.prod(c.dims[:mu], dtype=np.int64)) % c.dims[mu] for mu in range(4)], axis=1)
    n = np.where(x.sum(axis=1) % 2 == parity, n, n + 1)
    return cbs, n


def test_dhop_32x32x32x32_ls12_sampled(c3):
    c, w = c3
    x = c.half(3001)
    xf = oracle.embed(c.P, x, 0)  # input on even sites, output on odd
    cbs, sites = _sample_sites(c, 1, 5)
    expect = oracle.hop_sites(c.P, c.Ud, xf, sites)
    del xf
    xg = to_gpu(x)
    out = torch().empty_like(xg)
    dwf.dwf_dhop(c.ctx, 1, 0, xg, out)
    got = out[torch().from_numpy(cbs).cuda()].cpu().numpy()
    assert relerr(got, expect) < 1e-12
    # FP16 storage, FP32 arithmetic, in the benchmark's tuned schedule
    dwf.dwf_tune(c.ctx, dwf.DWF_F16, tuned_cache())
    a, b = c.lat.internal(dwf.DWF_F16), c.lat.internal(dwf.DWF_F16)
    dwf.dwf_import(c.ctx, 0, dwf.DWF_F16, xg, a)
    dwf.dwf_dhop_internal(c.ctx, dwf.DWF_F16, 1, 0, a, b)
    dwf.dwf_export(c.ctx, 0, dwf.DWF_F16, b, out)
    got = out[torch().from_numpy(cbs).cuda()].cpu().numpy()
    assert relerr(got, expect) < 2e-3


def test_mixed_cg_32x32x32x32_ls12_sampled_residual(c3):
    c, w = c3
    b = c.full(w.source_seeds[0])
    bg = to_gpu(b)
    x = torch().zeros_like(bg)
    dwf.dwf_tune(c.ctx, dwf.DWF_F16, tuned_cache())
    status, st = dwf.dwf_cg(c.ctx, bg, x, tol=w.tol, mode=dwf.DWF_SOLVE_MIXED_F16)
    print(st, flush=True)
    assert status == dwf.DWF_OK and st["res_normal"] <= w.tol * 1.0000001
    assert st["res_full"] < 1e-6
    xh = to_host(x)
    sites = np.random.default_rng(7).choice(c.P.V, 2 * NSAMPLE, replace=False)
    r = b[sites] - oracle.d5_sites(c.P, c.Ud, xh, sites)
    # the sampled residual is an unbiased estimate of the full one
    ratio = np.linalg.norm(r) / np.linalg.norm(b[sites])
    assert ratio < 5 * st["res_full"] + 1e-10


def test_batched_multishift_16x16x16x16_ls12():
    w = synth.WORKLOADS["16^4x12_multishift"]
    print("\n[16^4x12 multishift 8 rhs x 12 shifts]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    try:
        shifts = synth.rational_shifts()
        bs = [c.half(s) for s in w.source_seeds]
        xs = [torch().empty(c.P.half_shape(), dtype=torch().complex128, device="cuda")
              for _ in range(len(bs) * len(shifts))]
        status, st = dwf.dwf_multishift_cg(c.ctx, [to_gpu(v) for v in bs], shifts, xs, tol=w.tol,
                                           mode=dwf.DWF_SOLVE_F64)
        print(st[0], flush=True)
        assert status == dwf.DWF_OK
        assert all(s["converged"] == 1 and s["res_normal"] <= w.tol * 1.0000001 for s in st)
        rng = np.random.default_rng(11)
        for q in rng.choice(len(xs), 3, replace=False):
            j, k = divmod(int(q), len(shifts))
            xg = to_host(xs[q])
            ap = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, xg), True) + shifts[k] * xg
            assert np.linalg.norm(bs[j] - ap) / np.linalg.norm(bs[j]) < 1.01 * w.tol
    finally:
        c.close()
