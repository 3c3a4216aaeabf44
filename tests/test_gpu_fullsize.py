"""GPU parity at the full workload sizes, on outputs the oracle computes site by site.

* 32^4 x Ls=12 Dirichlet block (the benchmark lattice): the hop in FP64 and in
  the FP16 internal path with the autotuned schedule the benchmark uses,
  compared with the oracle at sampled sites; the mixed-precision CGNE solution
  checked by the oracle's D5 residual at sampled sites.
* 16^4 x Ls=12, 8 right-hand sides x 12 shifts: batched multi-shift CG in FP64
  and in FP32 storage with FP64 refinement, every (rhs, shift) converged, one
  pair per shift re-checked with the oracle's Mpc.
* 24^4 x Ls=12 periodic: FGCR with the trained network, its solution checked
  by the oracle's D5 residual at sampled sites.
* 32^4 x Ls=12: the committed trained networks with the matrix-core forward
  against the oracle's network on the whole lattice, and FGCR with each of
  them, its solution checked by the oracle's D5 at sampled sites.
* Chebyshev filter: every storage precision against the oracle on the whole
  16^4 x Ls=12 block; at 32^4 x Ls=12 its first orders and its three-term
  recurrence at the benchmark's orders, through the FP64 Schur operator.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf, synth
from gpu_helpers import SITE_TOL, TOL, Case, relerr, site_relerr, to_gpu, to_host, torch

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
    print(f"FP16 dhop at sampled sites: global {relerr(got, expect):.2e}, worst site {site_relerr(got, expect):.2e}",
          flush=True)
    assert relerr(got, expect) < 2e-3
    assert site_relerr(got, expect) < SITE_TOL[dwf.DWF_F16]
    # the other storage precisions, in the same schedule
    for prec in (dwf.DWF_F32, dwf.DWF_BF16):
        a, b = c.lat.internal(prec), c.lat.internal(prec)
        dwf.dwf_import(c.ctx, 0, prec, xg, a)
        dwf.dwf_dhop_internal(c.ctx, prec, 1, 0, a, b)
        dwf.dwf_export(c.ctx, 0, prec, b, out)
        del a, b
        got = out[torch().from_numpy(cbs).cuda()].cpu().numpy()
        print(f"prec {prec} dhop at sampled sites: global {relerr(got, expect):.2e}, "
              f"worst site {site_relerr(got, expect):.2e}", flush=True)
        assert relerr(got, expect) < TOL[prec]
        assert site_relerr(got, expect) < SITE_TOL[prec]


@pytest.mark.parametrize("src", range(4))
def test_mixed_cg_32x32x32x32_ls12_sampled_residual(c3, src):
    """Each of the workload's four sources, as the benchmark cycles them."""
    c, w = c3
    b = c.full(w.source_seeds[src])
    bg = to_gpu(b)
    x = torch().zeros_like(bg)
    dwf.dwf_tune(c.ctx, dwf.DWF_F16, tuned_cache())
    status, st = dwf.dwf_cg(c.ctx, bg, x, tol=w.tol, mode=dwf.DWF_SOLVE_MIXED_F16)
    print(st, flush=True)
    assert status == dwf.DWF_OK and st["res_normal"] <= w.tol * 1.0000001
    assert st["res_full"] < 1e-6
    xh = to_host(x)
    sites = np.random.default_rng(7 + src).choice(c.P.V, 2 * NSAMPLE, replace=False)
    r = b[sites] - oracle.d5_sites(c.P, c.Ud, xh, sites)
    # the sampled residual is an unbiased estimate of the full one
    ratio = np.linalg.norm(r) / np.linalg.norm(b[sites])
    assert ratio < 5 * st["res_full"] + 1e-10


@pytest.mark.parametrize("weights", ["ptc_4-4-4_8x8x8x8_ls8.npz", "ptc_4-12-12-12-4_8x8x8x8_ls8.npz"])
def test_network_32x32x32x32_ls12_matches_oracle(c3, weights):
    """The committed trained networks (the compact 4-4-4 one beats CG on this
    lattice) with the matrix-core forward (the launch configuration FGCR
    uses), against the oracle's network on the whole lattice.  Bound as for the small lattices
    (BF16 operands and activations: 2e-2 globally); every site's error is
    also bounded relative to the root-mean-square site norm, which catches
    a wrong tile, tail or Dirichlet face at any site without being fooled by
    sites whose exact output is small."""
    c, w = c3
    data = np.load(os.path.join(os.path.dirname(dwf.__file__), "weights", weights))
    chans = [int(v) for v in data["chans"]]
    flat = np.asarray(data["weights"])
    Ws, off = [], 0
    for l in range(len(chans) - 1):
        n = 11 * chans[l + 1] * chans[l]
        Ws.append(flat[off:off + n].reshape(11, chans[l + 1], chans[l]))
        off += n
    print(f"\n[32^4x12 network {chans}]", flush=True)
    net = dwf.dwf_net_create(c.ctx, chans)
    try:
        dwf.dwf_net_set_weights(net, flat)
        dwf.dwf_net_set_forward(net, dwf.DWF_NET_FWD_MFMA_BF16)
        x = c.half(77)
        out = torch().empty_like(to_gpu(x))
        dwf.dwf_precond_apply(c.ctx, net, to_gpu(x), out)
        got = to_host(out).reshape(-1, 12)
        want = oracle.net_apply(c.P, c.Ud, Ws, x).reshape(-1, 12)
        err = relerr(got, want)
        rms = np.sqrt(np.mean(np.sum(np.abs(want) ** 2, axis=1)))
        site = float(np.max(np.linalg.norm(got - want, axis=1)) / rms)
        print(f"relative error {err:.2e}, largest site error / rms site norm {site:.2e}", flush=True)
        assert err < 2e-2
        assert site < 0.1
    finally:
        dwf.dwf_net_destroy(net)


@pytest.mark.parametrize("weights", ["ptc_4-4-4_8x8x8x8_ls8.npz", "ptc_4-12-12-12-4_8x8x8x8_ls8.npz"])
def test_fgcr_learned_32x32x32x32_ls12_sampled_residual(c3, weights):
    """The benchmark's learned-preconditioner leg: FGCR(16) with a committed
    network, matrix-core forward, BF16 Krylov basis, on the first source, no
    CG fallback; it converges in the FP64 full residual, and its solution is
    checked by the oracle's D5 at sampled sites."""
    c, w = c3
    data = np.load(os.path.join(os.path.dirname(dwf.__file__), "weights", weights))
    print(f"\n[32^4x12 FGCR(16) + {weights}]", flush=True)
    net = dwf.dwf_net_create(c.ctx, [int(v) for v in data["chans"]])
    try:
        dwf.dwf_net_set_weights(net, data["weights"])
        dwf.dwf_net_set_forward(net, dwf.DWF_NET_FWD_MFMA_BF16)
        b = c.full(w.source_seeds[0])
        bg = to_gpu(b)
        x = torch().zeros_like(bg)
        dwf.dwf_tune(c.ctx, dwf.DWF_F16, tuned_cache())
        s, st = dwf.dwf_fgcr(c.ctx, net, bg, x, tol=w.tol, restart=16, maxit=2000, fallback=False,
                             mode=dwf.DWF_SOLVE_MIXED_BF16)
        print(f"status {s}: {st['iters']} steps {st['seconds']:.3f} s, full residual {st['res_full']:.2e}", flush=True)
        # FGCR stops on the Schur residual; the full one lands near it
        assert s == dwf.DWF_OK and st["fell_back"] == 0 and st["res_full"] <= 1.5 * w.tol
        xh = to_host(x)
        sites = np.random.default_rng(9).choice(c.P.V, 2 * NSAMPLE, replace=False)
        r = b[sites] - oracle.d5_sites(c.P, c.Ud, xh, sites)
        ratio = np.linalg.norm(r) / np.linalg.norm(b[sites])
        print(f"sampled oracle residual {ratio:.2e}", flush=True)
        assert ratio < 5 * st["res_full"] + 1e-10
    finally:
        dwf.dwf_net_destroy(net)


@pytest.mark.parametrize("mode", [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F32])
def test_batched_multishift_16x16x16x16_ls12(mode):
    """All 96 systems converge in the FP64 true residual (the library's own
    check); one system per shift, each with a different right-hand side, is
    re-checked with the oracle's Mpc (12 of 96).  The single-field and batched
    stencil launches run in the recorded tile schedules the benchmark applies."""
    w = synth.WORKLOADS["16^4x12_multishift"]
    print(f"\n[16^4x12 multishift 8 rhs x 12 shifts, mode {mode}]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    try:
        shifts = synth.rational_shifts()
        bs = [c.half(s) for s in w.source_seeds]
        xs = [torch().empty(c.P.half_shape(), dtype=torch().complex128, device="cuda")
              for _ in range(len(bs) * len(shifts))]
        prec = dwf.DWF_F32 if mode == dwf.DWF_SOLVE_MIXED_F32 else dwf.DWF_F64
        dwf.dwf_tune(c.ctx, prec, tuned_cache())
        dwf.dwf_tune_op(c.ctx, dwf.DWF_TUNE_BATCHED, prec, len(bs), tuned_cache())
        print(f"schedules: single {dwf.dwf_get_tile_schedule(c.ctx, dwf.DWF_K_STENCIL)}, batched "
              f"{dwf.dwf_get_tile_schedule(c.ctx, dwf.DWF_SCHED_STENCIL_BATCHED)}", flush=True)
        status, st = dwf.dwf_multishift_cg(c.ctx, [to_gpu(v) for v in bs], shifts, xs, tol=w.tol, mode=mode)
        print(f"status {status}, worst residual {max(s['res_normal'] for s in st):.2e}, "
              f"iterations {min(s['iters'] for s in st)}..{max(s['iters'] for s in st)}, "
              f"{st[0]['seconds']:.2f} s", flush=True)
        assert status == dwf.DWF_OK
        assert all(s["converged"] == 1 and s["res_normal"] <= w.tol * 1.0000001 for s in st)
        rng = np.random.default_rng(11)
        for k in range(len(shifts)):
            j = int(rng.integers(len(bs)))
            xg = to_host(xs[j * len(shifts) + k])
            ap = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, xg), True) + shifts[k] * xg
            res = np.linalg.norm(bs[j] - ap) / np.linalg.norm(bs[j])
            print(f"shift {shifts[k]:.2e} rhs {j}: oracle residual {res:.2e}", flush=True)
            assert res < 1.01 * w.tol
    finally:
        c.close()


def test_fgcr_learned_24x24x24x24_ls12_periodic():
    """The learned preconditioner's deployment lattice: FGCR(32) with the
    committed 4-12-12-12-4 network (trained on 8^4 x 8), matrix-core forward
    and BF16 Krylov basis, reaches 1e-8 in the FP64 full residual, checked by
    the oracle's D5 at sampled sites; plain FP64 CG on the same source is
    timed beside it (the comparison is reported, whatever its outcome)."""
    w = synth.WORKLOADS["24^4x12_fgcr"]
    path = os.path.join(os.path.dirname(dwf.__file__), "weights", "ptc_4-12-12-12-4_8x8x8x8_ls8.npz")
    data = np.load(path)
    print("\n[24^4x12 periodic, FGCR + trained network]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    net = dwf.dwf_net_create(c.ctx, [int(v) for v in data["chans"]])
    try:
        dwf.dwf_net_set_weights(net, data["weights"])
        dwf.dwf_net_set_forward(net, dwf.DWF_NET_FWD_MFMA_BF16)
        b = c.full(w.source_seeds[0])
        bg = to_gpu(b)
        x = torch().zeros_like(bg)
        s_cg, st_cg = dwf.dwf_cg(c.ctx, bg, x, tol=w.tol, mode=dwf.DWF_SOLVE_F64)
        assert s_cg == dwf.DWF_OK
        x.zero_()
        s1, st1 = dwf.dwf_fgcr(c.ctx, net, bg, x, tol=w.tol, restart=32, maxit=3000, fallback=False,
                               mode=dwf.DWF_SOLVE_MIXED_BF16)
        print(f"FP64 CG: {st_cg['iters']} iterations {st_cg['seconds']:.2f} s res {st_cg['res_full']:.2e}; "
              f"FGCR(32) + network: status {s1}, {st1['iters']} steps {st1['seconds']:.2f} s "
              f"res {st1['res_full']:.2e}", flush=True)
        # FGCR stops on the Schur residual; the full one lands near it
        assert s1 == dwf.DWF_OK and st1["fell_back"] == 0 and st1["res_full"] <= 1.5 * w.tol
        xh = to_host(x)
        sites = np.random.default_rng(8).choice(c.P.V, 2 * NSAMPLE, replace=False)
        r = b[sites] - oracle.d5_sites(c.P, c.U, xh, sites)
        ratio = np.linalg.norm(r) / np.linalg.norm(b[sites])
        print(f"sampled oracle residual {ratio:.2e}", flush=True)
        assert ratio < 5 * st1["res_full"] + 1e-10
    finally:
        dwf.dwf_net_destroy(net)
        c.close()


# unit roundoff of each storage precision (FP16 and BF16 relative to a site's scale)
UNIT = {dwf.DWF_F64: 1.1e-16, dwf.DWF_F32: 6e-8, dwf.DWF_F16: 4.9e-4, dwf.DWF_BF16: 3.9e-3}


def test_chebyshev_16x16x16x16_ls12_matches_oracle():
    """The Chebyshev filter (Sec. 2.4) in every storage precision on the
    16^4 x Ls=12 Dirichlet block, against the oracle's recurrence on the whole
    lattice.  hi is twice a four-step oracle power estimate of the top of
    A = Mpc^+ Mpc (an overestimate only widens the interval), lo = hi / 100.
    Bounds as on the small lattices: an error made at step j reaches step k
    through U_{k-j}, at most k - j + 1 on [-1, 1], so after k steps it is
    below (k + 1)(k + 2) u; the first two orders are also checked site by site
    (one application of A reads a site's 4-hop neighbourhood, hence 50 u)."""
    w = synth.WORKLOADS["16^4x12_dirichlet"]
    print("\n[16^4x12 dirichlet, Chebyshev filter against the oracle]", flush=True)
    c = Case(w.dims, w.Ls, mf=w.mf, dirichlet=w.dirichlet, eps=w.eps, seed=w.gauge_seed)
    try:
        v = c.half(2718)
        u = v / np.linalg.norm(v)
        for _ in range(4):
            u = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, u), True)
            lam = np.linalg.norm(u)
            u /= lam
        hi = 2.0 * lam
        lo = hi / 100
        orders = [0, 1, 2, 5, 8]
        want = oracle.chebyshev(c.P, c.Ud, v, lo, hi, orders)
        g = to_gpu(v)
        for prec in (dwf.DWF_F64, dwf.DWF_F32, dwf.DWF_F16, dwf.DWF_BF16):
            outs = [torch().empty_like(g) for _ in orders]
            dwf.dwf_chebyshev_filter(c.ctx, g, lo, hi, orders, outs, prec=prec)
            for k, o, e in zip(orders, outs, want):
                got = to_host(o)
                err, serr = relerr(got, e), site_relerr(got, e)
                print(f"prec {prec} order {k}: relative error {err:.2e}, worst site {serr:.2e}", flush=True)
                assert err < max(1e-11, (k + 1) * (k + 2) * UNIT[prec]), (prec, k)
                if k <= 1:
                    assert serr < max(1e-10, 50 * UNIT[prec]), (prec, k)
    finally:
        c.close()


@pytest.mark.parametrize("prec", [dwf.DWF_F64, dwf.DWF_F16])
def test_chebyshev_32x32x32x32_ls12_recurrence(c3, prec):
    """At 32^4 x Ls=12, where the oracle's recurrence takes minutes, the
    filter's outputs at the benchmark's orders and their neighbours are
    checked by what holds at any size: T_0 v = v, T_1 v = x(A) v and
    T_{k+1} v + T_{k-1} v = 2 x(A) T_k v, with x(A) = (2 A - (hi + lo)) /
    (hi - lo) applied in FP64 by the Schur operator (whose hop is checked
    against the oracle at sampled sites above).  The filter rounds each new
    vector once, and inside x(A) the stored Mpc w and A w, each scaled by
    2 / (hi - lo) against |A| <= hi: a step's residual is below about 9 u of
    the largest of its three vectors; the bound is 12 u (1e-12 in FP64)."""
    c, w = c3
    T = torch()
    print(f"\n[32^4x12 Chebyshev filter recurrence, prec {prec}]", flush=True)
    v = to_gpu(c.half(4242))

    def A(x):
        t, y = T.empty_like(x), T.empty_like(x)
        dwf.dwf_schur_apply(c.ctx, 0, x, t)
        dwf.dwf_schur_apply(c.ctx, 1, t, y)
        return y

    u = v / v.norm()
    for _ in range(20):
        u = A(u)
        lam = float(u.norm())
        u /= lam
    del u
    hi = 1.1 * lam
    lo = hi / 100
    a, sh = 2.0 / (hi - lo), -(hi + lo) / (hi - lo)
    orders = [0, 1, 7, 8, 9, 31, 32, 33]
    outs = [T.empty_like(v) for _ in orders]
    dwf.dwf_tune(c.ctx, dwf.DWF_F16, tuned_cache())
    dwf.dwf_chebyshev_filter(c.ctx, v, lo, hi, orders, outs, prec=prec)
    T.cuda.synchronize()
    bound = max(1e-12, 12 * UNIT[prec])
    out = dict(zip(orders, outs))
    e0 = float((out[0] - v).norm() / v.norm())
    x1 = a * A(v) + sh * v
    e1 = float((out[1] - x1).norm() / x1.norm())
    d = (out[1] - x1).reshape(-1, 12).norm(dim=1)
    n = x1.reshape(-1, 12).norm(dim=1)
    keep = n > 1e-6 * n.max()
    s1 = float((d[keep] / n[keep]).max())
    del x1, d, n, keep
    print(f"T_0 v - v: {e0:.2e}; T_1 v - x(A) v: {e1:.2e}, worst site {s1:.2e}", flush=True)
    assert e0 < UNIT[prec] + 1e-15 and e1 < bound and s1 < max(1e-10, 50 * UNIT[prec])
    for k in (8, 32):
        r = out[k + 1] + out[k - 1] - 2 * (a * A(out[k]) + sh * out[k])
        top = max(float(out[j].norm()) for j in (k - 1, k, k + 1))
        rel = float(r.norm()) / top
        print(f"order {k}: |T_(k+1) v + T_(k-1) v - 2 x(A) T_k v| / max norm = {rel:.2e} "
              f"(|T_k v| / |v| = {float(out[k].norm() / v.norm()):.3f})", flush=True)
        assert rel < bound, k
