"""GPU parity of the domain-boundary operators of the two-flavour boundary
action (Sec. 2.1): the link cut by a domain mask, D5 on full fields, the
projector P and the operators R and R^-1, against the oracle (pinned in
test_oracle_boundary.py), and the identities R R^-1 = P and D_dbar P = D_dbar
on the GPU at 8^4 x 8 and at the benchmark's 24^4 x 12 periodic split."""
import numpy as np
import pytest

import oracle
from oracle import Params
from paper_2203_17119_amd import dwf, synth
from gpu_helpers import relerr, to_gpu, to_host, torch
from helpers import coords

pytestmark = pytest.mark.gpu

B, C, M5, MF = 1.5, 0.5, 1.8, 0.1


def _mask_t(L, t_hi):
    return (coords(L)[:, 3] < t_hi).astype(np.int8)


def _mask_box(L, x_hi, t_hi):
    x = coords(L)
    return ((x[:, 0] < x_hi) & (x[:, 3] < t_hi)).astype(np.int8)


class BCase:
    """Full and cut contexts of one gauge field and domain mask."""

    def __init__(self, L, Ls, mask, seed, c=C):
        T = torch()
        self.L, self.Ls, self.mask = tuple(L), Ls, mask
        self.P = Params(L, Ls, B, c, M5, MF)
        self.U = synth.gauge_field(L, 0.5, seed)
        self.Uc = oracle.mask_cut(L, self.U, mask)
        self.mask_dev = T.from_numpy(mask.astype(np.int8)).cuda()
        self.full = dwf.Lattice(L, Ls, B, c, M5, MF, gauge=self.U)
        U_dev = to_gpu(self.U)
        self.Uc_dev = T.empty_like(U_dev)
        dwf.dwf_mask_links(self.full.ctx, self.mask_dev, U_dev, self.Uc_dev)
        self.cut = dwf.Lattice(L, Ls, B, c, M5, MF, gauge=self.Uc_dev)

    def field(self, seed):
        return synth.gaussian_fermion(self.L, self.Ls, seed)

    def close(self):
        self.full.close()
        self.cut.close()


SMALL = {
    "t_split": dict(L=(2, 2, 2, 4), Ls=4, mask=lambda L: _mask_t(L, 2), c=C),
    "xt_box": dict(L=(4, 2, 2, 6), Ls=2, mask=lambda L: _mask_box(L, 2, 3), c=C),
    # Shamir (c = 0): the projector is the orthogonal spin mask
    "t_split_shamir": dict(L=(2, 2, 2, 4), Ls=4, mask=lambda L: _mask_t(L, 2), c=0.0),
}


@pytest.fixture(scope="module", params=list(SMALL))
def small(request):
    cfg = SMALL[request.param]
    print(f"\n[boundary case {request.param}: {cfg['L']} ls{cfg['Ls']} c={cfg['c']}]", flush=True)
    c = BCase(cfg["L"], cfg["Ls"], cfg["mask"](cfg["L"]), seed=23, c=cfg["c"])
    yield request.param, c
    c.close()


def test_mask_links_matches_oracle(small):
    name, c = small
    got = to_host(c.Uc_dev)
    assert np.array_equal(got, c.Uc)
    assert (got == 0).sum() > 0


def test_d5_apply_matches_oracle(small):
    name, c = small
    for lat, U in ((c.full, c.U), (c.cut, c.Uc)):
        psi = c.field(31)
        out = torch().empty_like(to_gpu(psi))
        dwf.dwf_d5_apply(lat.ctx, to_gpu(psi), out)
        want = oracle.d5(c.P, U, psi)
        assert relerr(to_host(out), want) < 1e-13


def test_projector_matches_oracle(small):
    name, c = small
    psi = c.field(32)
    x = to_gpu(psi)
    out = torch().empty_like(x)
    dwf.dwf_boundary_project(c.full.ctx, c.mask_dev, x, out)
    want = oracle.boundary_projector(c.P, c.mask, psi)
    got = to_host(out)
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"{name}: |P psi - oracle| / max = {err:.2e}", flush=True)
    assert err < 1e-13
    # in place
    dwf.dwf_boundary_project(c.full.ctx, c.mask_dev, x, x)
    assert torch().equal(x, out)


@pytest.mark.parametrize("inverse", [False, True])
def test_r_matches_oracle(small, inverse):
    name, c = small
    psi = c.field(33)
    out = torch().empty_like(to_gpu(psi))
    s, st = dwf.dwf_boundary_apply(c.full.ctx, c.cut.ctx, c.mask_dev, to_gpu(psi), out, inverse=inverse,
                                   tol=1e-12, mode=dwf.DWF_SOLVE_F64)
    want = oracle.boundary_r(c.P, c.U, c.Uc, c.mask, psi, inverse=inverse)
    err = relerr(to_host(out), want)
    print(f"{name} {'R^-1' if inverse else 'R'}: rel err {err:.2e}, {st['iters']} CG iterations, "
          f"largest full residual {st['res_full']:.1e}", flush=True)
    assert s == dwf.DWF_OK and st["converged"] == 1
    assert err < 1e-8


def test_boundary_argument_errors(small):
    name, c = small
    T = torch()
    psi = to_gpu(c.field(34))
    out = T.empty_like(psi)
    for bad in (T.full_like(c.mask_dev, 1), T.zeros_like(c.mask_dev), c.mask_dev * 2):
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_boundary_project(c.full.ctx, bad, psi, out)
        assert e.value.status == dwf.DWF_EINVAL
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_boundary_apply(c.full.ctx, c.full.ctx, c.mask_dev, psi, out)
    assert e.value.status == dwf.DWF_EINVAL
    other = dwf.Lattice(c.L, c.Ls, B, c.P.c, M5, 2 * MF, gauge=c.Uc_dev)
    try:
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_boundary_apply(c.full.ctx, other.ctx, c.mask_dev, psi, out)
        assert e.value.status == dwf.DWF_EINVAL
    finally:
        other.close()
    shamir_b0 = dwf.Lattice(c.L, c.Ls, 0.0, 1.0, M5, MF, gauge=c.U)
    try:
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_boundary_project(shamir_b0.ctx, c.mask_dev, psi, out)
        assert e.value.status == dwf.DWF_ENOTSUP
    finally:
        shamir_b0.close()


def test_identities_8x8x8x8_ls8():
    """At 8^4 x 8 with Omega = {t < 4}: D_dbar P = D_dbar through the two
    contexts' D5, and R R^-1 = P, in FP64 and with mixed-precision solves."""
    print("\n[boundary 8x8x8x8 ls8, Omega = t < 4]", flush=True)
    L = (8, 8, 8, 8)
    c = BCase(L, 8, _mask_t(L, 4), seed=29)
    T = torch()
    try:
        psi = to_gpu(oracle.restrict(c.P, c.mask, c.field(35)))
        p = T.empty_like(psi)
        dwf.dwf_boundary_project(c.full.ctx, c.mask_dev, psi, p)

        def dbar(v):
            a, b = T.empty_like(v), T.empty_like(v)
            dwf.dwf_d5_apply(c.full.ctx, v, a)
            dwf.dwf_d5_apply(c.cut.ctx, v, b)
            return a - b

        want = dbar(psi)
        assert float((dbar(p) - want).norm() / want.norm()) < 1e-13
        for mode, tol, bound in ((dwf.DWF_SOLVE_F64, 1e-10, 1e-6), (dwf.DWF_SOLVE_MIXED_F16, 1e-10, 1e-6)):
            rinv = T.empty_like(psi)
            s1, st1 = dwf.dwf_boundary_apply(c.full.ctx, c.cut.ctx, c.mask_dev, psi, rinv, inverse=True, tol=tol,
                                             mode=mode)
            back = T.empty_like(psi)
            s2, st2 = dwf.dwf_boundary_apply(c.full.ctx, c.cut.ctx, c.mask_dev, rinv, back, tol=tol, mode=mode)
            err = float((back - p).norm() / p.norm())
            print(f"mode {mode}: |R R^-1 psi - P psi| / |P psi| = {err:.2e}; R^-1 {st1['iters']} iterations "
                  f"{st1['seconds']:.3f} s, R {st2['iters']} iterations {st2['seconds']:.3f} s", flush=True)
            assert s1 == dwf.DWF_OK and s2 == dwf.DWF_OK
            assert err < bound
    finally:
        c.close()


def test_boundary_apply_in_caller_workspace():
    """R^-1 with the full context's workspace carved from a torch buffer sized
    by dwf_workspace_bytes(DWF_OP_BOUNDARY): nothing allocated by the library
    on that context during the call, and the same result."""
    print("\n[boundary in caller workspace, 4x4x4x4 ls4]", flush=True)
    L = (4, 4, 4, 4)
    T = torch()
    ref_c, c = BCase(L, 4, _mask_t(L, 2), seed=37), BCase(L, 4, _mask_t(L, 2), seed=37)
    try:
        psi = to_gpu(c.field(38))
        want = T.empty_like(psi)
        dwf.dwf_boundary_apply(ref_c.full.ctx, ref_c.cut.ctx, ref_c.mask_dev, psi, want, inverse=True, tol=1e-10)
        # the cut context allocates its own buffers on first use; do that first
        got = T.empty_like(psi)
        dwf.dwf_boundary_apply(c.full.ctx, c.cut.ctx, c.mask_dev, psi, got, inverse=True, tol=1e-10, maxit=1)
        c.full.close()
        c.full = dwf.Lattice(L, 4, B, C, M5, MF, gauge=c.U)
        need = dwf.dwf_workspace_bytes(c.full.ctx, dwf.DWF_OP_BOUNDARY, dwf.DWF_SOLVE_F64)
        ws = T.empty(need, dtype=T.uint8, device="cuda")
        dwf.dwf_prepare_links(c.full.ctx, dwf.DWF_F64)
        dwf.dwf_set_workspace(c.full.ctx, ws)
        T.cuda.synchronize()
        before = T.cuda.mem_get_info()[0]
        s, st = dwf.dwf_boundary_apply(c.full.ctx, c.cut.ctx, c.mask_dev, psi, got, inverse=True, tol=1e-10)
        T.cuda.synchronize()
        after = T.cuda.mem_get_info()[0]
        used = dwf.dwf_workspace_used(c.full.ctx)
        print(f"need {need} B, used {used} B, free memory change {after - before} B", flush=True)
        assert s == dwf.DWF_OK and 0 < used <= need and after == before
        assert T.equal(got, want)
    finally:
        ref_c.close()
        c.close()


def test_boundary_24x24x24x24_ls12_periodic_split():
    """The benchmark's configuration: the 24^4 x 12 periodic lattice (mf 0.01,
    eps 0.7) split at t = 12, Omega = t < 12, solves in mixed FP16 storage to
    1e-8.  The cut links and the projector against the oracle on the whole
    lattice, D_dbar P = D_dbar through the two contexts' D5, and
    R R^-1 psi = P psi within 1e4 times the solves' tolerance, the ratio of
    the 8^4 x 8 test (three solves, each error amplified by the operators of
    the chain)."""
    w = synth.WORKLOADS["24^4x12_fgcr"]
    L = tuple(w.dims)
    print(f"\n[boundary {L} ls{w.Ls} periodic, Omega = t < {L[3] // 2}, mixed FP16 solves]", flush=True)
    T = torch()
    P = Params(L, w.Ls, w.b, w.c, w.M5, w.mf)
    U = synth.gauge_field(L, w.eps, w.gauge_seed)
    mask = _mask_t(L, L[3] // 2)
    mask_dev = T.from_numpy(mask).cuda()
    full = dwf.Lattice(L, w.Ls, w.b, w.c, w.M5, w.mf, w.dirichlet, gauge=U)
    cut = None
    try:
        U_dev = to_gpu(U)
        Uc_dev = T.empty_like(U_dev)
        dwf.dwf_mask_links(full.ctx, mask_dev, U_dev, Uc_dev)
        del U_dev
        assert np.array_equal(to_host(Uc_dev), oracle.mask_cut(L, U, mask))
        cut = dwf.Lattice(L, w.Ls, w.b, w.c, w.M5, w.mf, w.dirichlet, gauge=Uc_dev)
        del Uc_dev, U
        psi_h = synth.gaussian_fermion(L, w.Ls, w.source_seeds[0])
        psi = to_gpu(psi_h)
        p = T.empty_like(psi)
        dwf.dwf_boundary_project(full.ctx, mask_dev, psi, p)
        want = oracle.boundary_projector(P, mask, psi_h)
        err = float(np.abs(to_host(p) - want).max() / np.abs(want).max())
        print(f"|P psi - oracle| / max = {err:.2e}", flush=True)
        assert err < 1e-13
        del want, psi_h
        a, b = T.empty_like(psi), T.empty_like(psi)
        keep = T.from_numpy(mask.astype(np.float64)).cuda().reshape(-1, 1, 1, 1)

        def dbar(v):
            dwf.dwf_d5_apply(full.ctx, v, a)
            dwf.dwf_d5_apply(cut.ctx, v, b)
            return a - b

        on = psi * keep
        ref = dbar(on)
        e_dp = float((dbar(p) - ref).norm() / ref.norm())
        del on, ref, keep
        rinv, back = T.empty_like(psi), T.empty_like(psi)
        s1, st1 = dwf.dwf_boundary_apply(full.ctx, cut.ctx, mask_dev, psi, rinv, inverse=True, tol=w.tol,
                                         mode=dwf.DWF_SOLVE_MIXED_F16)
        s2, st2 = dwf.dwf_boundary_apply(full.ctx, cut.ctx, mask_dev, rinv, back, tol=w.tol,
                                         mode=dwf.DWF_SOLVE_MIXED_F16)
        err = float((back - p).norm() / p.norm())
        print(f"|D_dbar P psi - D_dbar psi| / |D_dbar psi| = {e_dp:.2e}; |R R^-1 psi - P psi| / |P psi| = "
              f"{err:.2e}; R^-1 {st1['iters']} iterations {st1['seconds']:.3f} s, R {st2['iters']} iterations "
              f"{st2['seconds']:.3f} s", flush=True)
        assert e_dp < 1e-13
        assert s1 == dwf.DWF_OK and s2 == dwf.DWF_OK
        assert err < 1e4 * w.tol
    finally:
        full.close()
        if cut is not None:
            cut.close()
