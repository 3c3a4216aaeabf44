"""GPU edge cases: degenerate inputs and parameters, argument errors that only
a live context can report, and run-to-run determinism of the solvers."""
import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf
from gpu_helpers import Case, relerr, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    print("\n[edge case 4^4x8]", flush=True)
    c = Case((4, 4, 4, 4), 8, mf=0.01, eps=0.4, seed=1001)
    yield c
    c.close()


@pytest.mark.parametrize("mode", [dwf.DWF_SOLVE_F64, dwf.DWF_SOLVE_MIXED_F16])
def test_zero_source_gives_zero_solution(c1, mode):
    b = torch().zeros(c1.P.full_shape(), dtype=torch().complex128, device="cuda")
    x = torch().ones_like(b)
    status, st = dwf.dwf_cg(c1.ctx, b, x, tol=1e-10, mode=mode)
    assert status == dwf.DWF_OK and st["converged"] == 1 and st["iters"] == 0
    assert float(x.abs().max()) == 0.0


def test_zero_source_fgcr_and_network(c1):
    b = torch().zeros(c1.P.full_shape(), dtype=torch().complex128, device="cuda")
    x = torch().ones_like(b)
    status, st = dwf.dwf_fgcr(c1.ctx, None, b, x, tol=1e-10, restart=8)
    assert status == dwf.DWF_OK and st["converged"] == 1
    assert float(x.abs().max()) == 0.0
    net = dwf.dwf_net_create(c1.ctx, [4, 8, 4])
    try:
        dwf.dwf_net_set_weights(net, np.ones(dwf.dwf_net_num_weights(net), dtype=np.complex64))
        z = torch().zeros(c1.P.half_shape(), dtype=torch().complex128, device="cuda")
        out = torch().ones_like(z)
        dwf.dwf_precond_apply(c1.ctx, net, z, out)
        assert float(out.abs().max()) == 0.0
    finally:
        dwf.dwf_net_destroy(net)


def test_shamir_ls1_is_wilson_and_solves():
    """b = 1, c = 0, Ls = 1: the red-black system of the Wilson operator."""
    c = Case((4, 2, 2, 4), 1, mf=0.2, eps=0.5, seed=71, b=1.0, c=0.0)
    try:
        x = c.half(72)
        out = torch().empty_like(to_gpu(x))
        for dagger in (0, 1):
            dwf.dwf_schur_apply(c.ctx, dagger, to_gpu(x), out)
            assert relerr(to_host(out), oracle.mpc(c.P, c.Ud, x, bool(dagger))) < 1e-12
        b = c.full(73)
        xs = torch().zeros_like(to_gpu(b))
        status, st = dwf.dwf_cg(c.ctx, to_gpu(b), xs, tol=1e-11)
        assert status == dwf.DWF_OK
        r = b - oracle.d5(c.P, c.Ud, to_host(xs))
        assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-9
    finally:
        c.close()


def test_all_faces_dirichlet_smallest_block():
    """2^4 block with all faces Dirichlet: in every direction half the links (those
    leaving through x_mu = 1) are zero, the other half connect the two layers."""
    c = Case((2, 2, 2, 2), 4, mf=0.05, dirichlet=(1, 1, 1, 1), eps=0.6, seed=74)
    try:
        x = c.half(75)
        out = torch().empty_like(to_gpu(x))
        for out_parity, dagger in [(1, 0), (0, 1)]:
            dwf.dwf_dhop(c.ctx, out_parity, dagger, to_gpu(x), out)
            assert relerr(to_host(out), c.oracle_dhop(x, out_parity, bool(dagger))) < 1e-12
        dwf.dwf_schur_apply(c.ctx, 0, to_gpu(x), out)
        assert relerr(to_host(out), oracle.mpc(c.P, c.Ud, x, False)) < 1e-12
    finally:
        c.close()


def test_mixed_cg_is_deterministic(c1):
    b = to_gpu(c1.full(76))
    xa = torch().zeros_like(b)
    xb = torch().zeros_like(b)
    _, sa = dwf.dwf_cg(c1.ctx, b, xa, tol=1e-9, mode=dwf.DWF_SOLVE_MIXED_F16)
    _, sb = dwf.dwf_cg(c1.ctx, b, xb, tol=1e-9, mode=dwf.DWF_SOLVE_MIXED_F16)
    assert sa["iters"] == sb["iters"] and sa["reliable_updates"] == sb["reliable_updates"]
    assert torch().equal(xa, xb)


def test_multishift_single_system_and_zero_shift(c1):
    b = c1.half(77)
    shifts = [0.0]
    xs = [torch().empty(c1.P.half_shape(), dtype=torch().complex128, device="cuda")]
    status, st = dwf.dwf_multishift_cg(c1.ctx, [to_gpu(b)], shifts, xs, tol=1e-9)
    assert status == dwf.DWF_OK and st[0]["converged"] == 1
    xg = to_host(xs[0])
    ap = oracle.mpc(c1.P, c1.Ud, oracle.mpc(c1.P, c1.Ud, xg), True)
    assert np.linalg.norm(b - ap) / np.linalg.norm(b) < 1.01e-9


def test_live_argument_errors(c1):
    b = to_gpu(c1.half(78))
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_multishift_cg(c1.ctx, [b] * 65, [0.1], [torch().empty_like(b) for _ in range(65)])
    assert e.value.status == dwf.DWF_EINVAL
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_multishift_cg(c1.ctx, [b], [-1.0], [torch().empty_like(b)])
    assert e.value.status == dwf.DWF_EINVAL
    full = torch().zeros(c1.P.full_shape(), dtype=torch().complex128, device="cuda")
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_fgcr(c1.ctx, None, full, torch().zeros_like(full), mode=dwf.DWF_SOLVE_MIXED_F16)
    assert e.value.status == dwf.DWF_ENOTSUP
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_net_create(c1.ctx, [4, 6, 4])
    assert e.value.status == dwf.DWF_ENOTSUP
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_set_tile_schedule(c1.ctx, dwf.DWF_K_STENCIL, 64, 1)  # 64 x Ls 8 > 256 lanes
    assert e.value.status == dwf.DWF_EINVAL
