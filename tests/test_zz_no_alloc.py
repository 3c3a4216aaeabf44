"""The Schur operator without device allocation (dwf_schur_apply_internal_noalloc)
against the allocating entry point dwf_schur_apply_internal: the same kernels
on the same input, so the outputs agree bit for bit.  Two lattices in a row,
the second smaller, share the fixed scratch array; sizes beyond it and
precisions whose links are not prepared are refused."""
import numpy as np
import pytest

from paper_2203_17119_amd import dwf
from gpu_helpers import Case, to_gpu, torch

pytestmark = pytest.mark.gpu


def internal(case, prec, seed):
    T = torch()
    canon = to_gpu(case.half(seed))
    buf = T.empty(dwf.dwf_field_bytes(case.ctx, 0, prec), dtype=T.uint8, device="cuda")
    dwf.dwf_import(case.ctx, 0, prec, canon, buf)
    return buf


def both(case, prec, dagger, seed):
    T = torch()
    a = internal(case, prec, seed)
    ref = T.empty_like(a)
    out = T.full_like(a, 0x5A)  # stale bytes: the call must overwrite every byte it owns
    dwf.dwf_schur_apply_internal(case.ctx, prec, dagger, a, ref)
    dwf.dwf_schur_apply_internal_noalloc(case.ctx, prec, dagger, a, out)
    T.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("prec", [dwf.DWF_F64, dwf.DWF_F32, dwf.DWF_F16, dwf.DWF_BF16])
def test_noalloc_matches_allocating_entry_point_two_sizes(prec):
    print(f"\n[noalloc prec {prec}: 8x8x8x8 ls8 then 4x4x4x4 ls6]", flush=True)
    big = Case((8, 8, 8, 8), 8, mf=0.02, dirichlet=(1, 1, 1, 1), eps=0.7, seed=61)
    small = Case((4, 4, 4, 4), 6, mf=0.05, eps=0.5, seed=62)
    try:
        for case, seed in ((big, 1), (small, 2)):
            for dagger in (0, 1):
                ref, out = both(case, prec, dagger, seed + 10 * dagger)
                assert np.array_equal(ref, out), (case.dims, prec, dagger)
                assert np.any(ref != 0)
    finally:
        big.close()
        small.close()


def test_noalloc_refuses_oversize_and_unprepared_links():
    print("\n[noalloc refusals: 16x16x16x16 ls12 FP64, unprepared FP16 links]", flush=True)
    T = torch()
    big = Case((16, 16, 16, 16), 12, mf=0.01, dirichlet=(1, 1, 1, 1), eps=0.7, seed=63)
    try:
        n = dwf.dwf_field_bytes(big.ctx, 0, dwf.DWF_F64)
        assert 2 * n > 128 << 20
        a = T.zeros(n, dtype=T.uint8, device="cuda")
        b = T.zeros_like(a)
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_schur_apply_internal_noalloc(big.ctx, dwf.DWF_F64, 0, a, b)
        assert e.value.status == dwf.DWF_EINVAL and "too large" in str(e.value)
        # FP16 links are prepared on first use by the allocating entry points only
        n16 = dwf.dwf_field_bytes(big.ctx, 0, dwf.DWF_F16)
        a16 = T.zeros(n16, dtype=T.uint8, device="cuda")
        b16 = T.zeros_like(a16)
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_schur_apply_internal_noalloc(big.ctx, dwf.DWF_F16, 0, a16, b16)
        assert e.value.status == dwf.DWF_EINVAL and "not prepared" in str(e.value)
        # after an allocating call in FP16 the same lattice fits (two FP16 fields, 41 MB)
        dwf.dwf_schur_apply_internal(big.ctx, dwf.DWF_F16, 0, a16, b16)
        c16 = T.full_like(a16, 0x33)
        dwf.dwf_schur_apply_internal_noalloc(big.ctx, dwf.DWF_F16, 0, a16, c16)
        T.cuda.synchronize()
        assert T.equal(b16, c16)
    finally:
        big.close()
