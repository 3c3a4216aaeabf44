"""GPU parity of the Chebyshev filter (dwf_chebyshev_filter) against the oracle's
recurrence, which the CPU tests pin to an eigendecomposition.

Tolerances: FP64 agrees to rounding (1e-11).  In a lower storage precision
every step rounds the new vector (unit roundoff u: FP32 6e-8, FP16 with site
scale 4.9e-4, BF16 3.9e-3); an error made at step j reaches step k through
the second-kind polynomial U_{k-j}, at most k - j + 1 in size on [-1, 1], so
after k steps the relative error is below (k + 1)(k + 2)/2 u.
"""
import numpy as np
import pytest

import oracle
from paper_2203_17119_amd import dwf
from gpu_helpers import Case, relerr, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

UNIT = {dwf.DWF_F64: 1e-13, dwf.DWF_F32: 6e-8, dwf.DWF_F16: 4.9e-4, dwf.DWF_BF16: 3.9e-3}
ORDERS = [0, 1, 2, 5, 8]


def bound(prec, k):
    return max(1e-11, 2.0 * (k + 1) * (k + 2) / 2 * UNIT[prec])


@pytest.fixture(scope="module", params=["4x2x2x4_ls8_dirichlet", "2x4x2x2_ls5"])
def case(request):
    print(f"\n[chebyshev case {request.param}]", flush=True)
    if request.param.endswith("ls8_dirichlet"):
        c = Case((4, 2, 2, 4), 8, mf=0.05, dirichlet=(1, 0, 0, 1), eps=0.5, seed=81)
    else:
        c = Case((2, 4, 2, 2), 5, mf=0.1, eps=0.5, seed=82)
    yield c
    c.close()


def spectrum_top(c, v):
    """upper bound of the spectrum of Mpc^+ Mpc from a few oracle power steps"""
    w = v / np.linalg.norm(v)
    for _ in range(30):
        w = oracle.mpc(c.P, c.Ud, oracle.mpc(c.P, c.Ud, w), True)
        lam = np.linalg.norm(w)
        w = w / lam
    return 1.1 * lam


@pytest.mark.parametrize("prec", [dwf.DWF_F64, dwf.DWF_F32, dwf.DWF_F16, dwf.DWF_BF16])
def test_chebyshev_matches_oracle(case, prec):
    v = case.half(83)
    hi = spectrum_top(case, v)
    lo = 0.02 * hi
    expect = oracle.chebyshev(case.P, case.Ud, v, lo, hi, ORDERS)
    outs = [torch().empty_like(to_gpu(v)) for _ in ORDERS]
    dwf.dwf_chebyshev_filter(case.ctx, to_gpu(v), lo, hi, ORDERS, outs, prec=prec)
    for k, o, e in zip(ORDERS, outs, expect):
        err = relerr(to_host(o), e)
        print(f"prec {prec} order {k}: relative error {err:.2e}", flush=True)
        assert err < bound(prec, k), (prec, k)


def test_chebyshev_single_orders_and_repeat_calls(case):
    """Order 0 alone is the input; a call for a single high order equals the same
    order taken from a longer list; and a second call on the same context gives
    the same bits (the workspace rotation starts afresh)."""
    v = case.half(84)
    hi = spectrum_top(case, v)
    g = to_gpu(v)
    o0 = torch().empty_like(g)
    dwf.dwf_chebyshev_filter(case.ctx, g, 0.0, hi, [0], [o0])
    assert relerr(to_host(o0), v) < 1e-15
    a = [torch().empty_like(g) for _ in range(3)]
    dwf.dwf_chebyshev_filter(case.ctx, g, 0.1 * hi, hi, [3, 6, 9], a)
    b = torch().empty_like(g)
    dwf.dwf_chebyshev_filter(case.ctx, g, 0.1 * hi, hi, [9], [b])
    assert torch().equal(a[2], b)
    c2 = [torch().empty_like(g) for _ in range(3)]
    dwf.dwf_chebyshev_filter(case.ctx, g, 0.1 * hi, hi, [3, 6, 9], c2)
    assert all(torch().equal(x, y) for x, y in zip(a, c2))


def test_chebyshev_argument_errors(case):
    """argument checks run before any device work"""
    g = to_gpu(case.half(85))
    o = torch().empty_like(g)
    for lo, hi, orders in [(1.0, 1.0, [1]), (-0.1, 1.0, [1]), (0.0, float("inf"), [1]), (0.0, 1.0, [2, 2]),
                           (0.0, 1.0, [3, 1]), (0.0, 1.0, [-1])]:
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_chebyshev_filter(case.ctx, g, lo, hi, orders, [o] * len(orders))
        assert e.value.status == dwf.DWF_EINVAL
    with pytest.raises(dwf.DWFError) as e:
        dwf.dwf_chebyshev_filter(case.ctx, g, 0.0, 1.0, list(range(65)), [o] * 65)
    assert e.value.status == dwf.DWF_EINVAL
