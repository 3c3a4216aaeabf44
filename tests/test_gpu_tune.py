"""The autotuner's search path (no cache entry): it times candidate schedules,
applies and records the winner, and a second call reads the record.  The
single-field and the batched (multi-shift) schedules are tuned and recorded
apart, keyed by the operation and the batch size.  Results do not depend on
the schedule: operator outputs and multi-shift solutions are bit-identical
across schedules."""
import json

import numpy as np
import pytest

from paper_2203_17119_amd import dwf, synth
from gpu_helpers import Case, to_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    print("\n[tuner: 8x8x8x8 ls8 dirichlet]", flush=True)
    c = Case((8, 8, 8, 8), 8, mf=0.02, dirichlet=(1, 1, 1, 1), eps=0.7, seed=91)
    yield c
    c.close()


def read_cache(path):
    with open(path) as fh:
        return [json.loads(line) for line in fh if line.strip()]


def test_single_field_search_and_record(case, tmp_path):
    path = str(tmp_path / "tune.jsonl")
    x = to_gpu(case.half(92))
    before = torch().empty_like(x)
    dwf.dwf_schur_apply(case.ctx, 0, x, before)
    ms = dwf.dwf_tune_op(case.ctx, dwf.DWF_TUNE_NORMAL, dwf.DWF_F16, 1, path)
    rec = read_cache(path)
    # the record keeps six significant digits of the time
    assert len(rec) == 1 and rec[0]["key"].endswith("/p2/d1111") and rec[0]["ms"] == pytest.approx(ms, rel=1e-5)
    sched = dwf.dwf_get_tile_schedule(case.ctx, dwf.DWF_K_STENCIL)
    print(f"single-field pick {sched} in {ms:.4f} ms (record {rec[0]})", flush=True)
    assert sched[1] == rec[0]["run"] and (rec[0]["sb"] == 0 or sched[0] == rec[0]["sb"])
    # the recorded pick is read back without timing
    dwf.dwf_set_tile_schedule(case.ctx, dwf.DWF_K_STENCIL, 3, 1)
    assert dwf.dwf_tune(case.ctx, dwf.DWF_F16, path) == pytest.approx(ms, rel=1e-5)
    assert len(read_cache(path)) == 1
    after = torch().empty_like(x)
    dwf.dwf_schur_apply(case.ctx, 0, x, after)
    assert torch().equal(before, after)


def test_batched_search_and_record(case, tmp_path):
    path = str(tmp_path / "tune.jsonl")
    T = torch()
    shifts = synth.rational_shifts(4, 1e-2, 1.0)
    bs = [to_gpu(case.half(s)) for s in (93, 94, 95, 96)]

    def solve():
        xs = [T.empty_like(bs[0]) for _ in range(len(bs) * len(shifts))]
        s, _ = dwf.dwf_multishift_cg(case.ctx, bs, shifts, xs, tol=1e-9, mode=dwf.DWF_SOLVE_MIXED_F32)
        assert s == dwf.DWF_OK
        return xs

    dwf.dwf_set_tile_schedule(case.ctx, dwf.DWF_SCHED_STENCIL_BATCHED, 5, 1)
    ref = solve()
    single = dwf.dwf_get_tile_schedule(case.ctx, dwf.DWF_K_STENCIL)
    ms = dwf.dwf_tune_op(case.ctx, dwf.DWF_TUNE_BATCHED, dwf.DWF_F32, 4, path)
    rec = read_cache(path)
    assert len(rec) == 1 and rec[0]["key"].endswith("/p1/d1111/batch4")
    sched = dwf.dwf_get_tile_schedule(case.ctx, dwf.DWF_SCHED_STENCIL_BATCHED)
    print(f"batched pick {sched} in {ms:.4f} ms (record {rec[0]})", flush=True)
    assert dwf.dwf_get_tile_schedule(case.ctx, dwf.DWF_K_STENCIL) == single  # the single-field one is untouched
    got = solve()
    for a, b in zip(got, ref):
        assert T.equal(a, b)
    # another batch size is another record
    dwf.dwf_tune_op(case.ctx, dwf.DWF_TUNE_BATCHED, dwf.DWF_F32, 2, path)
    keys = [r["key"] for r in read_cache(path)]
    assert len(keys) == 2 and keys[1].endswith("/batch2")


def test_tune_argument_errors(case):
    for args in [(7, dwf.DWF_F32, 1), (dwf.DWF_TUNE_NORMAL, dwf.DWF_F32, 2), (dwf.DWF_TUNE_BATCHED, dwf.DWF_F32, 0),
                 (dwf.DWF_TUNE_BATCHED, 9, 2)]:
        with pytest.raises(dwf.DWFError) as e:
            dwf.dwf_tune_op(case.ctx, *args)
        assert e.value.status == dwf.DWF_EINVAL


def test_multishift_tile_schedule_options(case):
    """dwf_solver_opts.tile_sb / tile_run: a fixed batched schedule and an
    autotuned one (tile_sb = -1) give bit-identical multi-shift solutions."""
    T = torch()
    shifts = synth.rational_shifts(3, 1e-2, 1.0)
    bs = [to_gpu(case.half(s)) for s in (97, 98)]

    def solve(**kw):
        xs = [T.empty_like(bs[0]) for _ in range(len(bs) * len(shifts))]
        s, _ = dwf.dwf_multishift_cg(case.ctx, bs, shifts, xs, tol=1e-9, mode=dwf.DWF_SOLVE_F64, **kw)
        assert s == dwf.DWF_OK
        return xs

    a = solve(tile_sb=3, tile_run=2)
    assert dwf.dwf_get_tile_schedule(case.ctx, dwf.DWF_SCHED_STENCIL_BATCHED) == (3, 2)
    b = solve(tile_sb=-1)
    print(f"autotuned batched schedule {dwf.dwf_get_tile_schedule(case.ctx, dwf.DWF_SCHED_STENCIL_BATCHED)}",
          flush=True)
    for u, v in zip(a, b):
        assert T.equal(u, v)
    with pytest.raises(dwf.DWFError) as e:
        solve(tile_sb=40, tile_run=1)  # 40 sites x Ls 8 > 256 lanes
    assert e.value.status == dwf.DWF_EINVAL
