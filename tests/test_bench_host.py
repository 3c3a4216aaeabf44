"""Host logic of the benchmark: the counter traffic it reports, and the
autotuner record it applies.  No GPU needed."""
import json
import os

import pytest

import bench


def test_traffic_reported_only_for_the_profiled_sources_and_schedule(tmp_path, monkeypatch):
    # the committed summary matches the committed stencil sources in the schedule it names
    text = open(bench.TRAFFIC_SUMMARY).read()
    sched = None
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("tile_schedule:"):
            sched = tuple(int(v) for v in line.split(":", 1)[1].split())
    assert sched is not None, "the counter summary names its tile schedule"
    t = bench.measured_traffic(sched)
    assert t is not None and t > 0
    # another schedule: the counters do not describe its launches
    assert bench.measured_traffic((sched[0] + 1, sched[1])) is None
    # other kernel sources: no traffic either
    fake = tmp_path / "summary.md"
    fake.write_text(text.replace("source_sha256: ", "source_sha256: 0"))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(fake))
    assert bench.measured_traffic(sched) is None
    # no summary at all
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic(sched) is None


def test_tune_record_is_well_formed():
    """Every line of the autotuner's record is one JSON object with a key, a
    schedule within the launch limits (sites per workgroup x Ls <= 256) and
    a positive time."""
    assert os.path.exists(bench.TUNE_CACHE)
    keys = set()
    with open(bench.TUNE_CACHE) as f:
        for line in f:
            if not line.strip():
                continue
            e = json.loads(line)
            assert set(e) == {"key", "sb", "run", "ms"}
            parts = e["key"].split("/")
            arch, dims, ls, prec, dirichlet = parts[:5]
            # the batched (multi-shift) schedule carries the batch size
            assert len(parts) == 5 or (len(parts) == 6 and parts[5].startswith("batch") and int(parts[5][5:]) >= 1)
            L = [int(v) for v in dims.split("x")]
            Ls = int(ls[2:])
            assert len(L) == 4 and Ls >= 1 and prec[0] == "p" and dirichlet[0] == "d"
            assert 0 <= e["sb"] and e["sb"] * Ls <= 256
            assert 1 <= e["run"] <= 1 << 20
            assert e["ms"] > 0
            keys.add(e["key"])
    # the benchmark lattice at FP16 storage has a recorded pick
    assert any(k.split("/")[1:4] == ["32x32x32x32", "Ls12", "p2"] for k in keys)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_more_than_one_gpu_is_refused(n, capsys, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", str(n)])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
