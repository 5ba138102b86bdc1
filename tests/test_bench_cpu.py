"""Host logic of bench.py: the launch planner and the argument handling the benchmark is run
with (no GPU)."""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("count,chunk,want", [
    (20, 100, [20]),
    (5, 100, [5]),
    (2000, 100, [100] * 20),
    (7, 3, [3, 3, 1]),
    (0, 100, []),
    (100, 100, [100]),
])
def test_plan_launches(count, chunk, want):
    got = bench.plan_launches(count, chunk)
    assert got == want
    assert sum(got) == count and all(1 <= c <= chunk for c in got)


def test_plan_launches_rejects_bad_chunk():
    with pytest.raises(ValueError):
        bench.plan_launches(10, 0)


@pytest.mark.parametrize("argv", [["--gpus", "1", "--steps", "20", "--warmup", "5"], [],
                                  ["--steps", "7", "--warmup", "3", "--chunk", "3"]])
def test_parse_accepts_driver_arguments(argv, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
    a = bench.parse()
    assert a.gpus == 1 and a.steps >= 1 and a.warmup >= 0
    # the planner covers both regions exactly, whatever the chunk
    assert sum(bench.plan_launches(a.steps, a.chunk)) == a.steps
    assert sum(bench.plan_launches(a.warmup, a.chunk)) == a.warmup


def test_more_than_one_gpu_exits_with_message(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
