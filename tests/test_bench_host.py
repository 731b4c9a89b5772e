"""Host logic of the benchmark (no GPU): the refusal of more than one GPU, the rule that counter
figures are reported only for the kernel source and launch parameters they were taken with,
and the algorithmic byte counts."""

import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == n and "one GPU" in line["error"]


def test_counter_figures_follow_source_and_params():
    b = _bench()
    entries = b.MEASURED["bp_traverse"]
    assert {tuple(sorted(e["params"].items())) for e in entries} == {(("trav_budget", 24),), (("trav_budget", 32),)}
    for e in entries:
        # the committed source is the one the figures were taken on
        assert b.measured("bp_traverse", "bytes", dict(e["params"], screen_blocks=1, row_blocks=1)) == e["bytes"]
        assert b.measured("bp_traverse", "valu_wave", e["params"]) == e["valu_wave"]
    # other launch parameters: no figure
    assert b.measured("bp_traverse", "bytes", {"trav_budget": 64}) is None
    # another source: no figure
    saved = [dict(e) for e in entries]
    try:
        for e in entries:
            e["sha256"] = "0" * 64
        assert b.measured("bp_traverse", "bytes", {"trav_budget": 24}) is None
    finally:
        b.MEASURED["bp_traverse"][:] = saved
    assert b.measured("screen", "bytes", {}) is None


def test_algorithmic_bytes():
    b = _bench()
    nv, nt, P, H, nnzb = 65_536, 130_050, 172_212, 498, 6_178
    # the traversal: every leaf record (64 B) and leaf box (32 B), the inner levels (~nt/3 boxes
    # of 32 B) and every pair written once (8 B)
    assert b.stage_bytes("bp_traverse", nv, nt, P, H, nnzb, 4) == 64 * nt + 32 * nt + 32 * nt // 3 + 8 * P
    # screening reads each pair, vertex and triangle once and writes the hit records
    assert b.stage_bytes("screen", nv, nt, P, H, nnzb, 4) == 8 * P + 24 * nv + 12 * nt + 80 * H
    # the assembly grows with the precision of the gradient and the Hessian blocks
    assert b.stage_bytes("assembly", nv, nt, P, H, nnzb, 8) > b.stage_bytes("assembly", nv, nt, P, H, nnzb, 4)
    assert b.stage_bytes("unknown", nv, nt, P, H, nnzb, 4) == 0
