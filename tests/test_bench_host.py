"""Host logic of the benchmark (no GPU): the refusal of more than one GPU, the rule that counter
figures are reported only for the kernel source and launch parameters they were taken with,
and the algorithmic byte counts."""

import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
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


def test_counter_figures_follow_source_and_params(monkeypatch):
    import hashlib

    b = _bench()
    src = "paper_2606_06511_amd/csrc/evaluate.hip"
    sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    table = {"screen": [{"bytes": 123, "valu_wave": 45, "sources": {src: sha}, "params": {"screen_blocks": 2048}},
                        {"bytes": 456, "valu_wave": 67, "sources": {src: "0" * 64}, "params": {}}]}
    monkeypatch.setattr(b, "MEASURED", table)
    # the committed source and the same launch parameter: the figure
    assert b.measured("screen", "bytes", {"screen_blocks": 2048, "row_blocks": 1}) == 123
    assert b.measured("screen", "valu_wave", {"screen_blocks": 2048}) == 45
    # another launch parameter, or a source that changed since: no figure
    assert b.measured("screen", "bytes", {"screen_blocks": 4096}) is None
    table["screen"][0]["sources"] = {src: "1" * 64}
    assert b.measured("screen", "bytes", {"screen_blocks": 2048}) is None
    assert b.measured("derivs", "bytes", {}) is None
    # every committed figure names sources that exist
    for entries in _bench().MEASURED.values():
        for e in entries:
            assert all(os.path.exists(os.path.join(ROOT, f)) for f in e["sources"])


@pytest.mark.parametrize("prec", [np.float32, np.float64])
def test_path_bytes_count_the_arrays(prec):
    """The path's algorithmic bytes are the sizes of the arrays one evaluation must read and
    write: the candidate list, triangles and positions in; every hit record out and back in;
    gradient, BSR values, column indices and row pointers, and the energy out."""
    b = _bench()
    nv, nt, P, H, nnzb = 1000, 1900, 5000, 37, 811
    s = np.dtype(prec).itemsize
    rec = np.dtype([("a", prec, 18), ("b", prec, 18), ("M", prec, 3), ("t", prec, 2), ("vid", np.int32, 6)])
    arrays_in = [np.zeros((P, 2), np.int32), np.zeros((nt, 3), np.int32), np.zeros((nv, 3), np.float64)]
    records = np.zeros(H, rec)
    arrays_out = [np.zeros((nv, 3), prec), np.zeros((nnzb, 3, 3), prec), np.zeros(nnzb, np.int32),
                  np.zeros(nv + 1, np.int32), np.zeros(1, np.float64)]
    want = sum(a.nbytes for a in arrays_in) + 2 * records.nbytes + sum(a.nbytes for a in arrays_out)
    assert b.path_bytes(nv, nt, P, H, nnzb, s) == want
    assert b.path_bytes(nv, nt, P, H, nnzb, s, flags=True) == want + np.zeros(P, np.uint8).nbytes
    # the screening stage reads the same inputs and writes each hit's geometry: pair key, pair
    # index, endpoint descriptor, the two interval ends and the six plane sides
    geom = np.dtype([("key", np.int64), ("pair", np.int32), ("desc", np.uint32), ("t", np.float64, 2),
                     ("da", np.float64, 3), ("db", np.float64, 3)])
    assert b.stage_bytes("screen", nv, nt, P, H, nnzb, s) == sum(a.nbytes for a in arrays_in) + H * geom.itemsize
