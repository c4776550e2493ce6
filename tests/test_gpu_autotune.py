"""The autotuner: every candidate gives identical bytes, the choice is
applied and cached per config class, and the tuned library stays exact."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import check, to_dev

pytestmark = pytest.mark.gpu


def test_autotune_small(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_1066_amd as fs
    from paper_1406_1066_amd import autotune
    monkeypatch.setenv("FSPARSE_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setenv("FSPARSE_TUNE_TABLE", "0")   # measure, not look up
    fs.set_tuning(reset=True)
    try:
        t = W.fem3d(20, 0.15, seed=5)
        ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
        r1 = autotune.tune(ii, jj, ss, t.m, t.n, reps=2)
        assert not r1["cached"]
        # every stage's candidates, less the launches already timed
        first = len({autotune._effective(dict(autotune.START, **c))
                     for c in autotune._candidates(autotune.STAGES[0])})
        nfresh = len(r1["times_ms"]) - len(autotune.REUSE_BLOCKS)
        assert first <= nfresh <= first + sum(
            len(v) for st in autotune.STAGES[1:] for v in st.values())
        assert json.dumps({k: v for k, v in r1["best"].items()
                           if k != "reuse_block"}, sort_keys=True) \
            in r1["times_ms"]
        cur = fs.get_tuning()
        for k, v in r1["best"].items():
            if k == "slot_values":
                assert cur[k] == fs.api.SLOT_VALUES[v]
            elif k != "bin_mode":
                assert cur[k] == v
        d = json.load(open(tmp_path / "tune.json"))
        assert r1["key"] in d
        r2 = autotune.tune(ii, jj, ss, t.m, t.n)
        assert r2["cached"] and r2["best"] == r1["best"]
        check(fs, t.ii, t.jj, t.ss, t.m, t.n)
        b = W.batched_fem2d(4, 1e3, 2e4, seed=3)
        bi, bj, bs, bm, bn = b.concat()
        r3 = autotune.tune(to_dev(bi), to_dev(bj), to_dev(bs), list(bm),
                           list(bn), trip_off=b.trip_off, reps=1)
        assert r3["key"] != r1["key"]
    finally:
        fs.set_tuning(reset=True)
