"""The committed labelled training systems of the parameter predictor: each
record must be the system the config-5 recipe draws for its index, and its
times must satisfy what branch-and-bound labelling guarantees (§V-E, §V-F:
the label is the fastest combination by measured time to 1e-10)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LABELS = os.path.join(ROOT, "paper_2105_07544_amd", "predictor_data", "config5_train.jsonl")
NCOMBO = 4 * 5 * 2  # restart {25,50,100,200} x degree {0,5,10,25,40} x {float32 IR, float64}
FIXED = 1 * (5 * 2) + 0 * 2 + 0  # (m = 50, d = 0, float32) in restart-major, degree, precision order


@pytest.fixture(scope="module")
def recs():
    with open(LABELS) as fh:
        return [json.loads(line) for line in fh if line.strip()]


def test_records_are_contiguous_and_complete(recs):
    assert len(recs) >= 1920
    assert [r["index"] for r in recs] == list(range(len(recs)))
    for r in recs:
        assert len(r["features"]) == 16 and all(math.isfinite(f) for f in r["features"])
        for key in ("times", "bounds", "iters", "capped"):
            assert len(r[key]) == NCOMBO, (r["index"], key)


def test_branch_and_bound_invariants(recs):
    for r in recs:
        t = np.array([np.inf if v is None else v for v in r["times"]])
        best = t.min()
        assert np.isfinite(best) and best > 0.0, r["index"]
        b = np.array(r["bounds"])
        capped = np.array(r["capped"])
        # a combination has no time exactly when it was stopped, and it was
        # stopped only once it had spent more than the best time found
        assert np.array_equal(~np.isfinite(t), capped), r["index"]
        assert np.all(b[capped] > best), r["index"]
        # a finished combination's bound is its time
        assert np.allclose(b[~capped], t[~capped]), r["index"]
        # the fixed combination runs first, so it always has a time or a bound
        assert b[FIXED] > 0.0 and r["iters"][FIXED] > 0, r["index"]


def test_records_match_the_config5_recipe(recs):
    # every 61st system regenerated from its index: kind, grid side, n, nnz
    for r in recs[::61]:
        s = W.config5_systems(1, seed=5, start=r["index"])[0]
        assert (s["kind"], s["N"], s["A"].n, s["A"].nnz) == (r["kind"], r["N"], r["n"], r["nnz"]), r["index"]


def test_kind_and_side_distribution(recs):
    n = len(recs)
    kinds = {k: sum(r["kind"] == k for r in recs) for k in ("convdiff", "laplace2d", "laplace3d")}
    assert sum(kinds.values()) == n
    # half, a quarter and a quarter, within five binomial standard deviations
    for k, p in (("convdiff", 0.5), ("laplace2d", 0.25), ("laplace3d", 0.25)):
        assert abs(kinds[k] - p * n) <= 5 * math.sqrt(n * p * (1 - p)), kinds
    side2 = [r["N"] for r in recs if r["kind"] != "laplace3d"]
    side3 = [r["N"] for r in recs if r["kind"] == "laplace3d"]
    assert 64 <= min(side2) and max(side2) <= 1024
    assert 16 <= min(side3) and max(side3) <= 101
    # uniform sides: the means within five standard errors of the midpoints
    assert abs(np.mean(side2) - 544.0) <= 5 * 277.4 / math.sqrt(len(side2))
    assert abs(np.mean(side3) - 58.5) <= 5 * 24.8 / math.sqrt(len(side3))
