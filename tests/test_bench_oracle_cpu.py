"""The benchmark's staged oracle leg (bench.staged_oracle: the unchanged oracle
functions spread over worker processes, particle chunks and kz-plane ranges) gives
the values of the oracle's own single-process solve.  CPU only."""

import os
import sys

import numpy as np

import apm_workloads as W
from oracle import apm_oracle as O

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _small():
    return W.workload_large_nested(root_n=16, sub_n=8, nlevels=3, npart=3000,
                                   with_velocities=False)


def _reference(w):
    rd = lambda a: np.asarray(a, np.float32).astype(np.float64)
    plan = O.OraclePlan(w.root_n, w.grids)
    return plan, O.solve(plan, rd(w.x), rd(w.y), rd(w.z), rd(w.m))


def test_staged_oracle_samples_match_the_solve():
    w = _small()
    plan, ref = _reference(w)
    got = bench.staged_oracle(w, full=False, workers=3)
    for gi, (idx, vals) in got["gmf_samples"].items():
        assert np.allclose(vals, ref["gmf"][gi].reshape(-1)[idx], rtol=1e-12, atol=1e-12)
    for gi, (cells, vals) in got["own_samples"].items():
        assert np.allclose(vals, ref["short"][gi].reshape(-1, 4)[cells], rtol=1e-11,
                           atol=1e-11 * np.abs(ref["short"][gi]).max())
    for gi, mass in got["mass"].items():
        assert abs(mass - ref["mass"][gi]) <= 1e-12 * abs(ref["mass"][gi])


def test_staged_oracle_full_matches_the_solve():
    w = _small()
    plan, ref = _reference(w)
    got = bench.staged_oracle(w, full=True, workers=3)
    assert np.array_equal(got["owner"], ref["owner"])
    for gi in range(len(w.grids)):
        sc = np.abs(ref["field"][gi]).max()
        assert np.allclose(got["gmf"][gi], ref["gmf"][gi], rtol=1e-12, atol=1e-12)
        assert np.allclose(got["short"][gi], ref["short"][gi], rtol=1e-11, atol=1e-11 * sc)
        assert np.allclose(got["field"][gi], ref["field"][gi], rtol=1e-11, atol=1e-11 * sc)
    own = ref["owner"] >= 0
    assert np.allclose(got["acc"][own], ref["acc"][own], rtol=1e-11,
                       atol=1e-11 * np.abs(ref["acc"]).max())
    assert np.allclose(got["pot"][own], ref["pot"][own], rtol=1e-11,
                       atol=1e-11 * np.abs(ref["pot"]).max())
    # the bench's error table on the oracle's own values is zero to rounding
    fake = dict(gmf=got["gmf"], own=[got["short"][i] for i in range(len(w.grids))],
                field=[got["field"][i] for i in range(len(w.grids))], owner=got["owner"],
                acc=got["acc"], pot=got["pot"],
                mass=[sum(got["mass"][g.index] for g in plan.level_grids(l))
                      for l in range(plan.nlevels)])
    grids = [dict(level=g.level) for g in plan.grids]
    e = bench.staged_errors(got, fake, grids)
    assert e["owner_mismatches"] == 0
    assert max(v for k, v in e.items() if isinstance(v, float)) < 1e-14
