"""The benchmark's contract on the host: one GPU only, and the roofline's byte basis
(the z pass's floor in a three-pass convolution) following from the workload's
geometry.  The geometry is taken from the oracle's own plan, which derives GMF boxes
and transform sizes independently of the library's plan.  CPU only."""

import os
import subprocess
import sys

import pytest

import apm_workloads as W
from oracle import apm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

P = pytest.importorskip("paper_1410_0010_amd")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus 2" in r.stderr and r.stdout.strip() == ""


def oracle_floor(w, esize):
    """Read and write the gz My (Mx/2+1) complex intermediate, read the octant."""
    b = 0
    for g in O.OraclePlan(w.root_n, w.grids).grids:
        Mx, My, Mz = (int(v) for v in g.M)
        gz = int(g.gmf_n[2])
        b += 2 * gz * My * (Mx // 2 + 1) * 2 * esize
        b += (Mx // 2 + 1) * (My // 2 + 1) * (Mz // 2 + 1) * esize
    return b


@pytest.mark.parametrize("name", ["large_nested", "plummer_gas", "plummer_nested", "clumps"])
def test_pass_b_floor_follows_the_geometry(name):
    small = dict(large_nested=dict(npart=10, with_velocities=False),
                 plummer_gas=dict(npart=10), plummer_nested=dict(npart=10),
                 clumps=dict(per_clump=2))[name]
    w = {"large_nested": W.workload_large_nested, "plummer_gas": W.workload_plummer_gas,
         "plummer_nested": W.workload_plummer_nested, "clumps": W.workload_clumps}[name](**small)
    plan = P.Plan(w.root_n, w.grids, boundary=w.boundary)
    for esize in (4, 8):
        assert bench.pass_b_floor(plan, esize) == oracle_floor(w, esize)


def test_large_workload_floor_is_the_documented_figure():
    # root 512^3 (1024^3 doubled transform, 512 GMF planes) + three 256^3 levels
    # (512^3 transforms, 262 GMF planes): 6.70 GB per step in FP32, 3.351 GB per
    # launch (two launches per step, one per transform length)
    w = W.workload_large_nested(npart=10, with_velocities=False)
    b = oracle_floor(w, 4)
    assert abs(b / 2 - 3.351e9) < 0.001e9
