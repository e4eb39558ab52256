"""Pins of the oracle's subcycled evolution (evolve_subcycled, the recursive level
stepping of Sec. 2 with dt_{l+1} = dt_l / 2, Eq. 10) against what the paper and the
mathematics fix:

* one step size on every level reduces each step to a single consistent solve at
  the mid-step positions, so an isolated particle crossing the levels keeps its
  velocity to rounding (Sec. 3.1: about 1e-14 without subcycling);
* a particle at rest sees the same fields at every time, so subcycling adds no
  force to it either: the time interpolation of the parent's field must have weights
  that sum to one;
* the self-force particle moves along the diagonal of a geometry symmetric under
  permutations of the axes, so its velocity error is the same in all three
  directions (Sec. 3.1 calls it symmetric in all directions);
* its size is of the order 1e-4 over t = 0.4 (Sec. 3.1, Fig. 2) with the particle's
  mass read as density 1 on a root cell (1/4096): the paper gives no G and no units
  for this test, and with G m = 1 the coarse levels' share of the particle's own
  field, taken at other times, changes the velocity by order one.
"""

import numpy as np

import apm_workloads as W
from oracle import apm_oracle as O


def self_force(mass, pos=(0.15, 0.15, 0.15), vel=1.0):
    w = W.workload_self_force(pos)
    w.m = np.array([mass])
    w.vx, w.vy, w.vz = (np.full(1, vel) for _ in range(3))
    return w, O.OraclePlan(w.root_n, w.grids)


def test_equal_steps_keep_the_velocity_across_levels():
    w, plan = self_force(1.0)
    r = O.evolve_subcycled(plan, w.x, w.y, w.z, w.vx, w.vy, w.vz, w.m, 3e-3, 70, ratio=1)
    assert r["level"][0] == 2                       # crossed levels 1 and 2
    dv = np.abs(r["vel"][:, 0, :] - 1.0).max()
    assert dv <= 1e-13, dv


def test_particle_at_rest_feels_no_force_with_subcycling():
    w, plan = self_force(1.0, pos=(0.45, 0.5, 0.55), vel=0.0)
    r = O.evolve_subcycled(plan, w.x, w.y, w.z, w.vx, w.vy, w.vz, w.m, 0.025, 3, ratio=2)
    assert r["level"][0] == 3
    assert np.abs(r["vel"]).max() <= 1e-13
    assert np.abs(r["pos"][-1, 0] - np.array([0.45, 0.5, 0.55])).max() <= 1e-13


def test_subcycled_self_force_symmetric_and_of_the_papers_order():
    w, plan = self_force(1.0 / 4096)
    r = O.evolve_subcycled(plan, w.x, w.y, w.z, w.vx, w.vy, w.vz, w.m, 0.025, 16, ratio=2)
    d = r["vel"][:, 0, :] - 1.0
    assert np.abs(d - d.mean(axis=1, keepdims=True)).max() <= 1e-12 * np.abs(d).max()
    dv = np.linalg.norm(d, axis=1) / np.sqrt(3.0)
    assert r["level"][0] == 3
    assert 1e-5 <= dv.max() <= 1e-3, dv.max()
