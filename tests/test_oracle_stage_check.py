"""Pins of the oracle's stage-1 Courant check (an option, off by default).

Sec. 2.1.2 calls the DG2 operators depth-positivity preserving under the
Courant bound Cr = 0.3.  The step size comes from the state at the start of
the step; on the floodplain's carved channel banks (1 m bed steps across one
2 m cell) stage 1 gives a thin film tens of m/s, stage 2 then breaks the
bound and mean depths go negative.  The check repeats stage 1 with the step
the bound allows for its result.

* off (or with a fixed step size), the checked step is the plain step;
* on the inflow mouth of the floodplain the unchecked run goes negative
  (after about 350 steps with the paper's end-of-stage treatment, within 30
  with the optional partly-wet rule), the checked run never does over 600
  steps, and loses little time;
* every accepted step satisfies the bound on its own stage-1 result.
"""
import math

import numpy as np
import torch

from oracle import dg2_oracle as O
from paper_2010_02003_amd import workloads as WL


def _run(sc, steps):
    U, bed, prm = O.setup(sc)
    t, hmin, first, dts = 0.0, 0.0, None, []
    for n in range(steps):
        dt = O.time_step(U, prm, t)
        if prm.stage_check > 0:
            U, dt = O.step_checked(U, t, bed, prm, dt)
        else:
            U = O.step(U, t, bed, prm, dt)
        t += dt
        dts.append(dt)
        m = float(U[0, 0].min())
        if m < 0.0 and first is None:
            first = n
        hmin = min(hmin, m)
    return t, hmin, first, dts, U


def test_check_off_or_fixed_dt_is_the_plain_step():
    modes, Z = WL.random_modes(30, 20, seed=3, slope=1.2)
    U = O.from_planes(modes)
    bed = O.bed_from_corners(Z)
    for check, fixed in ((0, 0.0), (3, 2e-3)):
        prm = O.Params(nx=30, ny=20, dx=2.0, dy=1.5, manning=0.03, stage_check=check, fixed_dt=fixed)
        a = O.step(U, 0.0, bed, prm, 2e-3)
        b, dt = O.step_checked(U, 0.0, bed, prm, 2e-3)
        assert dt == 2e-3 and torch.equal(a, b)


def _mouth(check, flat):
    sc = WL.floodplain_mouth(stage_check=check)
    sc.partly_wet_flat = flat
    return sc


def test_check_keeps_mean_depths_positive_on_steep_banks():
    t0, h0, first0, _, _ = _run(_mouth(0, False), 600)
    t1, h1, first1, dts, _ = _run(_mouth(3, False), 600)
    assert first0 is not None and first0 < 500 and h0 < -1e-5
    assert first1 is None and h1 >= 0.0
    assert t1 > 0.95 * t0


def test_check_keeps_mean_depths_positive_with_the_partly_wet_option():
    t0, h0, first0, _, _ = _run(_mouth(0, True), 200)
    t1, h1, first1, dts, _ = _run(_mouth(3, True), 200)
    assert first0 is not None and first0 < 30 and h0 < -1e-3
    assert first1 is None and h1 >= 0.0
    assert t1 > 0.95 * t0


def _urban_corner(n, check):
    full = WL.urban(precision="fp64")
    return WL.Scenario(name="urban_corner", nx=n, ny=n, dx=full.dx, dy=full.dy,
                       Z=full.Z[:n + 1, :n + 1].copy(), surface=np.zeros((n + 1, n + 1)), is_eta=False,
                       manning=full.manning[:n, :n].copy(), cfl=full.cfl, dt_max=full.dt_max,
                       rain=full.rain, stage_check=check)


def test_check_keeps_the_urban_corner_non_negative():
    """The 96 x 96 corner of the urban workload (half of it building blocks
    raised 10 m across one 0.5 m cell), rain from dry: the plain step goes
    negative after about 400 steps, the checked step never does."""
    _, h0, first0, _, _ = _run(_urban_corner(96, 0), 800)
    _, h1, first1, _, _ = _run(_urban_corner(96, 3), 800)
    assert first0 is not None and h0 < 0.0
    assert first1 is None and h1 >= 0.0


def test_accepted_steps_keep_the_courant_bound_on_stage_one():
    sc = WL.floodplain_mouth(stage_check=3)
    U, bed, prm = O.setup(sc)
    t, checked = 0.0, 0
    for n in range(60):
        dt0 = O.time_step(U, prm, t)
        Un, dt = O.step_checked(U, t, bed, prm, dt0)
        assert dt <= dt0
        _, U1 = O._stage1(U, t, bed, prm, dt)
        lim = prm.cfl * O.cfl_min(U1, prm)
        if dt < dt0:
            checked += 1
        # three repeats were enough on every step of this run
        assert dt <= lim * (1.0 + 1e-12) or math.isinf(lim)
        U, t = Un, t + dt
    assert checked > 10
