"""Pins of the oracle's water-level and open boundaries (the boundary kinds of
the paper's benchmark tests, Sec. 3: a water-level hydrograph at the west
boundary in Sec. 3.1.1), against exact solutions.

* a level boundary at the level of a lake at rest over a bumpy bed leaves it
  at rest (well balanced);
* a level boundary at depth h_b feeding a dry flat channel holds the
  critical state there: the depth converges to Ritter's dam-break fan of a
  reservoir of depth 9/4 h_b (whose depth at x = 0 is 4/9 of it);
* a subcritical level rise enters a lake as the exact solution of the
  Riemann problem between the boundary state and the lake: a bore, with a
  left wave of only third order in the jump (the invariant is a rarefaction
  relation), so the level just inside is the prescribed one to 3e-4 m;
* open boundaries let Stoker's dam-break waves leave a truncated domain: the
  depth converges to the exact infinite-domain solution;
* a uniform flow passes through open boundaries unchanged;
* water entering through a level boundary brings no tangential motion: in a
  lake drifting along the boundary, the tangential discharge converges to
  the exact solution, where the tangential velocity is a passive tracer,
  zero behind the contact;
* water leaving through a level boundary keeps its tangential velocity: an
  oblique stream at the prescribed level leaves unchanged.
"""
import math

import numpy as np
import torch

from oracle import dg2_oracle as O
from paper_2010_02003_amd import workloads as WL

from exact_riemann import exact_riemann, ritter

G = 9.81
F64 = torch.float64


def test_level_boundary_at_the_lake_level_keeps_the_lake_at_rest():
    sc = WL.dambreak_bump(nx=24, ny=20)
    U = O.initial_state(sc.Z, np.full_like(sc.Z, 1.0), True)
    bed = O.bed_from_corners(sc.Z)
    lev = [O.LevelBC(O.WEST, 3, 15, torch.tensor([0.0, 100.0], dtype=F64),
                     torch.tensor([1.0, 1.0], dtype=F64)),
           O.LevelBC(O.NORTH, 0, 23, torch.tensor([0.0], dtype=F64), torch.tensor([1.0], dtype=F64))]
    prm = O.Params(nx=24, ny=20, dx=1.0, dy=1.0, manning=0.03, levels=lev)
    assert float(O.spatial_operator(U, bed, prm, 0.0).abs().max()) < 1e-13
    r = O.run(U, bed, prm, steps=100)
    assert float(r.U[1:].abs().max()) < 1e-12


def _ritter_l1(nx, T=5.0, L=100.0, hb=0.4):
    dx = L / nx
    X, _ = WL.corner_xy(nx, 2, dx, dx)
    Z = np.zeros_like(X)
    U = O.initial_state(Z, np.zeros_like(Z), False)
    lev = [O.LevelBC(O.WEST, 0, 1, torch.tensor([0.0], dtype=F64), torch.tensor([hb], dtype=F64))]
    prm = O.Params(nx=nx, ny=2, dx=dx, dy=dx, cfl=0.3, levels=lev, dt_max=0.05)
    r = O.run(U, O.bed_from_corners(Z), prm, t_end=T)
    sub = 32
    xf = (np.arange(nx * sub) + 0.5) * dx / sub
    he, _ = ritter(2.25 * hb, xf / T)
    exact = he.reshape(nx, sub).mean(axis=1)
    h = r.U[0, 0, 0].numpy()
    return np.abs(h - exact).mean(), h, exact


def test_level_boundary_feeds_the_exact_ritter_fan():
    e1, h1, ex1 = _ritter_l1(100)
    e2, _, _ = _ritter_l1(200)
    e3, _, _ = _ritter_l1(400)
    assert e1 < 1e-2
    assert e2 < 0.7 * e1 and e3 < 0.7 * e2
    # the first cell follows the fan's critical state at the boundary
    assert abs(h1[0] - ex1[0]) < 1e-2 and abs(ex1[0] - 0.4) < 2e-2


def _bore_l1(nx, T=6.0, L=100.0, h0=1.0, hb=1.2):
    """Lake of depth h0 at rest, level hb > h0 imposed at x = 0: the exact
    solution is a single right-going bore from the boundary state (hb, ub),
    ub on the invariant u - 2c of the lake, into the lake."""
    dx = L / nx
    X, _ = WL.corner_xy(nx, 2, dx, dx)
    Z = np.zeros_like(X)
    U = O.initial_state(Z, np.full_like(Z, h0), False)
    lev = [O.LevelBC(O.WEST, 0, 1, torch.tensor([0.0], dtype=F64), torch.tensor([hb], dtype=F64))]
    prm = O.Params(nx=nx, ny=2, dx=dx, dy=dx, cfl=0.3, levels=lev)
    r = O.run(U, O.bed_from_corners(Z), prm, t_end=T)
    ub = 2.0 * (math.sqrt(G * hb) - math.sqrt(G * h0))
    sub = 32
    xf = (np.arange(nx * sub) + 0.5) * dx / sub
    he, ue, hs, us = exact_riemann(hb, ub, h0, 0.0, xf / T)
    exact = he.reshape(nx, sub).mean(axis=1)
    return np.abs(r.U[0, 0, 0].numpy() - exact).mean(), hs, us, ub


def test_level_boundary_drives_the_exact_bore_into_a_lake():
    e1, hs, us, ub = _bore_l1(100)
    e2, _, _, _ = _bore_l1(200)
    # the boundary state lies on the lake's outgoing invariant: the Riemann
    # problem between it and the lake is a bore and a weak left wave
    assert abs(hs - 1.2) < 5e-4 and abs(us - ub) < 2e-3
    assert e1 < 2e-3
    assert e2 < 0.8 * e1


def _open_stoker_l1(nx, T=8.0):
    x0, L = 30.0, 40.0
    dx = L / nx
    X, _ = WL.corner_xy(nx, 2, dx, dx, x0, 0.0)
    Z = np.zeros_like(X)
    U = O.initial_state(Z, np.where(X < 50.0, 1.0, 0.5), True)
    opens = [O.OpenBC(O.WEST, 0, 1), O.OpenBC(O.EAST, 0, 1)]
    prm = O.Params(nx=nx, ny=2, dx=dx, dy=dx, cfl=0.3, opens=opens, x0=x0)
    r = O.run(U, O.bed_from_corners(Z), prm, t_end=T)
    sub = 32
    xf = x0 + (np.arange(nx * sub) + 0.5) * dx / sub
    he, _, _, _ = exact_riemann(1.0, 0.0, 0.5, 0.0, (xf - 50.0) / T)
    exact = he.reshape(nx, sub).mean(axis=1)
    return np.abs(r.U[0, 0, 0].numpy() - exact).mean()


def test_open_boundaries_let_dam_break_waves_leave():
    """Domain [30, 70] m, dam at 50 m, t = 8 s: the rarefaction head (25 m) and
    the shock (73.7 m) have both left the domain through open boundaries."""
    e1 = _open_stoker_l1(80)
    e2 = _open_stoker_l1(160)
    assert e1 < 6e-3
    assert e2 < 0.75 * e1


def test_uniform_flow_passes_through_open_boundaries():
    nx, ny = 12, 5
    X, _ = WL.corner_xy(nx, ny, 1.0, 1.0)
    Z = np.zeros_like(X)
    h, u, v = 0.8, 0.6, -0.3
    U = O.initial_state(Z, np.full_like(Z, h), False, qx=np.full_like(Z, h * u), qy=np.full_like(Z, h * v))
    opens = [O.OpenBC(s, 0, (ny if s in (O.WEST, O.EAST) else nx) - 1) for s in range(4)]
    prm = O.Params(nx=nx, ny=ny, dx=1.0, dy=1.0, opens=opens)
    r = O.run(U, O.bed_from_corners(Z), prm, steps=50)
    assert float((r.U - U).abs().max()) < 1e-13


def _bore_with_current_l1(nx, T=20.0, L=100.0, h0=1.0, hb=1.5, v0=0.5):
    """A bore from a level rise entering a lake that drifts along the
    boundary at v0 (y-uniform, open north and south): water entering from
    the reservoir brings no tangential motion, so v is a passive tracer that
    is 0 behind the contact at the middle-state speed u* and v0 ahead of it."""
    dx = L / nx
    X, _ = WL.corner_xy(nx, 2, dx, dx)
    Z = np.zeros_like(X)
    U = O.initial_state(Z, np.full_like(Z, h0), False, qy=np.full_like(Z, h0 * v0))
    lev = [O.LevelBC(O.WEST, 0, 1, torch.tensor([0.0], dtype=F64), torch.tensor([hb], dtype=F64))]
    opens = [O.OpenBC(O.SOUTH, 0, nx - 1), O.OpenBC(O.NORTH, 0, nx - 1)]
    prm = O.Params(nx=nx, ny=2, dx=dx, dy=dx, cfl=0.3, levels=lev, opens=opens)
    r = O.run(U, O.bed_from_corners(Z), prm, t_end=T)
    ub = 2.0 * (math.sqrt(G * hb) - math.sqrt(G * h0))
    sub = 32
    xf = (np.arange(nx * sub) + 0.5) * dx / sub
    he, _, _, us = exact_riemann(hb, ub, h0, 0.0, xf / T)
    qy = np.where(xf / T < us, 0.0, he * v0).reshape(nx, sub).mean(axis=1)
    got = r.U[2, 0].numpy()
    assert np.allclose(got[0], got[1], rtol=0, atol=1e-13)  # stays y-uniform
    return np.abs(got[0] - qy).mean(), us


def test_level_boundary_inflow_brings_no_tangential_motion():
    e1, us = _bore_with_current_l1(100)
    e2, _ = _bore_with_current_l1(200)
    # the contact has moved u* T = 28 m into the domain: water behind it is
    # at rest along y; a ghost carrying the lake's v0 would leave qy ~ h v0
    # (0.75) there, an L1 error near 0.2.  HLL smears the contact, so the
    # error falls at about half order.
    assert us * 20.0 > 20.0
    assert e1 < 1e-2
    assert e2 < 0.85 * e1


def test_oblique_flow_leaves_through_a_level_boundary_unchanged():
    """Water leaving through a level boundary keeps its own tangential
    velocity: a uniform subcritical oblique stream at the prescribed level
    leaves through it with no change."""
    nx, ny = 12, 5
    X, _ = WL.corner_xy(nx, ny, 1.0, 1.0)
    Z = np.zeros_like(X)
    h, u, v = 0.8, -0.6, 0.4
    U = O.initial_state(Z, np.full_like(Z, h), False, qx=np.full_like(Z, h * u), qy=np.full_like(Z, h * v))
    lev = [O.LevelBC(O.WEST, 0, ny - 1, torch.tensor([0.0], dtype=F64), torch.tensor([h], dtype=F64))]
    opens = [O.OpenBC(O.EAST, 0, ny - 1), O.OpenBC(O.SOUTH, 0, nx - 1), O.OpenBC(O.NORTH, 0, nx - 1)]
    prm = O.Params(nx=nx, ny=ny, dx=1.0, dy=1.0, levels=lev, opens=opens)
    r = O.run(U, O.bed_from_corners(Z), prm, steps=50)
    assert float((r.U - U).abs().max()) < 1e-13
