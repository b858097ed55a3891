"""Pins of two oracle parts that no other test fixes independently.

Courant step (Sec. 2.1.2 gives Cr = 0.3; which speeds enter is a reading: the
directional minimum over wet cell means).
The pin measures the Courant number that the chosen step realises from the
definition of the Courant number, with the wave speeds taken a different
way: as the spectral radius of the Jacobians dF/dU and dG/dU of the physical
fluxes of Eq. (1), differentiated numerically and passed to numpy's
eigenvalue routine.  On grids with dx != dy, in both orientations, with
velocities of both signs and a dry cell carrying a large discharge, the
largest Courant number over the wet cells must be exactly Cr, and the step
must be dt_max when nothing is wet.  A swapped dx/dy, a missing absolute
value on a velocity or a dry cell taken into account all fail it.

Discharge inflow (a reading, the paper gives no boundary treatment: face
flux [q, q^2/h_b + g h_b^2/2], h_b the larger of the inner dummy depth and
the critical depth (q^2/g)^(1/3)).
A constant discharge entering a dry, flat, frictionless channel has an
exact solution: the boundary state is critical, and the flow beyond it is
Ritter's dam-break fan of a reservoir of depth 9/4 times the critical depth
(whose depth at x = 0 is 4/9 of the reservoir's and whose velocity there is
the critical one).  The oracle's depth must converge to that fan; the same
run with a planted mistake in the momentum flux (the 1/2 dropped from the
pressure term, the square of q dropped from the critical depth, the
advective term dropped) must not.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dg2_oracle as O
from paper_2010_02003_amd import workloads as WL

from exact_riemann import ritter

G = 9.81
F64 = torch.float64


def _phys_flux(h, qx, qy, axis):
    """Physical flux of Eq. (1) in direction x (axis 0) or y (axis 1)."""
    if axis == 0:
        return np.array([qx, qx * qx / h + 0.5 * G * h * h, qx * qy / h])
    return np.array([qy, qx * qy / h, qy * qy / h + 0.5 * G * h * h])


def _spectral_radius(h, qx, qy, axis):
    U = np.array([h, qx, qy])
    J = np.empty((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-6 * max(1.0, abs(U[k]))
        J[:, k] = (_phys_flux(*(U + e), axis) - _phys_flux(*(U - e), axis)) / (2.0 * e[k])
    return float(np.abs(np.linalg.eigvals(J)).max())


def _state(ny, nx, seed):
    rng = np.random.default_rng(seed)
    U = torch.zeros((3, 3, ny, nx), dtype=F64)
    U[0, 0] = torch.tensor(rng.uniform(0.05, 2.0, (ny, nx)))
    U[1, 0] = torch.tensor(rng.uniform(-3.0, 3.0, (ny, nx))) * U[0, 0]
    U[2, 0] = torch.tensor(rng.uniform(-3.0, 3.0, (ny, nx))) * U[0, 0]
    U[:, 1:] = torch.tensor(rng.uniform(-0.02, 0.02, (3, 2, ny, nx)))  # slopes play no part
    U[0, 0, 1, 2] = 5e-6  # a dry cell with a large discharge: ignored
    U[1, 0, 1, 2] = -40.0
    U[2, 0, 1, 2] = 25.0
    return U


@pytest.mark.parametrize("dx,dy", [(2.0, 0.5), (0.5, 2.0), (1.0, 3.0)])
@pytest.mark.parametrize("seed", [1, 2])
def test_courant_step_realises_cr_with_jacobian_wave_speeds(dx, dy, seed):
    ny, nx = 5, 6
    U = _state(ny, nx, seed)
    prm = O.Params(nx=nx, ny=ny, dx=dx, dy=dy, cfl=0.3, dt_max=100.0)
    dt = O.time_step(U, prm, 0.0)
    cr = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            h, qx, qy = (float(U[v, 0, j, i]) for v in range(3))
            if h <= prm.tol:
                continue
            cr[j, i] = dt * max(_spectral_radius(h, qx, qy, 0) / dx, _spectral_radius(h, qx, qy, 1) / dy)
    assert abs(cr.max() - 0.3) <= 1e-9
    assert np.all(cr <= 0.3 * (1.0 + 1e-9))


def test_courant_step_direction_decides_which_cell_is_fastest():
    """Two wet cells: one fast in x, one fast in y.  On a grid long in x the
    y-fast cell sets the step, on a grid long in y the x-fast cell does; a
    swapped dx/dy picks the other cell and a different step."""
    U = torch.zeros((3, 3, 1, 2), dtype=F64)
    U[0, 0] = 1.0
    U[1, 0, 0, 0] = -6.0  # u = -6 (negative: the absolute value matters)
    U[2, 0, 0, 1] = -6.0  # v = -6
    c = math.sqrt(G)
    for dx, dy in ((4.0, 1.0), (1.0, 4.0)):
        prm = O.Params(nx=2, ny=1, dx=dx, dy=dy, cfl=0.3, dt_max=100.0)
        dt = O.time_step(U, prm, 0.0)
        # the Courant number dt * speed / length of each cell's fastest direction
        crs = [dt * max(_spectral_radius(1.0, float(U[1, 0, 0, i]), float(U[2, 0, 0, i]), 0) / dx,
                        _spectral_radius(1.0, float(U[1, 0, 0, i]), float(U[2, 0, 0, i]), 1) / dy)
               for i in range(2)]
        fast = 1 if dy < dx else 0
        assert abs(crs[fast] - 0.3) <= 1e-9 and crs[1 - fast] < 0.3
        assert abs(_spectral_radius(1.0, -6.0, 0.0, 0) - (6.0 + c)) < 1e-6


def test_courant_step_with_nothing_wet_is_dt_max():
    U = torch.zeros((3, 3, 3, 4), dtype=F64)
    U[0, 0] = 1e-5  # at the tolerance: dry
    U[1, 0] = 3.0
    prm = O.Params(nx=4, ny=3, dx=1.0, dy=2.0, dt_max=0.7)
    assert O.time_step(U, prm, 0.0) == 0.7
    assert O.time_step(U, prm, 0.0, t_end=0.25) == 0.25


def _inflow_l1(nx, q=0.6, T=5.0, L=60.0):
    dx = L / nx
    Z = np.zeros((3, nx + 1))
    U = O.initial_state(Z, np.zeros_like(Z), False)
    infl = [O.InflowBC(O.WEST, 0, 1, torch.tensor([0.0], dtype=F64), torch.tensor([q * 2 * dx], dtype=F64))]
    prm = O.Params(nx=nx, ny=2, dx=dx, dy=dx, cfl=0.3, inflows=infl, dt_max=0.05)
    r = O.run(U, O.bed_from_corners(Z), prm, t_end=T)
    hc = (q * q / G) ** (1.0 / 3.0)
    sub = 32
    xf = (np.arange(nx * sub) + 0.5) * dx / sub
    he, _ = ritter(2.25 * hc, xf / T)
    exact = he.reshape(nx, sub).mean(axis=1)
    h = r.U[0, 0, 0].numpy()
    return float(np.abs(h - exact).mean()), h, exact, hc


def test_constant_inflow_into_a_dry_channel_is_ritters_fan():
    e1, h1, ex1, hc = _inflow_l1(60)
    e2, h2, ex2, _ = _inflow_l1(120)
    e3, h3, ex3, _ = _inflow_l1(240)
    assert e1 < 5e-3
    assert e2 < 0.8 * e1 and e3 < 0.5 * e2
    # the cells at the boundary follow the critical state: depth hc at x = 0
    assert abs(ex3[0] - hc) < 5e-3
    assert abs(h2[0] - ex2[0]) < 2e-3 and abs(h3[0] - ex3[0]) < 2e-3


def _bad_half(q_in, h_inner, g):
    hc = torch.pow(q_in * q_in / g, 1.0 / 3.0)
    hb = torch.maximum(h_inner, hc)
    z = torch.zeros_like(h_inner)
    return torch.stack([q_in + z, q_in * q_in / hb + g * hb * hb, z])


def _bad_floor(q_in, h_inner, g):
    hc = torch.pow(q_in / g, 1.0 / 3.0)  # the square of q dropped from the critical depth
    hb = torch.maximum(h_inner, hc)
    z = torch.zeros_like(h_inner)
    return torch.stack([q_in + z, q_in * q_in / hb + 0.5 * g * hb * hb, z])


def _bad_advective(q_in, h_inner, g):
    hc = torch.pow(q_in * q_in / g, 1.0 / 3.0)
    hb = torch.maximum(h_inner, hc)
    z = torch.zeros_like(h_inner)
    return torch.stack([q_in + z, 0.5 * g * hb * hb, z])


@pytest.mark.parametrize("bad", [_bad_half, _bad_floor, _bad_advective])
def test_inflow_pin_fails_on_a_planted_momentum_mistake(monkeypatch, bad):
    good, hg, exg, _ = _inflow_l1(120)
    monkeypatch.setattr(O, "inflow_face_flux", bad)
    wrong, hw, exw, _ = _inflow_l1(120)
    # the depth at the boundary is no longer the critical one
    assert abs(hg[0] - exg[0]) < 2e-3
    assert abs(hw[0] - exw[0]) > 2e-2


def _cfl_swapped(U, prm):
    h0 = U[0, 0]
    wet = h0 > prm.tol
    hs = torch.where(wet, h0, torch.ones_like(h0))
    u, v, c = torch.abs(U[1, 0] / hs), torch.abs(U[2, 0] / hs), torch.sqrt(prm.g * hs)
    m = torch.minimum(prm.dy / (u + c), prm.dx / (v + c))  # dx and dy swapped
    return float(torch.where(wet, m, torch.full_like(m, math.inf)).min())


def _cfl_signed(U, prm):
    h0 = U[0, 0]
    wet = h0 > prm.tol
    hs = torch.where(wet, h0, torch.ones_like(h0))
    u, v, c = U[1, 0] / hs, U[2, 0] / hs, torch.sqrt(prm.g * hs)  # no absolute values
    m = torch.minimum(prm.dx / (u + c), prm.dy / (v + c))
    return float(torch.where(wet, m, torch.full_like(m, math.inf)).min())


def _cfl_with_dry(U, prm):
    hs = torch.clamp(U[0, 0], min=1e-6)  # dry cells counted
    u, v, c = torch.abs(U[1, 0] / hs), torch.abs(U[2, 0] / hs), torch.sqrt(prm.g * hs)
    return float(torch.minimum(prm.dx / (u + c), prm.dy / (v + c)).min())


@pytest.mark.parametrize("bad", [_cfl_swapped, _cfl_signed, _cfl_with_dry])
def test_courant_pins_fail_on_a_planted_mistake(monkeypatch, bad):
    monkeypatch.setattr(O, "cfl_min", bad)
    failed = 0
    for check in (lambda: test_courant_step_realises_cr_with_jacobian_wave_speeds(2.0, 0.5, 1),
                  test_courant_step_direction_decides_which_cell_is_fastest):
        try:
            check()
        except AssertionError:
            failed += 1
    assert failed >= 1
