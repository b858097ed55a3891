"""Pins of the oracle's Roe flux option (Sec. 2.1.2 names Roe's solver).

Roe's linearisation resolves any single discontinuity that satisfies the
Rankine-Hugoniot conditions exactly, so across an isolated shock or shear
wave the flux must be the exact upwind flux; it is consistent; a mirror
state gives zero mass flux; the scheme stays well balanced; and dam breaks
converge to the exact solution: Stoker's (golden file) and a transonic
rarefaction, where a Roe scheme could admit an expansion shock, against a
textbook exact Riemann solver written out below.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import dg2_oracle as O
from paper_2010_02003_amd import workloads as WL

from exact_riemann import exact_riemann

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = 9.81
TOL = 1e-5
F64 = torch.float64


def _t(*a):
    return [torch.tensor([float(x)], dtype=F64) for x in a]


def _phys(h, u, v):
    return np.array([h * u, h * u * u + 0.5 * G * h * h, h * u * v])


def test_roe_is_consistent():
    rng = np.random.default_rng(3)
    for _ in range(50):
        h, u, v = rng.uniform(0.01, 3.0), rng.uniform(-3, 3), rng.uniform(-3, 3)
        F = O.roe_flux(*_t(h, u, v, h, u, v), G, TOL).numpy()[:, 0]
        assert np.allclose(F, _phys(h, u, v), rtol=1e-14, atol=1e-14)


def _shock_pair(hL, hR, s, family):
    """States on either side of a shock of speed s satisfying the jump
    conditions: mass flux m through the shock with m^2 = g hL hR (hL+hR)/2;
    family 3 (hL > hR, fluid crosses right to left) or 1 (hL < hR)."""
    m = math.sqrt(G * hL * hR * (hL + hR) / 2.0) * (-1.0 if family == 3 else 1.0)
    return hL, s + m / hL, hR, s + m / hR


@pytest.mark.parametrize("family", [1, 3])
@pytest.mark.parametrize("s", [-2.5, -0.4, 0.3, 1.7])
def test_roe_flux_is_exact_upwind_across_an_isolated_shock(family, s):
    hL, hR = (1.3, 0.6) if family == 3 else (0.6, 1.3)
    hL, uL, hR, uR = _shock_pair(hL, hR, s, family)
    v = 0.7  # same tangential velocity on both sides: a single wave
    FL, FR = _phys(hL, uL, v), _phys(hR, uR, v)
    # the pair satisfies the jump conditions F_R - F_L = s (U_R - U_L)
    dU = np.array([hR - hL, hR * uR - hL * uL, (hR - hL) * v])
    assert np.allclose(FR - FL, s * dU, atol=1e-12)
    F = O.roe_flux(*_t(hL, uL, v, hR, uR, v), G, TOL).numpy()[:, 0]
    assert np.allclose(F, FL if s > 0 else FR, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("u", [-0.8, 0.5])
def test_roe_flux_upwinds_a_shear_wave(u):
    h = 0.9
    F = O.roe_flux(*_t(h, u, 0.3, h, u, -1.1), G, TOL).numpy()[:, 0]
    want = _phys(h, u, 0.3 if u > 0 else -1.1)
    assert np.allclose(F, want, rtol=1e-13, atol=1e-13)


def test_roe_mirror_state_has_zero_mass_flux():
    rng = np.random.default_rng(4)
    for _ in range(20):
        h, u, v = rng.uniform(0.01, 2.0), rng.uniform(-2, 2), rng.uniform(-2, 2)
        F = O.roe_flux(*_t(h, u, v, h, -u, v), G, TOL).numpy()[:, 0]
        assert abs(F[0]) < 1e-14
        assert abs(F[2]) < 1e-14


def test_roe_with_a_dry_side_is_the_hll_flux():
    a = _t(1e-6, 0.0, 0.0, 0.8, -0.4, 0.2)
    assert torch.equal(O.roe_flux(*a, G, TOL), O.hll_flux(*a, G, TOL))


def test_roe_lake_at_rest_and_high_wall_stay_still():
    sc = WL.dambreak_bump(nx=24, ny=20)
    U = O.initial_state(sc.Z, np.full_like(sc.Z, 1.0), True)
    bed = O.bed_from_corners(sc.Z)
    prm = O.params_from_scenario(sc)
    prm.flux = "ROE"
    assert float(O.spatial_operator(U, bed, prm, 0.0).abs().max()) < 1e-13
    r = O.run(U, bed, prm, steps=100)
    assert float(r.U[1:].abs().max()) < 1e-12
    # water against a high wall, wet/dry front on the steep cell
    nx, ny = 20, 6
    X, _ = WL.corner_xy(nx, ny, 1.0, 1.0)
    Z = np.where(X <= 10, 0.0, 2.0)
    U = O.initial_state(Z, np.full_like(Z, 1.0), True)
    prm = O.Params(nx=nx, ny=ny, dx=1.0, dy=1.0, manning=0.02, flux="ROE")
    r = O.run(U, O.bed_from_corners(Z), prm, steps=200)
    assert float(r.U[1:].abs().max()) < 1e-13


def test_exact_riemann_solver_reproduces_stoker_golden():
    """The solver above, checked against the independently computed Stoker
    middle state (tests/golden/stoker_dambreak.json)."""
    s = json.load(open(os.path.join(GOLDEN, "stoker_dambreak.json")))
    _, _, hs, us = exact_riemann(s["h_L"], 0.0, s["h_R"], 0.0, np.array([0.0]))
    assert hs == pytest.approx(s["h_m"], rel=1e-12)
    assert us == pytest.approx(s["u_m"], rel=1e-12)


def _dam_break_l1(hL, hR, nx, flux, T):
    L = 100.0
    dx = L / nx
    X, _ = WL.corner_xy(nx, 2, dx, dx)
    Z = np.zeros_like(X)
    U = O.initial_state(Z, np.where(X < 50.0, hL, hR), True)
    prm = O.Params(nx=nx, ny=2, dx=dx, dy=dx, cfl=0.3, flux=flux)
    r = O.run(U, O.bed_from_corners(Z), prm, t_end=T)
    sub = 32
    xf = (np.arange(nx * sub) + 0.5) * dx / sub
    he, _, _, _ = exact_riemann(hL, 0.0, hR, 0.0, (xf - 50.0) / T)
    exact = he.reshape(nx, sub).mean(axis=1)
    h = r.U[0, 0, 0].numpy()
    return np.abs(h - exact).mean(), h, exact


def test_roe_stoker_dam_break_converges():
    e1, _, _ = _dam_break_l1(1.0, 0.5, 100, "ROE", 8.0)
    e2, _, _ = _dam_break_l1(1.0, 0.5, 200, "ROE", 8.0)
    assert e1 < 6e-3
    assert e2 < 0.75 * e1


def test_roe_transonic_rarefaction_converges_without_expansion_shock():
    """hL = 1, hR = 0.05: the left rarefaction fan straddles x/t = 0, where a
    first-order Roe scheme would admit an expansion shock.  With DG2 slopes
    the solution converges to the exact fan there, as fast as with HLL."""
    _, _, hs, us = exact_riemann(1.0, 0.0, 0.05, 0.0, np.array([0.0]))
    assert us - math.sqrt(G * hs) > 0.0  # the fan is transonic
    errs, near = [], []
    for nx in (100, 200, 400):
        e, h, ex = _dam_break_l1(1.0, 0.05, nx, "ROE", 5.0)
        k = slice(nx // 2 - nx // 20, nx // 2 + nx // 20)  # x in [45, 55] m around the sonic point
        errs.append(e)
        near.append(np.abs(h[k] - ex[k]).max())
    assert errs[0] < 8e-3
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]
    assert near[0] < 1.5e-2 and near[2] < 0.5 * near[0]
    e_hll, _, _ = _dam_break_l1(1.0, 0.05, 200, "HLL", 5.0)
    assert errs[1] < 1.1 * e_hll
