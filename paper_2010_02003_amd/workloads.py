"""Seeded synthetic inputs for the DG2 flood step.

This module only builds input data: corner-node DEMs, initial free-surface or
depth values at corner nodes, Manning fields, inflow hydrograph tables, rainfall
windows and gauge positions.  It contains none of the numerical method (no
modes, fluxes or updates), so both the HIP library and the CPU oracle can be
fed from it.

The paper runs its DG2 model on UK Environment Agency benchmark DEMs and
hydrographs (Sec. 3, Table 2) that are not available here.  The generators
below stand in for them with synthetic terrain at the paper's scales (Manning
0.01-0.04, inflow peaks of tens of m^3/s, runs of hours) and are the only
source of input data for tests and benchmarks.

Conventions
-----------
* ``nx`` cells in x (west -> east), ``ny`` cells in y (south -> north).
* Corner arrays have shape ``(ny + 1, nx + 1)``; element ``[j, i]`` sits at
  ``(x0 + i*dx, y0 + j*dy)``.
* Per-cell arrays have shape ``(ny, nx)`` with the cell centre at
  ``(x0 + (i + 0.5)*dx, y0 + (j + 0.5)*dy)``.
* Sides: 0 = west, 1 = east, 2 = south, 3 = north.  An inflow segment is a
  closed range of boundary cells ``[first, last]`` counted along the side
  (rows ``j`` for west/east, columns ``i`` for south/north).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


@dataclass
class Inflow:
    """Discharge hydrograph entering through one boundary segment."""

    side: int
    first: int
    last: int
    t: np.ndarray  # sample times (s), increasing
    Q: np.ndarray  # total discharge through the segment (m^3/s), >= 0


@dataclass
class Level:
    """Water-level hydrograph imposed along one boundary segment."""

    side: int
    first: int
    last: int
    t: np.ndarray  # sample times (s), increasing
    eta: np.ndarray  # free-surface elevation (m)


@dataclass
class Scenario:
    """Everything that defines one run: grid, inputs and run controls."""

    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    Z: np.ndarray  # corner DEM (ny+1, nx+1)
    surface: np.ndarray  # corner eta (is_eta) or h (ny+1, nx+1)
    is_eta: bool = True
    qx: Optional[np.ndarray] = None  # corner discharges, None = 0
    qy: Optional[np.ndarray] = None
    manning: object = 0.0  # float or (ny, nx) array
    cfl: float = 0.3
    dt_max: float = 1.0
    g: float = 9.81
    tol_dry: float = 1e-5
    theta: float = 10.0
    variant: str = "NL"  # "NL" or "LL"
    precision: str = "fp64"  # "fp64" or "fp32"
    flux: str = "HLL"  # face flux: "HLL" or "ROE"
    steps: Optional[int] = None
    t_end: Optional[float] = None
    fixed_dt: float = 0.0
    inflows: List[Inflow] = field(default_factory=list)
    levels: List[Level] = field(default_factory=list)
    opens: List[Tuple[int, int, int]] = field(default_factory=list)  # (side, first, last)
    rain: Optional[Tuple[float, float, float]] = None  # (rate m/s, t_begin, t_end)
    gauges: Optional[np.ndarray] = None  # (ng, 2) x, y in m
    x0: float = 0.0
    y0: float = 0.0
    stage_check: int = 0  # repeats of stage 1 allowed by the stage-1 Courant check (0: off)
    partly_wet_flat: bool = False  # optional partly-wet rule (not in the paper; off by default)

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def corner_xy(nx: int, ny: int, dx: float, dy: float, x0: float = 0.0, y0: float = 0.0):
    x = x0 + dx * np.arange(nx + 1, dtype=np.float64)
    y = y0 + dy * np.arange(ny + 1, dtype=np.float64)
    return np.meshgrid(x, y)  # X[j, i], Y[j, i]


def cell_xy(nx: int, ny: int, dx: float, dy: float, x0: float = 0.0, y0: float = 0.0):
    x = x0 + dx * (np.arange(nx, dtype=np.float64) + 0.5)
    y = y0 + dy * (np.arange(ny, dtype=np.float64) + 0.5)
    return np.meshgrid(x, y)


def fbm_surface(shape: Tuple[int, int], hurst: float, relief: float, seed: int) -> np.ndarray:
    """Fractional-Brownian surface by 2D spectral synthesis.

    Amplitude falls as |k|^-(H+1) with random phases and Gaussian weights, the
    mean (k = 0) is removed and the result is rescaled to [0, relief].
    """
    rng = np.random.default_rng(seed)
    ny, nx = shape
    kx = np.fft.fftfreq(nx)
    ky = np.fft.fftfreq(ny)
    KX, KY = np.meshgrid(kx, ky)
    K = np.sqrt(KX * KX + KY * KY)
    K[0, 0] = 1.0
    amp = K ** (-(hurst + 1.0))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    weight = rng.standard_normal(size=shape)
    field_ = np.real(np.fft.ifft2(amp * weight * np.exp(1j * phase)))
    lo, hi = field_.min(), field_.max()
    if hi - lo <= 0:
        return np.zeros(shape)
    return (field_ - lo) / (hi - lo) * relief


def triangular_hydrograph(peak: float, t_peak: float, t_stop: float) -> Tuple[np.ndarray, np.ndarray]:
    t = np.array([0.0, t_peak, t_stop], dtype=np.float64)
    Q = np.array([0.0, peak, 0.0], dtype=np.float64)
    return t, Q


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def dambreak_bump(nx: int = 128, ny: int = 128, dx: float = 1.0, variant: str = "NL",
                  precision: str = "fp64", steps: int = 500) -> Scenario:
    """Dam break over a Gaussian bump, reflective walls, 128 x 128 cells, dx = 1 m.

    Bed z = 0.3 exp(-((x-64)^2 + (y-64)^2)/200) m; free surface 1.0 m for
    x < 64 and 0.5 m for x >= 64 (a corner on x = 64 takes the x >= 64 value);
    zero velocity; Manning 0.03; Courant number 0.33; g = 9.81; 500 RK2 steps.
    The bump and the dam stay centred when the grid is refined or coarsened.
    """
    Lx = nx * dx
    Ly = ny * dx
    X, Y = corner_xy(nx, ny, dx, dx)
    xc, yc = 0.5 * Lx, 0.5 * Ly
    Z = 0.3 * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / 200.0)
    eta = np.where(X < xc, 1.0, 0.5)
    return Scenario(name="dambreak_bump_%dx%d" % (nx, ny), nx=nx, ny=ny, dx=dx, dy=dx, Z=Z,
                    surface=eta, is_eta=True, manning=0.03, cfl=0.33, dt_max=1.0,
                    variant=variant, precision=precision, steps=steps)


def channel_centreline(x: np.ndarray) -> np.ndarray:
    return 512.0 + 150.0 * np.sin(2.0 * np.pi * x / 680.0)


def floodplain(nx: int = 1024, ny: int = 512, dx: float = 2.0, variant: str = "NL",
               precision: str = "fp64", seed: int = 2, t_end: float = 10800.0) -> Scenario:
    """Synthetic floodplain, 1024 x 512 cells, dx = 2 m, initially dry.

    Bed: fBm (Hurst 0.7, relief 5 m, seeded) minus 2 m inside a 20 m wide
    meandering channel with centreline y = 512 + 150 sin(2 pi x / 680) m.
    West-edge inflow into the channel mouth (cells whose centres lie within
    10 m of the centreline at x = 0): triangular hydrograph 0 -> 20 m^3/s at
    30 min -> 0 at 60 min.  Manning 0.035, walls elsewhere, 3 h simulated.
    """
    X, Y = corner_xy(nx, ny, dx, dx)
    Z = fbm_surface((ny + 1, nx + 1), 0.7, 5.0, seed)
    in_channel = np.abs(Y - channel_centreline(X)) <= 10.0
    Z = Z - 2.0 * in_channel
    h = np.zeros_like(Z)
    yc = dx * (np.arange(ny) + 0.5)
    mouth = np.nonzero(np.abs(yc - channel_centreline(np.array(0.0))) <= 10.0)[0]
    t, Q = triangular_hydrograph(20.0, 1800.0, 3600.0)
    inflow = Inflow(WEST, int(mouth[0]), int(mouth[-1]), t, Q)
    gx = np.array([100.0, 400.0, 800.0, 1200.0, 1600.0, 2000.0])
    gauges = np.stack([gx, channel_centreline(gx)], axis=1)
    return Scenario(name="floodplain_%dx%d" % (nx, ny), nx=nx, ny=ny, dx=dx, dy=dx, Z=Z,
                    surface=h, is_eta=False, manning=0.035, cfl=0.3, dt_max=1.0,
                    variant=variant, precision=precision, t_end=t_end, inflows=[inflow],
                    gauges=gauges)


def floodplain_mouth(nx: int = 40, ny: int = 40, row0: int = 236, stage_check: int = 0,
                     precision: str = "fp64") -> Scenario:
    """The corner of the floodplain around its inflow mouth: columns 0..nx-1
    and rows row0..row0+ny-1 of the 1024 x 512 grid, with the same bed (the
    channel carved with 1 m steps across one cell), the same inflow (the
    whole mouth segment lies inside) and walls on the cut edges."""
    full = floodplain(precision=precision)
    b = full.inflows[0]
    assert row0 <= b.first and b.last < row0 + ny
    Z = full.Z[row0:row0 + ny + 1, 0:nx + 1].copy()
    return Scenario(name="floodplain_mouth_%dx%d" % (nx, ny), nx=nx, ny=ny, dx=full.dx, dy=full.dy, Z=Z,
                    surface=np.zeros_like(Z), is_eta=False, manning=full.manning, cfl=full.cfl,
                    dt_max=full.dt_max, precision=precision,
                    inflows=[Inflow(b.side, b.first - row0, b.last - row0, b.t, b.Q)],
                    y0=row0 * full.dy, stage_check=stage_check)


def urban(n: int = 4096, dx: float = 0.5, nblocks: int = 2000, precision: str = "fp32",
          seed: int = 3, steps: int = 2000, variant: str = "NL") -> Scenario:
    """Urban-like domain, 4096 x 4096 cells, dx = 0.5 m, from dry under rain.

    Bed: plane of slope 1e-3 in a seeded direction, shifted to be >= 0, plus
    ``nblocks`` axis-aligned rectangular building blocks (sides U[5, 40] m,
    uniform positions) raised by 10 m (overlaps are not stacked).
    Uniform rainfall 50 mm/h for 1 h.  Manning 0.02 on a street grid (10 m
    wide streets every 100 m) and 0.05 elsewhere.  Walls on all sides.
    Steps are capped at 0.02 s: the 10 m block walls rise over one 0.5 m cell
    (slope 20), and a rain film starting from rest there is accelerated at
    about g * 20 within a step, so larger steps drain wall cells negative
    before the Courant limit can react.
    """
    rng = np.random.default_rng(seed)
    L = n * dx
    X, Y = corner_xy(n, n, dx, dx)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    Z = 1e-3 * (X * np.cos(theta) + Y * np.sin(theta))
    Z = Z - Z.min()
    sides = rng.uniform(5.0, 40.0, size=(nblocks, 2))
    lower = rng.uniform(0.0, 1.0, size=(nblocks, 2)) * (L - sides)
    raised = np.zeros(Z.shape, dtype=bool)
    for k in range(nblocks):
        i0 = int(np.ceil(lower[k, 0] / dx))
        i1 = int(np.floor((lower[k, 0] + sides[k, 0]) / dx))
        j0 = int(np.ceil(lower[k, 1] / dx))
        j1 = int(np.floor((lower[k, 1] + sides[k, 1]) / dx))
        raised[j0:j1 + 1, i0:i1 + 1] = True
    Z = Z + 10.0 * raised
    h = np.zeros_like(Z)
    XC, YC = cell_xy(n, n, dx, dx)
    street = (np.mod(XC, 100.0) < 10.0) | (np.mod(YC, 100.0) < 10.0)
    manning = np.where(street, 0.02, 0.05)
    rain = (50e-3 / 3600.0, 0.0, 3600.0)
    g = np.array([[0.25 * L, 0.25 * L], [0.5 * L, 0.5 * L], [0.75 * L, 0.3 * L], [0.3 * L, 0.8 * L]])
    return Scenario(name="urban_%dx%d" % (n, n), nx=n, ny=n, dx=dx, dy=dx, Z=Z, surface=h,
                    is_eta=False, manning=manning, cfl=0.3, dt_max=0.02, variant=variant,
                    precision=precision, steps=steps, rain=rain, gauges=g)


def ensemble_member(k: int, seed: int = 4) -> Scenario:
    """Member ``k`` of the 256-scenario ensemble (uneven grid sizes).

    nx in {64, 128, 256, 512}, ny in {64, 128, 256}, dx = 2 m, fBm bed (Hurst
    0.7, relief 5 m, seed 1000 + k), Manning ~ U[0.02, 0.06], west-edge inflow
    over 20 m centred on the edge with a triangular hydrograph peaking at
    Q ~ U[5, 50] m^3/s at 30 min and ending at 60 min, initially dry.
    """
    rng = np.random.default_rng([seed, k])
    nx = int(rng.choice([64, 128, 256, 512]))
    ny = int(rng.choice([64, 128, 256]))
    n_m = float(rng.uniform(0.02, 0.06))
    peak = float(rng.uniform(5.0, 50.0))
    dx = 2.0
    Z = fbm_surface((ny + 1, nx + 1), 0.7, 5.0, 1000 + k)
    h = np.zeros_like(Z)
    mid = ny // 2
    first, last = mid - 5, mid + 4  # 10 cells = 20 m
    t, Q = triangular_hydrograph(peak, 1800.0, 3600.0)
    return Scenario(name="ens%03d_%dx%d" % (k, nx, ny), nx=nx, ny=ny, dx=dx, dy=dx, Z=Z,
                    surface=h, is_eta=False, manning=n_m, cfl=0.3, dt_max=1.0,
                    precision="fp32", steps=1000, inflows=[Inflow(WEST, first, last, t, Q)])


def ensemble(count: int = 256, seed: int = 4) -> List[Scenario]:
    return [ensemble_member(k, seed) for k in range(count)]


def adjoint_case(n: int = 512, dx: float = 2.0, seed: int = 5, steps: int = 2000,
                 block: int = 64, nsamples: int = 60, cfl: float = 0.3) -> Dict[str, object]:
    """Inputs of the gradient (adjoint) workload, 512 x 512 cells, dx = 2 m.

    Bed: fBm (seed, relief 5 m) plus a 3 m Gaussian bump (sigma 100 m) in the
    centre.  Lake at rest with a free surface 1 m above the highest bed point
    (fully wet).  Target Manning field: 8 x 8 blocks of 64 x 64 cells with
    n ~ U[0.02, 0.06]; the model starts from n = 0.04.  West-edge inflow over
    20 m centred on the edge, hydrograph given by ``nsamples`` samples evenly
    spread over the run T = steps dt (target: triangular, 0 at t = 0, peak
    20 m^3/s at T/3, 0 from 2T/3 on; model start: 0.8 x target).  Fixed step
    dt = 0.9 x the Courant step of the initial state, cfl min dx/sqrt(g h)
    over cell means (0.0596 s at 512 x 512).  Eight
    gauges at ((k + 1/2) L/8, L/2), k = 0..7 (L = n dx; 64 + 128 k m, 512 m).
    """
    rng = np.random.default_rng(seed)
    X, Y = corner_xy(n, n, dx, dx)
    L = n * dx
    Z = fbm_surface((n + 1, n + 1), 0.7, 5.0, seed)
    Z = Z + 3.0 * np.exp(-((X - 0.5 * L) ** 2 + (Y - 0.5 * L) ** 2) / (2.0 * 100.0 ** 2))
    eta = np.full_like(Z, Z.max() + 1.0)
    nb = n // block
    n_blocks_target = rng.uniform(0.02, 0.06, size=(nb, nb))
    mid = n // 2
    gauges = np.stack([(np.arange(8) + 0.5) * (L / 8.0), np.full(8, 0.5 * L)], axis=1)
    # Courant step of the initial lake: the deepest cell mean sets it
    zc = 0.25 * (Z[:-1, :-1] + Z[1:, :-1] + Z[:-1, 1:] + Z[1:, 1:])
    hmax = float((eta.max() - zc).max())
    dt = 0.9 * cfl * dx / np.sqrt(9.81 * hmax)
    T = steps * dt
    t_q = np.linspace(0.0, T, nsamples)
    Q_target = np.interp(t_q, [0.0, T / 3.0, 2.0 * T / 3.0, T], [0.0, 20.0, 0.0, 0.0])
    return dict(n=n, dx=dx, Z=Z, eta=eta, block=block, n_blocks_target=n_blocks_target,
                n_model=0.04, steps=steps, dt=dt, nsamples=nsamples, inflow_side=WEST,
                inflow_first=mid - 5, inflow_last=mid + 4, t_q=t_q, Q_target=Q_target,
                model_scale=0.8, gauges=gauges, checkpoint_every=100)


def thacker_bowl(dx: float = 40.0, L: float = 4000.0, h0: float = 1.0, r0: float = 2000.0,
                 g: float = 9.81, tau: float = 1756.2, precision: str = "fp64",
                 variant: str = "NL") -> Scenario:
    """Curved oscillatory flow in a frictionless parabolic bowl (Thacker's
    solution; the long-run test of Sec. 2.3, period tau = 1756.2 s).

    Domain [-L, L]^2 (8 km square), cells of dx (40 m: 200 x 200).  Bed
    z = -h0 (1 - r^2/a^2) with a chosen so that the period 2 pi a /
    sqrt(8 g h0) equals tau (a = 2476.7 m for h0 = 1 m, g = 9.81); r0 = 2000 m
    sets the amplitude A = (a^4 - r0^4)/(a^4 + r0^4).  At t = 0 the water is
    at rest with the concave surface of the exact solution (maximally dry).
    Walls far outside the wet region, no friction.  The exact solution is in
    ``thacker_exact``.
    """
    a = tau * np.sqrt(8.0 * g * h0) / (2.0 * np.pi)
    n = int(round(2.0 * L / dx))
    X, Y = corner_xy(n, n, dx, dx, -L, -L)
    Z = -h0 * (1.0 - (X * X + Y * Y) / (a * a))
    h, _, _ = thacker_exact(X, Y, 0.0, h0=h0, a=a, r0=r0, g=g)
    return Scenario(name="thacker_%dx%d" % (n, n), nx=n, ny=n, dx=dx, dy=dx, Z=Z, surface=h,
                    is_eta=False, manning=0.0, cfl=0.3, dt_max=1e6, g=g, variant=variant,
                    precision=precision, x0=-L, y0=-L)


def thacker_exact(x, y, t, h0: float = 1.0, a: float = None, r0: float = 2000.0,
                  g: float = 9.81, tau: float = 1756.2):
    """Thacker's curved oscillatory solution at time t: depth h >= 0 and the
    velocities (u, v), with a from tau when not given (as in thacker_bowl)."""
    if a is None:
        a = tau * np.sqrt(8.0 * g * h0) / (2.0 * np.pi)
    w = np.sqrt(8.0 * g * h0) / a
    A = (a ** 4 - r0 ** 4) / (a ** 4 + r0 ** 4)
    c, sn = np.cos(w * t), np.sin(w * t)
    r2 = (x * x + y * y) / (a * a)
    eta = h0 * (np.sqrt(1.0 - A * A) / (1.0 - A * c) - 1.0
                - r2 * ((1.0 - A * A) / (1.0 - A * c) ** 2 - 1.0))
    z = -h0 * (1.0 - r2)
    h = np.maximum(eta - z, 0.0)
    f = 0.5 * w * A * sn / (1.0 - A * c)
    wet = h > 0.0
    return h, np.where(wet, f * x, 0.0), np.where(wet, f * y, 0.0)


def random_modes(nx: int, ny: int, seed: int, wet_fraction: float = 0.8,
                 depth: float = 1.0, slope: float = 0.3, speed: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Random 9-plane mode state and 3-plane bed modes for single-stage checks.

    Returns ``(modes, bed)`` with ``modes`` shaped (9, ny, nx) in the plane
    order h0, h1x, h1y, qx0, qx1x, qx1y, qy0, qy1x, qy1y and ``bed`` shaped
    (ny+1, nx+1) corner elevations.  A ``1 - wet_fraction`` share of the cells
    is dry (depth below the drying tolerance or zero) with zero discharge, so
    wet/dry branches are exercised.  This builds raw coefficients only.
    """
    rng = np.random.default_rng(seed)
    h0 = depth * rng.uniform(0.2, 1.0, size=(ny, nx))
    dry = rng.uniform(size=(ny, nx)) > wet_fraction
    h0 = np.where(dry, rng.choice([0.0, 3e-6, 2e-5], size=(ny, nx)), h0)
    h1x = slope * h0 * rng.uniform(-1.0, 1.0, size=(ny, nx))
    h1y = slope * h0 * rng.uniform(-1.0, 1.0, size=(ny, nx))
    q = [speed * h0 * rng.uniform(-1.0, 1.0, size=(ny, nx)) for _ in range(6)]
    q = [np.where(dry, 0.0, a) for a in q]
    modes = np.stack([h0, h1x, h1y, q[0], 0.3 * q[1], 0.3 * q[2], q[3], 0.3 * q[4], 0.3 * q[5]])
    bed = 0.5 * rng.standard_normal(size=(ny + 1, nx + 1))
    return modes, bed
