"""Plain FP64 CPU oracle of the slope-decoupled DG2 shallow-water time step.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library never does, and the two share no code.

Everything is written with whole-array torch float64 CPU operations, one
operation per formula, on ghost-padded arrays, in the order in which the paper
describes the method (Sec. 2.1 of Ayog, Kesserwani, Shaw, Sharifian & Bau,
"Second-order discontinuous Galerkin flood model: comparison with
industry-standard finite volume models"):

  Sec. 2.1.1, Eq. (2)-(3)   planar modes (mean, x-slope, y-slope) per element,
                            initialised from corner-node values
  Sec. 2.1.2, Eq. (4)-(5)   face limits, positivity-preserving dummy limits,
                            wall revision of the bed, two-argument numerical
                            flux, dummy modes and the operators L0, L1x, L1y
  Sec. 2.1.2                explicit two-stage Runge-Kutta, Courant number
  Sec. 2.1.3                implicit friction splitting at the centre and the
                            four Gauss points, applied before the RK2 step
  Sec. 2.1.3, Eq. (6)-(7)   optional local slope limiting (DG2-LL)
  Eq. (11)-(12)             mass and energy diagnostics

For the adjoint, ``gauge_misfit_reference`` differentiates a gauge misfit
through this same step with torch's reverse-mode automatic differentiation
(Manning field and inflow hydrograph samples as parameters, fixed dt).

Readings taken where the paper is silent or ambiguous (the same ones the HIP
library implements):

  * flux: HLL with Toro's two-rarefaction wave-speed estimates and dry-bed
    speeds, zero flux when both sides are dry; optionally Roe's solver, the
    paper's own choice, without entropy fix and with HLL at faces that have
    a dry side;
  * Eq. (5b) is read as the y-directional average mode;
  * one revised bed value z* per face, using the depth limit on the west
    (south) side of that face;
  * velocities (and hence discharge and momentum fluxes) are zero wherever a
    depth is at or below the drying tolerance;
  * time step: Cr * min over wet cell means of min(dx/(|u|+c), dy/(|v|+c)),
    capped by dt_max and by the time left to the target;
  * RK2 is the SSP (Heun) average U^{n+1} = (W + U1 + dt L(U1)) / 2;
  * friction: implicit (exact) integral of the split friction ODE at frozen
    depth at the centre and the four Gauss points, once per time step with
    the full dt, increments added to the discharge modes;
  * walls: mirror ghost cells; discharge inflow: prescribed face flux;
    water-level boundary: a ghost at the prescribed level whose normal
    velocity keeps the outgoing Riemann invariant, inflow capped at critical
    speed; open boundary: a ghost holding the inside cell's mean state;
    rainfall: added to the mean depth mode before friction;
  * cells whose mean depth is at or below the drying tolerance get zero
    discharge modes after each stage; depths are never clipped.

Array layout: a state ``U`` is a tensor of shape (3, 3, ny, nx) indexed as
``U[var, mode, j, i]`` with var in (h, qx, qy) and mode in (0, 1x, 1y).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

F64 = torch.float64
SQRT3 = math.sqrt(3.0)
H, QX, QY = 0, 1, 2
M0, MX, MY = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3

# Mirror ghost signs (var x mode).  Reflection across an x-wall keeps the even
# fields h, qy and flips their x-slope; the normal discharge qx flips its mean
# and y-slope and keeps its x-slope.  Likewise for a y-wall.
_MIRROR_X = torch.tensor([[1.0, -1.0, 1.0], [-1.0, 1.0, -1.0], [1.0, -1.0, 1.0]], dtype=F64)
_MIRROR_Y = torch.tensor([[1.0, 1.0, -1.0], [1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]], dtype=F64)


def _t(a) -> torch.Tensor:
    return torch.as_tensor(a, dtype=F64)


# ---------------------------------------------------------------------------
# Sec. 2.1.1: modes from corner-node data (Eq. 3)
# ---------------------------------------------------------------------------

def face_centre_values(C: torch.Tensor):
    """Values at the face-centred nodes E, W, N, S averaged from corner values."""
    E = 0.5 * (C[:-1, 1:] + C[1:, 1:])
    W = 0.5 * (C[:-1, :-1] + C[1:, :-1])
    N = 0.5 * (C[1:, :-1] + C[1:, 1:])
    S = 0.5 * (C[:-1, :-1] + C[:-1, 1:])
    return E, W, N, S


def modes_from_corners(C) -> torch.Tensor:
    """Eq. (3): mean = (E + W)/2, x-slope = (E - W)/2, y-slope = (N - S)/2."""
    E, W, N, S = face_centre_values(_t(C))
    return torch.stack([0.5 * (E + W), 0.5 * (E - W), 0.5 * (N - S)])


@dataclass
class Bed:
    """Time-invariant bed modes (Eq. 3 applied to the DEM) and face values.

    ``zfx[j, i]`` is the bed at the centre of the x-face west of cell i (shape
    (ny, nx+1)); ``zfy[j, i]`` the bed at the y-face south of cell j (shape
    (ny+1, nx)).  Both neighbours of a face share that value, which is the
    continuity property that Eq. (3) gives the bed.
    """

    z: torch.Tensor  # (3, ny, nx): z0, z1x, z1y
    zfx: torch.Tensor
    zfy: torch.Tensor


def bed_from_corners(Z) -> Bed:
    Z = _t(Z)
    zfx = 0.5 * (Z[:-1, :] + Z[1:, :])
    zfy = 0.5 * (Z[:, :-1] + Z[:, 1:])
    return Bed(modes_from_corners(Z), zfx, zfy)


def initial_state(Z, surface, is_eta: bool = True, qx=None, qy=None) -> torch.Tensor:
    """Initial modes (Eq. 3) from corner values of the free surface or depth.

    Given a depth, its modes come from Eq. (3) directly.  Given a free surface
    eta, the depth modes are the eta modes minus the bed modes, so that a
    flat surface gives a discrete lake at rest (h1 = -z1); an element whose
    mean depth comes out negative (its mean bed lies above the surface) is
    set dry.  Face limits of a partly wet element may be negative; the dummy
    limits of Sec. 2.1.2 take care of them.
    """
    Z = _t(Z)
    s = _t(surface)
    if is_eta:
        h = modes_from_corners(s) - modes_from_corners(Z)
        h = torch.where(h[0] < 0.0, torch.zeros_like(h), h)
    else:
        h = modes_from_corners(s)
    zero = torch.zeros_like(Z)
    qx = zero if qx is None else _t(qx)
    qy = zero if qy is None else _t(qy)
    return torch.stack([h, modes_from_corners(qx), modes_from_corners(qy)])


# ---------------------------------------------------------------------------
# Problem parameters
# ---------------------------------------------------------------------------

@dataclass
class InflowBC:
    side: int
    first: int
    last: int
    t: torch.Tensor
    Q: torch.Tensor  # may require grad (adjoint reference)


@dataclass
class LevelBC:
    """Water-level boundary: the free-surface elevation eta(t) (piecewise
    linear in the samples, held outside) along a boundary segment."""
    side: int
    first: int
    last: int
    t: torch.Tensor
    eta: torch.Tensor


@dataclass
class OpenBC:
    """Open (transmissive) boundary segment."""
    side: int
    first: int
    last: int


@dataclass
class Params:
    nx: int
    ny: int
    dx: float
    dy: float
    g: float = 9.81
    tol: float = 1e-5
    cfl: float = 0.3
    dt_max: float = 1.0
    theta: float = 10.0
    variant: str = "NL"
    flux: str = "HLL"  # face flux: "HLL" (default reading) or "ROE" (the paper's choice)
    manning: object = 0.0  # float or (ny, nx) tensor
    inflows: List[InflowBC] = field(default_factory=list)
    levels: List[LevelBC] = field(default_factory=list)
    opens: List[OpenBC] = field(default_factory=list)
    rain: Optional[Tuple[float, float, float]] = None
    fixed_dt: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    # stage-1 Courant check (an option, off by default): up to this many
    # repeats of stage 1 with a smaller step when its result breaks Cr
    stage_check: int = 0
    # partly-wet rule (an option, off by default; not in the paper): after
    # each stage, elements with a wet mean and a face-limit depth at or below
    # tol drop their slope modes
    partly_wet_flat: bool = False


def _table_value(ts, vs, t: float):
    """Piecewise-linear interpolation of a time table, held constant outside."""
    ts = ts.to(F64)
    if t <= float(ts[0]):
        return vs[0]
    if t >= float(ts[-1]):
        return vs[-1]
    k = int(torch.searchsorted(ts, torch.tensor([t], dtype=F64), right=True)[0]) - 1
    w = (t - float(ts[k])) / (float(ts[k + 1]) - float(ts[k]))
    return vs[k] * (1.0 - w) + vs[k + 1] * w


def hydrograph_value(bc: InflowBC, t: float) -> torch.Tensor:
    """Discharge of an inflow hydrograph at time t."""
    return _table_value(bc.t, bc.Q, t)


# ---------------------------------------------------------------------------
# Boundary ghosts
# ---------------------------------------------------------------------------

def pad_mirror(U: torch.Tensor, mx=_MIRROR_X, my=_MIRROR_Y) -> torch.Tensor:
    """Surround the (..., ny, nx) mode field with one layer of mirror ghosts.

    Corner ghosts are never used by the five-point stencil and stay zero.
    """
    lead = U.shape[:-2]
    ny, nx = U.shape[-2:]
    P = torch.zeros(lead + (ny + 2, nx + 2), dtype=U.dtype)
    P[..., 1:-1, 1:-1] = U
    sx = mx.reshape(mx.shape + (1,))
    sy = my.reshape(my.shape + (1,))
    P[..., 1:-1, 0] = U[..., :, 0] * sx
    P[..., 1:-1, -1] = U[..., :, -1] * sx
    P[..., 0, 1:-1] = U[..., 0, :] * sy
    P[..., -1, 1:-1] = U[..., -1, :] * sy
    return P


def pad_bed(z: torch.Tensor) -> torch.Tensor:
    """Mirror ghosts for the bed modes: z is even across every wall."""
    mx = torch.tensor([1.0, -1.0, 1.0], dtype=F64)
    my = torch.tensor([1.0, 1.0, -1.0], dtype=F64)
    return pad_mirror(z, mx, my)


# ---------------------------------------------------------------------------
# Sec. 2.1.2: limits, dummy limits, flux
# ---------------------------------------------------------------------------

def dummy_limits(h, qn, qt, tol):
    """Positivity-preserving dummy limits: h* = max(0, h), q* = h* u.

    The velocities are q/h above the drying tolerance and zero otherwise.
    Returns (h*, u_n, u_t).
    """
    wet = h > tol
    hsafe = torch.where(wet, h, torch.ones_like(h))
    un = torch.where(wet, qn / hsafe, torch.zeros_like(h))
    ut = torch.where(wet, qt / hsafe, torch.zeros_like(h))
    return torch.clamp(h, min=0.0), un, ut


def physical_flux(h, un, ut, g):
    """Normal flux of the SWE (Eq. 1) from depth and velocities: [hu, hu^2 + gh^2/2, huv]."""
    q = h * un
    return torch.stack([q, q * un + 0.5 * g * h * h, q * ut])


def hll_flux(hL, uL, vL, hR, uR, vR, g, tol):
    """HLL numerical flux through a face with normal velocity u and tangential v.

    Wave speeds follow Toro's two-rarefaction estimates; a dry side uses the
    dry-bed front speed of the wet side.  Both sides dry gives zero flux.
    """
    cL = torch.sqrt(g * hL)
    cR = torch.sqrt(g * hR)
    ustar = 0.5 * (uL + uR) + cL - cR
    cstar = 0.5 * (cL + cR) + 0.25 * (uL - uR)
    dryL = hL <= tol
    dryR = hR <= tol
    sL = torch.where(dryL, uR - 2.0 * cR, torch.minimum(uL - cL, ustar - cstar))
    sR = torch.where(dryR, uL + 2.0 * cL, torch.maximum(uR + cR, ustar + cstar))
    FL = physical_flux(hL, uL, vL, g)
    FR = physical_flux(hR, uR, vR, g)
    UL = torch.stack([hL, hL * uL, hL * vL])
    UR = torch.stack([hR, hR * uR, hR * vR])
    middle = (sL < 0.0) & (sR > 0.0)
    den = torch.where(middle, sR - sL, torch.ones_like(sL))
    Fm = (sR * FL - sL * FR + sL * sR * (UR - UL)) / den
    F = torch.where(sL >= 0.0, FL, torch.where(sR <= 0.0, FR, Fm))
    both_dry = dryL & dryR
    return torch.where(both_dry, torch.zeros_like(F), F)


def roe_flux(hL, uL, vL, hR, uR, vR, g, tol):
    """Roe's approximate Riemann solver (named in Sec. 2.1.2) on the dummy limits.

    Roe averages u = (sqrt(hL) uL + sqrt(hR) uR)/(sqrt(hL) + sqrt(hR)), v alike,
    c = sqrt(g (hL + hR)/2); eigenvalues u - c, u, u + c with eigenvectors
    (1, u - c, v), (0, 0, 1), (1, u + c, v) and wave strengths from the jump
    in (h, hu, hv).  F = (F_L + F_R)/2 - sum |lambda_k| alpha_k r_k / 2.  The
    paper names no entropy fix and none is applied: with DG2 slopes a
    transonic rarefaction converges to the exact fan without one (tested),
    while Harten's fix with Harten-Hyman widths, fed by face-limit speeds,
    destabilised it.  A face with a side at or below the drying tolerance
    takes the HLL flux (dry-bed front speeds), since Roe averages need two
    wet states.
    """
    wet = (hL > tol) & (hR > tol)
    one = torch.ones_like(hL)
    hLw = torch.where(wet, hL, one)
    hRw = torch.where(wet, hR, one)
    rL, rR = torch.sqrt(hLw), torch.sqrt(hRw)
    uh = (rL * uL + rR * uR) / (rL + rR)
    vh = (rL * vL + rR * vR) / (rL + rR)
    ch = torch.sqrt(0.5 * g * (hLw + hRw))
    dh = hRw - hLw
    dq = hRw * uR - hLw * uL
    dr = hRw * vR - hLw * vL
    a1 = ((uh + ch) * dh - dq) / (2.0 * ch)
    a2 = dr - vh * dh
    a3 = (dq - (uh - ch) * dh) / (2.0 * ch)
    m1 = torch.abs(uh - ch)
    m3 = torch.abs(uh + ch)
    m2 = torch.abs(uh)
    FL = physical_flux(hLw, uL, vL, g)
    FR = physical_flux(hRw, uR, vR, g)
    diss = torch.stack([m1 * a1 + m3 * a3,
                        m1 * a1 * (uh - ch) + m3 * a3 * (uh + ch),
                        (m1 * a1 + m3 * a3) * vh + m2 * a2])
    F = 0.5 * (FL + FR) - 0.5 * diss
    return torch.where(wet, F, hll_flux(hL, uL, vL, hR, uR, vR, g, tol))


def face_flux(prm, hL, uL, vL, hR, uR, vR):
    """The two-argument face flux of Sec. 2.1.2 selected by prm.flux."""
    if prm.flux == "ROE":
        return roe_flux(hL, uL, vL, hR, uR, vR, prm.g, prm.tol)
    return hll_flux(hL, uL, vL, hR, uR, vR, prm.g, prm.tol)


def inflow_face_flux(q_in, h_inner, g):
    """Prescribed discharge through an inflow face (normal flux components).

    Mass flux q_in per unit width; momentum flux q_in^2/h_b + g h_b^2 / 2 with
    h_b the larger of the inner dummy depth and the critical depth of q_in.
    """
    hc = torch.pow(q_in * q_in / g, 1.0 / 3.0)
    hb = torch.maximum(h_inner, hc)
    mom = q_in * q_in / hb + 0.5 * g * hb * hb
    zero = torch.zeros_like(h_inner)
    return torch.stack([q_in + zero, mom, zero])


def _relu(a):
    return torch.clamp(a, min=0.0)


def spatial_operator(W: torch.Tensor, bed: Bed, prm: Params, t_stage: float) -> torch.Tensor:
    """The DG2 operators L0, L1x, L1y of Eq. (4) for every element.

    Face limits and dummy limits follow Sec. 2.1.2; the dummy modes follow
    Eq. (5) with (5b) read as the y-directional average mode.
    Returns a (3, 3, ny, nx) tensor laid out like the state.
    """
    g, tol, dx, dy = prm.g, prm.tol, prm.dx, prm.dy
    ny, nx = prm.ny, prm.nx
    P = pad_mirror(W)

    # ---- x-faces: face f (0..nx) separates padded columns f and f+1 --------
    Lc = P[:, :, 1:-1, :-1]
    Rc = P[:, :, 1:-1, 1:]
    hm, qxm, qym = (Lc[:, M0] + Lc[:, MX]).unbind(0)   # U_E^- of the west cell
    hp, qxp, qyp = (Rc[:, M0] - Rc[:, MX]).unbind(0)   # U_W^+ of the east cell
    hsm, um, vm = dummy_limits(hm, qxm, qym, tol)
    hsp, up, vp = dummy_limits(hp, qxp, qyp, tol)
    Fx = face_flux(prm, hsm, um, vm, hsp, up, vp)          # [mass, x-mom, y-mom]
    zsx = bed.zfx - _relu(-hm)                           # z* per x-face

    # ---- y-faces: face f (0..ny) separates padded rows f and f+1 ------------
    Sc = P[:, :, :-1, 1:-1]
    Nc = P[:, :, 1:, 1:-1]
    hn, qxn, qyn = (Sc[:, M0] + Sc[:, MY]).unbind(0)   # U_N^- of the south cell
    hs_, qxs, qys = (Nc[:, M0] - Nc[:, MY]).unbind(0)  # U_S^+ of the north cell
    hsn, vn, un_ = dummy_limits(hn, qyn, qxn, tol)      # normal velocity is v
    hss, vs, us = dummy_limits(hs_, qys, qxs, tol)
    Gn = face_flux(prm, hsn, vn, un_, hss, vs, us)       # [mass, y-mom, x-mom]
    Fy = torch.stack([Gn[0], Gn[2], Gn[1]])              # [mass, x-mom, y-mom]
    zsy = bed.zfy - _relu(-hn)

    # ---- inflow faces: prescribed flux replaces the wall flux ---------------
    Fx = Fx.clone()
    Fy = Fy.clone()
    for bc in prm.inflows:
        Q = hydrograph_value(bc, t_stage).to(F64)
        a, b = bc.first, bc.last + 1
        width = (b - a) * (dy if bc.side in (WEST, EAST) else dx)
        q_in = Q / width
        if float(q_in.detach()) == 0.0:
            continue
        if bc.side == WEST:
            f = inflow_face_flux(q_in, hsp[a:b, 0], g)
            Fx[:, a:b, 0] = torch.stack([f[0], f[1], f[2]])
        elif bc.side == EAST:
            f = inflow_face_flux(q_in, hsm[a:b, nx], g)
            Fx[:, a:b, nx] = torch.stack([-f[0], f[1], f[2]])
        elif bc.side == SOUTH:
            f = inflow_face_flux(q_in, hss[0, a:b], g)
            Fy[:, 0, a:b] = torch.stack([f[0], f[2], f[1]])
        else:
            f = inflow_face_flux(q_in, hsn[ny, a:b], g)
            Fy[:, ny, a:b] = torch.stack([-f[0], f[2], f[1]])

    # ---- water-level and open boundary faces ------------------------------
    # The outside of the face is a ghost state and the face flux is the
    # two-argument flux between inside and ghost, oriented along +x / +y.
    # Open boundary: the inside cell's mean state (zero gradient of the cell
    # average; copying the face limit itself leaves the slope equations of
    # the boundary cell without any upwinding, and an outgoing shock then
    # grows unstable).
    # Level boundary: depth h_b = max(0, eta(t) - z_face); normal velocity
    # from the Riemann invariant that leaves the domain (u - 2c at a west or
    # south face, u + 2c at an east or north face), so that a subcritical
    # boundary carries exactly the prescribed level; an inflow is capped at
    # critical speed c_b (a dry or supercritical inside sends no invariant
    # back); tangential velocity from the inside.
    def ghost_face(side, a, b, eta):
        if side in (WEST, EAST):
            col = 0 if side == WEST else nx
            if side == WEST:
                h_in, u_in, v_in = hsp[a:b, col], up[a:b, col], vp[a:b, col]
            else:
                h_in, u_in, v_in = hsm[a:b, col], um[a:b, col], vm[a:b, col]
            zf = bed.zfx[a:b, col]
        else:
            row = 0 if side == SOUTH else ny
            if side == SOUTH:  # y-face states in (h, normal v, tangential u)
                h_in, u_in, v_in = hss[row, a:b], vs[row, a:b], us[row, a:b]
            else:
                h_in, u_in, v_in = hsn[row, a:b], vn[row, a:b], un_[row, a:b]
            zf = bed.zfy[row, a:b]
        if eta is None:
            # the inside cell's mean state, through the dummy limit
            if side in (WEST, EAST):
                cc = 0 if side == WEST else nx - 1
                hm0, qn0, qt0 = W[H, M0][a:b, cc], W[QX, M0][a:b, cc], W[QY, M0][a:b, cc]
            else:
                rr = 0 if side == SOUTH else ny - 1
                hm0, qn0, qt0 = W[H, M0][rr, a:b], W[QY, M0][rr, a:b], W[QX, M0][rr, a:b]
            hg, ug, vg = dummy_limits(hm0, qn0, qt0, tol)
        else:
            hg = torch.clamp(eta - zf, min=0.0)
            cg, cin = torch.sqrt(g * hg), torch.sqrt(g * h_in)
            if side in (WEST, SOUTH):
                ug = torch.minimum(u_in - 2.0 * cin + 2.0 * cg, cg)
                entering = ug > 0.0
            else:
                ug = torch.maximum(u_in + 2.0 * cin - 2.0 * cg, -cg)
                entering = ug < 0.0
            # water entering from the reservoir brings no tangential motion;
            # water leaving keeps its own
            vg = torch.where(entering, torch.zeros_like(v_in), v_in)
        if side in (WEST, SOUTH):
            f = face_flux(prm, hg, ug, vg, h_in, u_in, v_in)
        else:
            f = face_flux(prm, h_in, u_in, v_in, hg, ug, vg)
        if side == WEST:
            Fx[:, a:b, 0] = f
        elif side == EAST:
            Fx[:, a:b, nx] = f
        elif side == SOUTH:
            Fy[:, 0, a:b] = torch.stack([f[0], f[2], f[1]])
        else:
            Fy[:, ny, a:b] = torch.stack([f[0], f[2], f[1]])

    for bc in prm.levels:
        ghost_face(bc.side, bc.first, bc.last + 1, _table_value(bc.t, bc.eta, t_stage).to(F64))
    for bc in prm.opens:
        ghost_face(bc.side, bc.first, bc.last + 1, None)

    # ---- per element: dummy modes (Eq. 5) and operators (Eq. 4) ------------
    FE, FW = Fx[:, :, 1:], Fx[:, :, :-1]
    GN, GS = Fy[:, 1:, :], Fy[:, :-1, :]
    # own dummy limits at E (the '-' side of face i+1) and W (the '+' side of face i)
    Em = torch.stack([hsm, hsm * um, hsm * vm])[:, :, 1:]
    Wp = torch.stack([hsp, hsp * up, hsp * vp])[:, :, :-1]
    Nm = torch.stack([hsn, hsn * un_, hsn * vn])[:, 1:, :]
    Sp = torch.stack([hss, hss * us, hss * vs])[:, :-1, :]
    U0x, U1x = 0.5 * (Em + Wp), 0.5 * (Em - Wp)
    U0y, U1y = 0.5 * (Nm + Sp), 0.5 * (Nm - Sp)
    zb1x = 0.5 * (zsx[:, 1:] - zsx[:, :-1])
    zb1y = 0.5 * (zsy[1:, :] - zsy[:-1, :])

    def flux_x_at(Uq):
        h_, un, ut = dummy_limits(Uq[0], Uq[1], Uq[2], tol)
        return physical_flux(h_, un, ut, g)

    def flux_y_at(Uq):
        h_, vn_, ut = dummy_limits(Uq[0], Uq[2], Uq[1], tol)
        f = physical_flux(h_, vn_, ut, g)
        return torch.stack([f[0], f[2], f[1]])

    Fgx = flux_x_at(U0x + U1x / SQRT3) + flux_x_at(U0x - U1x / SQRT3)
    Fgy = flux_y_at(U0y + U1y / SQRT3) + flux_y_at(U0y - U1y / SQRT3)

    zero = torch.zeros_like(zb1x)
    L0 = -(FE - FW) / dx - (GN - GS) / dy
    L0 = L0 - 2.0 * g * torch.stack([zero, U0x[0] * zb1x / dx, U0y[0] * zb1y / dy])
    L1x = -(3.0 / dx) * ((FE + FW) - Fgx + (2.0 * g / 3.0) * torch.stack([zero, U1x[0] * zb1x, zero]))
    L1y = -(3.0 / dy) * ((GN + GS) - Fgy + (2.0 * g / 3.0) * torch.stack([zero, zero, U1y[0] * zb1y]))
    return torch.stack([L0, L1x, L1y], dim=1)


# ---------------------------------------------------------------------------
# Sec. 2.1.3: friction splitting and local limiting
# ---------------------------------------------------------------------------

def friction_increment(h, qx, qy, n, dt, g, tol):
    """Implicit friction increment of the discharges at one point.

    The split friction ODE dq/dt = S_f = -C_f |V| q / h (Eq. 1, C_f = g n^2
    h^(-1/3), V the velocity) keeps the depth and the flow direction fixed,
    so over a step dt its implicit solution is exact:
    q_new = q / (1 + dt C_f |V| / h).  Returns q_new - q; zero where the
    point is dry, motionless or frictionless.
    """
    n = _t(n) if not torch.is_tensor(n) else n
    qq = qx * qx + qy * qy
    active = (h > tol) & (qq > 0.0) & (n > 0.0)
    hs = torch.where(active, h, torch.ones_like(h))
    V = torch.sqrt(torch.where(active, qq, torch.ones_like(h))) / hs
    Cf = g * n * n * torch.pow(hs, -1.0 / 3.0)
    factor = 1.0 / (1.0 + dt * Cf * V / hs)
    zero = torch.zeros_like(h)
    return (torch.where(active, qx * factor - qx, zero),
            torch.where(active, qy * factor - qy, zero))


def apply_friction(W: torch.Tensor, n, dt: float, g: float, tol: float) -> torch.Tensor:
    """Friction at the centre and the Gauss points G_x1,2 and G_y1,2 (Fig. 1).

    The centre increment goes to the mean discharges; the slope discharges get
    sqrt(3)/2 times the difference of the two Gauss-point increments, the
    exact inverse of evaluating the planar solution at x_c +- dx/(2 sqrt 3).
    Depth modes are unchanged.
    """
    h, qx, qy = W[H], W[QX], W[QY]
    pts = {
        "c": (h[M0], qx[M0], qy[M0]),
        "x+": (h[M0] + h[MX] / SQRT3, qx[M0] + qx[MX] / SQRT3, qy[M0] + qy[MX] / SQRT3),
        "x-": (h[M0] - h[MX] / SQRT3, qx[M0] - qx[MX] / SQRT3, qy[M0] - qy[MX] / SQRT3),
        "y+": (h[M0] + h[MY] / SQRT3, qx[M0] + qx[MY] / SQRT3, qy[M0] + qy[MY] / SQRT3),
        "y-": (h[M0] - h[MY] / SQRT3, qx[M0] - qx[MY] / SQRT3, qy[M0] - qy[MY] / SQRT3),
    }
    d = {k: friction_increment(*p, n, dt, g, tol) for k, p in pts.items()}
    half_r3 = 0.5 * SQRT3
    out = W.clone()
    for comp, var in ((0, QX), (1, QY)):
        out[var, M0] = W[var, M0] + d["c"][comp]
        out[var, MX] = W[var, MX] + half_r3 * (d["x+"][comp] - d["x-"][comp])
        out[var, MY] = W[var, MY] + half_r3 * (d["y+"][comp] - d["y-"][comp])
    return out


def minmod3(a, b, c):
    """Generalised minmod of three arguments (Eq. 7)."""
    pos = (a > 0) & (b > 0) & (c > 0)
    neg = (a < 0) & (b < 0) & (c < 0)
    mn = torch.minimum(torch.minimum(a, b), c)
    mx = torch.maximum(torch.maximum(a, b), c)
    return torch.where(pos, mn, torch.where(neg, mx, torch.zeros_like(a)))


def local_limit(W: torch.Tensor, bed: Bed, prm: Params) -> torch.Tensor:
    """Local slope limiting of Sec. 2.1.3 (DG2-LL), applied to a snapshot.

    For each direction and each of the components free-surface elevation
    h + z, qx and qy: the discontinuity detector of Eq. (6), written without
    division as max(|jump_E|, |jump_W|) > theta (dx/2) max|U0 -+ U1/sqrt 3|,
    triggers the minmod of Eq. (7) on that slope.  The depth slope is rebuilt
    as the limited surface slope minus the bed slope.  Limiting is switched
    off when the element or either neighbour in that direction is dry.
    Neighbours across walls are the mirror ghosts.
    """
    tol, theta = prm.tol, prm.theta
    P = pad_mirror(W)
    Zp = pad_bed(bed.z)
    out = W.clone()
    for mode, half, sl_c, sl_p, sl_m in (
        (MX, 0.5 * prm.dx, (slice(1, -1), slice(1, -1)), (slice(1, -1), slice(2, None)), (slice(1, -1), slice(0, -2))),
        (MY, 0.5 * prm.dy, (slice(1, -1), slice(1, -1)), (slice(2, None), slice(1, -1)), (slice(0, -2), slice(1, -1))),
    ):
        h0 = P[H, M0]
        wet = (h0[sl_c] > tol) & (h0[sl_p] > tol) & (h0[sl_m] > tol)
        for var in (H, QX, QY):
            if var == H:
                a0 = P[H, M0] + Zp[M0]
                a1 = P[H, mode] + Zp[mode]
            else:
                a0 = P[var, M0]
                a1 = P[var, mode]
            c0, c1 = a0[sl_c], a1[sl_c]
            jump_p = torch.abs((a0[sl_p] - a1[sl_p]) - (c0 + c1))
            jump_m = torch.abs((c0 - c1) - (a0[sl_m] + a1[sl_m]))
            scale = torch.maximum(torch.abs(c0 - c1 / SQRT3), torch.abs(c0 + c1 / SQRT3))
            detect = torch.maximum(jump_p, jump_m) > theta * half * scale
            act = detect & wet
            lim = minmod3(c1, a0[sl_p] - c0, c0 - a0[sl_m])
            if var == H:
                out[H, mode] = torch.where(act, lim - bed.z[mode], W[H, mode])
            else:
                out[var, mode] = torch.where(act, lim, W[var, mode])
    return out


# ---------------------------------------------------------------------------
# Sec. 2.1.2: time step and RK2
# ---------------------------------------------------------------------------

def cfl_min(U: torch.Tensor, prm: Params) -> float:
    """min over wet cell means of min(dx/(|u|+c), dy/(|v|+c)); +inf if none is wet."""
    h0 = U[H, M0]
    wet = h0 > prm.tol
    if not bool(wet.any()):
        return math.inf
    hs = torch.where(wet, h0, torch.ones_like(h0))
    u = torch.abs(U[QX, M0] / hs)
    v = torch.abs(U[QY, M0] / hs)
    c = torch.sqrt(prm.g * hs)
    m = torch.minimum(prm.dx / (u + c), prm.dy / (v + c))
    m = torch.where(wet, m, torch.full_like(m, math.inf))
    return float(m.min())


def time_step(U: torch.Tensor, prm: Params, t: float, t_end: float = math.inf) -> float:
    """Courant-limited step (Cr of Sec. 2.1.2), capped by dt_max and the time left."""
    if prm.fixed_dt > 0.0:
        dt = prm.fixed_dt
    else:
        dt = min(prm.cfl * cfl_min(U, prm), prm.dt_max)
    return min(dt, t_end - t)


def rain_depth(prm: Params, t: float, dt: float) -> float:
    if prm.rain is None:
        return 0.0
    rate, tb, te = prm.rain
    return rate * max(0.0, min(t + dt, te) - max(t, tb))


def wet_dry_fix(U: torch.Tensor, tol: float, partly_wet_flat: bool = False) -> torch.Tensor:
    """End-of-stage wet/dry treatment of the element modes.

    Dry elements are flagged by the mean depth alone (Sec. 2.1.3): an element
    whose mean depth is at or below tol gets zero discharge modes, and nothing
    else changes.  Mean depths are never changed, so mass is conserved
    exactly.

    With ``partly_wet_flat`` (an option that is not part of the paper's
    method), elements with a wet mean but a face-limit depth at or below tol
    also drop every slope mode, which makes them locally first order at the
    front.
    """
    h0 = U[H, M0]
    dry = h0 <= tol
    out = U.clone()
    zero = torch.zeros_like(h0)
    for var in (QX, QY):
        for m in (M0, MX, MY):
            out[var, m] = torch.where(dry, zero, U[var, m])
    if partly_wet_flat:
        lim = torch.minimum(torch.minimum(h0 + U[H, MX], h0 - U[H, MX]),
                            torch.minimum(h0 + U[H, MY], h0 - U[H, MY]))
        part = (~dry) & (lim <= tol)
        for var in (H, QX, QY):
            for m in (MX, MY):
                out[var, m] = torch.where(part, zero, out[var, m])
    return out


def _stage1(U: torch.Tensor, t: float, bed: Bed, prm: Params, dt: float):
    """Stage input W (rain, friction split, [LL]) and stage-1 result U1."""
    W = U.clone()
    W[H, M0] = W[H, M0] + rain_depth(prm, t, dt)
    W = apply_friction(W, prm.manning, dt, prm.g, prm.tol)
    if prm.variant == "LL":
        W = local_limit(W, bed, prm)
    U1 = wet_dry_fix(W + dt * spatial_operator(W, bed, prm, t), prm.tol, prm.partly_wet_flat)
    return W, U1


def _stage2(W: torch.Tensor, U1: torch.Tensor, t: float, bed: Bed, prm: Params, dt: float):
    if prm.variant == "LL":
        U1 = local_limit(U1, bed, prm)
    U2 = 0.5 * (W + U1 + dt * spatial_operator(U1, bed, prm, t + dt))
    return wet_dry_fix(U2, prm.tol, prm.partly_wet_flat)


def step(U: torch.Tensor, t: float, bed: Bed, prm: Params, dt: float):
    """One time step t -> t + dt: rain, friction, [LL], two RK2 stages."""
    W, U1 = _stage1(U, t, bed, prm, dt)
    return _stage2(W, U1, t, bed, prm, dt)


def step_checked(U: torch.Tensor, t: float, bed: Bed, prm: Params, dt: float):
    """A step whose stage-1 result also keeps the Courant number (an option).

    The step size of Sec. 2.1.2 comes from the state at the start of the
    step, but stage 1 can give a thin film on a steep bank tens of m/s, and
    stage 2 then breaks the Courant bound that keeps depths positive.  Here
    stage 1 is repeated (at most prm.stage_check times) with dt = Cr times the
    Courant minimum of its own result while dt exceeds that; the last attempt
    is kept.  With a fixed step size (or stage_check = 0) this is `step`.
    Returns the new state and the step size used.
    """
    W, U1 = _stage1(U, t, bed, prm, dt)
    if prm.fixed_dt <= 0.0:
        for _ in range(prm.stage_check):
            lim = prm.cfl * cfl_min(U1, prm)
            if not (dt > lim):
                break
            dt = lim
            W, U1 = _stage1(U, t, bed, prm, dt)
    return _stage2(W, U1, t, bed, prm, dt), dt


# ---------------------------------------------------------------------------
# Gauges and diagnostics
# ---------------------------------------------------------------------------

def gauge_cells(xy: np.ndarray, prm: Params):
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    i = np.clip(np.floor((xy[:, 0] - prm.x0) / prm.dx).astype(int), 0, prm.nx - 1)
    j = np.clip(np.floor((xy[:, 1] - prm.y0) / prm.dy).astype(int), 0, prm.ny - 1)
    xi = (xy[:, 0] - (prm.x0 + (i + 0.5) * prm.dx)) / (0.5 * prm.dx)
    zeta = (xy[:, 1] - (prm.y0 + (j + 0.5) * prm.dy)) / (0.5 * prm.dy)
    return i, j, xi, zeta


def sample_gauges(U: torch.Tensor, bed: Bed, prm: Params, xy) -> torch.Tensor:
    """h, eta = h + z, u, v of the planar solution (Eq. 2) at each gauge point."""
    i, j, xi, zeta = gauge_cells(xy, prm)
    out = []
    for k in range(len(i)):
        def at(var):
            return U[var, M0, j[k], i[k]] + xi[k] * U[var, MX, j[k], i[k]] + zeta[k] * U[var, MY, j[k], i[k]]
        h = at(H)
        z = bed.z[M0, j[k], i[k]] + xi[k] * bed.z[MX, j[k], i[k]] + zeta[k] * bed.z[MY, j[k], i[k]]
        wet = bool(h > prm.tol)
        u = at(QX) / h if wet else torch.zeros((), dtype=F64)
        v = at(QY) / h if wet else torch.zeros((), dtype=F64)
        out.append(torch.stack([h, h + z, u, v]))
    return torch.stack(out) if out else torch.zeros((0, 4), dtype=F64)


def mass(U: torch.Tensor, prm: Params) -> float:
    """Eq. (11): the integral of the planar depth over every element is h0 dx dy."""
    return float(U[H, M0].sum()) * prm.dx * prm.dy


def energy(U: torch.Tensor, bed: Bed, prm: Params) -> float:
    """Eq. (12) integrated with the 2 x 2 Gauss rule on each element."""
    g, tol = prm.g, prm.tol
    tot = torch.zeros((), dtype=F64)
    for a in (-1.0 / SQRT3, 1.0 / SQRT3):
        for b in (-1.0 / SQRT3, 1.0 / SQRT3):
            h = U[H, M0] + a * U[H, MX] + b * U[H, MY]
            qx = U[QX, M0] + a * U[QX, MX] + b * U[QX, MY]
            qy = U[QY, M0] + a * U[QY, MX] + b * U[QY, MY]
            z = bed.z[M0] + a * bed.z[MX] + b * bed.z[MY]
            wet = h > tol
            hs = torch.where(wet, h, torch.ones_like(h))
            kin = torch.where(wet, 0.5 * (qx * qx + qy * qy) / hs, torch.zeros_like(h))
            pot = 0.5 * g * ((h + z) ** 2 - z * z)
            tot = tot + (kin + pot).sum()
    return float(tot) * 0.25 * prm.dx * prm.dy


# ---------------------------------------------------------------------------
# Time stepping to a target time
# ---------------------------------------------------------------------------

@dataclass
class RunResult:
    U: torch.Tensor
    t: float
    steps: int
    dts: List[float]
    gauge_t: List[float]
    gauges: List[torch.Tensor]


def run(U: torch.Tensor, bed: Bed, prm: Params, steps: Optional[int] = None,
        t_end: float = math.inf, t0: float = 0.0, gauges=None,
        fixed_dts: Optional[Sequence[float]] = None) -> RunResult:
    """Advance ``steps`` steps, or until ``t_end`` (the last step lands on it).

    ``fixed_dts`` replaces the Courant step by the given sequence (used to
    replay another run's step sizes exactly).
    """
    t = t0
    n = 0
    dts, gts, gvals = [], [], []
    limit = steps if steps is not None else 1 << 62
    while n < limit:
        if fixed_dts is not None:
            if n >= len(fixed_dts):
                break
            dt = float(fixed_dts[n])
        else:
            dt = time_step(U, prm, t, t_end)
        if dt <= 0.0:
            break
        if prm.stage_check > 0:
            U, dt = step_checked(U, t, bed, prm, dt)
        else:
            U = step(U, t, bed, prm, dt)
        t = t_end if (t_end - t) == dt else t + dt
        n += 1
        dts.append(dt)
        if gauges is not None:
            gts.append(t)
            gvals.append(sample_gauges(U, bed, prm, gauges))
    return RunResult(U, t, n, dts, gts, gvals)


def params_from_scenario(sc) -> Params:
    """Build oracle parameters from a workloads.Scenario (plain attribute copy)."""
    man = sc.manning
    man = _t(man) if isinstance(man, np.ndarray) else float(man)
    infl = [InflowBC(b.side, b.first, b.last, _t(b.t), _t(b.Q)) for b in sc.inflows]
    levs = [LevelBC(b.side, b.first, b.last, _t(b.t), _t(b.eta)) for b in sc.levels]
    opens = [OpenBC(side, first, last) for side, first, last in sc.opens]
    return Params(nx=sc.nx, ny=sc.ny, dx=sc.dx, dy=sc.dy, g=sc.g, tol=sc.tol_dry, cfl=sc.cfl,
                  dt_max=sc.dt_max, theta=sc.theta, variant=sc.variant, manning=man,
                  inflows=infl, levels=levs, opens=opens, rain=sc.rain, fixed_dt=sc.fixed_dt,
                  x0=sc.x0, y0=sc.y0, flux=sc.flux, stage_check=sc.stage_check,
                  partly_wet_flat=bool(getattr(sc, "partly_wet_flat", False)))


def setup(sc):
    """(U0, bed, params) for a workloads.Scenario."""
    bed = bed_from_corners(sc.Z)
    U = initial_state(sc.Z, sc.surface, sc.is_eta, sc.qx, sc.qy)
    return U, bed, params_from_scenario(sc)


def to_planes(U: torch.Tensor) -> np.ndarray:
    """(3, 3, ny, nx) -> (9, ny, nx) numpy planes h0,h1x,h1y,qx0,...,qy1y."""
    return U.reshape(9, U.shape[-2], U.shape[-1]).detach().numpy().copy()


def from_planes(P) -> torch.Tensor:
    P = _t(np.asarray(P))
    return P.reshape(3, 3, P.shape[-2], P.shape[-1]).clone()


# ---------------------------------------------------------------------------
# Reverse-mode reference for the adjoint (gradients of a gauge misfit)
# ---------------------------------------------------------------------------

def gauge_misfit_reference(U0: torch.Tensor, bed: Bed, prm: Params, manning: torch.Tensor,
                           side: int, first: int, last: int, t_q: torch.Tensor, Q: torch.Tensor,
                           dt: float, steps: int, gauges, target: torch.Tensor):
    """Loss J = sum over steps n = 1..N and gauges g of (h_g(U^n) - target[n-1, g])^2
    for a fixed step dt, and its gradients with respect to the per-cell
    Manning field and the inflow hydrograph samples Q (at times t_q), by
    reverse-mode automatic differentiation through the oracle's step.

    Returns (J, dJ/dmanning, dJ/dQ) as float64 tensors.  Every step of the
    forward map is the plain oracle step above; torch's autograd supplies the
    exact reverse pass of that arithmetic (ties of min/max split the gradient
    evenly, derivatives of branch decisions are zero).
    """
    n = manning.detach().clone().requires_grad_(True)
    q = Q.detach().clone().requires_grad_(True)
    p = Params(**{**prm.__dict__})
    p.manning = n
    p.inflows = [InflowBC(side, first, last, t_q.to(F64), q)]
    p.fixed_dt = dt
    U = U0.clone()
    t = 0.0
    J = torch.zeros((), dtype=F64)
    for k in range(steps):
        U = step(U, t, bed, p, dt)
        t = t + dt
        h = sample_gauges(U, bed, p, gauges)[:, 0]
        J = J + ((h - target[k]) ** 2).sum()
    J.backward()
    return J.detach(), n.grad.detach().clone(), q.grad.detach().clone()
