// HIP kernels of the DG2 step for gfx950 (CDNA4, wave64).
//
// Stage kernels (one launch per RK stage, Sec. 2.1.2): every wavefront owns a
// strip of output columns plus one halo column on each side and marches up
// R rows of the grid.  Each lane holds one cell column.  For every row the
// lane builds the stage input (rain + friction split of Sec. 2.1.3 in stage
// 1), its four dummy face limits (Sec. 2.1.2), the north-face flux with the
// row above (kept in registers for the next row as its south face) and the
// east-face flux with the neighbouring lane; the west-face flux arrives from
// the lane to the west by a cross-lane shuffle.  Every face flux is
// evaluated once, nothing goes through LDS, and each state plane is read
// once per stage with unit-stride, wave-wide loads (structure of arrays).
//
// Stage 2 writes U^{n+1} in place over U^n (or into a separate buffer): a
// lane reads U^n only at the cell it writes, and halo lanes read only the
// stage-1 planes.  On request the NL stages also store the wet/dry decision
// of every result cell, which the adjoint step needs.  Stage 2's tail folds
// the Courant candidate of every new cell into a wave minimum and one atomic
// per wavefront; a single-thread plan kernel then turns the minimum into the
// next step size on the device, so queued steps never wait for the host.
//
// For DG2-NL the fused step kernel further down runs both stages in one
// pass, stage 1 a row ahead of stage 2 with its result in registers, and
// writes the new state to a second buffer.
//
// Tiles whose halo lies inside the grid run a form of the march with the
// boundary treatment compiled out (template flags); the fused kernel's
// interior form also runs two rows per loop iteration.  All forms do the
// same arithmetic, so results do not depend on which form a cell gets.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dg2_internal.h"

namespace dg2 {

template <typename real>
struct Row {
  real W[9];
  real eh, eu, ev, er;  // east face, west ('-') side: dummy h*, u, v and raw depth
  real wh, wu, wv;      // west face, east ('+') side
  real nh, nu, nv, nr;  // north face, south ('-') side, raw depth
  real sh, su, sv;      // south face, north ('+') side
};

template <typename real>
__device__ __forceinline__ void row_limits(Row<real> &r, real tol) {
  const real *W = r.W;
  r.er = W[0] + W[1];
  dummy_limit(r.er, W[3] + W[4], W[6] + W[7], tol, r.eh, r.eu, r.ev);
  dummy_limit(W[0] - W[1], W[3] - W[4], W[6] - W[7], tol, r.wh, r.wu, r.wv);
  r.nr = W[0] + W[2];
  dummy_limit(r.nr, W[3] + W[5], W[6] + W[8], tol, r.nh, r.nu, r.nv);
  dummy_limit(W[0] - W[2], W[3] - W[5], W[6] - W[8], tol, r.sh, r.su, r.sv);
}

// Flux through the y-face between a lower row and the row above it, as
// [mass, x-momentum, y-momentum].
template <int FLUX, typename real>
__device__ __forceinline__ void y_face(const Row<real> &lo, const Row<real> &hi, real g, real tol,
                                       real &G0, real &G1, real &G2) {
  real m, fn, ft;
  face_flux<FLUX>(lo.nh, lo.nv, lo.nu, hi.sh, hi.sv, hi.su, g, tol, m, fn, ft);
  G0 = m;
  G1 = ft;
  G2 = fn;
}

// DG2 operators of one element (Eq. 4) from its dummy face limits (carried
// in the row record), the four face fluxes and the revised bed slopes
// zbx = (z*_E - z*_W)/2, zby = (z*_N - z*_S)/2: dummy modes by Eq. (5),
// physical fluxes at the Gauss points U0 +- U1/sqrt(3), then L0, L1x, L1y.
template <typename real>
__device__ __forceinline__ void cell_operator(const Row<real> &cur, real FE0, real FE1, real FE2,
                                              real FW0, real FW1, real FW2, real GN0, real GN1,
                                              real GN2, real GS0, real GS1, real GS2, real zbx,
                                              real zby, real g, real tol, real idx, real idy,
                                              real *Lop) {
  const real half = real(0.5), is3 = real(kInvSqrt3), two_g = real(2) * g;
  const real tg3 = real(2) * g / real(3);
  const real e1 = cur.eh * cur.eu, e2 = cur.eh * cur.ev;
  const real w1 = cur.wh * cur.wu, w2 = cur.wh * cur.wv;
  const real A0 = half * (cur.eh + cur.wh), A1 = half * (e1 + w1), A2 = half * (e2 + w2);
  const real B0 = half * (cur.eh - cur.wh), B1 = half * (e1 - w1), B2 = half * (e2 - w2);
  const real n1 = cur.nh * cur.nu, n2 = cur.nh * cur.nv;
  const real s1 = cur.sh * cur.su, s2 = cur.sh * cur.sv;
  const real C0 = half * (cur.nh + cur.sh), C1 = half * (n1 + s1), C2 = half * (n2 + s2);
  const real D0 = half * (cur.nh - cur.sh), D1 = half * (n1 - s1), D2 = half * (n2 - s2);
  real Fp0, Fp1, Fp2, Fm0, Fm1, Fm2, Gp0, Gp1, Gp2, Gm0, Gm1, Gm2;
  flux_x(A0 + B0 * is3, A1 + B1 * is3, A2 + B2 * is3, g, tol, Fp0, Fp1, Fp2);
  flux_x(A0 - B0 * is3, A1 - B1 * is3, A2 - B2 * is3, g, tol, Fm0, Fm1, Fm2);
  flux_y(C0 + D0 * is3, C1 + D1 * is3, C2 + D2 * is3, g, tol, Gp0, Gp1, Gp2);
  flux_y(C0 - D0 * is3, C1 - D1 * is3, C2 - D2 * is3, g, tol, Gm0, Gm1, Gm2);
  const real m3x = real(-3) * idx, m3y = real(-3) * idy;
  Lop[0] = -(FE0 - FW0) * idx - (GN0 - GS0) * idy;
  Lop[3] = -(FE1 - FW1) * idx - (GN1 - GS1) * idy - two_g * A0 * zbx * idx;
  Lop[6] = -(FE2 - FW2) * idx - (GN2 - GS2) * idy - two_g * C0 * zby * idy;
  Lop[1] = m3x * ((FE0 + FW0) - (Fp0 + Fm0));
  Lop[4] = m3x * ((FE1 + FW1) - (Fp1 + Fm1) + tg3 * B0 * zbx);
  Lop[7] = m3x * ((FE2 + FW2) - (Fp2 + Fm2));
  Lop[2] = m3y * ((GN0 + GS0) - (Gp0 + Gm0));
  Lop[5] = m3y * ((GN1 + GS1) - (Gp1 + Gm1));
  Lop[8] = m3y * ((GN2 + GS2) - (Gp2 + Gm2) + tg3 * D0 * zby);
}

// One side's boundary segment as a lane sees it: kind (kBc*), whether this
// lane's current face lies on it, the stage value (unit discharge or level)
// and, for a level, the bed at the face.
template <typename real>
struct Bface {
  int kind;
  bool on;
  real val, zf;
};

// Bed value at the face of cell (j, i) on side 0..3 (W, E, S, N).
template <typename real>
__device__ __forceinline__ real face_bed(const Scen<real> &s, int j, int i, int side) {
  const unsigned off = (unsigned)(j * s.nx + i) * (unsigned)sizeof(real);
  const real z0 = ld_at(s.z, off);
  const real z1 = ld_at(s.z + (side < 2 ? 1 : 2) * s.P, off);
  return (side == 0 || side == 2) ? z0 - z1 : z0 + z1;
}

// Whether a side's segment is active at this stage: an inflow with zero
// discharge is a wall.
template <typename real>
__device__ __forceinline__ bool side_on(int kind, real val) {
  return kind == kBcInflow ? val != real(0) : (kind == kBcLevel || kind == kBcOpen);
}

// North face of a row (the y-face to the row above) as [mass, x-mom, y-mom];
// a boundary segment on the north wall replaces the flux.  dN = max(0, -h_N^-)
// for the wall revision of the bed at that face.
template <int FLUX, typename real>
__device__ __forceinline__ void north_face(const Row<real> &cur, const Row<real> &nxt,
                                           const Bface<real> &b, real g, real tol, real &G0,
                                           real &G1, real &G2, real &dN) {
  y_face<FLUX>(cur, nxt, g, tol, G0, G1, G2);
  dN = dmax(real(0), -cur.nr);
  if (b.on) {
    if (b.kind == kBcInflow) {
      inflow_flux(b.val, cur.nh, g, G0, G2);
      G0 = -G0;
      G1 = real(0);
    } else {
      real fn, ft;
      ghost_face_flux<FLUX>(b.kind, false, b.val, b.zf, cur.nh, cur.nv, cur.nu, cur.W[0], cur.W[6],
                            cur.W[3], g, tol, G0, fn, ft);
      G1 = ft;
      G2 = fn;
    }
  }
}

// South face of a row (the y-face to the row below, lo); a boundary segment
// on the south wall replaces the flux.  dS = max(0, -h_N^- of lo).
template <int FLUX, typename real>
__device__ __forceinline__ void south_face(const Row<real> &lo, const Row<real> &cur,
                                           const Bface<real> &b, real g, real tol, real &G0,
                                           real &G1, real &G2, real &dS) {
  y_face<FLUX>(lo, cur, g, tol, G0, G1, G2);
  dS = dmax(real(0), -lo.nr);
  if (b.on) {
    if (b.kind == kBcInflow) {
      inflow_flux(b.val, cur.sh, g, G0, G2);
      G1 = real(0);
    } else {
      real fn, ft;
      ghost_face_flux<FLUX>(b.kind, true, b.val, b.zf, cur.sh, cur.sv, cur.su, cur.W[0], cur.W[6],
                            cur.W[3], g, tol, G0, fn, ft);
      G1 = ft;
      G2 = fn;
    }
  }
}

// East face of every lane's cell (with the '+' limit of the lane to the east)
// and its west face (the east face of the lane to the west), with boundary
// segments on the west and east walls, and the wall-revision depths.  On
// the west wall the face is computed by the ghost lane west of the domain,
// whose row is the mirror image of the first cell (mean qx negated).
template <int FLUX, typename real>
__device__ __forceinline__ void east_west_faces(const Row<real> &cur, const Bface<real> &bW,
                                                const Bface<real> &bE, real g, real tol, real &FE0,
                                                real &FE1, real &FE2, real &FW0, real &FW1,
                                                real &FW2, real &dE, real &dW) {
  const real ph = __shfl_down(cur.wh, 1, 64);
  const real pu = __shfl_down(cur.wu, 1, 64);
  const real pv = __shfl_down(cur.wv, 1, 64);
  face_flux<FLUX>(cur.eh, cur.eu, cur.ev, ph, pu, pv, g, tol, FE0, FE1, FE2);
  if (bW.on) {
    if (bW.kind == kBcInflow) {
      inflow_flux(bW.val, ph, g, FE0, FE1);
      FE2 = real(0);
    } else {
      ghost_face_flux<FLUX>(bW.kind, true, bW.val, bW.zf, ph, pu, pv, cur.W[0], -cur.W[3], cur.W[6],
                            g, tol, FE0, FE1, FE2);
    }
  }
  if (bE.on) {
    if (bE.kind == kBcInflow) {
      inflow_flux(bE.val, cur.eh, g, FE0, FE1);
      FE0 = -FE0;
      FE2 = real(0);
    } else {
      ghost_face_flux<FLUX>(bE.kind, false, bE.val, bE.zf, cur.eh, cur.eu, cur.ev, cur.W[0], cur.W[3],
                            cur.W[6], g, tol, FE0, FE1, FE2);
    }
  }
  dE = dmax(real(0), -cur.er);
  FW0 = __shfl_up(FE0, 1, 64);
  FW1 = __shfl_up(FE1, 1, 64);
  FW2 = __shfl_up(FE2, 1, 64);
  dW = __shfl_up(dE, 1, 64);
}

// Stage-2 bookkeeping of a new cell state o: Courant candidate, NaN and
// negative-depth flags, and gauge samples of the planar solution (Eq. 2).
template <typename real>
__device__ __forceinline__ void new_state_checks(const Scen<real> &s, const real *o, long long cidx,
                                                 unsigned long long gmask, long long gslot, real g,
                                                 real tol, double &mloc, unsigned &flags) {
  const double m = cfl_candidate(o[0], o[3], o[6], g, tol, s.dx, s.dy);
  mloc = m < mloc ? m : mloc;
  if (o[0] != o[0]) flags |= kFlagNaN;
  if (o[0] < real(0)) flags |= kFlagNegative;
  if (gmask) {
    for (int k = 0; k < s.ng; ++k) {
      if (!((gmask >> k) & 1ull)) continue;
      if (s.g_cell[k] != (int)cidx) continue;
      const real xi = s.g_xi[k], ze = s.g_zeta[k];
      const real h = o[0] + xi * o[1] + ze * o[2];
      const real qx = o[3] + xi * o[4] + ze * o[5];
      const real qy = o[6] + xi * o[7] + ze * o[8];
      real *gb = s.g_buf + (gslot + k) * 4;
      gb[0] = h;
      gb[1] = h + s.g_z[k];
      gb[2] = h > tol ? qx / h : real(0);
      gb[3] = h > tol ? qy / h : real(0);
    }
  }
}

// Gauges inside this wavefront's output rectangle, as a bit mask.
template <typename real>
__device__ __forceinline__ unsigned long long gauge_mask(const Scen<real> &s, int c0, int cols,
                                                         int j0, int j1) {
  unsigned long long gmask = 0;
  for (int k = 0; k < s.ng; ++k) {
    const int gc = s.g_cell[k];
    const int gj = gc / s.nx, gi = gc - gj * s.nx;
    if (gj >= j0 && gj < j1 && gi >= c0 && gi < c0 + cols) gmask |= 1ull << k;
  }
  return gmask;
}

// Wave minimum of the Courant candidates and one atomic per wavefront on the
// order-preserving bit pattern of a positive double; flags are OR-ed in.
template <typename real>
__device__ __forceinline__ void publish_min(const Scen<real> &s, int lane, double mloc,
                                            unsigned flags) {
  const unsigned long long bits = wave_min_u64((unsigned long long)__double_as_longlong(mloc));
  const unsigned long long anyflag = __ballot(flags != 0);
  if (lane == 0 && bits != kInfBits) {
    const unsigned long long seen =
        __hip_atomic_load(&s.ctrl->minbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bits < seen) atomicMin(&s.ctrl->minbits, bits);
  }
  if (anyflag && flags) atomicOr(&s.ctrl->flags, flags);
}

// Raw planes of one row for the lane's column (clamped into the grid) and,
// in stage 1, its Manning value.
template <typename real, int STAGE>
struct Raw {
  real W[9];
  real n;
};

template <typename real, int STAGE>
__device__ __forceinline__ void load_raw(const Scen<real> &s, const real *src, int r, int ci,
                                         Raw<real, STAGE> &raw) {
  const int rs = r < 0 ? 0 : (r >= s.ny ? s.ny - 1 : r);
  const unsigned off = (unsigned)(rs * s.nx + ci) * (unsigned)sizeof(real);
#pragma unroll
  for (int k = 0; k < 9; ++k) raw.W[k] = ld_at(src + k * s.P, off);
  if (STAGE == 1) raw.n = s.n ? ld_at(s.n, off) : s.n_uniform;
}

// Stage input of one row from its raw planes: mirror ghosts, then in stage 1
// rain and the friction split, then the dummy face limits.
template <typename real, int STAGE>
__device__ __forceinline__ void build_row(const Raw<real, STAGE> &raw, int r, int ny, bool mx,
                                          real rain, real gdt, real tol, Row<real> &row) {
#pragma unroll
  for (int k = 0; k < 9; ++k) row.W[k] = raw.W[k];
  mirror(row.W, mx, (r < 0) || (r >= ny));
  if (STAGE == 1) {
    row.W[0] += rain;
    apply_friction(row.W, gdt * raw.n * raw.n, tol);
  }
  row_limits(row, tol);
}

// Per-cell data of an output row: bed slopes and, in stage 2, the state U^n
// and Manning value that rebuild the friction-split stage-1 input W1.
template <typename real, int STAGE>
struct Own {
  real z1x, z1y;
  real U[STAGE == 2 ? 9 : 1];
  real n;
};

template <typename real, int STAGE>
__device__ __forceinline__ void load_own(const Scen<real> &s, long long cidx, Own<real, STAGE> &o) {
  const unsigned off = (unsigned)cidx * (unsigned)sizeof(real);
  o.z1x = ld_at(s.z + s.P, off);
  o.z1y = ld_at(s.z + 2 * s.P, off);
  if (STAGE == 2) {
#pragma unroll
    for (int k = 0; k < 9; ++k) o.U[k] = ld_at(s.U + k * s.P, off);
    o.n = s.n ? ld_at(s.n, off) : s.n_uniform;
  }
}

// Software-pipelined march: the loads of the row after next are issued at
// the top of each iteration and consumed one iteration later, so they have a
// whole row of arithmetic to hide behind; a row's own data (bed slopes and,
// in stage 2, U^n and n) is loaded at the top of its iteration, ahead of the
// flux arithmetic of that row.  Prefetching the own data a row earlier as
// well costs more registers than it gains.
//
// Even segments march up and odd segments march down, so two neighbouring
// segments reach their common boundary at about the same time and each one's
// halo row is still in L2 when the other reads it.  The face between two
// rows is always y_face(lower, upper), so the direction changes no result.
// The carried face (CF, dC) is the south face of the current row when
// marching up and its north face when marching down.
// EDGE = false: an interior tile, whose boundary treatment is compiled out.
template <typename real, int STAGE, int FLUX, bool down, bool EDGE>
__device__ __forceinline__ void march_nl_dir(const Scen<real> &s, const Consts &c, int strip, int seg,
                                             int R, int lane) {
  const double dtd = s.ctrl->dt;
  if (!(dtd > 0.0)) return;

  const real dt = (real)dtd, g = (real)c.g, tol = (real)c.tol;
  const bool flat = c.flat != 0;
  const real half = real(0.5);
  const int i = strip * kStripNL + lane - 1;
  const int j0 = seg * R, j1 = min(j0 + R, s.ny);
  const int d = down ? -1 : 1;
  const int jfirst = down ? j1 - 1 : j0, jstop = down ? j0 - 1 : j1;
  const bool own = lane >= 1 && lane <= kStripNL && (!EDGE || i < s.nx);
  const int ci = !EDGE ? i : (i < 0 ? 0 : (i >= s.nx ? s.nx - 1 : i));
  const bool mx = EDGE && ((i < 0) || (i >= s.nx));
  const real rain = (real)s.ctrl->rain;
  const real gdt = g * dt;
  const real *src = STAGE == 1 ? s.U : s.U1;
  real *dst = STAGE == 1 ? s.U1 : s.Uout;

  const int si = STAGE - 1;
  const real qW = (real)s.ctrl->qin[0][si], qE = (real)s.ctrl->qin[1][si];
  const real qS = (real)s.ctrl->qin[2][si], qN = (real)s.ctrl->qin[3][si];
  const int kW = s.bkind[0], kE = s.bkind[1], kS = s.bkind[2], kN = s.bkind[3];
  const bool faceW = EDGE && (i == -1) && side_on(kW, qW);
  const bool faceE = EDGE && (i == s.nx - 1) && side_on(kE, qE);
  const bool colS = EDGE && side_on(kS, qS) && i >= s.seg_first[2] && i <= s.seg_last[2];
  const bool colN = EDGE && side_on(kN, qN) && i >= s.seg_first[3] && i <= s.seg_last[3];

  // gauges owned by this wavefront
  unsigned long long gmask = 0;
  long long gslot = 0;
  if (STAGE == 2 && s.ng > 0) {
    gmask = gauge_mask(s, strip * kStripNL, kStripNL, j0, j1);
    gslot = (s.ctrl->gauge_written % s.g_cap) * s.ng;
  }

  Row<real> cur, nxt;
  Raw<real, STAGE> rawA, rawN;
  Own<real, STAGE> ownC;
  real CF0, CF1, CF2, dC;
  {
    Row<real> back;
    load_raw<real, STAGE>(s, src, jfirst - d, ci, rawA);
    load_raw<real, STAGE>(s, src, jfirst, ci, rawN);
    build_row<real, STAGE>(rawA, jfirst - d, s.ny, mx, rain, gdt, tol, back);
    load_raw<real, STAGE>(s, src, jfirst + d, ci, rawA);
    build_row<real, STAGE>(rawN, jfirst, s.ny, mx, rain, gdt, tol, cur);
    if (!down) {
      const bool on = jfirst == 0 && colS;
      const Bface<real> bS{kS, on, qS, on && kS == kBcLevel ? face_bed(s, 0, i, 2) : real(0)};
      south_face<FLUX>(back, cur, bS, g, tol, CF0, CF1, CF2, dC);
    } else {
      const bool on = jfirst == s.ny - 1 && colN;
      const Bface<real> bN{kN, on, qN, on && kN == kBcLevel ? face_bed(s, s.ny - 1, i, 3) : real(0)};
      north_face<FLUX>(cur, back, bN, g, tol, CF0, CF1, CF2, dC);
    }
  }

  double mloc = __longlong_as_double((long long)kInfBits);
  unsigned flags = 0;

  for (int j = jfirst; j != jstop; j += d) {
    // prefetch: the row after next, and the own data of this row
    if (down ? (j - 2 >= j0 - 1) : (j + 2 <= j1)) load_raw<real, STAGE>(s, src, j + 2 * d, ci, rawN);
    if (own) load_own<real, STAGE>(s, (long long)j * s.nx + i, ownC);

    build_row<real, STAGE>(rawA, j + d, s.ny, mx, rain, gdt, tol, nxt);

    real GN0, GN1, GN2, dN, GS0, GS1, GS2, dS;
    if (!down) {
      const bool on = j == s.ny - 1 && colN;
      const Bface<real> bN{kN, on, qN, on && kN == kBcLevel ? face_bed(s, s.ny - 1, i, 3) : real(0)};
      north_face<FLUX>(cur, nxt, bN, g, tol, GN0, GN1, GN2, dN);
      GS0 = CF0;
      GS1 = CF1;
      GS2 = CF2;
      dS = dC;
    } else {
      const bool on = j == 0 && colS;
      const Bface<real> bS{kS, on, qS, on && kS == kBcLevel ? face_bed(s, 0, i, 2) : real(0)};
      south_face<FLUX>(nxt, cur, bS, g, tol, GS0, GS1, GS2, dS);
      GN0 = CF0;
      GN1 = CF1;
      GN2 = CF2;
      dN = dC;
    }
    real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
    const bool onW = faceW && j >= s.seg_first[0] && j <= s.seg_last[0];
    const bool onE = faceE && j >= s.seg_first[1] && j <= s.seg_last[1];
    const Bface<real> bW{kW, onW, qW, onW && kW == kBcLevel ? face_bed(s, j, 0, 0) : real(0)};
    const Bface<real> bE{kE, onE, qE, onE && kE == kBcLevel ? face_bed(s, j, s.nx - 1, 1) : real(0)};
    east_west_faces<FLUX>(cur, bW, bE, g, tol, FE0, FE1, FE2, FW0, FW1, FW2, dE, dW);

    if (own) {
      const long long cidx = (long long)j * s.nx + i;
      real W1[9];
      if (STAGE == 2) {
#pragma unroll
        for (int k = 0; k < 9; ++k) W1[k] = ownC.U[k];
        W1[0] += rain;
        apply_friction(W1, gdt * ownC.n * ownC.n, tol);
      }
      real Lop[9];
      cell_operator(cur, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                    ownC.z1x - half * dE + half * dW, ownC.z1y - half * dN + half * dS, g, tol,
                    s.idx, s.idy, Lop);
      real o[9];
      if (STAGE == 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k) o[k] = cur.W[k] + dt * Lop[k];
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) o[k] = half * (W1[k] + cur.W[k] + dt * Lop[k]);
      }
      const unsigned code = wet_dry_fix(o, tol, flat);
      const unsigned off = (unsigned)cidx * (unsigned)sizeof(real);
#pragma unroll
      for (int k = 0; k < 9; ++k) st_at(dst + k * s.P, off, o[k]);
      if (s.mask) s.mask[cidx] = (unsigned char)code;

      if (STAGE == 2) new_state_checks(s, o, cidx, gmask, gslot, g, tol, mloc, flags);
    }

    cur = nxt;
    rawA = rawN;
    if (!down) {
      CF0 = GN0;
      CF1 = GN1;
      CF2 = GN2;
      dC = dN;
    } else {
      CF0 = GS0;
      CF1 = GS1;
      CF2 = GS2;
      dC = dS;
    }
  }

  if (STAGE == 2) publish_min(s, lane, mloc, flags);
}

// Stage 1 of an interior tile (rows j0 - 1 .. j0 + R and columns i0 - 1 ..
// i0 + 62 inside the grid) runs a march with the boundary treatment compiled
// out (same arithmetic, bitwise equal): 7 % faster in FP64, 2 % in FP32.
// Stage 2 keeps one march, whose FP64 form ran 2 % slower split.
template <typename real, int STAGE, int FLUX>
__device__ __forceinline__ void march_nl(const Scen<real> &s, const Consts &c, int strip, int seg,
                                         int R, int lane) {
  const int j0 = seg * R;
  const bool in = STAGE == 1 && strip >= 1 && strip * kStripNL + 62 <= s.nx - 1 && j0 >= 1 &&
                  j0 + R <= s.ny - 1;
  if (seg & 1) {
    if (in)
      march_nl_dir<real, STAGE, FLUX, true, false>(s, c, strip, seg, R, lane);
    else
      march_nl_dir<real, STAGE, FLUX, true, true>(s, c, strip, seg, R, lane);
  } else {
    if (in)
      march_nl_dir<real, STAGE, FLUX, false, false>(s, c, strip, seg, R, lane);
    else
      march_nl_dir<real, STAGE, FLUX, false, true>(s, c, strip, seg, R, lane);
  }
}

// Work item of a wavefront.  Workgroups go to the 8 XCDs round-robin
// (workgroup b on XCD b % 8); they are renumbered so that each XCD works
// through one contiguous range of items, where neighbouring strips and row
// segments share cache lines (strip edges, halo rows) in the same L2.
// Stage 1 walks the items in the opposite order to stage 2, so that each
// stage starts on the rows the previous one wrote last, which are still in
// the Infinity Cache.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b & 7, k = b >> 3;
  const int per = G >> 3, rem = G & 7;
  return x * per + (x < rem ? x : rem) + k;
}

template <int STAGE>
__device__ __forceinline__ int stage_item(const Launch &L, int &item) {
  item = xcd_block(blockIdx.x, gridDim.x) * L.wpb + (threadIdx.x >> 6);
  if (item >= L.nitems) return 0;
  if (STAGE == 1) item = L.nitems - 1 - item;
  return 1;
}

template <typename real, int STAGE, int FLUX>
__global__ void __launch_bounds__(256, 2) k_stage_nl(Scen<real> s, Consts c, Launch L) {
  int item;
  if (!stage_item<STAGE>(L, item)) return;
  march_nl<real, STAGE, FLUX>(s, c, item % L.nstrips, item / L.nstrips, L.R, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Fused DG2-NL step: both RK stages of Sec. 2.1.2 in one pass.
//
// A wavefront owns 60 output columns (lanes 2..61) and R output rows.  Stage
// 1 marches one row ahead of stage 2 over the output rows and the row beyond
// each end, on every lane; its result U1 stays in registers and feeds stage 2
// of the row behind, which takes U1 of the rows on either side and of the
// lanes on either side (valid on lanes 1..62).  A step thus reads a cell's
// state, Manning value and bed slopes once (plus halos) and writes the new
// state once, and U1 never goes to memory.  The new state goes to a second
// buffer, since neighbouring wavefronts still read U^n; the host then swaps
// the two.  Each cell is computed by the same device functions in the same
// order as by the two stage kernels, so the results are bitwise equal.
// ---------------------------------------------------------------------------

// Face between row r of the march and the next row r + d (the north face of
// r when marching up, its south face when marching down), with a boundary
// segment where that face is the grid edge.
template <int FLUX, bool down, typename real>
__device__ __forceinline__ void face_ahead(const Scen<real> &s, int r, int i, const Row<real> &cur,
                                           const Row<real> &nxt, bool colS, bool colN, real qS,
                                           real qN, real g, real tol, real &F0, real &F1, real &F2,
                                           real &dF) {
  const int kS = s.bkind[2], kN = s.bkind[3];
  if (!down) {
    const bool on = r == s.ny - 1 && colN;
    const Bface<real> b{kN, on, qN, on && kN == kBcLevel ? face_bed(s, s.ny - 1, i, 3) : real(0)};
    north_face<FLUX>(cur, nxt, b, g, tol, F0, F1, F2, dF);
  } else {
    const bool on = r == 0 && colS;
    const Bface<real> b{kS, on, qS, on && kS == kBcLevel ? face_bed(s, 0, i, 2) : real(0)};
    south_face<FLUX>(nxt, cur, b, g, tol, F0, F1, F2, dF);
  }
}

// Face between the previous row r - d (back) and row r.
template <int FLUX, bool down, typename real>
__device__ __forceinline__ void face_behind(const Scen<real> &s, int r, int i, const Row<real> &back,
                                            const Row<real> &cur, bool colS, bool colN, real qS,
                                            real qN, real g, real tol, real &F0, real &F1, real &F2,
                                            real &dF) {
  const int kS = s.bkind[2], kN = s.bkind[3];
  if (!down) {
    const bool on = r == 0 && colS;
    const Bface<real> b{kS, on, qS, on && kS == kBcLevel ? face_bed(s, 0, i, 2) : real(0)};
    south_face<FLUX>(back, cur, b, g, tol, F0, F1, F2, dF);
  } else {
    const bool on = r == s.ny - 1 && colN;
    const Bface<real> b{kN, on, qN, on && kN == kBcLevel ? face_bed(s, s.ny - 1, i, 3) : real(0)};
    north_face<FLUX>(cur, back, b, g, tol, F0, F1, F2, dF);
  }
}

// East and west faces of row r in stage k (0 or 1) of the fused march.
template <int FLUX, typename real>
__device__ __forceinline__ void fused_x_faces(const Scen<real> &s, int r, const Row<real> &cur,
                                              bool faceW, bool faceE, real qW, real qE, real g,
                                              real tol, real &FE0, real &FE1, real &FE2, real &FW0,
                                              real &FW1, real &FW2, real &dE, real &dW) {
  const int kW = s.bkind[0], kE = s.bkind[1];
  const bool onW = faceW && r >= s.seg_first[0] && r <= s.seg_last[0];
  const bool onE = faceE && r >= s.seg_first[1] && r <= s.seg_last[1];
  const Bface<real> bW{kW, onW, qW, onW && kW == kBcLevel ? face_bed(s, r, 0, 0) : real(0)};
  const Bface<real> bE{kE, onE, qE, onE && kE == kBcLevel ? face_bed(s, r, s.nx - 1, 1) : real(0)};
  east_west_faces<FLUX>(cur, bW, bE, g, tol, FE0, FE1, FE2, FW0, FW1, FW2, dE, dW);
}

// The row beyond the grid edge next to a row: its mirror image in y.
template <typename real>
__device__ __forceinline__ void ghost_row_y(const Row<real> &r, real tol, Row<real> &gh) {
#pragma unroll
  for (int k = 0; k < 9; ++k) gh.W[k] = r.W[k];
  mirror(gh.W, false, true);
  row_limits(gh, tol);
}

// Values one row of the fused march hands to the next.
template <typename real>
struct FusedCarry {
  Row<real> A;       // stage-1 input of the current row
  Raw<real, 1> raw;  // raw planes of the row after it
  real CA[4];        // stage-1 face behind the current row (3 fluxes, bed-step term)
  Row<real> B;       // U1 of the row behind (stage 2 outputs it next)
  real CB[4];        // stage-2 face behind that row
  real W1[9];        // stage-1 input of the row behind
  real zx, zy;       // bed slopes of the row behind
};

// Whether a fused tile and its halo lie inside the grid: rows j0 - 2 .. j1 + 1
// and columns i0 - 2 .. i0 + 61 (i0 = 60 strip, j1 = j0 + R).  Such a tile has
// no boundary face, ghost lane, ghost row or clamped column.
template <typename real>
__device__ __forceinline__ bool fused_xin(const Scen<real> &s, int strip) {
  return strip >= 1 && strip * kStripF + 61 <= s.nx - 1;
}
template <typename real>
__device__ __forceinline__ bool fused_yin(const Scen<real> &s, int seg, int R) {
  const int j0 = seg * R;
  return j0 >= 2 && j0 + R + 1 <= s.ny - 1;
}

// CHECK: a trial of the stage-1 Courant check.  s.ctrl is then the check's
// staging block: the launch returns at once unless it is armed, and the
// Courant minimum of the stage-1 result over the output cells goes to its
// minbits1 (the new state's minimum and flags to its minbits and flags).
// XE / YE: the tile touches the west or east / the south or north grid edge;
// without them (an interior tile) the march runs two rows per iteration.
// Dropping a boundary treatment a tile does not need leaves the march fewer
// live scalars and branches (same arithmetic, bitwise equal results).
template <typename real, int FLUX, bool down, bool CHECK, bool XE, bool YE>
__device__ __forceinline__ void march_fused_dir(const Scen<real> &s, const Consts &c, int strip,
                                                int seg, int R, int lane) {
  if (CHECK && s.ctrl->aux == 0u) return;
  const double dtd = s.ctrl->dt;
  if (!(dtd > 0.0)) {
    // an idle step (a run-to target was reached): the host swaps the two
    // state buffers after every step, so the state is carried over unchanged
    const int i = strip * kStripF + lane - 2;
    if (lane >= 2 && lane <= kStripF + 1 && i < s.nx) {
      for (int j = seg * R; j < min(seg * R + R, s.ny); ++j) {
        const unsigned off = (unsigned)(j * s.nx + i) * (unsigned)sizeof(real);
#pragma unroll
        for (int k = 0; k < 9; ++k) st_at(s.Uout + k * s.P, off, ld_at(s.U + k * s.P, off));
      }
    }
    return;
  }

  const real dt = (real)dtd, g = (real)c.g, tol = (real)c.tol;
  const bool flat = c.flat != 0;
  const real half = real(0.5);
  const int ny = s.ny;
  const int i = strip * kStripF + lane - 2;
  const int j0 = seg * R, j1 = min(j0 + R, ny);
  const int d = down ? -1 : 1;
  const int jfirst = down ? j1 - 1 : j0, jlast = down ? j0 : j1 - 1;
  // stage-1 rows: the output rows and the row beyond each end, inside the grid
  const int afirst = min(max(jfirst - d, 0), ny - 1);
  const int alast = min(max(jlast + d, 0), ny - 1);
  const int astop = alast + d;
  const bool own = lane >= 2 && lane <= kStripF + 1 && (!XE || i < s.nx);
  const int ci = !XE ? i : (i < 0 ? 0 : (i >= s.nx ? s.nx - 1 : i));
  const bool mx = XE && ((i < 0) || (i >= s.nx));
  // whether this strip holds the ghost lane west (i = -1) or east (i = nx) of the grid
  const bool wedge = XE && strip == 0;
  const bool eedge = XE && s.nx - strip * kStripF + 2 <= 63;
  const real rain = (real)s.ctrl->rain;
  const real gdt = g * dt;
  const real *src = s.U;
  real *dst = s.Uout;

  // boundary segments of each stage (stage values of the unit discharge or level)
  const int kW = s.bkind[0], kE = s.bkind[1], kS = s.bkind[2], kN = s.bkind[3];
  const real qW1 = (real)s.ctrl->qin[0][0], qE1 = (real)s.ctrl->qin[1][0];
  const real qS1 = (real)s.ctrl->qin[2][0], qN1 = (real)s.ctrl->qin[3][0];
  const real qW2 = (real)s.ctrl->qin[0][1], qE2 = (real)s.ctrl->qin[1][1];
  const real qS2 = (real)s.ctrl->qin[2][1], qN2 = (real)s.ctrl->qin[3][1];
  const bool inS = i >= s.seg_first[2] && i <= s.seg_last[2];
  const bool inN = i >= s.seg_first[3] && i <= s.seg_last[3];
  const bool faceW1 = XE && (i == -1) && side_on(kW, qW1);
  const bool faceW2 = XE && (i == -1) && side_on(kW, qW2);
  const bool faceE1 = XE && (i == s.nx - 1) && side_on(kE, qE1);
  const bool faceE2 = XE && (i == s.nx - 1) && side_on(kE, qE2);
  const bool colS1 = YE && side_on(kS, qS1) && inS, colS2 = YE && side_on(kS, qS2) && inS;
  const bool colN1 = YE && side_on(kN, qN1) && inN, colN2 = YE && side_on(kN, qN2) && inN;

  unsigned long long gmask = 0;
  long long gslot = 0;
  if (s.ng > 0) {
    gmask = gauge_mask(s, strip * kStripF, kStripF, j0, j1);
    gslot = (s.ctrl->gauge_written % s.g_cap) * s.ng;
  }

  double mloc = __longlong_as_double((long long)kInfBits);
  double m1loc = mloc;
  unsigned flags = 0;
  if constexpr (!XE && !YE) {
    // Interior tiles: the row loop written out twice per iteration, with the
    // values carried from row to row in two slots that swap roles, so no
    // register is copied between rows.
    FusedCarry<real> K[2];
    {
      Row<real> back;
      load_raw<real, 1>(s, src, afirst - d, ci, K[0].raw);
      load_raw<real, 1>(s, src, afirst, ci, K[1].raw);
      build_row<real, 1>(K[0].raw, afirst - d, ny, mx, rain, gdt, tol, back);
      load_raw<real, 1>(s, src, afirst + d, ci, K[0].raw);
      build_row<real, 1>(K[1].raw, afirst, ny, mx, rain, gdt, tol, K[0].A);
      face_behind<FLUX, down>(s, afirst, i, back, K[0].A, colS1, colN1, qS1, qN1, g, tol, K[0].CA[0],
                              K[0].CA[1], K[0].CA[2], K[0].CA[3]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) K[0].CB[k] = 0;
    K[0].zx = 0;
    K[0].zy = 0;
    auto row = [&](int r, FusedCarry<real> &kc, FusedCarry<real> &kn) __attribute__((always_inline)) {
      if (down ? (r - 2 >= alast - 1) : (r + 2 <= alast + 1))
        load_raw<real, 1>(s, src, r + 2 * d, ci, kn.raw);
      const unsigned offA = (unsigned)(r * s.nx + ci) * (unsigned)sizeof(real);
      const real zx = ld_at(s.z + s.P, offA), zy = ld_at(s.z + 2 * s.P, offA);

      // ---- stage 1 on row r ----
      build_row<real, 1>(kc.raw, r + d, ny, mx, rain, gdt, tol, kn.A);
      face_ahead<FLUX, down>(s, r, i, kc.A, kn.A, colS1, colN1, qS1, qN1, g, tol, kn.CA[0], kn.CA[1],
                             kn.CA[2], kn.CA[3]);
      real u1[9];
      {
        real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
        fused_x_faces<FLUX>(s, r, kc.A, faceW1, faceE1, qW1, qE1, g, tol, FE0, FE1, FE2, FW0, FW1, FW2,
                            dE, dW);
        const real *CN = down ? kc.CA : kn.CA, *CS = down ? kn.CA : kc.CA;
        const real GN0 = CN[0], GN1 = CN[1], GN2 = CN[2];
        const real GS0 = CS[0], GS1 = CS[1], GS2 = CS[2];
        const real dN = down ? kc.CA[3] : kn.CA[3], dS = down ? kn.CA[3] : kc.CA[3];
        real Lop[9];
        cell_operator(kc.A, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                      zx - half * dE + half * dW, zy - half * dN + half * dS, g, tol, s.idx, s.idy,
                      Lop);
#pragma unroll
        for (int k = 0; k < 9; ++k) u1[k] = kc.A.W[k] + dt * Lop[k];
        (void)wet_dry_fix(u1, tol, flat);
        if (CHECK && own && r >= j0 && r < j1) {
          const double m = cfl_candidate(u1[0], u1[3], u1[6], g, tol, s.dx, s.dy);
          m1loc = m < m1loc ? m : m1loc;
        }
      }
      // ghost lanes beyond the grid take U1 of the edge column (mirrored when the row is built)
      if (wedge) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const real v = __shfl_down(u1[k], 1, 64);
          if (i == -1) u1[k] = v;
        }
      }
      if (eedge) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const real v = __shfl_up(u1[k], 1, 64);
          if (i == s.nx) u1[k] = v;
        }
      }

      // ---- stage 2: U1 of row r arrives ----
      {
        Raw<real, 2> rb;
#pragma unroll
        for (int k = 0; k < 9; ++k) rb.W[k] = u1[k];
        build_row<real, 2>(rb, r, ny, mx, rain, gdt, tol, kn.B);
      }
      if (r == afirst) {
        if (YE && afirst == jfirst) {
          // the row before the first output row is beyond the grid edge
          Row<real> gh;
          ghost_row_y(kn.B, tol, gh);
          face_behind<FLUX, down>(s, r, i, gh, kn.B, colS2, colN2, qS2, qN2, g, tol, kn.CB[0], kn.CB[1],
                                  kn.CB[2], kn.CB[3]);
        }
      } else {
        const int kB = r - d;
        face_ahead<FLUX, down>(s, kB, i, kc.B, kn.B, colS2, colN2, qS2, qN2, g, tol, kn.CB[0], kn.CB[1],
                               kn.CB[2], kn.CB[3]);
        if (kB >= j0 && kB < j1) {
          // output row kB
          real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
          fused_x_faces<FLUX>(s, kB, kc.B, faceW2, faceE2, qW2, qE2, g, tol, FE0, FE1, FE2, FW0, FW1,
                              FW2, dE, dW);
          if (own) {
            const real *CN = down ? kc.CB : kn.CB, *CS = down ? kn.CB : kc.CB;
            const real GN0 = CN[0], GN1 = CN[1], GN2 = CN[2];
            const real GS0 = CS[0], GS1 = CS[1], GS2 = CS[2];
            const real dN = down ? kc.CB[3] : kn.CB[3], dS = down ? kn.CB[3] : kc.CB[3];
            real Lop[9];
            cell_operator(kc.B, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                          kc.zx - half * dE + half * dW, kc.zy - half * dN + half * dS, g, tol, s.idx,
                          s.idy, Lop);
            real o[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) o[k] = half * (kc.W1[k] + kc.B.W[k] + dt * Lop[k]);
            (void)wet_dry_fix(o, tol, flat);
            const long long cidx = (long long)kB * s.nx + i;
            const unsigned off = (unsigned)cidx * (unsigned)sizeof(real);
#pragma unroll
            for (int k = 0; k < 9; ++k) st_at(dst + k * s.P, off, o[k]);
            new_state_checks(s, o, cidx, gmask, gslot, g, tol, mloc, flags);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) kn.W1[k] = kc.A.W[k];
      kn.zx = zx;
      kn.zy = zy;
      };
    int r = afirst;
    int left = (astop - afirst) * d;
    for (; left >= 2; left -= 2, r += 2 * d) {
      row(r, K[0], K[1]);
      row(r + d, K[1], K[0]);
    }
    if (left == 1) row(r, K[0], K[1]);
  } else {
    // stage 1 march state: current row, raw planes of the next two rows, face behind
    Row<real> curA;
    Raw<real, 1> rawA, rawN;
    real CA0, CA1, CA2, dCA;
    {
      Row<real> back;
      load_raw<real, 1>(s, src, afirst - d, ci, rawA);
      load_raw<real, 1>(s, src, afirst, ci, rawN);
      build_row<real, 1>(rawA, afirst - d, ny, mx, rain, gdt, tol, back);
      load_raw<real, 1>(s, src, afirst + d, ci, rawA);
      build_row<real, 1>(rawN, afirst, ny, mx, rain, gdt, tol, curA);
      face_behind<FLUX, down>(s, afirst, i, back, curA, colS1, colN1, qS1, qN1, g, tol, CA0, CA1, CA2,
                              dCA);
    }
    // stage 2 state: U1 row behind, the face behind it, and its stage-1 input and bed slopes
    Row<real> curB;
    real CB0 = 0, CB1 = 0, CB2 = 0, dCB = 0;
    real W1p[9];
    real zxp = 0, zyp = 0;


    for (int r = afirst; r != astop; r += d) {
      if (down ? (r - 2 >= alast - 1) : (r + 2 <= alast + 1))
        load_raw<real, 1>(s, src, r + 2 * d, ci, rawN);
      const unsigned offA = (unsigned)(r * s.nx + ci) * (unsigned)sizeof(real);
      const real zx = ld_at(s.z + s.P, offA), zy = ld_at(s.z + 2 * s.P, offA);

      // ---- stage 1 on row r ----
      Row<real> nxtA;
      build_row<real, 1>(rawA, r + d, ny, mx, rain, gdt, tol, nxtA);
      real FA0, FA1, FA2, dFA;
      face_ahead<FLUX, down>(s, r, i, curA, nxtA, colS1, colN1, qS1, qN1, g, tol, FA0, FA1, FA2, dFA);
      real u1[9];
      {
        real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
        fused_x_faces<FLUX>(s, r, curA, faceW1, faceE1, qW1, qE1, g, tol, FE0, FE1, FE2, FW0, FW1, FW2,
                            dE, dW);
        const real GN0 = down ? CA0 : FA0, GN1 = down ? CA1 : FA1, GN2 = down ? CA2 : FA2;
        const real GS0 = down ? FA0 : CA0, GS1 = down ? FA1 : CA1, GS2 = down ? FA2 : CA2;
        const real dN = down ? dCA : dFA, dS = down ? dFA : dCA;
        real Lop[9];
        cell_operator(curA, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                      zx - half * dE + half * dW, zy - half * dN + half * dS, g, tol, s.idx, s.idy,
                      Lop);
#pragma unroll
        for (int k = 0; k < 9; ++k) u1[k] = curA.W[k] + dt * Lop[k];
        (void)wet_dry_fix(u1, tol, flat);
        if (CHECK && own && r >= j0 && r < j1) {
          const double m = cfl_candidate(u1[0], u1[3], u1[6], g, tol, s.dx, s.dy);
          m1loc = m < m1loc ? m : m1loc;
        }
      }
      // ghost lanes beyond the grid take U1 of the edge column (mirrored when the row is built)
      if (wedge) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const real v = __shfl_down(u1[k], 1, 64);
          if (i == -1) u1[k] = v;
        }
      }
      if (eedge) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const real v = __shfl_up(u1[k], 1, 64);
          if (i == s.nx) u1[k] = v;
        }
      }

      // ---- stage 2: U1 of row r arrives ----
      Row<real> nxtB;
      {
        Raw<real, 2> rb;
#pragma unroll
        for (int k = 0; k < 9; ++k) rb.W[k] = u1[k];
        build_row<real, 2>(rb, r, ny, mx, rain, gdt, tol, nxtB);
      }
      if (r == afirst) {
        if (YE && afirst == jfirst) {
          // the row before the first output row is beyond the grid edge
          Row<real> gh;
          ghost_row_y(nxtB, tol, gh);
          face_behind<FLUX, down>(s, r, i, gh, nxtB, colS2, colN2, qS2, qN2, g, tol, CB0, CB1, CB2,
                                  dCB);
        }
      } else {
        const int kB = r - d;
        real FB0, FB1, FB2, dFB;
        face_ahead<FLUX, down>(s, kB, i, curB, nxtB, colS2, colN2, qS2, qN2, g, tol, FB0, FB1, FB2,
                               dFB);
        if (kB >= j0 && kB < j1) {
          // output row kB
          real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
          fused_x_faces<FLUX>(s, kB, curB, faceW2, faceE2, qW2, qE2, g, tol, FE0, FE1, FE2, FW0, FW1,
                              FW2, dE, dW);
          if (own) {
            const real GN0 = down ? CB0 : FB0, GN1 = down ? CB1 : FB1, GN2 = down ? CB2 : FB2;
            const real GS0 = down ? FB0 : CB0, GS1 = down ? FB1 : CB1, GS2 = down ? FB2 : CB2;
            const real dN = down ? dCB : dFB, dS = down ? dFB : dCB;
            real Lop[9];
            cell_operator(curB, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                          zxp - half * dE + half * dW, zyp - half * dN + half * dS, g, tol, s.idx,
                          s.idy, Lop);
            real o[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) o[k] = half * (W1p[k] + curB.W[k] + dt * Lop[k]);
            (void)wet_dry_fix(o, tol, flat);
            const long long cidx = (long long)kB * s.nx + i;
            const unsigned off = (unsigned)cidx * (unsigned)sizeof(real);
#pragma unroll
            for (int k = 0; k < 9; ++k) st_at(dst + k * s.P, off, o[k]);
            new_state_checks(s, o, cidx, gmask, gslot, g, tol, mloc, flags);
          }
        }
        CB0 = FB0;
        CB1 = FB1;
        CB2 = FB2;
        dCB = dFB;
      }
      curB = nxtB;
#pragma unroll
      for (int k = 0; k < 9; ++k) W1p[k] = curA.W[k];
      zxp = zx;
      zyp = zy;

      curA = nxtA;
      rawA = rawN;
      CA0 = FA0;
      CA1 = FA1;
      CA2 = FA2;
      dCA = dFA;
    }

    if (YE && alast == jlast) {
      // the row after the last output row is beyond the grid edge
      Row<real> gh;
      ghost_row_y(curB, tol, gh);
      real FB0, FB1, FB2, dFB;
      face_ahead<FLUX, down>(s, jlast, i, curB, gh, colS2, colN2, qS2, qN2, g, tol, FB0, FB1, FB2, dFB);
      real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
      fused_x_faces<FLUX>(s, jlast, curB, faceW2, faceE2, qW2, qE2, g, tol, FE0, FE1, FE2, FW0, FW1,
                          FW2, dE, dW);
      if (own) {
        const real GN0 = down ? CB0 : FB0, GN1 = down ? CB1 : FB1, GN2 = down ? CB2 : FB2;
        const real GS0 = down ? FB0 : CB0, GS1 = down ? FB1 : CB1, GS2 = down ? FB2 : CB2;
        const real dN = down ? dCB : dFB, dS = down ? dFB : dCB;
        real Lop[9];
        cell_operator(curB, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                      zxp - half * dE + half * dW, zyp - half * dN + half * dS, g, tol, s.idx, s.idy,
                      Lop);
        real o[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) o[k] = half * (W1p[k] + curB.W[k] + dt * Lop[k]);
        (void)wet_dry_fix(o, tol, flat);
        const long long cidx = (long long)jlast * s.nx + i;
        const unsigned off = (unsigned)cidx * (unsigned)sizeof(real);
#pragma unroll
        for (int k = 0; k < 9; ++k) st_at(dst + k * s.P, off, o[k]);
        new_state_checks(s, o, cidx, gmask, gslot, g, tol, mloc, flags);
      }
    }

  }

  publish_min(s, lane, mloc, flags);
  if (CHECK) {
    const unsigned long long b1 = wave_min_u64((unsigned long long)__double_as_longlong(m1loc));
    if (lane == 0 && b1 != kInfBits) atomicMin(&s.ctrl->minbits1, b1);
  }
}

// One tile of the fused march: the instantiation without the boundary
// treatment a tile does not need (west/east edge, south/north edge).
template <typename real, int FLUX, bool down, bool CHECK>
__device__ __forceinline__ void fused_tile(const Scen<real> &s, const Consts &c, int strip, int seg,
                                           int R, int lane) {
  const bool xin = fused_xin(s, strip), yin = fused_yin(s, seg, R);
  if (xin && yin)
    march_fused_dir<real, FLUX, down, CHECK, false, false>(s, c, strip, seg, R, lane);
  else if (yin)
    march_fused_dir<real, FLUX, down, CHECK, true, false>(s, c, strip, seg, R, lane);
  else if (xin)
    march_fused_dir<real, FLUX, down, CHECK, false, true>(s, c, strip, seg, R, lane);
  else
    march_fused_dir<real, FLUX, down, CHECK, true, true>(s, c, strip, seg, R, lane);
}

template <typename real, int FLUX, bool CHECK>
__global__ void __launch_bounds__(256, sizeof(real) == 8 ? 1 : 3) k_step_nl(Scen<real> s, Consts c, Launch L) {
  int item;
  if (!stage_item<2>(L, item)) return;
  const int strip = item % L.nstrips, seg = item / L.nstrips;
  if (seg & 1)
    fused_tile<real, FLUX, true, CHECK>(s, c, strip, seg, L.R, threadIdx.x & 63);
  else
    fused_tile<real, FLUX, false, CHECK>(s, c, strip, seg, L.R, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// DG2-LL: local slope limiting (Sec. 2.1.3, Eq. 6-7) before each stage.
//
// Halo of two cells: a wavefront owns 60 output columns (lanes 2..61) and a
// lane keeps three consecutive rows of the unlimited stage input.  Row r is
// limited in x with its neighbours from the lanes on either side (cross-lane
// shuffles) and in y with rows r-1 and r+1 from its own registers.  Ghost
// cells at distance d mirror the cell at distance d-1 inside the wall, so the
// limiter evaluated on a ghost lane or row gives exactly the mirror image of
// the limited interior cell, as a ghost of the limited state must be.
// Stage 1 also stores the limited stage-1 input W1 for the RK average of
// stage 2, which therefore reads neither U^n nor the Manning plane.
// ---------------------------------------------------------------------------

// Reflect an index up to two cells outside [0, n) back inside; m tells
// whether an odd number of reflections was used.  Lanes beyond the grid (dead
// lanes of the last strip) are clamped; their values are never used.
__device__ __forceinline__ int reflect2(int i, int n, bool &m) {
  m = false;
  if (i < 0) {
    i = -i - 1;
    m = true;
  }
  if (i >= n) {
    i = 2 * n - i - 1;
    m = !m;
  }
  if (i < 0) {
    i = -i - 1;
    m = !m;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Unlimited stage input of one row and its bed modes.
template <typename real>
struct RowLL {
  real W[9];
  real z0, z1x, z1y;
};

template <typename real, int STAGE>
__device__ __forceinline__ void load_row_ll(const Scen<real> &s, const real *src, int r, int ci,
                                            bool mx, real rain, real gdt, real tol,
                                            RowLL<real> &row) {
  bool my;
  const int rs = reflect2(r, s.ny, my);
  const unsigned off = (unsigned)(rs * s.nx + ci) * (unsigned)sizeof(real);
#pragma unroll
  for (int k = 0; k < 9; ++k) row.W[k] = ld_at(src + k * s.P, off);
  row.z0 = ld_at(s.z, off);
  row.z1x = ld_at(s.z + s.P, off);
  row.z1y = ld_at(s.z + 2 * s.P, off);
  real n = s.n_uniform;
  if (STAGE == 1 && s.n) n = ld_at(s.n, off);
  mirror(row.W, mx, my);
  if (mx) row.z1x = -row.z1x;
  if (my) row.z1y = -row.z1y;
  if (STAGE == 1) {
    row.W[0] += rain;
    apply_friction(row.W, gdt * n * n, tol);
  }
}

template <typename real>
__device__ __forceinline__ real minmod3(real a, real b, real c) {
  if (a > real(0) && b > real(0) && c > real(0)) return dmin(dmin(a, b), c);
  if (a < real(0) && b < real(0) && c < real(0)) return dmax(dmax(a, b), c);
  return real(0);
}

// One slope of Eq. (6)-(7) for a component with mean c0 and slope c1 in the
// element, neighbours (p0, p1) ahead and (m0, m1) behind: the detector
// max(|jump_p|, |jump_m|) > theta (d/2) max|c0 -+ c1/sqrt3| written without
// division, then the generalised minmod.  Returns true and the limited slope
// in out when limiting applies.
template <typename real>
__device__ __forceinline__ bool ll_slope(real c0, real c1, real p0, real p1, real m0, real m1,
                                         real thr, real &out) {
  const real jp = fabs((p0 - p1) - (c0 + c1));
  const real jm = fabs((c0 - c1) - (m0 + m1));
  const real is3 = real(kInvSqrt3);
  const real sc = dmax(fabs(c0 - c1 * is3), fabs(c0 + c1 * is3));
  if (!(dmax(jp, jm) > thr * sc)) return false;
  out = minmod3(c1, p0 - c0, c0 - m0);
  return true;
}

// Limited copy of the middle row c (rows m below, p above); x neighbours come
// from the adjacent lanes.  thx = theta dx/2, thy = theta dy/2.
template <typename real>
__device__ __forceinline__ void limit_row(const RowLL<real> &m, const RowLL<real> &c,
                                          const RowLL<real> &p, real thx, real thy, real tol,
                                          real *out) {
#pragma unroll
  for (int k = 0; k < 9; ++k) out[k] = c.W[k];
  const real e0 = c.W[0] + c.z0, ex = c.W[1] + c.z1x, ey = c.W[2] + c.z1y;  // eta modes
  // x direction: neighbours from the lanes on either side
  const real h0E = __shfl_down(c.W[0], 1, 64), h0W = __shfl_up(c.W[0], 1, 64);
  const real e0E = __shfl_down(e0, 1, 64), e0W = __shfl_up(e0, 1, 64);
  const real exE = __shfl_down(ex, 1, 64), exW = __shfl_up(ex, 1, 64);
  const real u0E = __shfl_down(c.W[3], 1, 64), u0W = __shfl_up(c.W[3], 1, 64);
  const real uxE = __shfl_down(c.W[4], 1, 64), uxW = __shfl_up(c.W[4], 1, 64);
  const real v0E = __shfl_down(c.W[6], 1, 64), v0W = __shfl_up(c.W[6], 1, 64);
  const real vxE = __shfl_down(c.W[7], 1, 64), vxW = __shfl_up(c.W[7], 1, 64);
  real lim;
  if (c.W[0] > tol && h0E > tol && h0W > tol) {
    if (ll_slope(e0, ex, e0E, exE, e0W, exW, thx, lim)) out[1] = lim - c.z1x;
    if (ll_slope(c.W[3], c.W[4], u0E, uxE, u0W, uxW, thx, lim)) out[4] = lim;
    if (ll_slope(c.W[6], c.W[7], v0E, vxE, v0W, vxW, thx, lim)) out[7] = lim;
  }
  // y direction: rows below and above
  if (c.W[0] > tol && p.W[0] > tol && m.W[0] > tol) {
    if (ll_slope(e0, ey, p.W[0] + p.z0, p.W[2] + p.z1y, m.W[0] + m.z0, m.W[2] + m.z1y, thy, lim))
      out[2] = lim - c.z1y;
    if (ll_slope(c.W[3], c.W[5], p.W[3], p.W[5], m.W[3], m.W[5], thy, lim)) out[5] = lim;
    if (ll_slope(c.W[6], c.W[8], p.W[6], p.W[8], m.W[6], m.W[8], thy, lim)) out[8] = lim;
  }
}

template <typename real>
__device__ __forceinline__ void limited_row(const RowLL<real> &m, const RowLL<real> &c,
                                            const RowLL<real> &p, real thx, real thy, real tol,
                                            Row<real> &row) {
  limit_row(m, c, p, thx, thy, tol, row.W);
  row_limits(row, tol);
}

// EDGE = false: an interior tile (rows j0 - 2 .. j0 + R + 1 and columns
// i0 - 2 .. i0 + 61 inside the grid), whose boundary treatment is compiled out.
template <typename real, int STAGE, int FLUX, bool EDGE>
__device__ __forceinline__ void march_ll_tile(const Scen<real> &s, const Consts &c, int strip, int seg,
                                              int R, int lane) {
  const double dtd = s.ctrl->dt;
  if (!(dtd > 0.0)) return;

  const real dt = (real)dtd, g = (real)c.g, tol = (real)c.tol;
  const bool flat = c.flat != 0;
  const real half = real(0.5);
  const real thx = (real)(c.theta * 0.5 * (double)s.dx), thy = (real)(c.theta * 0.5 * (double)s.dy);
  const int i = strip * kStripLL + lane - 2;
  const int j0 = seg * R, j1 = min(j0 + R, s.ny);
  const bool own = lane >= 2 && lane < 2 + kStripLL && (!EDGE || i < s.nx);
  bool mx = false;
  const int ci = EDGE ? reflect2(i, s.nx, mx) : i;
  const real rain = (real)s.ctrl->rain;
  const real gdt = g * dt;
  const real *src = STAGE == 1 ? s.U : s.U1;
  real *dst = STAGE == 1 ? s.U1 : s.Uout;

  const int si = STAGE - 1;
  const real qW = (real)s.ctrl->qin[0][si], qE = (real)s.ctrl->qin[1][si];
  const real qS = (real)s.ctrl->qin[2][si], qN = (real)s.ctrl->qin[3][si];
  const int kW = s.bkind[0], kE = s.bkind[1], kS = s.bkind[2], kN = s.bkind[3];
  const bool faceW = EDGE && (i == -1) && side_on(kW, qW);
  const bool faceE = EDGE && (i == s.nx - 1) && side_on(kE, qE);
  const bool colS = EDGE && side_on(kS, qS) && i >= s.seg_first[2] && i <= s.seg_last[2];
  const bool colN = EDGE && side_on(kN, qN) && i >= s.seg_first[3] && i <= s.seg_last[3];

  unsigned long long gmask = 0;
  long long gslot = 0;
  if (STAGE == 2 && s.ng > 0) {
    gmask = gauge_mask(s, strip * kStripLL, kStripLL, j0, j1);
    gslot = (s.ctrl->gauge_written % s.g_cap) * s.ng;
  }

  RowLL<real> ra, rb, rc;  // unlimited input of rows j-1, j, j+1 (shifted as the march goes)
  Row<real> cur, nxt;      // limited rows j and j+1 with their dummy limits
  real GS0, GS1, GS2, dS;
  {
    RowLL<real> rz;
    Row<real> prev;
    load_row_ll<real, STAGE>(s, src, j0 - 2, ci, mx, rain, gdt, tol, rz);
    load_row_ll<real, STAGE>(s, src, j0 - 1, ci, mx, rain, gdt, tol, ra);
    load_row_ll<real, STAGE>(s, src, j0, ci, mx, rain, gdt, tol, rb);
    load_row_ll<real, STAGE>(s, src, j0 + 1, ci, mx, rain, gdt, tol, rc);
    limited_row(rz, ra, rb, thx, thy, tol, prev);
    limited_row(ra, rb, rc, thx, thy, tol, cur);
    const bool on = j0 == 0 && colS;
    const Bface<real> bS{kS, on, qS, on && kS == kBcLevel ? face_bed(s, 0, i, 2) : real(0)};
    south_face<FLUX>(prev, cur, bS, g, tol, GS0, GS1, GS2, dS);
  }

  double mloc = __longlong_as_double((long long)kInfBits);
  unsigned flags = 0;

  for (int j = j0; j < j1; ++j) {
    // ra, rb, rc hold rows j-1, j, j+1 (unlimited); bring in row j+2
    RowLL<real> rd;
    load_row_ll<real, STAGE>(s, src, j + 2, ci, mx, rain, gdt, tol, rd);
    real W1[9];
    const long long cidx = (long long)j * s.nx + i;
    const unsigned off = (unsigned)cidx * (unsigned)sizeof(real);
    if (STAGE == 2 && own) {
#pragma unroll
      for (int k = 0; k < 9; ++k) W1[k] = ld_at(s.W1 + k * s.P, off);
    }
    limited_row(rb, rc, rd, thx, thy, tol, nxt);

    real GN0, GN1, GN2, dN;
    const bool onN = j == s.ny - 1 && colN;
    const Bface<real> bN{kN, onN, qN, onN && kN == kBcLevel ? face_bed(s, s.ny - 1, i, 3) : real(0)};
    north_face<FLUX>(cur, nxt, bN, g, tol, GN0, GN1, GN2, dN);
    real FE0, FE1, FE2, FW0, FW1, FW2, dE, dW;
    const bool onW = faceW && j >= s.seg_first[0] && j <= s.seg_last[0];
    const bool onE = faceE && j >= s.seg_first[1] && j <= s.seg_last[1];
    const Bface<real> bW{kW, onW, qW, onW && kW == kBcLevel ? face_bed(s, j, 0, 0) : real(0)};
    const Bface<real> bE{kE, onE, qE, onE && kE == kBcLevel ? face_bed(s, j, s.nx - 1, 1) : real(0)};
    east_west_faces<FLUX>(cur, bW, bE, g, tol, FE0, FE1, FE2, FW0, FW1, FW2, dE, dW);

    if (own) {
      real Lop[9];
      cell_operator(cur, FE0, FE1, FE2, FW0, FW1, FW2, GN0, GN1, GN2, GS0, GS1, GS2,
                    rb.z1x - half * dE + half * dW, rb.z1y - half * dN + half * dS, g, tol, s.idx,
                    s.idy, Lop);
      real o[9];
      if (STAGE == 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k) o[k] = cur.W[k] + dt * Lop[k];
#pragma unroll
        for (int k = 0; k < 9; ++k) st_at(s.W1 + k * s.P, off, cur.W[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) o[k] = half * (W1[k] + cur.W[k] + dt * Lop[k]);
      }
      wet_dry_fix(o, tol, flat);
#pragma unroll
      for (int k = 0; k < 9; ++k) st_at(dst + k * s.P, off, o[k]);
      if (STAGE == 2) new_state_checks(s, o, cidx, gmask, gslot, g, tol, mloc, flags);
    }

    ra = rb;
    rb = rc;
    rc = rd;
    cur = nxt;
    GS0 = GN0;
    GS1 = GN1;
    GS2 = GN2;
    dS = dN;
  }

  if (STAGE == 2) publish_min(s, lane, mloc, flags);
}

template <typename real, int STAGE, int FLUX>
__device__ __forceinline__ void march_ll(const Scen<real> &s, const Consts &c, int strip, int seg,
                                         int R, int lane) {
  const int j0 = seg * R;
  const bool in = strip >= 1 && strip * kStripLL + 61 <= s.nx - 1 && j0 >= 2 &&
                  j0 + R + 1 <= s.ny - 1;
  if (in)
    march_ll_tile<real, STAGE, FLUX, false>(s, c, strip, seg, R, lane);
  else
    march_ll_tile<real, STAGE, FLUX, true>(s, c, strip, seg, R, lane);
}

template <typename real, int STAGE, int FLUX>
__global__ void __launch_bounds__(256, 2) k_stage_ll(Scen<real> s, Consts c, Launch L) {
  int item;
  if (!stage_item<STAGE>(L, item)) return;
  march_ll<real, STAGE, FLUX>(s, c, item % L.nstrips, item / L.nstrips, L.R, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Batched ensemble: one persistent launch per stage advances every scenario
// of a batch.  The work list holds (scenario, strip, segment) items of all
// scenarios; the resident wavefronts stride through it, each item running the
// same march as the single-scenario kernels on that scenario's buffers with
// that scenario's own dt, time, inflows and Courant minimum.  Items of
// scenarios that are idle (dt = 0, e.g. already at their target time) return
// at once.
// ---------------------------------------------------------------------------

struct Item {
  int sid, strip, seg, pad;
};

template <typename real, int STAGE, int VARIANT, int FLUX>
__global__ void __launch_bounds__(256, 2) k_batch_stage(const Scen<real> *__restrict__ scens,
                                                     const Item *__restrict__ items, int nitems,
                                                     Consts c, int R, int wpb) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * wpb;
  for (int it = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6)); it < nitems;
       it += nw) {
    const int sid = __builtin_amdgcn_readfirstlane(items[it].sid);
    const int strip = __builtin_amdgcn_readfirstlane(items[it].strip);
    const int seg = __builtin_amdgcn_readfirstlane(items[it].seg);
    const Scen<real> s = scens[sid];
    if (VARIANT == 1)
      march_ll<real, STAGE, FLUX>(s, c, strip, seg, R, lane);
    else
      march_nl<real, STAGE, FLUX>(s, c, strip, seg, R, lane);
  }
}

// Fused step (both RK stages, DG2-NL) for a batch: the same
// persistent stride over the work items, each running the fused march on its
// scenario; the scenario table gives each member's current state (U) and
// the buffer its next state goes to (Uout).
template <typename real, int FLUX>
__global__ void __launch_bounds__(256, sizeof(real) == 8 ? 1 : 3) k_batch_step(const Scen<real> *__restrict__ scens,
                                                    const Item *__restrict__ items, int nitems,
                                                    Consts c, int R, int wpb) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * wpb;
  for (int it = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6)); it < nitems;
       it += nw) {
    const int sid = __builtin_amdgcn_readfirstlane(items[it].sid);
    const int strip = __builtin_amdgcn_readfirstlane(items[it].strip);
    const int seg = __builtin_amdgcn_readfirstlane(items[it].seg);
    const Scen<real> s = scens[sid];
    // two forms only (interior, and every edge): ensemble members are small,
    // so edge tiles are common, and the smaller kernel ran 0.9 % faster on
    // the 256-member ensemble than with the four forms of k_step_nl
    const bool in = fused_xin(s, strip) && fused_yin(s, seg, R);
    if (seg & 1) {
      if (in)
        march_fused_dir<real, FLUX, true, false, false, false>(s, c, strip, seg, R, lane);
      else
        march_fused_dir<real, FLUX, true, false, true, true>(s, c, strip, seg, R, lane);
    } else {
      if (in)
        march_fused_dir<real, FLUX, false, false, false, false>(s, c, strip, seg, R, lane);
      else
        march_fused_dir<real, FLUX, false, false, true, true>(s, c, strip, seg, R, lane);
    }
  }
}

// ---------------------------------------------------------------------------
// Step planner: one thread.  Finishes a step (t += dt, counters, gauge time),
// takes the Courant minimum of the new state, and plans the next step size,
// rain depth and stage inflows.
// ---------------------------------------------------------------------------

// Piecewise-linear hydrograph value at time x, held constant outside the
// samples.  k is the interval of a previous lookup at an earlier or equal
// time (the planner's times only grow); the scan continues from there.
__device__ double hydrograph_at(int n, const double *t, const double *Q, double x, int &k) {
  if (x <= t[0]) return Q[0];
  if (x >= t[n - 1]) return Q[n - 1];
  if (k < 0 || k > n - 2 || !(t[k] <= x)) k = 0;
  while (k + 1 < n && t[k + 1] <= x) ++k;
  const double w = (x - t[k]) / (t[k + 1] - t[k]);
  return Q[k] * (1.0 - w) + Q[k + 1] * w;
}

// The hydrograph samples a lookup usually needs (both ends and the hinted
// interval), loaded together up front; lookups whose time falls in the
// hinted interval then need no further load.
struct HydHint {
  int n, k;
  double t0, tn, tk, tk1, Q0, Qn, Qk, Qk1;
};
__device__ __forceinline__ HydHint hyd_hint(int n, const double *t, const double *Q, int k) {
  HydHint h;
  h.n = n;
  h.k = k < 0 ? 0 : (k > n - 2 ? (n >= 2 ? n - 2 : 0) : k);
  const int k1 = h.k + 1 < n ? h.k + 1 : n - 1;
  h.t0 = t[0];
  h.tn = t[n - 1];
  h.tk = t[h.k];
  h.tk1 = t[k1];
  h.Q0 = Q[0];
  h.Qn = Q[n - 1];
  h.Qk = Q[h.k];
  h.Qk1 = Q[k1];
  return h;
}
// hydrograph_at with the samples of a hint; k as there.  Bitwise the same
// value and interval: a time in [t_k, t_k+1) of a sorted table has k as its
// interval whatever the scan starts from.
__device__ __forceinline__ double hydrograph_hinted(const HydHint &h, const double *t,
                                                    const double *Q, double x, int &k) {
  if (x <= h.t0) return h.Q0;
  if (x >= h.tn) return h.Qn;
  if (k == h.k && h.tk <= x && x < h.tk1) {
    const double w = (x - h.tk) / (h.tk1 - h.tk);
    return h.Qk * (1.0 - w) + h.Qk1 * w;
  }
  return hydrograph_at(h.n, t, Q, x, k);
}

// The pending step from time t with size dt: its rain depth and the
// boundary values (unit inflow or level) at the two stage times.
__device__ void set_step(Ctrl *c, const PlanArgs &p, double dt) {
  const double t = c->t;
  c->dt = dt;
  c->rain = p.rain_rate > 0.0 ? p.rain_rate * fmax(0.0, fmin(t + dt, p.rain_te) - fmax(t, p.rain_tb))
                              : 0.0;
  for (int sd = 0; sd < 4; ++sd) {
    if (p.nhyd[sd] > 0) {
      int k = c->hyd_k[sd];
      const HydHint h = hyd_hint(p.nhyd[sd], p.hyd_t[sd], p.hyd_Q[sd], k);
      c->qin[sd][0] = hydrograph_hinted(h, p.hyd_t[sd], p.hyd_Q[sd], t, k) / p.seg_len[sd];
      const int k0 = k;
      c->qin[sd][1] = hydrograph_hinted(h, p.hyd_t[sd], p.hyd_Q[sd], t + dt, k) / p.seg_len[sd];
      c->hyd_k[sd] = k0;
    } else {
      c->qin[sd][0] = 0.0;
      c->qin[sd][1] = 0.0;
    }
  }
}

__device__ void plan_next(Ctrl *c, const PlanArgs &p) {
  const double t = c->t;
  const double cand = p.fixed_dt > 0.0 ? p.fixed_dt : fmin(p.cfl * c->cflmin, p.dt_max);
  double dt = fmin(cand, c->t_end - t);
  if (!(dt > 0.0)) dt = 0.0;
  set_step(c, p, dt);
}

__device__ void plan_step(Ctrl *c, const PlanArgs &p, int mode, double t_end, int set_tend) {
  if (set_tend) c->t_end = t_end;
  if (mode == kPlanFinishStep) {
    const double dt = c->dt;
    if (!(dt > 0.0)) return;  // the queued step was idle
    const double t0 = c->t;
    const double t1 = (dt == c->t_end - t0) ? c->t_end : t0 + dt;
    c->t = t1;
    c->last_dt = dt;
    c->step += 1;
    if (p.ng > 0) {
      p.gauge_t[c->gauge_written % p.gauge_cap] = t1;
      c->gauge_written += 1;
    }
    mode = kPlanFromMin;
  }
  if (mode == kPlanFromMin) {
    c->cflmin = __longlong_as_double((long long)c->minbits);
    c->minbits = kInfBits;
  }
  plan_next(c, p);
  if (p.hist) {
    const long long m = c->step - p.hist_base;
    if (m >= 0 && m < p.hist_len) p.hist[m] = *c;
  }
}

__global__ void k_plan(Ctrl *c, PlanArgs p, int mode, double t_end, int set_tend) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctrl cl = *c;
  plan_step(&cl, p, mode, t_end, set_tend);
  *c = cl;
}

// Stage-1 Courant check (an option; one thread).  After stage 1 (first) or a
// repeat of it, the Courant minimum of the stage-1 result has been gathered
// in r->minbits.  If the pending step is larger than Cr times that minimum
// (and a repeat is left), shrink it, plan it anew and arm the repeat block r,
// whose copy of the step makes the next stage-1 launch on r run; otherwise
// disarm r, so the remaining repeat launches return at once.  A fixed step
// size is never changed.
__global__ void k_stage_check(Ctrl *c, Ctrl *r, PlanArgs p, int first, int last) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!first && r->aux == 0u) return;
  const double m1 = __longlong_as_double((long long)r->minbits);
  r->minbits = kInfBits;
  const double lim = p.cfl * m1;
  if (!last && p.fixed_dt <= 0.0 && c->dt > lim) {
    set_step(c, p, lim);
    r->dt = c->dt;
    r->rain = c->rain;
    for (int sd = 0; sd < 4; ++sd) {
      r->qin[sd][0] = c->qin[sd][0];
      r->qin[sd][1] = c->qin[sd][1];
    }
    r->aux = 1u;
  } else {
    r->dt = 0.0;
    r->aux = 0u;
  }
}

// One thread per scenario of a batch.
__global__ void k_plan_batch(Ctrl *const *ctrls, const PlanArgs *pa, int n, int mode,
                             double t_end, int set_tend) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  // private copies: every load is issued at once, and the planner's stores
  // cannot alias the arguments it reads afterwards
  Ctrl *const cp = ctrls[k];
  const PlanArgs p = pa[k];
  Ctrl c = *cp;
  plan_step(&c, p, mode, t_end, set_tend);
  *cp = c;
}

// Courant minimum of the state s.U, into *bits (after the state was set from
// the host, or of a stage-1 result for the stage-1 Courant check); returns at
// once when a gate block is given and its step is idle.
template <typename real>
__global__ void __launch_bounds__(256) k_cfl(Scen<real> s, Consts c, const Ctrl *gate,
                                             unsigned long long *bits) {
  if (gate && !(gate->dt > 0.0)) return;
  const long long n = (long long)s.nx * s.ny;
  const real g = (real)c.g, tol = (real)c.tol;
  double m = __longlong_as_double((long long)kInfBits);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const double v = cfl_candidate(s.U[k], s.U[3 * s.P + k], s.U[6 * s.P + k], g, tol, s.dx, s.dy);
    m = v < m ? v : m;
  }
  const unsigned long long mb = wave_min_u64((unsigned long long)__double_as_longlong(m));
  if ((threadIdx.x & 63) == 0 && mb != kInfBits) atomicMin(bits, mb);
}

// Diagnostics: per-block partial sums (mass, energy, min depth, NaN count),
// then one block reduces the partials in a fixed order.
template <typename real>
__global__ void __launch_bounds__(256) k_diag(Scen<real> s, Consts c, double *part) {
  __shared__ double sh[4][256];
  const long long n = (long long)s.nx * s.ny;
  const double g = c.g, tol = c.tol;
  double mass = 0.0, en = 0.0, mn = __longlong_as_double((long long)kInfBits), nan = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const double h0 = s.U[k];
    mass += h0;
    mn = h0 < mn ? h0 : mn;
    if (h0 != h0) nan += 1.0;
    double e = 0.0;
    for (int a = -1; a <= 1; a += 2) {
      for (int b = -1; b <= 1; b += 2) {
        const double xa = a * kInvSqrt3, yb = b * kInvSqrt3;
        const double h = h0 + xa * (double)s.U[s.P + k] + yb * (double)s.U[2 * s.P + k];
        const double qx = (double)s.U[3 * s.P + k] + xa * (double)s.U[4 * s.P + k] +
                          yb * (double)s.U[5 * s.P + k];
        const double qy = (double)s.U[6 * s.P + k] + xa * (double)s.U[7 * s.P + k] +
                          yb * (double)s.U[8 * s.P + k];
        const double z = (double)s.z[k] + xa * (double)s.z[s.P + k] + yb * (double)s.z[2 * s.P + k];
        const double kin = h > tol ? 0.5 * (qx * qx + qy * qy) / h : 0.0;
        e += kin + 0.5 * g * ((h + z) * (h + z) - z * z);
      }
    }
    en += e;
  }
  const int t = threadIdx.x;
  sh[0][t] = mass;
  sh[1][t] = en;
  sh[2][t] = mn;
  sh[3][t] = nan;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      sh[0][t] += sh[0][t + w];
      sh[1][t] += sh[1][t + w];
      sh[2][t] = fmin(sh[2][t], sh[2][t + w]);
      sh[3][t] += sh[3][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[4 * blockIdx.x + 0] = sh[0][0];
    part[4 * blockIdx.x + 1] = sh[1][0];
    part[4 * blockIdx.x + 2] = sh[2][0];
    part[4 * blockIdx.x + 3] = sh[3][0];
  }
}

// Sums the per-block records and scales the two sums (mass by sm, energy by
// se; the library's own diagnostics pass 1 and scale on the host).
__global__ void __launch_bounds__(256) k_diag_final(const double *part, int nb, double *out, double sm,
                                                    double se) {
  __shared__ double sh[4][256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0, m = __longlong_as_double((long long)kInfBits), d = 0.0;
  for (int k = t; k < nb; k += 256) {
    a += part[4 * k];
    b += part[4 * k + 1];
    m = fmin(m, part[4 * k + 2]);
    d += part[4 * k + 3];
  }
  sh[0][t] = a;
  sh[1][t] = b;
  sh[2][t] = m;
  sh[3][t] = d;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      sh[0][t] += sh[0][t + w];
      sh[1][t] += sh[1][t + w];
      sh[2][t] = fmin(sh[2][t], sh[2][t + w]);
      sh[3][t] += sh[3][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = sh[0][0] * sm;
    out[1] = sh[1][0] * se;
    out[2] = sh[2][0];
    out[3] = sh[3][0];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

Launch make_launch(int nx, int ny, int cols, int R, int wpb, int items, int rmax) {
  Launch L;
  L.nstrips = (nx + cols - 1) / cols;
  if (R <= 0) {
    // aim at `items` wavefronts (stage kernels: ~34k, about ten rounds of the
    // ~3k resident slots, so the last round is short; the halo rows are
    // mostly L2 hits, the work items of one XCD being neighbours)
    long long r = (long long)L.nstrips * ny / items;
    R = (int)(r < 4 ? 4 : (r > rmax ? rmax : r));
  }
  if (R > ny) R = ny;
  L.R = R;
  L.wpb = (wpb == 1 || wpb == 2 || wpb == 4) ? wpb : 4;
  L.nitems = L.nstrips * ((ny + R - 1) / R);
  return L;
}

// Kernel instantiation for (stage, variant, flux).
template <typename real, int STAGE, int FLUX>
void queue_stage_kernel(int variant, const Scen<real> &s, const Consts &c, const Launch &L,
                        hipStream_t st) {
  const dim3 block(64 * L.wpb);
  const dim3 grid((L.nitems + L.wpb - 1) / L.wpb);
  if (variant == 1)
    hipLaunchKernelGGL((k_stage_ll<real, STAGE, FLUX>), grid, block, 0, st, s, c, L);
  else
    hipLaunchKernelGGL((k_stage_nl<real, STAGE, FLUX>), grid, block, 0, st, s, c, L);
}

template <typename real>
hipError_t launch_stage(int stage, int variant, const Scen<real> &s, const Consts &c,
                        const Launch &L, hipStream_t st) {
  if (c.flux == kFluxRoe) {
    if (stage == 1)
      queue_stage_kernel<real, 1, kFluxRoe>(variant, s, c, L, st);
    else
      queue_stage_kernel<real, 2, kFluxRoe>(variant, s, c, L, st);
  } else {
    if (stage == 1)
      queue_stage_kernel<real, 1, kFluxHLL>(variant, s, c, L, st);
    else
      queue_stage_kernel<real, 2, kFluxHLL>(variant, s, c, L, st);
  }
  return hipGetLastError();
}

template <typename real>
hipError_t launch_fused(const Scen<real> &s, const Consts &c, const Launch &L, hipStream_t st,
                        bool check) {
  const dim3 block(64 * L.wpb);
  const dim3 grid((L.nitems + L.wpb - 1) / L.wpb);
  if (c.flux == kFluxRoe) {
    if (check)
      hipLaunchKernelGGL((k_step_nl<real, kFluxRoe, true>), grid, block, 0, st, s, c, L);
    else
      hipLaunchKernelGGL((k_step_nl<real, kFluxRoe, false>), grid, block, 0, st, s, c, L);
  } else {
    if (check)
      hipLaunchKernelGGL((k_step_nl<real, kFluxHLL, true>), grid, block, 0, st, s, c, L);
    else
      hipLaunchKernelGGL((k_step_nl<real, kFluxHLL, false>), grid, block, 0, st, s, c, L);
  }
  return hipGetLastError();
}

// Stage-1 Courant check with the fused step kernel: the step is tried whole
// (the state at its start stays in place), against the staging block r.
// k_fused_check_begin copies the pending step into r and arms it; after each
// trial k_fused_check either shrinks r's step to Cr times the Courant minimum
// of the trial's stage-1 result (the next trial runs) or accepts the trial:
// its step size, rain, stage boundary values, the new state's Courant
// minimum and flags go to the context's block c, and r is disarmed.  Trial
// k computes stage 1 exactly as the k-th repeat of the per-stage check does,
// so both paths accept the same step size.
__global__ void k_fused_check_begin(const Ctrl *c, Ctrl *r) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  *r = *c;
  r->minbits = kInfBits;
  r->minbits1 = kInfBits;
  r->flags = 0u;
  r->aux = 1u;
}

__global__ void k_fused_check(Ctrl *c, Ctrl *r, PlanArgs p, int last) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (r->aux == 0u) return;
  const double m1 = __longlong_as_double((long long)r->minbits1);
  r->minbits1 = kInfBits;
  const double lim = p.cfl * m1;
  if (!last && p.fixed_dt <= 0.0 && r->dt > lim) {
    set_step(r, p, lim);
    r->minbits = kInfBits;
    r->flags = 0u;
  } else {
    c->dt = r->dt;
    c->rain = r->rain;
    for (int sd = 0; sd < 4; ++sd) {
      c->qin[sd][0] = r->qin[sd][0];
      c->qin[sd][1] = r->qin[sd][1];
      c->hyd_k[sd] = r->hyd_k[sd];
    }
    if (r->minbits < c->minbits) c->minbits = r->minbits;
    c->flags |= r->flags;
    r->minbits = kInfBits;
    r->aux = 0u;
  }
}

hipError_t launch_fused_check(Ctrl *ctrl, Ctrl *rep, const PlanArgs &p, int begin, int last,
                              hipStream_t st) {
  if (begin)
    hipLaunchKernelGGL(k_fused_check_begin, dim3(1), dim3(64), 0, st, ctrl, rep);
  else
    hipLaunchKernelGGL(k_fused_check, dim3(1), dim3(64), 0, st, ctrl, rep, p, last);
  return hipGetLastError();
}

hipError_t launch_plan(Ctrl *ctrl, const PlanArgs &p, int mode, double t_end, int set_tend,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(64), 0, st, ctrl, p, mode, t_end, set_tend);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_cfl(const Scen<real> &s, const Consts &c, hipStream_t st, const Ctrl *gate,
                      unsigned long long *bits) {
  const long long n = (long long)s.nx * s.ny;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_cfl<real>), dim3((unsigned)blocks), dim3(256), 0, st, s, c, gate,
                     bits ? bits : &s.ctrl->minbits);
  return hipGetLastError();
}

hipError_t launch_stage_check(Ctrl *ctrl, Ctrl *rep, const PlanArgs &p, int first, int last,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_stage_check, dim3(1), dim3(64), 0, st, ctrl, rep, p, first, last);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_diag(const Scen<real> &s, const Consts &c, double *partials, int nblocks,
                       double *out4, hipStream_t st, double sm, double se) {
  hipLaunchKernelGGL((k_diag<real>), dim3(nblocks), dim3(256), 0, st, s, c, partials);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, partials, nblocks, out4, sm, se);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free diagnostics entry point: the per-block
// records of the reduction (4 doubles per block), in a file-scope device
// array that each GPU holds once for the life of the process.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current and kept here.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kScratchRecords * 4];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_records(double **ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

template <typename real, int STAGE, int FLUX>
void queue_batch_kernel(int variant, const Scen<real> *scens, const Item *it, int nitems,
                        const Consts &c, int R, int wpb, int blocks, hipStream_t st) {
  const dim3 block(64 * wpb), grid(blocks);
  if (variant == 1)
    hipLaunchKernelGGL((k_batch_stage<real, STAGE, 1, FLUX>), grid, block, 0, st, scens, it, nitems,
                       c, R, wpb);
  else
    hipLaunchKernelGGL((k_batch_stage<real, STAGE, 0, FLUX>), grid, block, 0, st, scens, it, nitems,
                       c, R, wpb);
}

template <typename real>
hipError_t launch_batch_stage(int stage, int variant, const Scen<real> *scens, const void *items,
                              int nitems, const Consts &c, int R, int wpb, int blocks,
                              hipStream_t st) {
  const Item *it = (const Item *)items;
  if (c.flux == kFluxRoe) {
    if (stage == 1)
      queue_batch_kernel<real, 1, kFluxRoe>(variant, scens, it, nitems, c, R, wpb, blocks, st);
    else
      queue_batch_kernel<real, 2, kFluxRoe>(variant, scens, it, nitems, c, R, wpb, blocks, st);
  } else {
    if (stage == 1)
      queue_batch_kernel<real, 1, kFluxHLL>(variant, scens, it, nitems, c, R, wpb, blocks, st);
    else
      queue_batch_kernel<real, 2, kFluxHLL>(variant, scens, it, nitems, c, R, wpb, blocks, st);
  }
  return hipGetLastError();
}

// Scenarios still running (dt > 0 and t below their target) and the OR of
// their error flags, for the host's progress check: out[0] = count, out[1] = flags.
__global__ void k_batch_status(Ctrl *const *ctrls, int n, unsigned *out) {
  __shared__ unsigned cnt, fl;
  if (threadIdx.x == 0) {
    cnt = 0;
    fl = 0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const Ctrl *c = ctrls[k];
    if (c->dt > 0.0 && c->t < c->t_end) atomicAdd(&cnt, 1u);
    if (c->flags) atomicOr(&fl, c->flags);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = cnt;
    out[1] = fl;
  }
}

hipError_t launch_batch_status(Ctrl *const *ctrls, int n, unsigned *out, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_status, dim3(1), dim3(256), 0, st, ctrls, n, out);
  return hipGetLastError();
}

// Workgroups of the persistent batched launch: the number that can be
// resident at once for this kernel and workgroup size on the device.
template <typename real, int STAGE, int FLUX>
hipError_t batch_occupancy(int variant, int threads, int *per) {
  return variant == 1
             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_batch_stage<real, STAGE, 1, FLUX>,
                                                            threads, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_batch_stage<real, STAGE, 0, FLUX>,
                                                            threads, 0);
}

template <typename real>
int batch_blocks(int stage, int variant, int flux, int wpb) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
  const int threads = 64 * wpb;
  hipError_t e;
  if (flux == kFluxRoe)
    e = stage == 1 ? batch_occupancy<real, 1, kFluxRoe>(variant, threads, &per)
                   : batch_occupancy<real, 2, kFluxRoe>(variant, threads, &per);
  else
    e = stage == 1 ? batch_occupancy<real, 1, kFluxHLL>(variant, threads, &per)
                   : batch_occupancy<real, 2, kFluxHLL>(variant, threads, &per);
  if (e != hipSuccess || per < 1) per = 1;
  return per * cus;
}
template int batch_blocks<double>(int, int, int, int);
template int batch_blocks<float>(int, int, int, int);

template <typename real>
int batch_fused_blocks(int flux, int wpb) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
  const int threads = 64 * wpb;
  const hipError_t e =
      flux == kFluxRoe
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_step<real, kFluxRoe>, threads, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_step<real, kFluxHLL>, threads, 0);
  if (e != hipSuccess || per < 1) per = 1;
  return per * cus;
}

template <typename real>
hipError_t launch_batch_fused(const Scen<real> *scens, const void *items, int nitems, const Consts &c,
                              int R, int wpb, int blocks, hipStream_t st) {
  const Item *it = (const Item *)items;
  const dim3 block(64 * wpb), grid(blocks);
  if (c.flux == kFluxRoe)
    hipLaunchKernelGGL((k_batch_step<real, kFluxRoe>), grid, block, 0, st, scens, it, nitems, c, R, wpb);
  else
    hipLaunchKernelGGL((k_batch_step<real, kFluxHLL>), grid, block, 0, st, scens, it, nitems, c, R, wpb);
  return hipGetLastError();
}

template int batch_fused_blocks<float>(int, int);
template int batch_fused_blocks<double>(int, int);
template hipError_t launch_batch_fused<float>(const Scen<float> *, const void *, int, const Consts &, int,
                                              int, int, hipStream_t);
template hipError_t launch_batch_fused<double>(const Scen<double> *, const void *, int, const Consts &,
                                               int, int, int, hipStream_t);

hipError_t launch_plan_batch(Ctrl *const *ctrls, const PlanArgs *pa, int n, int mode, double t_end,
                             int set_tend, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_batch, dim3((n + 63) / 64), dim3(64), 0, st, ctrls, pa, n, mode, t_end,
                     set_tend);
  return hipGetLastError();
}

template hipError_t launch_batch_stage<double>(int, int, const Scen<double> *, const void *, int,
                                               const Consts &, int, int, int, hipStream_t);
template hipError_t launch_batch_stage<float>(int, int, const Scen<float> *, const void *, int,
                                              const Consts &, int, int, int, hipStream_t);
template hipError_t launch_stage<double>(int, int, const Scen<double> &, const Consts &,
                                         const Launch &, hipStream_t);
template hipError_t launch_stage<float>(int, int, const Scen<float> &, const Consts &,
                                        const Launch &, hipStream_t);
template hipError_t launch_fused<float>(const Scen<float> &, const Consts &, const Launch &,
                                        hipStream_t, bool);
template hipError_t launch_fused<double>(const Scen<double> &, const Consts &, const Launch &,
                                        hipStream_t, bool);
template hipError_t launch_cfl<double>(const Scen<double> &, const Consts &, hipStream_t, const Ctrl *,
                                       unsigned long long *);
template hipError_t launch_cfl<float>(const Scen<float> &, const Consts &, hipStream_t, const Ctrl *,
                                      unsigned long long *);
template hipError_t launch_diag<double>(const Scen<double> &, const Consts &, double *, int, double *,
                                        hipStream_t, double, double);
template hipError_t launch_diag<float>(const Scen<float> &, const Consts &, double *, int, double *,
                                       hipStream_t, double, double);

}  // namespace dg2
