// Device-side building blocks of the DG2 step (gfx950, wave64).
//
// Pointwise formulas of Sec. 2.1.2-2.1.3 of the paper: dummy limits, the
// HLL face flux, the physical flux at Gauss points and the implicit friction
// split.  Templated on the arithmetic type (double or float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dg2 {

constexpr double kInvSqrt3 = 0.57735026918962576451;   // Gauss points at +-1/sqrt(3), Eq. (4b-c)
constexpr double kHalfSqrt3 = 0.86602540378443864676;  // slope from two Gauss values
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;   // +inf as double bits

// Device-resident step control.  One per context (or per scenario in a
// batch).  Only the single-thread plan kernel writes t, dt, rain and qin;
// the stage kernels read them, so a queued step never needs the host.
struct Ctrl {
  double t;            // time of the current state
  double dt;           // size of the pending step, <= 0: idle
  double t_end;        // run-to target, +inf when none
  double rain;         // rain depth added by the pending step
  double qin[4][2];    // per side at the two stage times: unit inflow, or water level
  double cflmin;       // min_c m_c of the current state (+inf: nothing wet)
  double last_dt;      // size of the last completed step
  long long step;      // completed steps
  unsigned long long minbits;  // running min of m_c for the next step (double bits)
  unsigned int flags;  // bit 0: NaN, bit 1: negative mean depth
  unsigned int aux;    // repeat block of the stage-1 Courant check: armed flag
  long long gauge_written;  // samples recorded since the gauge record was reset
  int hyd_k[4];        // per side: hydrograph interval of the last lookup (search hint)
  unsigned long long minbits1;  // staging block of the stage-1 Courant check: running
                                // min of m_c over the stage-1 result (double bits)
};

enum : unsigned { kFlagNaN = 1u, kFlagNegative = 2u };

// Parameters of the step planner (host-side constants of one context).
struct PlanArgs {
  double cfl, dt_max, fixed_dt;
  double rain_rate, rain_tb, rain_te;
  int nhyd[4];
  const double *hyd_t[4];
  const double *hyd_Q[4];
  double seg_len[4];
  int ng;          // gauges (for the time record)
  int gauge_cap;
  double *gauge_t;
  // optional record of each planned step: hist[step - hist_base] = Ctrl
  // for 0 <= step - hist_base < hist_len (the adjoint's segment recompute)
  Ctrl *hist;
  long long hist_base;
  int hist_len;
};

// Arithmetic kernels by precision.  Every operand here is a positive normal
// number (depths above the drying tolerance, positive wave-speed gaps) or,
// for the square root, zero, so no range scaling or special-case handling is
// needed.  FP32 uses the hardware reciprocal, square root, exp2 and log2
// (about 1 ulp); the FP32 path is held to a stated depth error.  FP64
// refines the hardware estimates by Newton's method instead of calling the
// correctly rounded division and square root sequences (whose scaling and
// fix-up steps cost a third of the FP64 stage kernels' time): the
// reciprocal takes two Newton steps on the estimate of v_rcp_f64, a quotient
// one correction of a * (1/b), the square root one Newton step on the
// estimate of v_sqrt_f64, h^(-1/3) two Newton steps on an FP32 estimate;
// each result is within an ulp or two of the correctly rounded one.
template <typename real> __device__ __forceinline__ real dsqrt(real x);
template <> __device__ __forceinline__ double dsqrt<double>(double x) {
  // y + (x - y^2) / (2 y) on the hardware estimate y
  const double y = __builtin_amdgcn_sqrt(x);
  const double r = __builtin_amdgcn_rcp(y);
  const double e = __builtin_fma(-y, y, x);
  return x > 0.0 ? __builtin_fma(0.5 * e, r, y) : 0.0;
}
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <typename real> __device__ __forceinline__ real drcp(real x);
template <> __device__ __forceinline__ double drcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
template <> __device__ __forceinline__ float drcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename real> __device__ __forceinline__ real ddiv(real a, real b);
template <> __device__ __forceinline__ double ddiv<double>(double a, double b) {
  const double r = drcp<double>(b);
  const double q = a * r;
  return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
template <> __device__ __forceinline__ float ddiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// h^(-7/3) for a depth h above the drying tolerance
template <typename real> __device__ __forceinline__ real pow_m7_3(real h);
// h^(-1/3) for a depth above the drying tolerance: an FP32 estimate
// exp2(-log2(h)/3), then two Newton steps on y^-3 = h in FP64,
// y <- y + y (1 - h y^3) / 3 (the error squares at each step: ~1e-7, ~1e-14,
// then rounding).  Depths below 1e-30 (not expected: tol_dry is far above)
// take the library's rcbrt.
__device__ __forceinline__ double rcbrt_pos(double h) {
  if (__builtin_expect(h < 1e-30, 0)) return rcbrt(h);
  double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)h) * (-1.0f / 3.0f));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double e = __builtin_fma(-h, y * y * y, 1.0);
    y = __builtin_fma(y * (1.0 / 3.0), e, y);
  }
  return y;
}
template <> __device__ __forceinline__ double pow_m7_3<double>(double h) {
  const double rc = rcbrt_pos(h), rc2 = rc * rc;
  return (rc2 * rc2) * (rc2 * rc);
}
template <> __device__ __forceinline__ float pow_m7_3<float>(float h) {
  return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(h) * (-7.0f / 3.0f));
}
template <typename real> __device__ __forceinline__ real dcbrt(real x);
template <> __device__ __forceinline__ double dcbrt<double>(double x) { return cbrt(x); }
template <> __device__ __forceinline__ float dcbrt<float>(float x) { return cbrtf(x); }

// Element of a plane at a 32-bit byte offset: plane bases stay in scalar
// registers and each lane supplies only its 32-bit offset (one plane is
// below 4 GiB), which saves the 64-bit address arithmetic per access.
template <typename real>
__device__ __forceinline__ real ld_at(const real *plane, unsigned off) {
  return *reinterpret_cast<const real *>(reinterpret_cast<const char *>(plane) + off);
}
template <typename real>
__device__ __forceinline__ void st_at(real *plane, unsigned off, real v) {
  *reinterpret_cast<real *>(reinterpret_cast<char *>(plane) + off) = v;
}

template <typename real> __device__ __forceinline__ real dmax(real a, real b) { return a > b ? a : b; }
template <typename real> __device__ __forceinline__ real dmin(real a, real b) { return a < b ? a : b; }

// Positivity-preserving dummy limit (Sec. 2.1.2): h* = max(0, h), velocities
// q/h above the drying tolerance and zero otherwise.
template <typename real>
__device__ __forceinline__ void dummy_limit(real h, real qx, real qy, real tol, real &hs, real &u,
                                            real &v) {
  hs = h > real(0) ? h : real(0);
  if (h > tol) {
    const real r = drcp(h);
    u = qx * r;
    v = qy * r;
  } else {
    u = real(0);
    v = real(0);
  }
}

// HLL flux through a face with normal velocity u and tangential velocity v.
// Wave speeds: Toro's two-rarefaction estimates, dry-bed front speeds when a
// side is dry, zero flux when both are.  F = [h u, h u^2 + g h^2/2, h u v].
template <typename real>
__device__ __forceinline__ void hll(real hL, real uL, real vL, real hR, real uR, real vR, real g,
                                    real tol, real &F0, real &F1, real &F2) {
  const bool dryL = hL <= tol, dryR = hR <= tol;
  if (dryL && dryR) {
    F0 = F1 = F2 = real(0);
    return;
  }
  const real cL = dsqrt(g * hL), cR = dsqrt(g * hR);
  const real us = real(0.5) * (uL + uR) + cL - cR;
  const real cs = real(0.5) * (cL + cR) + real(0.25) * (uL - uR);
  const real sL = dryL ? uR - real(2) * cR : dmin(uL - cL, us - cs);
  const real sR = dryR ? uL + real(2) * cL : dmax(uR + cR, us + cs);
  const real qL = hL * uL, qR = hR * uR;
  const real FL0 = qL, FL1 = qL * uL + real(0.5) * g * hL * hL, FL2 = qL * vL;
  const real FR0 = qR, FR1 = qR * uR + real(0.5) * g * hR * hR, FR2 = qR * vR;
  if constexpr (sizeof(real) == 8) {
    // FP64: one formula for the three wave regimes (sl = min(sL, 0) and
    // sr = max(sR, 0) give F_L when sL >= 0 and F_R when sR <= 0), which
    // replaces six 64-bit selects by two min/max
    const real sl = dmin(sL, real(0)), sr = dmax(sR, real(0));
    const real inv = drcp(sr - sl);
    const real ss = sl * sr;
    F0 = (sr * FL0 - sl * FR0 + ss * (hR - hL)) * inv;
    F1 = (sr * FL1 - sl * FR1 + ss * (qR - qL)) * inv;
    F2 = (sr * FL2 - sl * FR2 + ss * (hR * vR - hL * vL)) * inv;
  } else if (sL >= real(0)) {
    F0 = FL0; F1 = FL1; F2 = FL2;
  } else if (sR <= real(0)) {
    F0 = FR0; F1 = FR1; F2 = FR2;
  } else {
    const real inv = drcp(sR - sL);
    const real ss = sL * sR;
    F0 = (sR * FL0 - sL * FR0 + ss * (hR - hL)) * inv;
    F1 = (sR * FL1 - sL * FR1 + ss * (qR - qL)) * inv;
    F2 = (sR * FL2 - sL * FR2 + ss * (hR * vR - hL * vL)) * inv;
  }
}

// Roe's approximate Riemann solver (the paper's choice, Sec. 2.1.2) on wet
// dummy limits: Roe averages u = (sqrt(hL) uL + sqrt(hR) uR)/(sqrt(hL) +
// sqrt(hR)) (v alike) and c = sqrt(g (hL + hR)/2), three waves with
// eigenvalues u - c, u, u + c, no entropy fix:
// F = (F_L + F_R)/2 - sum |lambda_k| alpha_k r_k / 2.  A face with a side at
// or below the drying tolerance takes the HLL flux.
template <typename real>
__device__ __forceinline__ void roe(real hL, real uL, real vL, real hR, real uR, real vR, real g,
                                    real tol, real &F0, real &F1, real &F2) {
  if (!(hL > tol && hR > tol)) {
    hll(hL, uL, vL, hR, uR, vR, g, tol, F0, F1, F2);
    return;
  }
  const real rL = dsqrt(hL), rR = dsqrt(hR);
  const real ir = drcp(rL + rR);
  const real uh = (rL * uL + rR * uR) * ir, vh = (rL * vL + rR * vR) * ir;
  const real ch = dsqrt(real(0.5) * g * (hL + hR));
  const real qL = hL * uL, qR = hR * uR;
  const real dh = hR - hL, dq = qR - qL, dr = hR * vR - hL * vL;
  const real i2c = drcp(real(2) * ch);
  const real l1 = uh - ch, l3 = uh + ch;
  const real m1 = fabs(l1) * (((uh + ch) * dh - dq) * i2c);  // |lambda_1| alpha_1
  const real m3 = fabs(l3) * ((dq - (uh - ch) * dh) * i2c);  // |lambda_3| alpha_3
  const real m2 = fabs(uh) * (dr - vh * dh);                 // |lambda_2| alpha_2
  const real FL1 = qL * uL + real(0.5) * g * hL * hL, FR1 = qR * uR + real(0.5) * g * hR * hR;
  F0 = real(0.5) * ((qL + qR) - (m1 + m3));
  F1 = real(0.5) * ((FL1 + FR1) - (m1 * l1 + m3 * l3));
  F2 = real(0.5) * ((qL * vL + qR * vR) - ((m1 + m3) * vh + m2));
}

// The two-argument face flux, chosen at compile time.
enum : int { kFluxHLL = 0, kFluxRoe = 1 };

// Boundary kinds of a side's segment (the values of dg2_bc).
enum : int { kBcWall = 0, kBcInflow = 1, kBcLevel = 2, kBcOpen = 3 };

template <int FLUX, typename real>
__device__ __forceinline__ void face_flux(real hL, real uL, real vL, real hR, real uR, real vR,
                                          real g, real tol, real &F0, real &F1, real &F2) {
  if (FLUX == kFluxRoe)
    roe(hL, uL, vL, hR, uR, vR, g, tol, F0, F1, F2);
  else
    hll(hL, uL, vL, hR, uR, vR, g, tol, F0, F1, F2);
}

// Flux through a water-level or open boundary face, along the face normal.
// (h, un, ut) is the inside dummy limit at the face, (hm, qnm, qtm) the
// inside cell's mean state, zf the bed at the face and eta the prescribed
// level; inside_plus: the inside lies on the + side (west and south faces).
// Level: ghost depth max(0, eta - zf), normal velocity keeping the outgoing
// Riemann invariant (u - 2c inside a west/south face, u + 2c inside an
// east/north face), an inflow capped at the critical speed, tangential
// velocity zero where the ghost's flow enters the domain, else from inside.
// Open: the ghost holds the inside cell's mean state.
template <int FLUX, typename real>
__device__ __forceinline__ void ghost_face_flux(int kind, bool inside_plus, real eta, real zf,
                                                real h, real un, real ut, real hm, real qnm,
                                                real qtm, real g, real tol, real &F0, real &Fn,
                                                real &Ft) {
  real hg, ug, vg;
  if (kind == kBcLevel) {
    hg = dmax(real(0), eta - zf);
    const real cg = dsqrt(g * hg), ci = dsqrt(g * h);
    ug = inside_plus ? dmin(un - real(2) * ci + real(2) * cg, cg)
                     : dmax(un + real(2) * ci - real(2) * cg, -cg);
    // reservoir water enters without tangential motion; leaving water keeps its own
    const bool entering = inside_plus ? ug > real(0) : ug < real(0);
    vg = entering ? real(0) : ut;
  } else {
    dummy_limit(hm, qnm, qtm, tol, hg, ug, vg);
  }
  if (inside_plus)
    face_flux<FLUX>(hg, ug, vg, h, un, ut, g, tol, F0, Fn, Ft);
  else
    face_flux<FLUX>(h, un, ut, hg, ug, vg, g, tol, F0, Fn, Ft);
}

// Prescribed discharge q through an inflow face: normal flux components
// [q, q^2/h_b + g h_b^2/2, 0], h_b = max(inner dummy depth, critical depth).
template <typename real>
__device__ __forceinline__ void inflow_flux(real q, real h_inner, real g, real &F0, real &F1) {
  const real hc = dcbrt(q * q / g);
  const real hb = dmax(h_inner, hc);
  F0 = q;
  F1 = ddiv(q * q, hb) + real(0.5) * g * hb * hb;
}

// Physical x-flux at a point (Eq. 1), velocity zeroed at or below tol.
template <typename real>
__device__ __forceinline__ void flux_x(real h, real qx, real qy, real g, real tol, real &F0,
                                       real &F1, real &F2) {
  const real hp = h > real(0) ? h : real(0);
  const real pres = real(0.5) * g * hp * hp;
  if (h > tol) {
    const real r = drcp(h);
    const real u = qx * r, v = qy * r;
    const real q = hp * u;
    F0 = q;
    F1 = q * u + pres;
    F2 = q * v;
  } else {
    F0 = real(0);
    F1 = pres;
    F2 = real(0);
  }
}

// Physical y-flux at a point, returned as [mass, x-momentum, y-momentum].
template <typename real>
__device__ __forceinline__ void flux_y(real h, real qx, real qy, real g, real tol, real &G0,
                                       real &G1, real &G2) {
  const real hp = h > real(0) ? h : real(0);
  const real pres = real(0.5) * g * hp * hp;
  if (h > tol) {
    const real r = drcp(h);
    const real u = qx * r, v = qy * r;
    const real q = hp * v;
    G0 = q;
    G1 = q * u;
    G2 = q * v + pres;
  } else {
    G0 = real(0);
    G1 = real(0);
    G2 = pres;
  }
}

// Implicit friction increment at one point.  The split friction ODE
// dq/dt = -C_f |V| q / h (C_f = g n^2 h^(-1/3)) keeps h and the flow direction,
// so its implicit solution over dt is exact: q_new = q / (1 + b |q|) with
// b = dt g n^2 h^(-7/3).  gn2dt = g n^2 dt.
template <typename real>
__device__ __forceinline__ void friction_point(real h, real qx, real qy, real gn2dt, real tol,
                                               real &dqx, real &dqy) {
  const real qq = qx * qx + qy * qy;
  if (h > tol && qq > real(0)) {
    const real b = gn2dt * pow_m7_3(h);
    const real bq = b * dsqrt(qq);
    const real f = ddiv(bq, real(1) + bq);
    dqx = -qx * f;
    dqy = -qy * f;
  } else {
    dqx = real(0);
    dqy = real(0);
  }
}

// Friction split on a planar element (Sec. 2.1.3, Fig. 1): increments at the
// centre and at G_x+-, G_y+- = U0 +- U1/sqrt(3); the centre increment goes to
// the mean discharges, sqrt(3)/2 times the Gauss difference to the slopes.
// W: [h0,h1x,h1y,qx0,qx1x,qx1y,qy0,qy1x,qy1y].
template <typename real>
__device__ __forceinline__ void apply_friction(real *W, real gn2dt, real tol) {
  if (!(gn2dt > real(0))) return;
  const real is3 = real(kInvSqrt3), hs3 = real(kHalfSqrt3);
  real cx, cy, pxx, pxy, mxx, mxy, pyx, pyy, myx, myy;
  friction_point(W[0], W[3], W[6], gn2dt, tol, cx, cy);
  friction_point(W[0] + W[1] * is3, W[3] + W[4] * is3, W[6] + W[7] * is3, gn2dt, tol, pxx, pxy);
  friction_point(W[0] - W[1] * is3, W[3] - W[4] * is3, W[6] - W[7] * is3, gn2dt, tol, mxx, mxy);
  friction_point(W[0] + W[2] * is3, W[3] + W[5] * is3, W[6] + W[8] * is3, gn2dt, tol, pyx, pyy);
  friction_point(W[0] - W[2] * is3, W[3] - W[5] * is3, W[6] - W[8] * is3, gn2dt, tol, myx, myy);
  W[3] += cx;
  W[4] += hs3 * (pxx - mxx);
  W[5] += hs3 * (pyx - myx);
  W[6] += cy;
  W[7] += hs3 * (pxy - mxy);
  W[8] += hs3 * (pyy - myy);
}

// Mirror ghost across an x-wall (mx) and/or a y-wall (my): the normal
// discharge is odd, h and the tangential discharge are even.
template <typename real>
__device__ __forceinline__ void mirror(real *W, bool mx, bool my) {
  if (mx) {
    W[1] = -W[1];
    W[3] = -W[3];
    W[5] = -W[5];
    W[7] = -W[7];
  }
  if (my) {
    W[2] = -W[2];
    W[5] = -W[5];
    W[6] = -W[6];
    W[7] = -W[7];
  }
}

// End-of-stage wet/dry treatment.  Dry elements are flagged by the mean
// depth alone (Sec. 2.1.3): an element with mean depth <= tol gets zero
// discharge modes.  Mean depths stay, so mass is exact.  With `flat` (an
// option outside the paper's method) a wet element with a face-limit depth
// <= tol also drops every slope mode (locally first order at the front).
// Returns the decision: 1 dry, 2 partly wet and flattened, 0 unchanged.
template <typename real>
__device__ __forceinline__ unsigned wet_dry_fix(real *o, real tol, bool flat) {
  if (!(o[0] > tol)) {
#pragma unroll
    for (int k = 3; k < 9; ++k) o[k] = real(0);
    return 1u;
  }
  if (flat) {
    const real ax = fabs(o[1]), ay = fabs(o[2]);
    if (o[0] - (ax > ay ? ax : ay) <= tol) {
      o[1] = o[2] = o[4] = o[5] = o[7] = o[8] = real(0);
      return 2u;
    }
  }
  return 0u;
}

// Courant candidate m_c = min(dx/(|u|+c), dy/(|v|+c)) of a wet mean state.
template <typename real>
__device__ __forceinline__ double cfl_candidate(real h0, real qx0, real qy0, real g, real tol,
                                                real dx, real dy) {
  if (!(h0 > tol)) return __longlong_as_double((long long)kInfBits);
  const real u = fabs(ddiv(qx0, h0)), v = fabs(ddiv(qy0, h0));
  const real c = dsqrt(g * h0);
  const real m = dmin(ddiv(dx, u + c), ddiv(dy, v + c));
  return (double)m;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

}  // namespace dg2
