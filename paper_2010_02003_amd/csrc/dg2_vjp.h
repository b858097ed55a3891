// Reverse-mode (vector-Jacobian) building blocks of the DG2-NL step, FP64.
//
// Each function recomputes its piece of the forward step of Sec. 2.1.2-2.1.3
// (same formulas as dg2_device.h) and returns the adjoint of its inputs for
// a given adjoint of its outputs.  Conventions: a min/max whose arguments tie
// sends half of the adjoint to each argument; branch decisions (wet/dry
// tests, upwind choices, clamps) carry no adjoint; sqrt(g h) has zero
// derivative at h = 0.  All functions are __host__ __device__ so that a CPU
// program can check them against central differences.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace dg2 {
namespace adj {

constexpr double kIs3 = 0.57735026918962576451;
constexpr double kHs3 = 0.86602540378443864676;

__host__ __device__ inline double dmax(double a, double b) { return a > b ? a : b; }
__host__ __device__ inline double dmin(double a, double b) { return a < b ? a : b; }

// ---- dummy limit (Sec. 2.1.2): (h, qn, qt) -> (h*, un, ut) ------------------
__host__ __device__ inline void dummy(double h, double qn, double qt, double tol, double &hs,
                                      double &un, double &ut) {
  hs = h > 0.0 ? h : 0.0;
  if (h > tol) {
    un = qn / h;
    ut = qt / h;
  } else {
    un = 0.0;
    ut = 0.0;
  }
}

__host__ __device__ inline void dummy_vjp(double h, double qn, double qt, double tol, double lhs,
                                          double lun, double lut, double &lh, double &lqn,
                                          double &lqt) {
  lh = h >= 0.0 ? lhs : 0.0;
  lqn = 0.0;
  lqt = 0.0;
  if (h > tol) {
    const double un = qn / h, ut = qt / h;
    lqn = lun / h;
    lqt = lut / h;
    lh += -(un * lun + ut * lut) / h;
  }
}

// ---- physical normal flux from (h, un, ut): [h u, h u^2 + g h^2/2, h u v] --
__host__ __device__ inline void pflux(double h, double u, double v, double g, double *F) {
  const double q = h * u;
  F[0] = q;
  F[1] = q * u + 0.5 * g * h * h;
  F[2] = q * v;
}

__host__ __device__ inline void pflux_vjp(double h, double u, double v, double g, const double *lF,
                                          double &lh, double &lu, double &lv) {
  lh = lF[0] * u + lF[1] * (u * u + g * h) + lF[2] * u * v;
  lu = lF[0] * h + lF[1] * 2.0 * h * u + lF[2] * h * v;
  lv = lF[2] * h * u;
}

// min/max with the even split of the adjoint on ties
__host__ __device__ inline double min_vjp_a(double a, double b) { return a < b ? 1.0 : (a == b ? 0.5 : 0.0); }
__host__ __device__ inline double max_vjp_a(double a, double b) { return a > b ? 1.0 : (a == b ? 0.5 : 0.0); }

// ---- HLL flux (reading R1) and its adjoint ------------------------------------
__host__ __device__ inline void hll(double hL, double uL, double vL, double hR, double uR,
                                    double vR, double g, double tol, double *F) {
  const bool dryL = hL <= tol, dryR = hR <= tol;
  if (dryL && dryR) {
    F[0] = F[1] = F[2] = 0.0;
    return;
  }
  const double cL = sqrt(g * hL), cR = sqrt(g * hR);
  const double us = 0.5 * (uL + uR) + cL - cR;
  const double cs = 0.5 * (cL + cR) + 0.25 * (uL - uR);
  const double sL = dryL ? uR - 2.0 * cR : dmin(uL - cL, us - cs);
  const double sR = dryR ? uL + 2.0 * cL : dmax(uR + cR, us + cs);
  double FL[3], FR[3];
  pflux(hL, uL, vL, g, FL);
  pflux(hR, uR, vR, g, FR);
  if (sL >= 0.0) {
    for (int k = 0; k < 3; ++k) F[k] = FL[k];
  } else if (sR <= 0.0) {
    for (int k = 0; k < 3; ++k) F[k] = FR[k];
  } else {
    const double UL[3] = {hL, hL * uL, hL * vL}, UR[3] = {hR, hR * uR, hR * vR};
    const double D = sR - sL;
    for (int k = 0; k < 3; ++k) F[k] = (sR * FL[k] - sL * FR[k] + sL * sR * (UR[k] - UL[k])) / D;
  }
}

// in: lF[3]; out: adjoints of (hL, uL, vL, hR, uR, vR) in l[6]
__host__ __device__ inline void hll_vjp(double hL, double uL, double vL, double hR, double uR,
                                        double vR, double g, double tol, const double *lF,
                                        double *l) {
  for (int k = 0; k < 6; ++k) l[k] = 0.0;
  const bool dryL = hL <= tol, dryR = hR <= tol;
  if (dryL && dryR) return;
  const double cL = sqrt(g * hL), cR = sqrt(g * hR);
  const double us = 0.5 * (uL + uR) + cL - cR;
  const double cs = 0.5 * (cL + cR) + 0.25 * (uL - uR);
  const double aL = uL - cL, bL = us - cs, aR = uR + cR, bR = us + cs;
  const double sL = dryL ? uR - 2.0 * cR : dmin(aL, bL);
  const double sR = dryR ? uL + 2.0 * cL : dmax(aR, bR);
  double FL[3], FR[3];
  pflux(hL, uL, vL, g, FL);
  pflux(hR, uR, vR, g, FR);
  double lFL[3] = {0, 0, 0}, lFR[3] = {0, 0, 0};
  double lsL = 0.0, lsR = 0.0;
  double lUL[3] = {0, 0, 0}, lUR[3] = {0, 0, 0};
  if (sL >= 0.0) {
    for (int k = 0; k < 3; ++k) lFL[k] = lF[k];
  } else if (sR <= 0.0) {
    for (int k = 0; k < 3; ++k) lFR[k] = lF[k];
  } else {
    const double UL[3] = {hL, hL * uL, hL * vL}, UR[3] = {hR, hR * uR, hR * vR};
    const double D = sR - sL;
    for (int k = 0; k < 3; ++k) {
      const double dU = UR[k] - UL[k];
      const double Fk = (sR * FL[k] - sL * FR[k] + sL * sR * dU) / D;
      lFL[k] = lF[k] * sR / D;
      lFR[k] = -lF[k] * sL / D;
      lUR[k] = lF[k] * sL * sR / D;
      lUL[k] = -lUR[k];
      lsL += lF[k] * (-FR[k] + sR * dU + Fk) / D;
      lsR += lF[k] * (FL[k] + sL * dU - Fk) / D;
    }
  }
  // wave speeds -> (uL, uR, cL, cR)
  double luL = 0, luR = 0, lcL = 0, lcR = 0;
  if (dryL) {
    luR += lsL;
    lcR += -2.0 * lsL;
  } else {
    const double wa = min_vjp_a(aL, bL), wb = min_vjp_a(bL, aL);
    luL += wa * lsL;
    lcL += -wa * lsL;
    // us - cs = uL/4 + 3 uR/4 + cL/2 - 3 cR/2
    luL += 0.25 * wb * lsL;
    luR += 0.75 * wb * lsL;
    lcL += 0.5 * wb * lsL;
    lcR += -1.5 * wb * lsL;
  }
  if (dryR) {
    luL += lsR;
    lcL += 2.0 * lsR;
  } else {
    const double wa = max_vjp_a(aR, bR), wb = max_vjp_a(bR, aR);
    luR += wa * lsR;
    lcR += wa * lsR;
    // us + cs = 3 uL/4 + uR/4 + 3 cL/2 - cR/2
    luL += 0.75 * wb * lsR;
    luR += 0.25 * wb * lsR;
    lcL += 1.5 * wb * lsR;
    lcR += -0.5 * wb * lsR;
  }
  // U = (h, h u, h v)
  double lh, lu, lv;
  pflux_vjp(hL, uL, vL, g, lFL, lh, lu, lv);
  l[0] += lh + lUL[0] + uL * lUL[1] + vL * lUL[2];
  l[1] += lu + hL * lUL[1] + luL;
  l[2] += lv + hL * lUL[2];
  pflux_vjp(hR, uR, vR, g, lFR, lh, lu, lv);
  l[3] += lh + lUR[0] + uR * lUR[1] + vR * lUR[2];
  l[4] += lu + hR * lUR[1] + luR;
  l[5] += lv + hR * lUR[2];
  if (cL > 0.0) l[0] += lcL * g / (2.0 * cL);
  if (cR > 0.0) l[3] += lcR * g / (2.0 * cR);
}

// ---- physical flux at a Gauss point from (h, qn, qt) via the dummy limit ----
__host__ __device__ inline void gflux(double h, double qn, double qt, double g, double tol,
                                      double *F) {
  double hs, un, ut;
  dummy(h, qn, qt, tol, hs, un, ut);
  pflux(hs, un, ut, g, F);
}

__host__ __device__ inline void gflux_vjp(double h, double qn, double qt, double g, double tol,
                                          const double *lF, double &lh, double &lqn, double &lqt) {
  double hs, un, ut;
  dummy(h, qn, qt, tol, hs, un, ut);
  double lhs, lun, lut;
  pflux_vjp(hs, un, ut, g, lF, lhs, lun, lut);
  dummy_vjp(h, qn, qt, tol, lhs, lun, lut, lh, lqn, lqt);
}

// ---- inflow face flux (reading R12), normal components [F0, F1] -------------
__host__ __device__ inline void inflow(double q, double h_in, double g, double &F0, double &F1) {
  const double hc = cbrt(q * q / g);
  const double hb = dmax(h_in, hc);
  F0 = q;
  F1 = q * q / hb + 0.5 * g * hb * hb;
}

__host__ __device__ inline void inflow_vjp(double q, double h_in, double g, double lF0, double lF1,
                                           double &lq, double &lh_in) {
  const double hc = cbrt(q * q / g);
  const double hb = dmax(h_in, hc);
  const double lhb = lF1 * (-q * q / (hb * hb) + g * hb);
  lq = lF0 + lF1 * 2.0 * q / hb;
  lh_in = max_vjp_a(h_in, hc) * lhb;
  if (q != 0.0) lq += max_vjp_a(hc, h_in) * lhb * (2.0 / 3.0) * hc / q;
}

// ---- friction at one point (reading R8): increment and its adjoint ----------
// a = dt g n^2 |q| h^(-7/3); dq = -q a / (1 + a)
__host__ __device__ inline void fric_point(double h, double qx, double qy, double n, double gdt,
                                           double tol, double &dx, double &dy) {
  const double qq = qx * qx + qy * qy;
  if (h > tol && qq > 0.0 && n > 0.0) {
    const double rc = 1.0 / cbrt(h);
    const double rc2 = rc * rc;
    const double a = gdt * n * n * sqrt(qq) * (rc2 * rc2) * (rc2 * rc);
    const double f = a / (1.0 + a);
    dx = -qx * f;
    dy = -qy * f;
  } else {
    dx = 0.0;
    dy = 0.0;
  }
}

// in: adjoints of (dx, dy); out: adjoints of (h, qx, qy) and of n
__host__ __device__ inline void fric_point_vjp(double h, double qx, double qy, double n, double gdt,
                                               double tol, double ldx, double ldy, double &lh,
                                               double &lqx, double &lqy, double &ln) {
  lh = lqx = lqy = ln = 0.0;
  const double qq = qx * qx + qy * qy;
  if (!(h > tol && qq > 0.0 && n > 0.0)) return;
  const double rc = 1.0 / cbrt(h);
  const double rc2 = rc * rc;
  const double a = gdt * n * n * sqrt(qq) * (rc2 * rc2) * (rc2 * rc);
  const double f = a / (1.0 + a);
  const double dfda = 1.0 / ((1.0 + a) * (1.0 + a));
  const double S = -(ldx * qx + ldy * qy) * dfda;  // adjoint of a
  lqx = -ldx * f + S * a * qx / qq;
  lqy = -ldy * f + S * a * qy / qq;
  lh = S * a * (-7.0 / 3.0) / h;
  ln = S * a * 2.0 / n;
}

// Friction split of a planar element, forward: W[9] from U[9].
__host__ __device__ inline void fric_elem(const double *U, double n, double gdt, double tol,
                                          double *W) {
  for (int k = 0; k < 9; ++k) W[k] = U[k];
  double cx, cy, pxx, pxy, mxx, mxy, pyx, pyy, myx, myy;
  fric_point(U[0], U[3], U[6], n, gdt, tol, cx, cy);
  fric_point(U[0] + U[1] * kIs3, U[3] + U[4] * kIs3, U[6] + U[7] * kIs3, n, gdt, tol, pxx, pxy);
  fric_point(U[0] - U[1] * kIs3, U[3] - U[4] * kIs3, U[6] - U[7] * kIs3, n, gdt, tol, mxx, mxy);
  fric_point(U[0] + U[2] * kIs3, U[3] + U[5] * kIs3, U[6] + U[8] * kIs3, n, gdt, tol, pyx, pyy);
  fric_point(U[0] - U[2] * kIs3, U[3] - U[5] * kIs3, U[6] - U[8] * kIs3, n, gdt, tol, myx, myy);
  W[3] += cx;
  W[4] += kHs3 * (pxx - mxx);
  W[5] += kHs3 * (pyx - myx);
  W[6] += cy;
  W[7] += kHs3 * (pxy - mxy);
  W[8] += kHs3 * (pyy - myy);
}

// Friction split, adjoint: lU[9] (overwritten) and ln (added) from lW[9].
__host__ __device__ inline void fric_elem_vjp(const double *U, double n, double gdt, double tol,
                                              const double *lW, double *lU, double &ln) {
  for (int k = 0; k < 9; ++k) lU[k] = lW[k];
  // (point offset sign, slope index) for centre, G_x+, G_x-, G_y+, G_y-
  const int slope[5] = {-1, 1, 1, 2, 2};
  const double sgn[5] = {0.0, 1.0, -1.0, 1.0, -1.0};
  for (int p = 0; p < 5; ++p) {
    const int m = slope[p];
    const double o = sgn[p] * kIs3;
    const double h = m < 0 ? U[0] : U[0] + o * U[m];
    const double qx = m < 0 ? U[3] : U[3] + o * U[3 + m];
    const double qy = m < 0 ? U[6] : U[6] + o * U[6 + m];
    double ldx, ldy;
    if (m < 0) {
      ldx = lW[3];
      ldy = lW[6];
    } else {
      ldx = sgn[p] * kHs3 * lW[3 + m];
      ldy = sgn[p] * kHs3 * lW[6 + m];
    }
    double lh, lqx, lqy, lnp;
    fric_point_vjp(h, qx, qy, n, gdt, tol, ldx, ldy, lh, lqx, lqy, lnp);
    ln += lnp;
    lU[0] += lh;
    lU[3] += lqx;
    lU[6] += lqy;
    if (m >= 0) {
      lU[m] += o * lh;
      lU[3 + m] += o * lqx;
      lU[6 + m] += o * lqy;
    }
  }
}

}  // namespace adj
}  // namespace dg2
