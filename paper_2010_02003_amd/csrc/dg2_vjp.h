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
    const double r = 1.0 / h;
    un = qn * r;
    ut = qt * r;
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
    const double r = 1.0 / h;
    const double un = qn * r, ut = qt * r;
    lqn = lun * r;
    lqt = lut * r;
    lh += -(un * lun + ut * lut) * r;
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

// ---- HLL flux (Toro wave speeds) and its adjoint -----------------------------
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
    const double iD = 1.0 / (sR - sL);
    for (int k = 0; k < 3; ++k) F[k] = (sR * FL[k] - sL * FR[k] + sL * sR * (UR[k] - UL[k])) * iD;
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
    const double iD = 1.0 / (sR - sL);
    for (int k = 0; k < 3; ++k) {
      const double dU = UR[k] - UL[k];
      const double Fk = (sR * FL[k] - sL * FR[k] + sL * sR * dU) * iD;
      const double l = lF[k] * iD;
      lFL[k] = l * sR;
      lFR[k] = -l * sL;
      lUR[k] = l * sL * sR;
      lUL[k] = -lUR[k];
      lsL += l * (-FR[k] + sR * dU + Fk);
      lsR += l * (FL[k] + sL * dU - Fk);
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

// ---- prescribed inflow face flux, normal components [F0, F1] ----------------
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
  const double rb = 1.0 / hb;
  const double lhb = lF1 * (-q * q * rb * rb + g * hb);
  lq = lF0 + lF1 * 2.0 * q * rb;
  lh_in = max_vjp_a(h_in, hc) * lhb;
  if (q != 0.0) lq += max_vjp_a(hc, h_in) * lhb * (2.0 / 3.0) * hc / q;
}

// ---- implicit friction at one point: increment and its adjoint --------------
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
  const double Sa = S * a, Saq = Sa / qq;
  lqx = -ldx * f + Saq * qx;
  lqy = -ldy * f + Saq * qy;
  lh = Sa * (-7.0 / 3.0) / h;
  ln = Sa * 2.0 / n;
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


// ---- wet/dry treatment at the end of a stage ---------------------------------
// Code of the decision taken on a stage output: 1 = dry (discharge modes set
// to zero, Sec. 2.1.3), 2 = partly wet with the optional partly-wet rule on
// (every slope mode set to zero), 0 = unchanged.
// The adjoint of the treatment zeroes the same entries of the adjoint.
__host__ __device__ inline void apply_mask(unsigned char m, double *v) {
  if (m & 1u) {
    for (int k = 3; k < 9; ++k) v[k] = 0.0;
  }
  if (m & 2u) {
    v[1] = v[2] = v[4] = v[5] = v[7] = v[8] = 0.0;
  }
}

// ---- the DG2 operator L of Eq. (4) at one stage -----------------------------
// Everything the adjoint of L needs: the stage input X (the state L was
// evaluated at), the adjoint of the stage output before its wet/dry
// treatment together with the treatment's codes, and the problem data.
struct OpAdj {
  const double *X;            // 9 planes of P elements
  const double *lam;          // 9 planes: adjoint of the stage output
  const unsigned char *mask;  // wet/dry code per cell of the stage output (nullptr: none)
  const double *z;            // bed modes z0, z1x, z1y (3 planes)
  int nx, ny;
  long long P;
  double idx, idy, g, tol;
  int seg_first[4], seg_last[4];  // inflow segment per side (first > last: none)
  double q[4];                    // unit discharge per side at this stage time (0: wall)
};

// Adjoint of the operator at the stage input of cell c, from the adjoint of
// the operator's output mu_c = mask_c(lam_c).
__host__ __device__ inline void load_mu(const OpAdj &a, long long c, double *mu) {
  for (int k = 0; k < 9; ++k) mu[k] = a.lam[k * a.P + c];
  if (a.mask) apply_mask(a.mask[c], mu);
}

// Raw face limits of a planar element (Sec. 2.1.2) and their dummy values.
struct Limits {
  double r[4][3];  // raw (h, qx, qy) at E, W, N, S
  double d[4][3];  // dummy (h*, u, v) at E, W, N, S
};

__host__ __device__ inline void limits(const double *X, double tol, Limits &L) {
  const double sgn[4] = {1.0, -1.0, 1.0, -1.0};
  for (int f = 0; f < 4; ++f) {
    const int m = f < 2 ? 1 : 2;
    L.r[f][0] = X[0] + sgn[f] * X[m];
    L.r[f][1] = X[3] + sgn[f] * X[3 + m];
    L.r[f][2] = X[6] + sgn[f] * X[6 + m];
    dummy(L.r[f][0], L.r[f][1], L.r[f][2], tol, L.d[f][0], L.d[f][1], L.d[f][2]);
  }
}

enum { kE = 0, kW = 1, kN = 2, kS = 3 };

// One face limit of a planar element: raw (h, qx, qy) and dummy (h*, u, v).
__host__ __device__ inline void face_limit(const double *X, int f, double tol, double *r, double *d) {
  const double sg = (f == kE || f == kN) ? 1.0 : -1.0;
  const int m = f < 2 ? 1 : 2;
  r[0] = X[0] + sg * X[m];
  r[1] = X[3] + sg * X[3 + m];
  r[2] = X[6] + sg * X[6 + m];
  dummy(r[0], r[1], r[2], tol, d[0], d[1], d[2]);
}

__host__ __device__ inline double hstar(double h) { return h > 0.0 ? h : 0.0; }

__host__ __device__ inline double relu_neg(double h) { return h < 0.0 ? -h : 0.0; }
// d relu(-h)/dh with the subgradient -1 taken at h = 0
__host__ __device__ inline double relu_neg_d(double h) { return h <= 0.0 ? -1.0 : 0.0; }

__host__ __device__ inline void load9(const double *base, long long P, long long c, double *v) {
  for (int k = 0; k < 9; ++k) v[k] = base[k * P + c];
}

// JT = (dL/dX)^T mu gathered at cell (i, j), where mu is the adjoint of L at
// every cell (the operator of a cell depends on its own modes and on those of
// its four neighbours through the face fluxes and the wall-revised bed).
// lq[side] receives the adjoint of the unit discharge of an inflow face of
// this cell on that side (0 when there is none).  Wall ghosts are mirror
// images of the cell (walls as mirror ghost cells), so their dependence folds
// back onto the cell; ghosts carry no operator of their own.
__host__ __device__ inline void operator_vjp(const OpAdj &a, int i, int j, double *JT, double *lq) {
  const long long P = a.P;
  const long long c = (long long)j * a.nx + i;
  const double g = a.g, tol = a.tol, idx = a.idx, idy = a.idy;
  double X[9], mu[9];
  load9(a.X, P, c, X);
  load_mu(a, c, mu);
  Limits Lc;
  limits(X, tol, Lc);
  for (int k = 0; k < 9; ++k) JT[k] = 0.0;
  for (int s = 0; s < 4; ++s) lq[s] = 0.0;
  // adjoints of the dummy values (h*, u, v) at each face, and of the raw depths
  double ld[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double lr[4] = {0, 0, 0, 0};
  const double *dE = Lc.d[kE], *dW = Lc.d[kW], *dN = Lc.d[kN], *dS = Lc.d[kS];

  // bed revision of the neighbours that uses this cell's raw depth
  double lzb_east = 0.0, lzb_north = 0.0;
  double dWv, dSv;  // wall-revision depths of the west and south faces

  // ---- east face -------------------------------------------------------
  {
    double lF[3], l[6];
    for (int k = 0; k < 3; ++k) lF[k] = -idx * (mu[3 * k] + 3.0 * mu[3 * k + 1]);
    if (i + 1 < a.nx) {
      double Xb[9], mb[9], rb[3], db[3];
      load9(a.X, P, c + 1, Xb);
      load_mu(a, c + 1, mb);
      face_limit(Xb, kW, tol, rb, db);
      for (int k = 0; k < 3; ++k) lF[k] += idx * (mb[3 * k] - 3.0 * mb[3 * k + 1]);
      hll_vjp(dE[0], dE[1], dE[2], db[0], db[1], db[2], g, tol, lF, l);
      for (int k = 0; k < 3; ++k) ld[kE][k] += l[k];
      const double ehb = hstar(Xb[0] + Xb[1]);
      const double A0 = 0.5 * (ehb + db[0]), B0 = 0.5 * (ehb - db[0]);
      lzb_east = -2.0 * g * idx * (A0 * mb[3] + B0 * mb[4]);
    } else if (a.q[1] != 0.0 && j >= a.seg_first[1] && j <= a.seg_last[1]) {
      // east inflow: F = [-q, q^2/h_b + g h_b^2/2, 0]
      double lqq, lh;
      inflow_vjp(a.q[1], dE[0], g, -lF[0], lF[1], lqq, lh);
      ld[kE][0] += lh;
      lq[1] += lqq;
    } else {
      // wall: the ghost's west limit is (h*, -u, v) of this east limit
      hll_vjp(dE[0], dE[1], dE[2], dE[0], -dE[1], dE[2], g, tol, lF, l);
      ld[kE][0] += l[0] + l[3];
      ld[kE][1] += l[1] - l[4];
      ld[kE][2] += l[2] + l[5];
    }
  }
  // ---- west face -------------------------------------------------------
  {
    double lF[3], l[6];
    for (int k = 0; k < 3; ++k) lF[k] = idx * (mu[3 * k] - 3.0 * mu[3 * k + 1]);
    if (i > 0) {
      double Xa[9], ma[9], ra[3], da[3];
      load9(a.X, P, c - 1, Xa);
      load_mu(a, c - 1, ma);
      face_limit(Xa, kE, tol, ra, da);
      for (int k = 0; k < 3; ++k) lF[k] -= idx * (ma[3 * k] + 3.0 * ma[3 * k + 1]);
      hll_vjp(da[0], da[1], da[2], dW[0], dW[1], dW[2], g, tol, lF, l);
      for (int k = 0; k < 3; ++k) ld[kW][k] += l[3 + k];
      dWv = relu_neg(ra[0]);
    } else {
      if (a.q[0] != 0.0 && j >= a.seg_first[0] && j <= a.seg_last[0]) {
        double lqq, lh;
        inflow_vjp(a.q[0], dW[0], g, lF[0], lF[1], lqq, lh);
        ld[kW][0] += lh;
        lq[0] += lqq;
      } else {
        hll_vjp(dW[0], -dW[1], dW[2], dW[0], dW[1], dW[2], g, tol, lF, l);
        ld[kW][0] += l[3] + l[0];
        ld[kW][1] += l[4] - l[1];
        ld[kW][2] += l[5] + l[2];
      }
      dWv = relu_neg(Lc.r[kW][0]);  // the ghost's east depth is this west depth
    }
  }
  // ---- north face: G = [mass, x-mom, y-mom], HLL in (h, v, u) order ---------
  {
    double lG[3], lF[3], l[6];
    for (int k = 0; k < 3; ++k) lG[k] = -idy * (mu[3 * k] + 3.0 * mu[3 * k + 2]);
    if (j + 1 < a.ny) {
      double Xb[9], mb[9], rb[3], db[3];
      load9(a.X, P, c + a.nx, Xb);
      load_mu(a, c + a.nx, mb);
      face_limit(Xb, kS, tol, rb, db);
      for (int k = 0; k < 3; ++k) lG[k] += idy * (mb[3 * k] - 3.0 * mb[3 * k + 2]);
      lF[0] = lG[0]; lF[1] = lG[2]; lF[2] = lG[1];
      hll_vjp(dN[0], dN[2], dN[1], db[0], db[2], db[1], g, tol, lF, l);
      ld[kN][0] += l[0];
      ld[kN][2] += l[1];
      ld[kN][1] += l[2];
      const double nhb = hstar(Xb[0] + Xb[2]);
      const double C0 = 0.5 * (nhb + db[0]), D0 = 0.5 * (nhb - db[0]);
      lzb_north = -2.0 * g * idy * (C0 * mb[6] + D0 * mb[8]);
    } else if (a.q[3] != 0.0 && i >= a.seg_first[3] && i <= a.seg_last[3]) {
      // north inflow: G = [-q, 0, q^2/h_b + g h_b^2/2]
      double lqq, lh;
      inflow_vjp(a.q[3], dN[0], g, -lG[0], lG[2], lqq, lh);
      ld[kN][0] += lh;
      lq[3] += lqq;
    } else {
      // wall: the ghost's south limit is (h*, -v, u) in (h, v, u) order
      lF[0] = lG[0]; lF[1] = lG[2]; lF[2] = lG[1];
      hll_vjp(dN[0], dN[2], dN[1], dN[0], -dN[2], dN[1], g, tol, lF, l);
      ld[kN][0] += l[0] + l[3];
      ld[kN][2] += l[1] - l[4];
      ld[kN][1] += l[2] + l[5];
    }
  }
  // ---- south face --------------------------------------------------------
  {
    double lG[3], lF[3], l[6];
    for (int k = 0; k < 3; ++k) lG[k] = idy * (mu[3 * k] - 3.0 * mu[3 * k + 2]);
    if (j > 0) {
      double Xa[9], ma[9], ra[3], da[3];
      load9(a.X, P, c - a.nx, Xa);
      load_mu(a, c - a.nx, ma);
      face_limit(Xa, kN, tol, ra, da);
      for (int k = 0; k < 3; ++k) lG[k] -= idy * (ma[3 * k] + 3.0 * ma[3 * k + 2]);
      lF[0] = lG[0]; lF[1] = lG[2]; lF[2] = lG[1];
      hll_vjp(da[0], da[2], da[1], dS[0], dS[2], dS[1], g, tol, lF, l);
      ld[kS][0] += l[3];
      ld[kS][2] += l[4];
      ld[kS][1] += l[5];
      dSv = relu_neg(ra[0]);
    } else {
      if (a.q[2] != 0.0 && i >= a.seg_first[2] && i <= a.seg_last[2]) {
        // south inflow: G = [q, 0, q^2/h_b + g h_b^2/2]
        double lqq, lh;
        inflow_vjp(a.q[2], dS[0], g, lG[0], lG[2], lqq, lh);
        ld[kS][0] += lh;
        lq[2] += lqq;
      } else {
        lF[0] = lG[0]; lF[1] = lG[2]; lF[2] = lG[1];
        hll_vjp(dS[0], -dS[2], dS[1], dS[0], dS[2], dS[1], g, tol, lF, l);
        ld[kS][0] += l[3] + l[0];
        ld[kS][2] += l[4] - l[1];
        ld[kS][1] += l[5] + l[2];
      }
      dSv = relu_neg(Lc.r[kS][0]);
    }
  }

  // ---- the cell's own terms: Gauss-point fluxes and bed source ------------
  const double is3 = kIs3;
  const double E[3] = {dE[0], dE[0] * dE[1], dE[0] * dE[2]};
  const double Wc[3] = {dW[0], dW[0] * dW[1], dW[0] * dW[2]};
  const double N[3] = {dN[0], dN[0] * dN[1], dN[0] * dN[2]};
  const double S[3] = {dS[0], dS[0] * dS[1], dS[0] * dS[2]};
  double A[3], B[3], C[3], D[3];
  for (int k = 0; k < 3; ++k) {
    A[k] = 0.5 * (E[k] + Wc[k]);
    B[k] = 0.5 * (E[k] - Wc[k]);
    C[k] = 0.5 * (N[k] + S[k]);
    D[k] = 0.5 * (N[k] - S[k]);
  }
  const double zbx = a.z[P + c] - 0.5 * relu_neg(Lc.r[kE][0]) + 0.5 * dWv;
  const double zby = a.z[2 * P + c] - 0.5 * relu_neg(Lc.r[kN][0]) + 0.5 * dSv;
  double lA[3] = {0, 0, 0}, lB[3] = {0, 0, 0}, lC[3] = {0, 0, 0}, lD[3] = {0, 0, 0};
  {
    const double lF[3] = {3.0 * idx * mu[1], 3.0 * idx * mu[4], 3.0 * idx * mu[7]};
    for (int p = 0; p < 2; ++p) {
      const double o = p == 0 ? is3 : -is3;
      double lh, lqx, lqy;
      gflux_vjp(A[0] + o * B[0], A[1] + o * B[1], A[2] + o * B[2], g, tol, lF, lh, lqx, lqy);
      lA[0] += lh; lA[1] += lqx; lA[2] += lqy;
      lB[0] += o * lh; lB[1] += o * lqx; lB[2] += o * lqy;
    }
  }
  {
    // y Gauss flux [mass, x-mom, y-mom] is the normal flux of (h, qy, qx) reordered
    const double lG[3] = {3.0 * idy * mu[2], 3.0 * idy * mu[5], 3.0 * idy * mu[8]};
    const double lF[3] = {lG[0], lG[2], lG[1]};
    for (int p = 0; p < 2; ++p) {
      const double o = p == 0 ? is3 : -is3;
      double lh, lqy, lqx;
      gflux_vjp(C[0] + o * D[0], C[2] + o * D[2], C[1] + o * D[1], g, tol, lF, lh, lqy, lqx);
      lC[0] += lh; lC[1] += lqx; lC[2] += lqy;
      lD[0] += o * lh; lD[1] += o * lqx; lD[2] += o * lqy;
    }
  }
  // bed source: L0 of qx has -2g A0 zbx/dx, L1x of qx has -2g B0 zbx/dx (and y alike)
  lA[0] += -2.0 * g * idx * zbx * mu[3];
  lB[0] += -2.0 * g * idx * zbx * mu[4];
  lC[0] += -2.0 * g * idy * zby * mu[6];
  lD[0] += -2.0 * g * idy * zby * mu[8];
  const double lzbx = -2.0 * g * idx * (A[0] * mu[3] + B[0] * mu[4]);
  const double lzby = -2.0 * g * idy * (C[0] * mu[6] + D[0] * mu[8]);
  // zbx = z1x - relu(-h_E)/2 + relu(-h_W of the west neighbour or wall ghost)/2
  lr[kE] += (-0.5 * lzbx + 0.5 * lzb_east) * relu_neg_d(Lc.r[kE][0]);
  lr[kN] += (-0.5 * lzby + 0.5 * lzb_north) * relu_neg_d(Lc.r[kN][0]);
  if (i == 0) lr[kW] += 0.5 * lzbx * relu_neg_d(Lc.r[kW][0]);
  if (j == 0) lr[kS] += 0.5 * lzby * relu_neg_d(Lc.r[kS][0]);
  // dummy modes of Eq. (5) from the conserved dummy limits (h*, h* u, h* v)
  double lcons[4][3];
  for (int k = 0; k < 3; ++k) {
    lcons[kE][k] = 0.5 * (lA[k] + lB[k]);
    lcons[kW][k] = 0.5 * (lA[k] - lB[k]);
    lcons[kN][k] = 0.5 * (lC[k] + lD[k]);
    lcons[kS][k] = 0.5 * (lC[k] - lD[k]);
  }
  const double *dd[4] = {dE, dW, dN, dS};
  for (int f = 0; f < 4; ++f) {
    ld[f][0] += lcons[f][0] + dd[f][1] * lcons[f][1] + dd[f][2] * lcons[f][2];
    ld[f][1] += dd[f][0] * lcons[f][1];
    ld[f][2] += dd[f][0] * lcons[f][2];
  }
  // dummy limits -> raw limits -> modes
  const double sgn[4] = {1.0, -1.0, 1.0, -1.0};
  for (int f = 0; f < 4; ++f) {
    double rh, rqx, rqy;
    dummy_vjp(Lc.r[f][0], Lc.r[f][1], Lc.r[f][2], tol, ld[f][0], ld[f][1], ld[f][2], rh, rqx, rqy);
    rh += lr[f];
    const int m = f < 2 ? 1 : 2;
    JT[0] += rh;
    JT[m] += sgn[f] * rh;
    JT[3] += rqx;
    JT[3 + m] += sgn[f] * rqx;
    JT[6] += rqy;
    JT[6 + m] += sgn[f] * rqy;
  }
}

}  // namespace adj
}  // namespace dg2
