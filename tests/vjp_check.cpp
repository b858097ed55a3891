// Host-side check of the reverse-mode building blocks in dg2_vjp.h against
// central differences of their own forward functions.  Built and run by
// tests/test_vjp_host.py; exits non-zero when any directional derivative
// disagrees beyond the truncation error of the difference quotient.
#include <cmath>
#include <cstdio>
#include <random>

#include "dg2_vjp.h"

using namespace dg2::adj;

namespace {

std::mt19937_64 rng(7);
double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

int failures = 0;
double worst = 0.0;

// Fourth-order central difference of f at 0 with step e.
template <typename F>
double cdiff(F f, double e) {
  return (8.0 * (f(e) - f(-e)) - (f(2 * e) - f(-2 * e))) / (12.0 * e);
}

// Compare <lambda, J v> from central differences with <J^T lambda, v>,
// relative to their size plus a scale for sums that cancel.
void report(const char *what, double fd, double ad, double scale) {
  const double err = std::fabs(fd - ad) / (std::fabs(fd) + std::fabs(ad) + scale);
  worst = err > worst ? err : worst;
  const bool ok = err < 1e-6;
  if (!ok) {
    ++failures;
    if (failures < 20) std::printf("FAIL %s fd=%.12e ad=%.12e rel=%.2e\n", what, fd, ad, err);
  }
}

const double g = 9.81, tol = 1e-5;

void check_hll(const char *what, double hL, double uL, double vL, double hR, double uR, double vR) {
  double lF[3] = {U(-1, 1), U(-1, 1), U(-1, 1)};
  double x[6] = {hL, uL, vL, hR, uR, vR};
  double v[6];
  for (double &d : v) d = U(-1, 1);
  // keep the depth perturbation from crossing the drying tolerance
  const double eps = 1e-4;
  auto f = [&](double s) {
    double y[6], F[3];
    for (int k = 0; k < 6; ++k) y[k] = x[k] + s * v[k] * (k % 3 == 0 ? 1e-3 * x[k] : 1.0);
    hll(y[0], y[1], y[2], y[3], y[4], y[5], g, tol, F);
    return lF[0] * F[0] + lF[1] * F[1] + lF[2] * F[2];
  };
  const double fd = cdiff(f, eps);
  double l[6];
  hll_vjp(hL, uL, vL, hR, uR, vR, g, tol, lF, l);
  double ad = 0;
  for (int k = 0; k < 6; ++k) ad += l[k] * v[k] * (k % 3 == 0 ? 1e-3 * x[k] : 1.0);
  report(what, fd, ad, 1e-12);
}

void check_gflux() {
  const double h = U(0.05, 3), qn = U(-2, 2), qt = U(-2, 2);
  double lF[3] = {U(-1, 1), U(-1, 1), U(-1, 1)}, v[3] = {U(-1, 1), U(-1, 1), U(-1, 1)};
  const double eps = 1e-4;
  auto f = [&](double s) {
    double F[3];
    gflux(h + s * v[0], qn + s * v[1], qt + s * v[2], g, tol, F);
    return lF[0] * F[0] + lF[1] * F[1] + lF[2] * F[2];
  };
  double lh, lqn, lqt;
  gflux_vjp(h, qn, qt, g, tol, lF, lh, lqn, lqt);
  report("gflux", cdiff(f, eps), lh * v[0] + lqn * v[1] + lqt * v[2], 1e-12);
}

void check_inflow(const char *what, double q, double h_in) {
  const double l0 = U(-1, 1), l1 = U(-1, 1), vq = U(-1, 1), vh = U(-1, 1);
  const double eps = 1e-4;
  auto f = [&](double s) {
    double F0, F1;
    inflow(q + s * vq, h_in + s * vh, g, F0, F1);
    return l0 * F0 + l1 * F1;
  };
  double lq, lh;
  inflow_vjp(q, h_in, g, l0, l1, lq, lh);
  report(what, cdiff(f, eps), lq * vq + lh * vh, 1e-12);
}

void check_fric_elem(const char *what, double h0) {
  double Ux[9] = {h0, U(-0.2, 0.2) * h0, U(-0.2, 0.2) * h0, U(-1, 1), U(-0.3, 0.3), U(-0.3, 0.3),
                  U(-1, 1), U(-0.3, 0.3), U(-0.3, 0.3)};
  const double n = U(0.02, 0.06), gdt = g * U(0.05, 2.0);
  double lW[9], v[9], vn = U(-1, 1);
  for (int k = 0; k < 9; ++k) {
    lW[k] = U(-1, 1);
    v[k] = U(-1, 1) * (k < 3 ? 0.01 * h0 : 0.1);
  }
  const double eps = 1e-3;
  auto f = [&](double s) {
    double Y[9], W[9];
    for (int k = 0; k < 9; ++k) Y[k] = Ux[k] + s * v[k];
    fric_elem(Y, n + s * vn * 0.01, gdt, tol, W);
    double acc = 0;
    for (int k = 0; k < 9; ++k) acc += lW[k] * W[k];
    return acc;
  };
  double lU[9], ln = 0;
  fric_elem_vjp(Ux, n, gdt, tol, lW, lU, ln);
  double ad = ln * vn * 0.01, mag = std::fabs(ad);
  for (int k = 0; k < 9; ++k) {
    ad += lU[k] * v[k];
    mag += std::fabs(lU[k] * v[k]);
  }
  report(what, cdiff(f, eps), ad, mag);
}

}  // namespace

int main() {
  for (int rep = 0; rep < 2000; ++rep) {
    // both wet, subcritical
    check_hll("hll wet", U(0.1, 3), U(-1, 1), U(-1, 1), U(0.1, 3), U(-1, 1), U(-1, 1));
    // supercritical to the right / left
    check_hll("hll sL>0", U(0.1, 0.5), U(4, 8), U(-1, 1), U(0.1, 0.5), U(4, 8), U(-1, 1));
    check_hll("hll sR<0", U(0.1, 0.5), U(-8, -4), U(-1, 1), U(0.1, 0.5), U(-8, -4), U(-1, 1));
    // one side dry (depth below the tolerance, zero velocity by the dummy limit)
    check_hll("hll dryL", U(0, 5e-6), 0.0, 0.0, U(0.1, 2), U(-1, 1), U(-1, 1));
    check_hll("hll dryR", U(0.1, 2), U(-1, 1), U(-1, 1), U(0, 5e-6), 0.0, 0.0);
    check_gflux();
    check_inflow("inflow critical", U(0.5, 3), U(0.01, 0.1));
    check_inflow("inflow inner", U(0.01, 0.3), U(0.5, 2));
    check_fric_elem("friction deep", U(0.3, 3));
    check_fric_elem("friction thin", U(0.002, 0.02));
  }
  std::printf("vjp_check: %d failures, largest relative difference %.2e\n", failures, worst);
  return failures ? 1 : 0;
}
