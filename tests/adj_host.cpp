// Host build of the operator adjoint in dg2_vjp.h over a whole grid, for
// tests/test_vjp_host.py to compare with reverse-mode differentiation of the
// oracle's spatial operator.  Planes are unpadded (stride nx * ny).
#include "dg2_vjp.h"

extern "C" void op_vjp_grid(const double *X, const double *lam, const unsigned char *mask,
                            const double *z, int nx, int ny, double dx, double dy, double g,
                            double tol, const int *seg_first, const int *seg_last, const double *q,
                            double *JT, double *lq_sum) {
  dg2::adj::OpAdj a{};
  a.X = X;
  a.lam = lam;
  a.mask = mask;
  a.z = z;
  a.nx = nx;
  a.ny = ny;
  a.P = (long long)nx * ny;
  a.idx = 1.0 / dx;
  a.idy = 1.0 / dy;
  a.g = g;
  a.tol = tol;
  for (int s = 0; s < 4; ++s) {
    a.seg_first[s] = seg_first[s];
    a.seg_last[s] = seg_last[s];
    a.q[s] = q[s];
    lq_sum[s] = 0.0;
  }
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      double out[9], lq[4];
      dg2::adj::operator_vjp(a, i, j, out, lq);
      const long long c = (long long)j * nx + i;
      for (int k = 0; k < 9; ++k) JT[k * a.P + c] = out[k];
      for (int s = 0; s < 4; ++s) lq_sum[s] += lq[s];
    }
  }
}
