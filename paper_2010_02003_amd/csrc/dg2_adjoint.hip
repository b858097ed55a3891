// Adjoint (reverse mode) of the DG2-NL time step: gradients of a loss on the
// gauge depths with respect to the per-cell Manning coefficient and the
// samples of one inflow hydrograph.
//
// Forward: the production stage kernels advance the state with a fixed step
// size, record the gauge depths after every step and keep a checkpoint of
// the state (and the device step record) every K steps.
//
// Backward: segments are taken from the last to the first.  A segment is
// recomputed from its checkpoint with the same production kernels, which
// now also keep every step's state U^n, stage-1 result U1^n, the wet/dry
// decisions of both stages and the step record.  The forward run already
// keeps these for its last segment, so that one is not recomputed (with a
// checkpoint interval of at least the step count nothing is: the whole
// trajectory stays in HBM, about 2 states per step).  The steps of the
// segment are then reversed, each with two gather kernels (one thread per
// cell):
//
//   stage 2:  U^{n+1} = fix(0.5 (W + U1 + dt L(U1)))
//             lam_U1 = 0.5 mu2 + 0.5 dt (dL/dU1)^T mu2,  mu2 = mask2(lam)
//             (the kernel also rebuilds W = friction(U^n + rain) per cell)
//   stage 1:  U1 = fix(W + dt L(W))
//             lam_W = 0.5 mu2 + mu1 + dt (dL/dW)^T mu1,   mu1 = mask1(lam_U1)
//             lam_U^n = (dW/dU^n)^T lam_W (friction split), dJ/dn += ...
//             plus the loss's own seed at the gauges of U^n.
//
// The adjoint of each cell's operator gathers the face-flux adjoints of its
// four faces from its own and its neighbours' mu (dg2_vjp.h).  The adjoint of
// the control side's unit discharge is written per face and per stage into
// a slot of its own, and the host maps these onto the hydrograph samples with
// the interpolation weights of each stage time, so the result does not
// depend on the order of floating-point atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/dg2.h"
#include "dg2_ctx.h"
#include "dg2_device.h"
#include "dg2_internal.h"
#include "dg2_vjp.h"

using namespace dg2;

namespace {

// Geometry and problem data shared by every reverse step.
struct AdjGeom {
  const double *z;  // bed modes (3 planes)
  const double *n;  // per-cell Manning or nullptr
  double n_uniform;
  int nx, ny;
  long long P;
  double idx, idy, g, tol;
  int seg_first[4], seg_last[4];
  int ctl_side, ctl_first, ctl_len;  // control inflow side (-1: none)
  int ng;
  const int *g_cell;
  const double *g_xi, *g_zeta;
};

// Data of one step of the recomputed trajectory.
struct AdjStep {
  const double *U;         // U^n
  const double *U1;        // stage-1 result
  const unsigned char *m1; // wet/dry codes of the stage-1 result
  const unsigned char *m2; // wet/dry codes of U^{n+1}
  const Ctrl *ctrl;        // step record: dt, rain, stage inflows
  double *lamq;            // 2 x ctl_len slots: control discharge adjoint per stage and face
};

constexpr int kBX = 64, kBY = 4;

__device__ __forceinline__ adj::OpAdj op_args(const AdjGeom &G, const double *X, const double *lam,
                                              const unsigned char *mask, const Ctrl *ctrl, int si) {
  adj::OpAdj a;
  a.X = X;
  a.lam = lam;
  a.mask = mask;
  a.z = G.z;
  a.nx = G.nx;
  a.ny = G.ny;
  a.P = G.P;
  a.idx = G.idx;
  a.idy = G.idy;
  a.g = G.g;
  a.tol = G.tol;
  for (int s = 0; s < 4; ++s) {
    a.seg_first[s] = G.seg_first[s];
    a.seg_last[s] = G.seg_last[s];
    a.q[s] = ctrl->qin[s][si];
  }
  return a;
}

// Face index of cell (i, j) on the control side, or -1.
__device__ __forceinline__ int control_face(const AdjGeom &G, int i, int j) {
  switch (G.ctl_side) {
    case 0: return i == 0 ? j - G.ctl_first : -1;
    case 1: return i == G.nx - 1 ? j - G.ctl_first : -1;
    case 2: return j == 0 ? i - G.ctl_first : -1;
    case 3: return j == G.ny - 1 ? i - G.ctl_first : -1;
    default: return -1;
  }
}

__global__ void __launch_bounds__(kBX *kBY)
    k_adj_stage2(AdjGeom G, AdjStep S, const double *__restrict__ lam, double *__restrict__ lamU1,
                 double *__restrict__ Wout) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
  if (i >= G.nx || j >= G.ny) return;
  const long long c = (long long)j * G.nx + i;
  const double dt = S.ctrl->dt;
  const adj::OpAdj a = op_args(G, S.U1, lam, S.m2, S.ctrl, 1);
  double JT[9], lq[4], mu[9];
  adj::operator_vjp(a, i, j, JT, lq);
  adj::load_mu(a, c, mu);
  for (int k = 0; k < 9; ++k) lamU1[k * G.P + c] = 0.5 * mu[k] + (0.5 * dt) * JT[k];
  const int f = control_face(G, i, j);
  if (f >= 0 && f < G.ctl_len) S.lamq[G.ctl_len + f] = (0.5 * dt) * lq[G.ctl_side];
  // stage-1 input W of this cell, exactly as the forward stage kernel forms it
  double W[9];
  for (int k = 0; k < 9; ++k) W[k] = S.U[k * G.P + c];
  const double g = G.g;
  const double gdt = g * dt;
  const double n = G.n ? G.n[c] : G.n_uniform;
  W[0] += S.ctrl->rain;
  apply_friction(W, gdt * n * n, G.tol);
  for (int k = 0; k < 9; ++k) Wout[k * G.P + c] = W[k];
}

__global__ void __launch_bounds__(kBX *kBY)
    k_adj_stage1(AdjGeom G, AdjStep S, const double *__restrict__ W,
                 const double *__restrict__ lamU1, double *lam, double *__restrict__ gn,
                 const double *__restrict__ seed) {
  const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
  if (i >= G.nx || j >= G.ny) return;
  const long long c = (long long)j * G.nx + i;
  const double dt = S.ctrl->dt;
  const adj::OpAdj a = op_args(G, W, lamU1, S.m1, S.ctrl, 0);
  double JT[9], lq[4], mu1[9], mu2[9], lW[9], lU[9];
  adj::operator_vjp(a, i, j, JT, lq);
  adj::load_mu(a, c, mu1);
  for (int k = 0; k < 9; ++k) mu2[k] = lam[k * G.P + c];
  adj::apply_mask(S.m2[c], mu2);
  for (int k = 0; k < 9; ++k) lW[k] = 0.5 * mu2[k] + mu1[k] + dt * JT[k];
  const int f = control_face(G, i, j);
  if (f >= 0 && f < G.ctl_len) S.lamq[f] = dt * lq[G.ctl_side];
  // friction split of Y = U^n + rain (the rain only shifts the mean depth)
  double Y[9];
  for (int k = 0; k < 9; ++k) Y[k] = S.U[k * G.P + c];
  Y[0] += S.ctrl->rain;
  const double n = G.n ? G.n[c] : G.n_uniform;
  double ln = 0.0;
  adj::fric_elem_vjp(Y, n, G.g * dt, G.tol, lW, lU, ln);
  // the loss's seed at the gauges sampled on U^n
  if (seed) {
    for (int k = 0; k < G.ng; ++k) {
      if (G.g_cell[k] != (int)c) continue;
      const double r = seed[k];
      lU[0] += r;
      lU[1] += r * G.g_xi[k];
      lU[2] += r * G.g_zeta[k];
    }
  }
  for (int k = 0; k < 9; ++k) lam[k * G.P + c] = lU[k];
  gn[c] += ln;
}

// lam = 0 except the seed of the last gauge sample; gn = 0.
__global__ void __launch_bounds__(256) k_adj_init(AdjGeom G, double *lam, double *gn,
                                                  const double *__restrict__ seed) {
  const long long n = (long long)G.ny * G.nx;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < G.ng; ++k) {
      if (G.g_cell[k] != (int)c) continue;
      v[0] += seed[k];
      v[1] += seed[k] * G.g_xi[k];
      v[2] += seed[k] * G.g_zeta[k];
    }
    for (int k = 0; k < 9; ++k) lam[k * G.P + c] = k < 3 ? v[k] : 0.0;
    gn[c] = 0.0;
  }
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================

struct dg2_adj {
  dg2_ctx *ctx = nullptr;
  int steps = 0, K = 0, nseg = 0;
  int side = -1, ctl_len = 0, nhyd = 0;
  double seg_len = 1.0;
  std::vector<double> hyd_t;  // host copy of the control hydrograph times
  size_t sb = 0;              // bytes of one 9-plane state
  double *U0 = nullptr;       // initial state
  Ctrl *ctrl0 = nullptr;      // initial step record
  Ctrl *actrl = nullptr;      // running step record
  double *ckpt = nullptr;     // nseg states
  Ctrl *ckctrl = nullptr;     // nseg step records
  double *Useg = nullptr;     // K + 1 states
  double *U1seg = nullptr;    // K stage-1 results
  unsigned char *mseg = nullptr;  // 2 K wet/dry code planes
  Ctrl *ctrlseg = nullptr;    // K step records
  int held = -1;              // the segment whose steps the segment buffers hold (-1: none)
  double *lam = nullptr, *lamU1 = nullptr, *Wbuf = nullptr, *gn = nullptr;
  double *lamq = nullptr;     // steps x 2 x ctl_len
  double *seed = nullptr;     // steps x ng
  double *g_buf = nullptr, *g_t = nullptr;  // forward gauge record
  bool forward_done = false;
  double t0 = 0.0;
  long long step0 = 0;  // the context's step count at U^0
  double ms_fwd = 0.0, ms_bwd = 0.0;
  std::string err;
};

namespace {

thread_local std::string g_adj_error;

dg2_status afail(dg2_adj *a, dg2_status s, const std::string &m) {
  if (a)
    a->err = m;
  else
    g_adj_error = m;
  return s;
}

dg2_status ahip(dg2_adj *a, hipError_t e, const char *what) {
  return afail(a, e == hipErrorOutOfMemory ? DG2_ENOMEM : DG2_EHIP,
               std::string(what) + ": " + hipGetErrorString(e));
}

#define ACHK(a, expr, what)                          \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return ahip(a, _e, what);  \
  } while (0)

AdjGeom geom(const dg2_adj *a) {
  const dg2_ctx *c = a->ctx;
  AdjGeom G{};
  G.z = (const double *)c->z;
  G.n = c->has_ncell ? (const double *)c->n : nullptr;
  G.n_uniform = c->n_uniform;
  G.nx = c->cfg.nx;
  G.ny = c->cfg.ny;
  G.P = c->P;
  G.idx = 1.0 / c->cfg.dx;
  G.idy = 1.0 / c->cfg.dy;
  G.g = c->cfg.g;
  G.tol = c->cfg.tol_dry;
  for (int k = 0; k < 4; ++k) {
    const bool on = side_table_on(c, k);
    G.seg_first[k] = on ? c->seg_first[k] : 1;
    G.seg_last[k] = on ? c->seg_last[k] : 0;
  }
  G.ctl_side = a->side;
  G.ctl_first = a->side >= 0 ? c->seg_first[a->side] : 0;
  G.ctl_len = a->ctl_len;
  G.ng = c->ng;
  G.g_cell = c->g_cell;
  G.g_xi = (const double *)c->g_xi;
  G.g_zeta = (const double *)c->g_zeta;
  return G;
}

// Production stage-kernel arguments on the adjoint's own buffers.
Scen<double> fwd_scen(const dg2_adj *a, const double *U, double *U1, double *Uout,
                      unsigned char *mask, bool gauges) {
  Scen<double> s = scen<double>(a->ctx);
  s.U = U;
  s.U1 = U1;
  s.Uout = Uout;
  s.mask = mask;
  s.W1 = nullptr;
  s.ctrl = a->actrl;
  if (gauges) {
    s.g_buf = a->g_buf;
    s.g_cap = a->steps;
  } else {
    s.ng = 0;
  }
  return s;
}

PlanArgs fwd_plan(const dg2_adj *a, bool gauges) {
  PlanArgs p = plan_args(a->ctx);
  if (gauges) {
    p.gauge_cap = a->steps;
    p.gauge_t = a->g_t;
  } else {
    p.ng = 0;
  }
  return p;
}

double *state(double *base, const dg2_adj *a, long long k) {
  return (double *)((char *)base + (size_t)k * a->sb);
}

hipError_t queue_fwd_step(dg2_adj *a, const Scen<double> &s1, const Scen<double> &s2,
                          const PlanArgs &pa) {
  const dg2_ctx *c = a->ctx;
  const Launch L = stage_launch_of(c);
  hipError_t e = launch_stage<double>(1, DG2_NL, s1, consts(c), L, c->stream);
  if (e == hipSuccess) e = launch_stage<double>(2, DG2_NL, s2, consts(c), L, c->stream);
  if (e == hipSuccess) e = launch_plan(a->actrl, pa, kPlanFinishStep, 0.0, 0, c->stream);
  return e;
}

// Interpolation weights of the hydrograph at time x (the step planner's rule).
void hat_weights(const std::vector<double> &t, double x, int &k0, double &w0, int &k1, double &w1) {
  const int n = (int)t.size();
  if (x <= t[0]) {
    k0 = k1 = 0;
    w0 = 1.0;
    w1 = 0.0;
    return;
  }
  if (x >= t[n - 1]) {
    k0 = k1 = n - 1;
    w0 = 1.0;
    w1 = 0.0;
    return;
  }
  int k = 0;
  while (k + 1 < n && t[k + 1] <= x) ++k;
  const double w = (x - t[k]) / (t[k + 1] - t[k]);
  k0 = k;
  k1 = k + 1;
  w0 = 1.0 - w;
  w1 = w;
}

}  // namespace

extern "C" {

const char *dg2_adj_last_error(const dg2_adj *a) { return a ? a->err.c_str() : g_adj_error.c_str(); }

void dg2_adj_destroy(dg2_adj *a) {
  if (!a) return;
  if (a->ctx && a->ctx->stream) (void)hipStreamSynchronize(a->ctx->stream);
  void *bufs[] = {a->U0, a->ctrl0, a->actrl, a->ckpt, a->ckctrl, a->Useg, a->U1seg, a->mseg,
                  a->ctrlseg, a->lam, a->lamU1, a->Wbuf, a->gn, a->lamq, a->seed, a->g_buf, a->g_t};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete a;
}

dg2_status dg2_adj_create(dg2_ctx *c, int32_t steps, int32_t every, int32_t side, dg2_adj **out) {
  if (!out) return afail(nullptr, DG2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!c) return afail(nullptr, DG2_EINVAL, "ctx is NULL");
  if (c->f32 || c->cfg.variant != DG2_NL || c->cfg.flux != DG2_FLUX_HLL)
    return afail(nullptr, DG2_EUNSUPPORTED, "the adjoint step is FP64 DG2-NL with the HLL flux only");
  if (!(c->fixed_dt > 0)) return afail(nullptr, DG2_ESTATE, "the adjoint needs a fixed step size");
  if (c->ng < 1) return afail(nullptr, DG2_ESTATE, "the adjoint needs at least one gauge");
  if (steps < 1 || every < 1) return afail(nullptr, DG2_EINVAL, "steps and checkpoint interval must be >= 1");
  if (side < -1 || side > 3) return afail(nullptr, DG2_EINVAL, "bad control side");
  if (side >= 0 && !(c->bkind[side] == DG2_BC_INFLOW_Q && side_table_on(c, side)))
    return afail(nullptr, DG2_ESTATE, "the control side has no inflow hydrograph");
  for (int k = 0; k < 4; ++k)
    if (side_active(c, k) && c->bkind[k] != DG2_BC_INFLOW_Q)
      return afail(nullptr, DG2_EUNSUPPORTED, "the adjoint step handles walls and discharge inflows only");

  dg2_adj *a = new (std::nothrow) dg2_adj();
  if (!a) return afail(nullptr, DG2_ENOMEM, "host allocation failed");
  a->ctx = c;
  a->steps = steps;
  a->K = every < steps ? every : steps;
  a->nseg = (steps + a->K - 1) / a->K;
  a->side = side;
  a->sb = 9 * (size_t)c->P * sizeof(double);
  auto bail = [&](dg2_status s) {
    g_adj_error = a->err;
    dg2_adj_destroy(a);
    return s;
  };
  if (side >= 0) {
    a->ctl_len = c->seg_last[side] - c->seg_first[side] + 1;
    a->nhyd = c->nhyd[side];
    const double d = (side == DG2_WEST || side == DG2_EAST) ? c->cfg.dy : c->cfg.dx;
    a->seg_len = a->ctl_len * d;
    a->hyd_t.resize(a->nhyd);
  }
  const size_t P = (size_t)c->P;
  const int K = a->K, ng = c->ng;
  struct {
    void **p;
    size_t bytes;
  } req[] = {
      {(void **)&a->U0, a->sb},
      {(void **)&a->ctrl0, sizeof(Ctrl)},
      {(void **)&a->actrl, sizeof(Ctrl)},
      {(void **)&a->ckpt, a->sb * a->nseg},
      {(void **)&a->ckctrl, sizeof(Ctrl) * a->nseg},
      {(void **)&a->Useg, a->sb * (K + 1)},
      {(void **)&a->U1seg, a->sb * K},
      {(void **)&a->mseg, P * 2 * K},
      {(void **)&a->ctrlseg, sizeof(Ctrl) * K},
      {(void **)&a->lam, a->sb},
      {(void **)&a->lamU1, a->sb},
      {(void **)&a->Wbuf, a->sb},
      {(void **)&a->gn, P * sizeof(double)},
      {(void **)&a->lamq, sizeof(double) * 2 * (size_t)steps * (a->ctl_len > 0 ? a->ctl_len : 1)},
      {(void **)&a->seed, sizeof(double) * (size_t)steps * ng},
      {(void **)&a->g_buf, sizeof(double) * 4 * (size_t)steps * ng},
      {(void **)&a->g_t, sizeof(double) * (size_t)steps},
  };
  for (auto &r : req) {
    hipError_t e = hipMalloc(r.p, r.bytes);
    if (e != hipSuccess) return bail(ahip(a, e, "adjoint buffers"));
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(a->U0, c->U, a->sb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && side >= 0)
    e = hipMemcpyAsync(a->hyd_t.data(), c->hyd_t[side], a->nhyd * sizeof(double),
                       hipMemcpyDeviceToHost, c->stream);
  // the initial step record: the context's time, nothing latched, no target
  Ctrl h{};
  if (e == hipSuccess) e = hipMemcpyAsync(&h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  h.flags = 0;
  h.gauge_written = 0;
  h.t_end = std::numeric_limits<double>::infinity();
  h.minbits = kInfBits;
  if (e == hipSuccess) e = hipMemcpyAsync(a->ctrl0, &h, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(ahip(a, e, "adjoint setup"));
  a->t0 = h.t;
  a->step0 = h.step;
  *out = a;
  return DG2_OK;
}

dg2_status dg2_adj_forward(dg2_adj *a, const double *n_cell, const double *Q, double *gauge_h) {
  if (!a) return DG2_EINVAL;
  dg2_ctx *c = a->ctx;
  if (n_cell) {
    if (dg2_set_manning(c, n_cell, 0.0) != DG2_OK)
      return afail(a, DG2_EINVAL, std::string("Manning field: ") + c->err);
  }
  if (Q) {
    if (a->side < 0) return afail(a, DG2_ESTATE, "no control hydrograph");
    for (int k = 0; k < a->nhyd; ++k)
      if (!std::isfinite(Q[k]) || Q[k] < 0) return afail(a, DG2_EINVAL, "Q must be finite and >= 0");
    ACHK(a, hipMemcpyAsync(c->hyd_Q[a->side], Q, a->nhyd * sizeof(double), hipMemcpyHostToDevice,
                           c->stream), "hydrograph");
    ACHK(a, hipStreamSynchronize(c->stream), "hydrograph");
  }
  hipStream_t st = c->stream;
  hipEvent_t ev[2];
  ACHK(a, hipEventCreate(&ev[0]), "event");
  ACHK(a, hipEventCreate(&ev[1]), "event");
  // initial state and step record; the gauge record restarts
  ACHK(a, hipMemcpyAsync(a->Useg, a->U0, a->sb, hipMemcpyDeviceToDevice, st), "forward");
  ACHK(a, hipMemcpyAsync(a->actrl, a->ctrl0, sizeof(Ctrl), hipMemcpyDeviceToDevice, st), "forward");
  const PlanArgs pa = fwd_plan(a, true);
  ACHK(a, launch_plan(a->actrl, pa, kPlanOnly, std::numeric_limits<double>::infinity(), 1, st), "plan");
  const Scen<double> s = fwd_scen(a, a->Useg, a->U1seg, a->Useg, nullptr, true);
  // the last segment's steps go to the segment buffers, as the backward
  // run's recompute would put them there, with the step records
  const int last0 = (a->nseg - 1) * a->K;
  PlanArgs pl = pa;
  pl.hist = a->ctrlseg;
  pl.hist_len = a->K;
  pl.hist_base = a->step0 + last0;
  a->held = -1;
  const size_t P = (size_t)c->P;
  ACHK(a, hipEventRecord(ev[0], st), "event");
  for (int n = 0; n < a->steps; ++n) {
    if (n % a->K == 0) {
      const int k = n / a->K;
      ACHK(a, hipMemcpyAsync(state(a->ckpt, a, k), a->Useg, a->sb, hipMemcpyDeviceToDevice, st), "checkpoint");
      ACHK(a, hipMemcpyAsync(a->ckctrl + k, a->actrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, st), "checkpoint");
    }
    if (n < last0) {
      ACHK(a, queue_fwd_step(a, s, s, pa), "forward step");
      continue;
    }
    const int m = n - last0;
    if (m == 0)
      ACHK(a, hipMemcpyAsync(a->ctrlseg, a->actrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, st), "segment");
    const Scen<double> s1 = fwd_scen(a, state(a->Useg, a, m), state(a->U1seg, a, m), nullptr,
                                     a->mseg + (size_t)(2 * m) * P, true);
    const Scen<double> s2 = fwd_scen(a, state(a->Useg, a, m), state(a->U1seg, a, m),
                                     state(a->Useg, a, m + 1), a->mseg + (size_t)(2 * m + 1) * P, true);
    ACHK(a, queue_fwd_step(a, s1, s2, pl), "forward step");
  }
  ACHK(a, hipEventRecord(ev[1], st), "event");
  ACHK(a, hipEventSynchronize(ev[1]), "forward");
  float ms = 0;
  (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
  a->ms_fwd = ms;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  Ctrl h{};
  ACHK(a, hipMemcpy(&h, a->actrl, sizeof(Ctrl), hipMemcpyDeviceToHost), "forward");
  if (h.flags & kFlagNaN) return afail(a, DG2_ENUMERIC, "NaN in the forward state");
  if (h.gauge_written != a->steps) return afail(a, DG2_ESTATE, "forward steps were idle");
  const int ng = c->ng;
  if (gauge_h) {
    std::vector<double> rec((size_t)a->steps * ng * 4);
    ACHK(a, hipMemcpy(rec.data(), a->g_buf, rec.size() * sizeof(double), hipMemcpyDeviceToHost), "gauges");
    for (int n = 0; n < a->steps; ++n)
      for (int k = 0; k < ng; ++k) gauge_h[(size_t)n * ng + k] = rec[((size_t)n * ng + k) * 4];
  }
  a->held = a->nseg - 1;
  a->forward_done = true;
  return DG2_OK;
}

dg2_status dg2_adj_backward(dg2_adj *a, const double *dL_dh, double *grad_n, double *grad_Q) {
  if (!a) return DG2_EINVAL;
  if (!a->forward_done) return afail(a, DG2_ESTATE, "dg2_adj_forward must run first");
  if (!dL_dh) return afail(a, DG2_EINVAL, "dL_dh is NULL");
  dg2_ctx *c = a->ctx;
  hipStream_t st = c->stream;
  const int ng = c->ng, N = a->steps, K = a->K;
  for (size_t k = 0; k < (size_t)N * ng; ++k)
    if (!std::isfinite(dL_dh[k])) return afail(a, DG2_EINVAL, "dL_dh has non-finite values");
  ACHK(a, hipMemcpyAsync(a->seed, dL_dh, sizeof(double) * N * ng, hipMemcpyHostToDevice, st), "seed");
  const AdjGeom G = geom(a);
  const size_t P = (size_t)c->P;
  const dim3 blk(kBX, kBY), grd((G.nx + kBX - 1) / kBX, (G.ny + kBY - 1) / kBY);
  const int L = a->ctl_len > 0 ? a->ctl_len : 1;
  hipEvent_t ev[2];
  ACHK(a, hipEventCreate(&ev[0]), "event");
  ACHK(a, hipEventCreate(&ev[1]), "event");
  ACHK(a, hipEventRecord(ev[0], st), "event");
  hipLaunchKernelGGL(k_adj_init, dim3(1024), dim3(256), 0, st, G, a->lam, a->gn,
                     (const double *)(a->seed + (size_t)(N - 1) * ng));
  ACHK(a, hipGetLastError(), "adjoint init");
  // the planner records each recomputed step's plan in ctrlseg
  PlanArgs pa = fwd_plan(a, false);
  pa.hist = a->ctrlseg;
  pa.hist_len = K;
  for (int sg = a->nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * K, len = (N - n0) < K ? (N - n0) : K;
    // recompute the segment, keeping every step, unless the buffers hold it
    if (a->held != sg) {
      a->held = -1;
      ACHK(a, hipMemcpyAsync(a->Useg, state(a->ckpt, a, sg), a->sb, hipMemcpyDeviceToDevice, st),
           "restore");
      ACHK(a, hipMemcpyAsync(a->actrl, a->ckctrl + sg, sizeof(Ctrl), hipMemcpyDeviceToDevice, st),
           "restore");
      ACHK(a, hipMemcpyAsync(a->ctrlseg, a->ckctrl + sg, sizeof(Ctrl), hipMemcpyDeviceToDevice, st),
           "restore");
      pa.hist_base = a->step0 + n0;
      for (int m = 0; m < len; ++m) {
        const Scen<double> s1 = fwd_scen(a, state(a->Useg, a, m), state(a->U1seg, a, m), nullptr,
                                         a->mseg + (size_t)(2 * m) * P, false);
        const Scen<double> s2 = fwd_scen(a, state(a->Useg, a, m), state(a->U1seg, a, m),
                                         state(a->Useg, a, m + 1), a->mseg + (size_t)(2 * m + 1) * P,
                                         false);
        ACHK(a, queue_fwd_step(a, s1, s2, pa), "recompute step");
      }
      a->held = sg;
    }
    // reverse the segment's steps
    for (int m = len - 1; m >= 0; --m) {
      const int n = n0 + m;
      AdjStep S;
      S.U = state(a->Useg, a, m);
      S.U1 = state(a->U1seg, a, m);
      S.m1 = a->mseg + (size_t)(2 * m) * P;
      S.m2 = a->mseg + (size_t)(2 * m + 1) * P;
      S.ctrl = a->ctrlseg + m;
      S.lamq = a->lamq + (size_t)n * 2 * L;
      hipLaunchKernelGGL(k_adj_stage2, grd, blk, 0, st, G, S, (const double *)a->lam, a->lamU1, a->Wbuf);
      const double *sd = n >= 1 ? a->seed + (size_t)(n - 1) * ng : nullptr;
      hipLaunchKernelGGL(k_adj_stage1, grd, blk, 0, st, G, S, (const double *)a->Wbuf,
                         (const double *)a->lamU1, a->lam, a->gn, sd);
      ACHK(a, hipGetLastError(), "adjoint step");
    }
  }
  ACHK(a, hipEventRecord(ev[1], st), "event");
  ACHK(a, hipEventSynchronize(ev[1]), "backward");
  float ms = 0;
  (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
  a->ms_bwd = ms;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (grad_n)
    ACHK(a, hipMemcpy(grad_n, a->gn, sizeof(double) * c->ncell, hipMemcpyDeviceToHost), "grad n");
  if (grad_Q && a->side >= 0) {
    std::vector<double> lq((size_t)N * 2 * L);
    std::vector<double> tt(N);
    ACHK(a, hipMemcpy(lq.data(), a->lamq, lq.size() * sizeof(double), hipMemcpyDeviceToHost), "grad Q");
    ACHK(a, hipMemcpy(tt.data(), a->g_t, N * sizeof(double), hipMemcpyDeviceToHost), "grad Q");
    for (int k = 0; k < a->nhyd; ++k) grad_Q[k] = 0.0;
    const double dt = c->fixed_dt;
    for (int n = 0; n < N; ++n) {
      const double tn = n == 0 ? a->t0 : tt[n - 1];
      for (int si = 0; si < 2; ++si) {
        double sum = 0.0;
        for (int f = 0; f < a->ctl_len; ++f) sum += lq[((size_t)n * 2 + si) * L + f];
        int k0, k1;
        double w0, w1;
        hat_weights(a->hyd_t, si == 0 ? tn : tn + dt, k0, w0, k1, w1);
        grad_Q[k0] += sum * w0 / a->seg_len;
        grad_Q[k1] += sum * w1 / a->seg_len;
      }
    }
  }
  return DG2_OK;
}

dg2_status dg2_adj_timing(const dg2_adj *a, double *ms_forward, double *ms_backward) {
  if (!a) return DG2_EINVAL;
  if (ms_forward) *ms_forward = a->ms_fwd;
  if (ms_backward) *ms_backward = a->ms_bwd;
  return DG2_OK;
}

}  // extern "C"
