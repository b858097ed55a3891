// C-ABI runtime of the DG2 library: context, device buffers, problem setup,
// step queueing, run-to-time, gauges, diagnostics and timing.
//
// The host side only moves data and queues kernels; every arithmetic step
// of the time integration runs in the HIP kernels of dg2_kernels.hip.  The
// one-off setup arithmetic (bed and initial modes from corner values, Eq. 3)
// is done here in double precision before upload.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dg2.h"
#include "dg2_ctx.h"
#include "dg2_tune_cache.h"
#include "dg2_internal.h"

using namespace dg2;

namespace {

thread_local std::string g_create_error;

constexpr int kMaxGauges = 64;

}  // namespace

namespace {

dg2_status fail(dg2_ctx *c, dg2_status s, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return s;
}

dg2_status hipfail(dg2_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? DG2_ENOMEM : DG2_EHIP, m);
}

#define HIPCHK(ctx, expr, what)                  \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return hipfail(ctx, _e, what); \
  } while (0)

bool finite_all(const double *a, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) return false;
  return true;
}

// Eq. (3) from corner values: face-centre averages, then mean and slopes.
void corner_modes(const double *C, int nx, int ny, double *m0, double *m1x, double *m1y) {
  const int w = nx + 1;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const double E = 0.5 * (C[j * w + i + 1] + C[(j + 1) * w + i + 1]);
      const double W = 0.5 * (C[j * w + i] + C[(j + 1) * w + i]);
      const double N = 0.5 * (C[(j + 1) * w + i] + C[(j + 1) * w + i + 1]);
      const double S = 0.5 * (C[j * w + i] + C[j * w + i + 1]);
      const size_t c = (size_t)j * nx + i;
      m0[c] = 0.5 * (E + W);
      m1x[c] = 0.5 * (E - W);
      m1y[c] = 0.5 * (N - S);
    }
  }
}

// Copy n doubles from host into a device array of the context precision.
dg2_status upload(dg2_ctx *c, void *dst, const double *src, size_t n) {
  if (!c->f32) {
    HIPCHK(c, hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, c->stream), "upload");
  } else {
    std::vector<float> tmp(n);
    for (size_t k = 0; k < n; ++k) tmp[k] = (float)src[k];
    HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), n * 4, hipMemcpyHostToDevice, c->stream), "upload");
    HIPCHK(c, hipStreamSynchronize(c->stream), "upload sync");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "upload sync");
  return DG2_OK;
}

dg2_status download(dg2_ctx *c, double *dst, const void *src, size_t n) {
  if (!c->f32) {
    HIPCHK(c, hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, c->stream), "download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "download sync");
  } else {
    std::vector<float> tmp(n);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, c->stream), "download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "download sync");
    for (size_t k = 0; k < n; ++k) dst[k] = tmp[k];
  }
  return DG2_OK;
}

// A stage kernel on the context's buffers; ctrl != nullptr replaces the
// context's control block (the repeat block of the stage-1 Courant check).
hipError_t queue_stage(dg2_ctx *c, int stage, Ctrl *ctrl = nullptr) {
  const Launch L = stage_launch_of(c);
  if (c->f32) {
    Scen<float> s = scen<float>(c);
    if (ctrl) s.ctrl = ctrl;
    return launch_stage<float>(stage, c->cfg.variant, s, consts(c), L, c->stream);
  }
  Scen<double> s = scen<double>(c);
  if (ctrl) s.ctrl = ctrl;
  return launch_stage<double>(stage, c->cfg.variant, s, consts(c), L, c->stream);
}

// Courant minimum of the stage-1 result into the repeat block, then the
// check; attempt 0 follows the first stage 1, attempt k its k-th repeat.
hipError_t queue_stage_check(dg2_ctx *c, int attempt) {
  const Ctrl *gate = attempt == 0 ? nullptr : c->ctrl2;
  hipError_t e;
  if (c->f32) {
    Scen<float> s = scen<float>(c);
    s.U = (const float *)c->U1;
    e = launch_cfl<float>(s, consts(c), c->stream, gate, &c->ctrl2->minbits);
  } else {
    Scen<double> s = scen<double>(c);
    s.U = (const double *)c->U1;
    e = launch_cfl<double>(s, consts(c), c->stream, gate, &c->ctrl2->minbits);
  }
  if (e != hipSuccess) return e;
  return launch_stage_check(c->ctrl, c->ctrl2, plan_args(c), attempt == 0, attempt == c->stage_check,
                            c->stream);
}

hipError_t queue_plan(dg2_ctx *c, int mode, double t_end = 0.0, int set_tend = 0) {
  return launch_plan(c->ctrl, plan_args(c), mode, t_end, set_tend, c->stream);
}

// Both stages in one kernel into the second buffer, which becomes the state.
template <typename real>
hipError_t queue_fused_as(dg2_ctx *c) {
  Scen<real> s = scen<real>(c);
  s.Uout = (real *)c->U1;
  hipError_t e;
  if (c->stage_check > 0) {
    // trials of the whole step against the staging block; once one is
    // accepted the remaining trial launches return at once
    const PlanArgs pa = plan_args(c);
    s.ctrl = c->ctrl2;
    e = launch_fused_check(c->ctrl, c->ctrl2, pa, 1, 0, c->stream);
    for (int k = 0; k <= c->stage_check && e == hipSuccess; ++k) {
      e = launch_fused<real>(s, consts(c), fused_launch_of(c), c->stream, true);
      if (e == hipSuccess) e = launch_fused_check(c->ctrl, c->ctrl2, pa, 0, k == c->stage_check, c->stream);
    }
  } else {
    e = launch_fused<real>(s, consts(c), fused_launch_of(c), c->stream);
  }
  if (e == hipSuccess) std::swap(c->U, c->U1);
  return e;
}
hipError_t queue_fused(dg2_ctx *c) { return c->f32 ? queue_fused_as<float>(c) : queue_fused_as<double>(c); }

dg2_status queue_step(dg2_ctx *c, hipEvent_t *ev = nullptr) {
  if (fused_active(c)) {
    if (ev) HIPCHK(c, hipEventRecord(ev[0], c->stream), "event");
    HIPCHK(c, queue_fused(c), "step launch");
    if (ev) HIPCHK(c, hipEventRecord(ev[1], c->stream), "event");
    HIPCHK(c, queue_plan(c, kPlanFinishStep), "plan launch");
    return DG2_OK;
  }
  if (ev) HIPCHK(c, hipEventRecord(ev[0], c->stream), "event");
  HIPCHK(c, queue_stage(c, 1), "stage 1 launch");
  if (c->stage_check > 0) {
    // repeats of stage 1 with a smaller step; each returns at once unless
    // the check before it armed the repeat block
    HIPCHK(c, queue_stage_check(c, 0), "stage check launch");
    for (int k = 1; k <= c->stage_check; ++k) {
      HIPCHK(c, queue_stage(c, 1, c->ctrl2), "stage 1 repeat launch");
      HIPCHK(c, queue_stage_check(c, k), "stage check launch");
    }
  }
  if (ev) HIPCHK(c, hipEventRecord(ev[1], c->stream), "event");
  HIPCHK(c, queue_stage(c, 2), "stage 2 launch");
  if (ev) HIPCHK(c, hipEventRecord(ev[2], c->stream), "event");
  HIPCHK(c, queue_plan(c, kPlanFinishStep), "plan launch");
  return DG2_OK;
}

// Courant minimum of the state just uploaded, then plan the first step.
dg2_status prime(dg2_ctx *c) {
  const unsigned long long inf = kInfBits;
  HIPCHK(c, hipMemcpyAsync(&c->ctrl->minbits, &inf, 8, hipMemcpyHostToDevice, c->stream), "prime");
  hipError_t e = c->f32 ? launch_cfl<float>(scen<float>(c), consts(c), c->stream)
                        : launch_cfl<double>(scen<double>(c), consts(c), c->stream);
  HIPCHK(c, e, "cfl launch");
  HIPCHK(c, queue_plan(c, kPlanFromMin), "plan launch");
  HIPCHK(c, hipStreamSynchronize(c->stream), "prime sync");
  return DG2_OK;
}

dg2_status read_ctrl(dg2_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->hctrl, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream),
         "ctrl read");
  HIPCHK(c, hipStreamSynchronize(c->stream), "ctrl sync");
  return DG2_OK;
}

dg2_status latched(dg2_ctx *c) {
  if (c->hctrl->flags & kFlagNaN) return fail(c, DG2_ENUMERIC, "NaN in the state");
  return DG2_OK;
}

dg2_status alloc(dg2_ctx *c, void **p, size_t bytes, const char *what) {
  HIPCHK(c, hipMalloc(p, bytes), what);
  HIPCHK(c, hipMemsetAsync(*p, 0, bytes, c->stream), what);
  return DG2_OK;
}

dg2_status reset_time(dg2_ctx *c, double t) {
  Ctrl h{};
  h.t = t;
  h.dt = 0.0;
  h.t_end = std::numeric_limits<double>::infinity();
  h.cflmin = std::numeric_limits<double>::infinity();
  h.minbits = kInfBits;
  h.step = 0;
  h.gauge_written = 0;
  *c->hctrl = h;
  HIPCHK(c, hipMemcpyAsync(c->ctrl, c->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream), "ctrl");
  HIPCHK(c, hipStreamSynchronize(c->stream), "ctrl");
  c->g_read = 0;
  return DG2_OK;
}

}  // namespace

namespace {
// Cache key of a context's step: architecture, precision, variant, flux,
// kernel form (fused step or per-stage kernels) and size class.
std::string tune_key(const dg2_ctx *c) {
  char b[256];
  std::snprintf(b, sizeof(b), "%s|%s|%s|%s|%s|%lldx%lld", device_arch().c_str(), c->f32 ? "fp32" : "fp64",
                c->cfg.variant == DG2_LL ? "LL" : "NL", c->cfg.flux == DG2_FLUX_ROE ? "ROE" : "HLL",
                fused_active(c) ? "fused" : "stages", size_class(c->cfg.nx), size_class(c->cfg.ny));
  return b;
}
}  // namespace

extern "C" {

void dg2_config_default(dg2_config *cfg, int32_t nx, int32_t ny, double dx, double dy) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->nx = nx;
  cfg->ny = ny;
  cfg->dx = dx;
  cfg->dy = dy;
  cfg->prec = DG2_FP64;
  cfg->variant = DG2_NL;
  cfg->g = 9.81;
  cfg->cfl = 0.3;
  cfg->tol_dry = 1e-5;
  cfg->ll_threshold = 10.0;
  cfg->dt_max = 1.0;
}

const char *dg2_last_error(const dg2_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

void dg2_destroy(dg2_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  void *bufs[] = {c->U_own, c->U1_own, c->W1, c->z, c->n, c->ctrl, c->ctrl2, c->g_cell, c->g_xi,
                  c->g_zeta, c->g_z, c->g_buf, c->g_t, c->diag_part, c->diag_out};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  for (int s = 0; s < 4; ++s) {
    if (c->hyd_t[s]) (void)hipFree(c->hyd_t[s]);
    if (c->hyd_Q[s]) (void)hipFree(c->hyd_Q[s]);
  }
  if (c->hctrl) (void)hipHostFree(c->hctrl);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

dg2_status dg2_create(const dg2_config *cfg, dg2_ctx **out) {
  if (!out) return fail(nullptr, DG2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, DG2_EINVAL, "cfg is NULL");
  if (cfg->nx < 1 || cfg->ny < 1) return fail(nullptr, DG2_EINVAL, "nx and ny must be >= 1");
  // one plane must stay below 4 GiB (32-bit in-plane offsets in the kernels)
  if ((long long)cfg->nx * cfg->ny * (cfg->prec == DG2_FP32 ? 4 : 8) >= (1ll << 32))
    return fail(nullptr, DG2_EINVAL, "grid too large: nx*ny must be < 2^29 (FP64) or 2^30 (FP32)");
  if (!(cfg->dx > 0) || !(cfg->dy > 0) || !std::isfinite(cfg->dx) || !std::isfinite(cfg->dy))
    return fail(nullptr, DG2_EINVAL, "dx and dy must be positive");
  if (!(cfg->g > 0) || !(cfg->cfl > 0) || !(cfg->tol_dry > 0) || !(cfg->dt_max > 0) ||
      !(cfg->ll_threshold >= 0) || !std::isfinite(cfg->x0) || !std::isfinite(cfg->y0))
    return fail(nullptr, DG2_EINVAL, "g, cfl, tol_dry, dt_max must be > 0 and ll_threshold >= 0");
  if (cfg->prec != DG2_FP64 && cfg->prec != DG2_FP32) return fail(nullptr, DG2_EINVAL, "bad prec");
  if (cfg->variant != DG2_NL && cfg->variant != DG2_LL) return fail(nullptr, DG2_EINVAL, "bad variant");
  if (cfg->flux != DG2_FLUX_HLL && cfg->flux != DG2_FLUX_ROE) return fail(nullptr, DG2_EINVAL, "bad flux");

  dg2_ctx *c = new (std::nothrow) dg2_ctx();
  if (!c) return fail(nullptr, DG2_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->f32 = cfg->prec == DG2_FP32;
  c->esz = c->f32 ? 4 : 8;
  c->ncell = (long long)cfg->nx * cfg->ny;
  // plane stride: a multiple of 64 elements plus a skew of 576, so that the
  // same cell of different planes does not fall on the same HBM channel and
  // bank when nx * ny is a large power of two (about 2 % faster at 4096^2)
  c->P = (c->ncell + 63) / 64 * 64 + 576;
  auto bail = [&](dg2_status s) {
    g_create_error = c->err;
    dg2_destroy(c);
    return s;
  };
  hipError_t e;
  if (cfg->hip_stream) {
    c->stream = (hipStream_t)cfg->hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hipfail(c, e, "stream create"));
    c->own_stream = true;
  }
  // set-up of the allocation-free diagnostics: the device address of its
  // scratch on this device (looked up once per device)
  {
    double *records = nullptr;
    e = scratch_records(&records);
    if (e != hipSuccess) return bail(hipfail(c, e, "scratch address"));
  }
  const size_t pb = (size_t)c->P * c->esz;
  dg2_status s;
  if ((s = alloc(c, &c->U_own, 9 * pb, "state")) != DG2_OK) return bail(s);
  c->U = c->U_own;
  if ((s = alloc(c, &c->U1_own, 9 * pb, "stage buffer")) != DG2_OK) return bail(s);
  c->U1 = c->U1_own;
  if ((s = alloc(c, &c->z, 3 * pb, "bed")) != DG2_OK) return bail(s);
  if (cfg->variant == DG2_LL && (s = alloc(c, &c->W1, 9 * pb, "limited stage input")) != DG2_OK)
    return bail(s);
  if ((s = alloc(c, (void **)&c->ctrl, sizeof(Ctrl), "ctrl")) != DG2_OK) return bail(s);
  if ((s = alloc(c, (void **)&c->ctrl2, sizeof(Ctrl), "ctrl")) != DG2_OK) return bail(s);
  {
    Ctrl rep{};
    rep.minbits = kInfBits;
    rep.minbits1 = kInfBits;
    e = hipMemcpy(c->ctrl2, &rep, sizeof(Ctrl), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hipfail(c, e, "ctrl"));
  }
  if ((s = alloc(c, (void **)&c->diag_part, kDiagBlocks * 4 * sizeof(double), "diag")) != DG2_OK)
    return bail(s);
  if ((s = alloc(c, (void **)&c->diag_out, 4 * sizeof(double), "diag")) != DG2_OK) return bail(s);
  e = hipHostMalloc((void **)&c->hctrl, sizeof(Ctrl), hipHostMallocDefault);
  if (e != hipSuccess) return bail(hipfail(c, e, "pinned ctrl"));
  c->zc.assign((size_t)(cfg->nx + 1) * (cfg->ny + 1), 0.0);
  c->z0.assign(c->ncell, 0.0);
  c->z1x.assign(c->ncell, 0.0);
  c->z1y.assign(c->ncell, 0.0);
  if ((s = reset_time(c, 0.0)) != DG2_OK) return bail(s);
  if ((s = prime(c)) != DG2_OK) return bail(s);
  *out = c;
  return DG2_OK;
}

dg2_status dg2_set_dem_corners(dg2_ctx *c, const double *z) {
  if (!c) return DG2_EINVAL;
  if (!z) return fail(c, DG2_EINVAL, "z is NULL");
  const size_t nc = (size_t)(c->cfg.nx + 1) * (c->cfg.ny + 1);
  if (!finite_all(z, nc)) return fail(c, DG2_EINVAL, "DEM has non-finite values");
  c->zc.assign(z, z + nc);
  corner_modes(z, c->cfg.nx, c->cfg.ny, c->z0.data(), c->z1x.data(), c->z1y.data());
  dg2_status s;
  if ((s = upload(c, plane(c->z, c, 0), c->z0.data(), c->ncell)) != DG2_OK) return s;
  if ((s = upload(c, plane(c->z, c, 1), c->z1x.data(), c->ncell)) != DG2_OK) return s;
  if ((s = upload(c, plane(c->z, c, 2), c->z1y.data(), c->ncell)) != DG2_OK) return s;
  return DG2_OK;
}

dg2_status dg2_set_manning(dg2_ctx *c, const double *n_cell, double n_uniform) {
  if (!c) return DG2_EINVAL;
  if (n_cell) {
    for (long long k = 0; k < c->ncell; ++k)
      if (!(n_cell[k] >= 0) || !std::isfinite(n_cell[k]))
        return fail(c, DG2_EINVAL, "Manning values must be finite and >= 0");
    if (!c->n) {
      dg2_status s = alloc(c, &c->n, (size_t)c->P * c->esz, "manning");
      if (s != DG2_OK) return s;
    }
    dg2_status s = upload(c, c->n, n_cell, c->ncell);
    if (s != DG2_OK) return s;
    c->has_ncell = true;
  } else {
    if (!(n_uniform >= 0) || !std::isfinite(n_uniform))
      return fail(c, DG2_EINVAL, "Manning value must be finite and >= 0");
    c->has_ncell = false;
    c->n_uniform = n_uniform;
  }
  return DG2_OK;
}

dg2_status dg2_set_state(dg2_ctx *c, const double *m, double t) {
  if (!c) return DG2_EINVAL;
  if (!m) return fail(c, DG2_EINVAL, "modes9 is NULL");
  if (!std::isfinite(t)) return fail(c, DG2_EINVAL, "t must be finite");
  const size_t n = (size_t)c->ncell;
  if (!finite_all(m, 9 * n)) return fail(c, DG2_EINVAL, "state has non-finite values");
  for (size_t k = 0; k < n; ++k)
    if (m[k] < 0) return fail(c, DG2_EINVAL, "mean depth h0 must be >= 0");
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  for (int k = 0; k < 9; ++k) {
    dg2_status s = upload(c, plane(c->U, c, k), m + k * n, n);
    if (s != DG2_OK) return s;
  }
  dg2_status s = reset_time(c, t);
  if (s != DG2_OK) return s;
  return prime(c);
}

dg2_status dg2_set_initial_corners(dg2_ctx *c, const double *surf, int32_t is_eta, const double *qx,
                                   const double *qy) {
  if (!c) return DG2_EINVAL;
  if (!surf) return fail(c, DG2_EINVAL, "surface is NULL");
  const int nx = c->cfg.nx, ny = c->cfg.ny;
  const size_t nc = (size_t)(nx + 1) * (ny + 1), n = (size_t)c->ncell;
  if (!finite_all(surf, nc) || (qx && !finite_all(qx, nc)) || (qy && !finite_all(qy, nc)))
    return fail(c, DG2_EINVAL, "initial condition has non-finite values");
  if (!is_eta)
    for (size_t k = 0; k < nc; ++k)
      if (surf[k] < 0) return fail(c, DG2_EINVAL, "depths must be >= 0");
  std::vector<double> m(9 * n, 0.0);
  corner_modes(surf, nx, ny, &m[0], &m[n], &m[2 * n]);
  if (is_eta) {
    for (size_t k = 0; k < n; ++k) {
      double h0 = m[k] - c->z0[k], h1 = m[n + k] - c->z1x[k], h2 = m[2 * n + k] - c->z1y[k];
      if (h0 < 0) h0 = h1 = h2 = 0.0;
      m[k] = h0;
      m[n + k] = h1;
      m[2 * n + k] = h2;
    }
  }
  if (qx) corner_modes(qx, nx, ny, &m[3 * n], &m[4 * n], &m[5 * n]);
  if (qy) corner_modes(qy, nx, ny, &m[6 * n], &m[7 * n], &m[8 * n]);
  return dg2_set_state(c, m.data(), 0.0);
}

dg2_status dg2_get_state(dg2_ctx *c, double *m, double *t, int64_t *step, double *last_dt) {
  if (!c) return DG2_EINVAL;
  const size_t n = (size_t)c->ncell;
  if (m) {
    for (int k = 0; k < 9; ++k) {
      dg2_status s = download(c, m + k * n, plane(c->U, c, k), n);
      if (s != DG2_OK) return s;
    }
  }
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) return s;
  if (t) *t = c->hctrl->t;
  if (step) *step = c->hctrl->step;
  if (last_dt) *last_dt = c->hctrl->last_dt;
  return latched(c);
}

dg2_status dg2_set_boundary(dg2_ctx *c, int32_t side, int32_t bc, int32_t first, int32_t last) {
  if (!c) return DG2_EINVAL;
  if (side < 0 || side > 3) return fail(c, DG2_EINVAL, "bad side");
  const int len = (side == DG2_WEST || side == DG2_EAST) ? c->cfg.ny : c->cfg.nx;
  if (bc == DG2_BC_WALL) {
    c->bkind[side] = DG2_BC_WALL;
  } else if (bc == DG2_BC_INFLOW_Q || bc == DG2_BC_LEVEL || bc == DG2_BC_OPEN) {
    if (first < 0 || last >= len || first > last) return fail(c, DG2_EINVAL, "bad segment");
    c->bkind[side] = bc;
    c->seg_first[side] = first;
    c->seg_last[side] = last;
  } else {
    return fail(c, DG2_EINVAL, "bad boundary type");
  }
  HIPCHK(c, queue_plan(c, kPlanOnly), "plan");
  return DG2_OK;
}

namespace {

// Store a side's time table (discharge or water level) on the device.
dg2_status set_side_table(dg2_ctx *c, int32_t side, const double *t, const double *v, int32_t n,
                          int kind) {
  if (side < 0 || side > 3) return fail(c, DG2_EINVAL, "bad side");
  if (!t || !v || n < 1) return fail(c, DG2_EINVAL, "need n >= 1 samples");
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(t[k]) || !std::isfinite(v[k]))
      return fail(c, DG2_EINVAL, "hydrograph values must be finite");
    if (kind == DG2_BC_INFLOW_Q && v[k] < 0) return fail(c, DG2_EINVAL, "discharges must be >= 0");
    if (k > 0 && !(t[k] > t[k - 1])) return fail(c, DG2_EINVAL, "hydrograph times must increase");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  if (c->hyd_t[side]) (void)hipFree(c->hyd_t[side]);
  if (c->hyd_Q[side]) (void)hipFree(c->hyd_Q[side]);
  c->hyd_t[side] = c->hyd_Q[side] = nullptr;
  c->nhyd[side] = 0;
  HIPCHK(c, hipMalloc((void **)&c->hyd_t[side], n * 8), "hydrograph");
  HIPCHK(c, hipMalloc((void **)&c->hyd_Q[side], n * 8), "hydrograph");
  HIPCHK(c, hipMemcpy(c->hyd_t[side], t, n * 8, hipMemcpyHostToDevice), "hydrograph");
  HIPCHK(c, hipMemcpy(c->hyd_Q[side], v, n * 8, hipMemcpyHostToDevice), "hydrograph");
  c->nhyd[side] = n;
  c->hyd_kind[side] = kind;
  HIPCHK(c, queue_plan(c, kPlanOnly), "plan");
  return DG2_OK;
}

}  // namespace

dg2_status dg2_set_inflow_hydrograph(dg2_ctx *c, int32_t side, const double *t, const double *Q,
                                     int32_t n) {
  if (!c) return DG2_EINVAL;
  return set_side_table(c, side, t, Q, n, DG2_BC_INFLOW_Q);
}

dg2_status dg2_set_level_hydrograph(dg2_ctx *c, int32_t side, const double *t, const double *eta,
                                    int32_t n) {
  if (!c) return DG2_EINVAL;
  return set_side_table(c, side, t, eta, n, DG2_BC_LEVEL);
}

dg2_status dg2_set_rainfall(dg2_ctx *c, double rate, double tb, double te) {
  if (!c) return DG2_EINVAL;
  if (!(rate >= 0) || !std::isfinite(rate) || !std::isfinite(tb) || !std::isfinite(te) || te < tb)
    return fail(c, DG2_EINVAL, "rain needs rate >= 0 and t_begin <= t_end");
  c->rain_rate = rate;
  c->rain_tb = tb;
  c->rain_te = te;
  HIPCHK(c, queue_plan(c, kPlanOnly), "plan");
  return DG2_OK;
}

dg2_status dg2_set_fixed_dt(dg2_ctx *c, double dt) {
  if (!c) return DG2_EINVAL;
  if (!std::isfinite(dt)) return fail(c, DG2_EINVAL, "dt must be finite");
  c->fixed_dt = dt > 0 ? dt : 0.0;
  HIPCHK(c, queue_plan(c, kPlanOnly), "plan");
  return DG2_OK;
}

dg2_status dg2_set_gauges(dg2_ctx *c, const double *xy, int32_t n, int32_t cap) {
  if (!c) return DG2_EINVAL;
  if (n < 0 || n > kMaxGauges) return fail(c, DG2_EINVAL, "0 <= n <= 64 gauges");
  if (n > 0 && !xy) return fail(c, DG2_EINVAL, "xy is NULL");
  const dg2_config &g = c->cfg;
  std::vector<int> cell(n);
  std::vector<double> xi(n), ze(n), zp(n);
  for (int k = 0; k < n; ++k) {
    const double x = xy[2 * k], y = xy[2 * k + 1];
    if (!(x >= g.x0 && x <= g.x0 + g.nx * g.dx && y >= g.y0 && y <= g.y0 + g.ny * g.dy))
      return fail(c, DG2_EINVAL, "gauge outside the domain");
    int i = (int)std::floor((x - g.x0) / g.dx), j = (int)std::floor((y - g.y0) / g.dy);
    i = i < 0 ? 0 : (i >= g.nx ? g.nx - 1 : i);
    j = j < 0 ? 0 : (j >= g.ny ? g.ny - 1 : j);
    cell[k] = j * g.nx + i;
    xi[k] = (x - (g.x0 + (i + 0.5) * g.dx)) / (0.5 * g.dx);
    ze[k] = (y - (g.y0 + (j + 0.5) * g.dy)) / (0.5 * g.dy);
    const size_t cc = cell[k];
    zp[k] = c->z0[cc] + xi[k] * c->z1x[cc] + ze[k] * c->z1y[cc];
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  void *old[] = {c->g_cell, c->g_xi, c->g_zeta, c->g_z, c->g_buf, c->g_t};
  for (void *b : old)
    if (b) (void)hipFree(b);
  c->g_cell = nullptr;
  c->g_xi = c->g_zeta = c->g_z = c->g_buf = nullptr;
  c->g_t = nullptr;
  c->ng = 0;
  c->gcap = 0;
  if (n > 0) {
    const int capv = cap > 0 ? cap : 65536;
    dg2_status s;
    if ((s = alloc(c, (void **)&c->g_cell, n * sizeof(int), "gauges")) != DG2_OK) return s;
    if ((s = alloc(c, &c->g_xi, n * c->esz, "gauges")) != DG2_OK) return s;
    if ((s = alloc(c, &c->g_zeta, n * c->esz, "gauges")) != DG2_OK) return s;
    if ((s = alloc(c, &c->g_z, n * c->esz, "gauges")) != DG2_OK) return s;
    if ((s = alloc(c, &c->g_buf, (size_t)capv * n * 4 * c->esz, "gauge record")) != DG2_OK) return s;
    if ((s = alloc(c, (void **)&c->g_t, (size_t)capv * sizeof(double), "gauge record")) != DG2_OK)
      return s;
    HIPCHK(c, hipMemcpy(c->g_cell, cell.data(), n * sizeof(int), hipMemcpyHostToDevice), "gauges");
    if ((s = upload(c, c->g_xi, xi.data(), n)) != DG2_OK) return s;
    if ((s = upload(c, c->g_zeta, ze.data(), n)) != DG2_OK) return s;
    if ((s = upload(c, c->g_z, zp.data(), n)) != DG2_OK) return s;
    c->ng = n;
    c->gcap = capv;
  }
  // restart the record
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) return s;
  const long long zero = 0;
  HIPCHK(c, hipMemcpyAsync(&c->ctrl->gauge_written, &zero, sizeof(zero), hipMemcpyHostToDevice,
                           c->stream), "gauges");
  HIPCHK(c, hipStreamSynchronize(c->stream), "gauges");
  c->g_read = 0;
  return DG2_OK;
}

dg2_status dg2_step(dg2_ctx *c, int32_t nsteps) {
  if (!c) return DG2_EINVAL;
  if (nsteps < 0) return fail(c, DG2_EINVAL, "nsteps must be >= 0");
  HIPCHK(c, queue_plan(c, kPlanOnly, std::numeric_limits<double>::infinity(), 1), "plan");
  for (int k = 0; k < nsteps; ++k) {
    dg2_status s = queue_step(c);
    if (s != DG2_OK) return s;
  }
  return DG2_OK;
}

dg2_status dg2_run_to(dg2_ctx *c, double T) {
  if (!c) return DG2_EINVAL;
  if (!std::isfinite(T)) return fail(c, DG2_EINVAL, "T must be finite");
  HIPCHK(c, queue_plan(c, kPlanOnly, T, 1), "plan");
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) return s;
  if ((s = latched(c)) != DG2_OK) return s;
  if (!(c->hctrl->t < T)) return DG2_OK;
  // queue chunks of steps; the chunk after the one that reaches T only holds
  // idle steps (dt = 0) that return at once.
  const int chunk = 32;
  long long guard = 0;
  hipEvent_t ev;
  HIPCHK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  Ctrl *snap = c->hctrl;
  dg2_status st = DG2_OK;
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      if ((st = queue_step(c)) != DG2_OK) break;
    }
    if (st != DG2_OK) break;
    hipError_t e = hipMemcpyAsync(snap, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipEventRecord(ev, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev);
    if (e != hipSuccess) {
      st = hipfail(c, e, "run_to");
      break;
    }
    if (snap->flags & kFlagNaN) {
      st = latched(c);
      break;
    }
    if (!(snap->t < T)) break;
    if (!(snap->dt > 0)) {
      st = fail(c, DG2_ENUMERIC, "time step collapsed to zero before reaching T");
      break;
    }
    guard += chunk;
    if (guard > (1ll << 31)) {
      st = fail(c, DG2_ESTATE, "run_to exceeded 2^31 steps");
      break;
    }
  }
  (void)hipEventDestroy(ev);
  return st;
}

dg2_status dg2_sync(dg2_ctx *c) {
  if (!c) return DG2_EINVAL;
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) return s;
  return latched(c);
}

dg2_status dg2_read_gauges(dg2_ctx *c, double *out, double *t, int32_t max_samples, int32_t *ns) {
  if (!c) return DG2_EINVAL;
  if (ns) *ns = 0;
  if (c->ng == 0) return fail(c, DG2_ESTATE, "no gauges set");
  if (max_samples < 0 || (max_samples > 0 && (!out || !t)))
    return fail(c, DG2_EINVAL, "need output buffers");
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) return s;
  const long long written = c->hctrl->gauge_written;
  long long avail = written - c->g_read;
  bool lost = false;
  if (avail > c->gcap) {
    c->g_read = written - c->gcap;
    avail = c->gcap;
    lost = true;
  }
  const long long take = avail < max_samples ? avail : max_samples;
  const int ng = c->ng;
  const size_t per = (size_t)ng * 4;
  std::vector<double> tmp(per);
  for (long long k = 0; k < take; ++k) {
    const long long slot = (c->g_read + k) % c->gcap;
    s = download(c, tmp.data(), (char *)c->g_buf + slot * per * c->esz, per);
    if (s != DG2_OK) return s;
    std::memcpy(out + k * per, tmp.data(), per * sizeof(double));
    HIPCHK(c, hipMemcpy(t + k, c->g_t + slot, sizeof(double), hipMemcpyDeviceToHost), "gauge t");
  }
  c->g_read += take;
  if (ns) *ns = (int32_t)take;
  if ((s = latched(c)) != DG2_OK) return s;
  if (lost) return fail(c, DG2_ESTATE, "gauge record overflowed; oldest samples lost");
  return DG2_OK;
}

dg2_status dg2_diagnostics(dg2_ctx *c, double *mass, double *energy, double *min_h) {
  if (!c) return DG2_EINVAL;
  hipError_t e = c->f32 ? launch_diag<float>(scen<float>(c), consts(c), c->diag_part, kDiagBlocks,
                                             c->diag_out, c->stream)
                        : launch_diag<double>(scen<double>(c), consts(c), c->diag_part, kDiagBlocks,
                                              c->diag_out, c->stream);
  HIPCHK(c, e, "diagnostics");
  double h[4];
  HIPCHK(c, hipMemcpyAsync(h, c->diag_out, sizeof(h), hipMemcpyDeviceToHost, c->stream), "diag");
  HIPCHK(c, hipStreamSynchronize(c->stream), "diag");
  const double area = c->cfg.dx * c->cfg.dy;
  if (mass) *mass = h[0] * area;
  if (energy) *energy = h[1] * 0.25 * area;
  if (min_h) *min_h = h[2];
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) return s;
  if (h[3] > 0) return fail(c, DG2_ENUMERIC, "NaN in the state");
  return latched(c);
}

dg2_status dg2_diagnostics_noalloc(const void *state, const void *bed, int32_t nx, int32_t ny,
                                   int64_t plane_stride, int32_t prec, double dx, double dy, double g,
                                   double tol_dry, double *out4, void *hip_stream) {
  if (!state || !bed || !out4) return fail(nullptr, DG2_EINVAL, "state, bed and out4 must not be NULL");
  if (prec != DG2_FP64 && prec != DG2_FP32) return fail(nullptr, DG2_EINVAL, "bad prec");
  const size_t esz = prec == DG2_FP32 ? 4 : 8;
  if (((uintptr_t)state | (uintptr_t)bed) % esz != 0 || (uintptr_t)out4 % 8 != 0)
    return fail(nullptr, DG2_EINVAL, "misaligned pointer");
  if (nx < 1 || ny < 1) return fail(nullptr, DG2_EINVAL, "nx and ny must be >= 1");
  if (plane_stride < (int64_t)nx * ny) return fail(nullptr, DG2_EINVAL, "plane_stride must be >= nx*ny");
  if (!(dx > 0) || !(dy > 0) || !(g > 0) || !(tol_dry > 0) || !std::isfinite(dx) || !std::isfinite(dy))
    return fail(nullptr, DG2_EINVAL, "dx, dy, g and tol_dry must be positive");
  double *records = nullptr;
  hipError_t e = scratch_records(&records);
  if (e != hipSuccess) return hipfail(nullptr, e, "scratch address");
  Consts k{};
  k.g = g;
  k.tol = tol_dry;
  const double area = dx * dy;
  const hipStream_t st = (hipStream_t)hip_stream;
  if (prec == DG2_FP32) {
    Scen<float> sc{};
    sc.U = (const float *)state;
    sc.z = (const float *)bed;
    sc.nx = nx;
    sc.ny = ny;
    sc.P = plane_stride;
    e = launch_diag<float>(sc, k, records, kScratchRecords, out4, st, area, 0.25 * area);
  } else {
    Scen<double> sc{};
    sc.U = (const double *)state;
    sc.z = (const double *)bed;
    sc.nx = nx;
    sc.ny = ny;
    sc.P = plane_stride;
    e = launch_diag<double>(sc, k, records, kScratchRecords, out4, st, area, 0.25 * area);
  }
  if (e != hipSuccess) return hipfail(nullptr, e, "diagnostics launch");
  return DG2_OK;
}

dg2_status dg2_time_kernels(dg2_ctx *c, int32_t nsteps, double *ms1, double *ms2, double *msstep) {
  if (!c) return DG2_EINVAL;
  if (nsteps < 1) return fail(c, DG2_EINVAL, "nsteps must be >= 1");
  HIPCHK(c, queue_plan(c, kPlanOnly, std::numeric_limits<double>::infinity(), 1), "plan");
  const bool fused = fused_active(c);  // one kernel per step: no stage-2 time
  std::vector<hipEvent_t> ev(3 * nsteps + 1);
  for (auto &e : ev) HIPCHK(c, hipEventCreate(&e), "event");
  dg2_status st = DG2_OK;
  for (int k = 0; k < nsteps && st == DG2_OK; ++k) st = queue_step(c, &ev[3 * k]);
  if (st == DG2_OK) {
    hipError_t e = hipEventRecord(ev[3 * nsteps], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[3 * nsteps]);
    if (e != hipSuccess) st = hipfail(c, e, "timing");
  }
  double a = 0, b = 0, w = 0;
  if (st == DG2_OK) {
    for (int k = 0; k < nsteps; ++k) {
      float t1 = 0, t2 = 0;
      (void)hipEventElapsedTime(&t1, ev[3 * k], ev[3 * k + 1]);
      if (!fused) (void)hipEventElapsedTime(&t2, ev[3 * k + 1], ev[3 * k + 2]);
      a += t1;
      b += t2;
    }
    float tw = 0;
    (void)hipEventElapsedTime(&tw, ev[0], ev[3 * nsteps]);
    w = tw;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (st != DG2_OK) return st;
  if (ms1) *ms1 = a / nsteps;
  if (ms2) *ms2 = b / nsteps;
  if (msstep) *msstep = w / nsteps;
  return dg2_sync(c);
}

dg2_status dg2_set_stage_check(dg2_ctx *c, int32_t repeats) {
  if (!c) return DG2_EINVAL;
  if (repeats < 0 || repeats > 8) return fail(c, DG2_EINVAL, "repeats must be 0..8");
  c->stage_check = repeats;
  return DG2_OK;
}

dg2_status dg2_set_partly_wet_flat(dg2_ctx *c, int32_t on) {
  if (!c) return DG2_EINVAL;
  if (on != 0 && on != 1) return fail(c, DG2_EINVAL, "on must be 0 or 1");
  c->partly_wet_flat = on;
  return DG2_OK;
}

dg2_status dg2_set_step_kernel(dg2_ctx *c, int32_t fused) {
  if (!c) return DG2_EINVAL;
  if (fused != 0 && fused != 1) return fail(c, DG2_EINVAL, "fused must be 0 or 1");
  c->fused_user = fused;
  return DG2_OK;
}

dg2_status dg2_set_launch(dg2_ctx *c, int32_t rows, int32_t wpb) {
  if (!c) return DG2_EINVAL;
  if (wpb != 1 && wpb != 2 && wpb != 4) return fail(c, DG2_EINVAL, "waves per block must be 1, 2 or 4");
  c->R_user = rows > 0 ? rows : 0;
  c->wpb_user = wpb;
  return DG2_OK;
}

dg2_status dg2_set_tune_cache(dg2_ctx *c, const char *path) {
  if (!c) return DG2_EINVAL;
  c->tune_path = path ? path : "";
  return DG2_OK;
}

dg2_status dg2_get_launch(const dg2_ctx *c, int32_t *rows, int32_t *waves, int32_t *from_cache) {
  if (!c) return DG2_EINVAL;
  const Launch L = launch_of(c);
  if (rows) *rows = L.R;
  if (waves) *waves = L.wpb;
  if (from_cache) *from_cache = c->tuned_from_cache;
  return DG2_OK;
}

dg2_status dg2_autotune(dg2_ctx *c, double budget_ms, int32_t *rows) {
  if (!c) return DG2_EINVAL;
  if (!(budget_ms > 0)) return fail(c, DG2_EINVAL, "budget must be > 0");
  c->tuned_from_cache = 0;
  const std::string key = tune_key(c);
  if (!c->tune_path.empty()) {
    const auto m = read_tune_cache(c->tune_path);
    const auto it = m.find(key);
    if (it != m.end() && it->second.rows >= 1 &&
        (it->second.waves == 1 || it->second.waves == 2 || it->second.waves == 4)) {
      c->R_user = it->second.rows;
      c->wpb_user = it->second.waves;
      c->tuned_from_cache = 1;
      if (rows) *rows = launch_of(c).R;
      return DG2_OK;
    }
  }
  const size_t bytes = 9 * (size_t)c->P * c->esz;
  void *save = nullptr;
  HIPCHK(c, hipMalloc(&save, bytes), "autotune");
  HIPCHK(c, hipMemcpyAsync(save, c->U, bytes, hipMemcpyDeviceToDevice, c->stream), "autotune");
  dg2_status s = read_ctrl(c);
  if (s != DG2_OK) {
    (void)hipFree(save);
    return s;
  }
  const Ctrl keep = *c->hctrl;
  const int keepR = c->R_user, keepW = c->wpb_user;
  // candidates: the built-in shape first, then rows per wavefront x
  // wavefronts per workgroup, while the time budget lasts
  std::vector<std::pair<int, int>> cand;
  c->R_user = 0;
  c->wpb_user = 4;
  cand.push_back({launch_of(c).R, 4});
  for (int W : {4, 2, 1})
    for (int R : {4, 8, 16, 24, 32, 48, 64, 96})
      if (R <= c->cfg.ny && !(R == cand[0].first && W == 4)) cand.push_back({R, W});
  double best = 1e300, spent = 0;
  int bestR = cand[0].first, bestW = 4;
  for (const auto &rw : cand) {
    c->R_user = rw.first;
    c->wpb_user = rw.second;
    double ms = 0;
    s = dg2_time_kernels(c, 3, nullptr, nullptr, &ms);
    HIPCHK(c, hipMemcpyAsync(c->U, save, bytes, hipMemcpyDeviceToDevice, c->stream), "autotune");
    *c->hctrl = keep;
    HIPCHK(c, hipMemcpyAsync(c->ctrl, c->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream), "autotune");
    HIPCHK(c, hipStreamSynchronize(c->stream), "autotune");
    if (s != DG2_OK) break;
    if (ms < best) {
      best = ms;
      bestR = rw.first;
      bestW = rw.second;
    }
    spent += 4 * ms;
    if (spent > budget_ms) break;
  }
  (void)hipFree(save);
  if (s != DG2_OK) {
    c->R_user = keepR;
    c->wpb_user = keepW;
    return s;
  }
  c->R_user = bestR;
  c->wpb_user = bestW;
  if (rows) *rows = bestR;
  if (!c->tune_path.empty()) {
    TuneEntry e;
    e.rows = bestR;
    e.waves = bestW;
    e.ms = best;
    if (!write_tune_cache(c->tune_path, key, e))
      return fail(c, DG2_EINVAL, "cannot write the tune cache " + c->tune_path);
  }
  return DG2_OK;
}

dg2_status dg2_state_layout(const dg2_ctx *c, size_t *bytes, size_t *stride) {
  if (!c) return DG2_EINVAL;
  if (bytes) *bytes = 9 * (size_t)c->P * c->esz;
  if (stride) *stride = (size_t)c->P;
  return DG2_OK;
}

dg2_status dg2_bind_device_state(dg2_ctx *c, void *ptr, size_t bytes) {
  if (!c) return DG2_EINVAL;
  const size_t need = 9 * (size_t)c->P * c->esz;
  void *target = ptr ? ptr : c->U_own;
  if (ptr && (bytes < need || ((uintptr_t)ptr & 255)))
    return fail(c, DG2_EINVAL, "device buffer too small or not 256-byte aligned");
  if (target != c->U)
    HIPCHK(c, hipMemcpyAsync(target, c->U, need, hipMemcpyDeviceToDevice, c->stream), "bind");
  HIPCHK(c, hipStreamSynchronize(c->stream), "bind");
  // the state now lives in target; the other library buffer is the stage buffer
  c->U = target;
  c->U1 = c->U1_own;
  return DG2_OK;
}

}  // extern "C"

// ===========================================================================
// Batched ensemble
// ===========================================================================

struct BatchItem {
  int sid, strip, seg, pad;
};

struct dg2_batch {
  std::vector<dg2_ctx *> m;
  std::string tune_path;  // dg2_batch_set_tune_cache (empty: none)
  int tuned_from_cache = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int f32 = 0, variant = 0;
  Consts consts{};
  void *d_scens = nullptr;
  BatchItem *d_items = nullptr;
  int nitems = 0, items_cap = 0;
  Ctrl **d_ctrls = nullptr;
  PlanArgs *d_plan = nullptr;
  unsigned *d_status = nullptr, *h_status = nullptr;
  int R = 0, R_user = 0, wpb = 4, graph_steps = 16;
  int blocks1 = 0, blocks2 = 0;
  std::vector<void *> seenU;  // members' state buffers as the batch last left them
  // fused step kernel: both RK stages per launch; each step writes every
  // member's next state into its other buffer, using scenario table `par`
  // (0: U -> U1, 1: U1 -> U as uploaded), and the host swaps the members'
  // buffers after queueing it.  Graphs hold an even number of steps and are
  // recaptured when they would start at the other parity.
  bool fused = false;
  int par = 0, graph_par = 0, blocksF = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_batch_error;

dg2_status bfail(dg2_batch *b, dg2_status s, const std::string &msg) {
  if (b)
    b->err = msg;
  else
    g_batch_error = msg;
  return s;
}

dg2_status bhip(dg2_batch *b, hipError_t e, const char *what) {
  return bfail(b, e == hipErrorOutOfMemory ? DG2_ENOMEM : DG2_EHIP,
               std::string(what) + ": " + hipGetErrorString(e));
}

#define BCHK(b, expr, what)                               \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return bhip(b, _e, what);       \
  } while (0)

void drop_graph(dg2_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

int batch_cols(const dg2_batch *b) {
  return b->fused ? kStripF : (b->variant == 1 ? kStripLL : kStripNL);
}

// Rows per wavefront: ~16k items over the whole batch (fused step: ~8.8k,
// since each item also computes two halo rows of stage 1), 4..32.
int batch_rows(const dg2_batch *b) {
  if (b->R_user > 0) return b->R_user;
  const int cols = batch_cols(b);
  long long lanes_rows = 0;
  for (auto *c : b->m) lanes_rows += (long long)((c->cfg.nx + cols - 1) / cols) * c->cfg.ny;
  long long r = lanes_rows / (b->fused ? 8800 : 16384);
  return (int)(r < 4 ? 4 : (r > 32 ? 32 : r));
}

dg2_status build_items(dg2_batch *b) {
  b->R = batch_rows(b);
  const int cols = batch_cols(b);
  std::vector<BatchItem> items;
  for (size_t k = 0; k < b->m.size(); ++k) {
    const dg2_config &g = b->m[k]->cfg;
    const int ns = (g.nx + cols - 1) / cols, ng = (g.ny + b->R - 1) / b->R;
    for (int sg = 0; sg < ng; ++sg)
      for (int st = 0; st < ns; ++st) items.push_back(BatchItem{(int)k, st, sg, 0});
  }
  if ((int)items.size() > b->items_cap) {
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    BCHK(b, hipMalloc((void **)&b->d_items, items.size() * sizeof(BatchItem)), "batch items");
    b->items_cap = (int)items.size();
  }
  BCHK(b, hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice),
       "batch items");
  b->nitems = (int)items.size();
  drop_graph(b);
  return DG2_OK;
}

template <typename real>
dg2_status upload_scens(dg2_batch *b) {
  std::vector<Scen<real>> sc;
  std::vector<PlanArgs> pa;
  std::vector<Ctrl *> ctrls;
  for (auto *c : b->m) {
    Scen<real> s = scen<real>(c);
    if (b->fused) s.Uout = (real *)c->U1;
    sc.push_back(s);
    pa.push_back(plan_args(c));
    ctrls.push_back(c->ctrl);
  }
  if (b->fused) {
    // table 1: the buffers the other way round
    for (auto *c : b->m) {
      Scen<real> s = scen<real>(c);
      s.U = (const real *)c->U1;
      s.U1 = (real *)c->U;
      s.Uout = (real *)c->U;
      sc.push_back(s);
    }
  }
  const size_t n = b->m.size();
  b->seenU.clear();
  for (auto *c : b->m) b->seenU.push_back(c->U);
  b->par = 0;
  BCHK(b, hipMemcpy(b->d_scens, sc.data(), sc.size() * sizeof(Scen<real>), hipMemcpyHostToDevice),
       "scenarios");
  BCHK(b, hipMemcpy(b->d_plan, pa.data(), n * sizeof(PlanArgs), hipMemcpyHostToDevice), "plans");
  BCHK(b, hipMemcpy(b->d_ctrls, ctrls.data(), n * sizeof(Ctrl *), hipMemcpyHostToDevice), "ctrls");
  return DG2_OK;
}

hipError_t batch_stage(dg2_batch *b, int stage) {
  const int blocks = stage == 1 ? b->blocks1 : b->blocks2;
  if (b->f32)
    return launch_batch_stage<float>(stage, b->variant, (const Scen<float> *)b->d_scens, b->d_items,
                                     b->nitems, b->consts, b->R, b->wpb, blocks, b->stream);
  return launch_batch_stage<double>(stage, b->variant, (const Scen<double> *)b->d_scens, b->d_items,
                                    b->nitems, b->consts, b->R, b->wpb, blocks, b->stream);
}

hipError_t batch_plan(dg2_batch *b, int mode, double t_end = 0.0, int set_tend = 0) {
  return launch_plan_batch(b->d_ctrls, b->d_plan, (int)b->m.size(), mode, t_end, set_tend, b->stream);
}

dg2_status batch_queue_step(dg2_batch *b) {
  if (b->fused) {
    // the scenario table holds Scen<real> of the batch's precision
    const size_t at = (size_t)b->par * b->m.size();
    const hipError_t e =
        b->f32 ? launch_batch_fused<float>((const Scen<float> *)b->d_scens + at, b->d_items, b->nitems,
                                           b->consts, b->R, b->wpb, b->blocksF, b->stream)
               : launch_batch_fused<double>((const Scen<double> *)b->d_scens + at, b->d_items, b->nitems,
                                            b->consts, b->R, b->wpb, b->blocksF, b->stream);
    BCHK(b, e, "batch step");
    BCHK(b, batch_plan(b, kPlanFinishStep), "batch plan");
    b->par ^= 1;
    for (size_t k = 0; k < b->m.size(); ++k) {
      std::swap(b->m[k]->U, b->m[k]->U1);
      b->seenU[k] = b->m[k]->U;
    }
    return DG2_OK;
  }
  BCHK(b, batch_stage(b, 1), "batch stage 1");
  BCHK(b, batch_stage(b, 2), "batch stage 2");
  BCHK(b, batch_plan(b, kPlanFinishStep), "batch plan");
  return DG2_OK;
}

dg2_status ensure_graph(dg2_batch *b) {
  if (b->gexec && b->fused && b->graph_par != b->par) drop_graph(b);
  if (b->gexec || b->graph_steps <= 1) return DG2_OK;
  b->graph_par = b->par;
  BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "graph capture");
  dg2_status st = DG2_OK;
  for (int k = 0; k < b->graph_steps && st == DG2_OK; ++k) st = batch_queue_step(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (st != DG2_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return bhip(b, e, "graph capture");
  b->graph = g;
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return bhip(b, e, "graph instantiate");
  }
  return DG2_OK;
}

// Queue n steps: whole graphs, then the remainder as eager launches.
dg2_status batch_setup(dg2_batch *b);

dg2_status batch_queue_steps(dg2_batch *b, int n) {
  // a member stepped alone with the fused step kernel has its state in its
  // other buffer now: upload the scenarios again
  bool moved = false;
  for (size_t k = 0; k < b->m.size(); ++k) moved = moved || b->m[k]->U != b->seenU[k];
  if (moved) {
    for (auto *c : b->m) BCHK(b, hipStreamSynchronize(c->stream), "member sync");
    dg2_status su = batch_setup(b);
    if (su != DG2_OK) return su;
  }
  dg2_status st = ensure_graph(b);
  if (st != DG2_OK) return st;
  int done = 0;
  if (b->gexec) {
    for (; done + b->graph_steps <= n; done += b->graph_steps)
      BCHK(b, hipGraphLaunch(b->gexec, b->stream), "graph launch");
  }
  for (; done < n; ++done)
    if ((st = batch_queue_step(b)) != DG2_OK) return st;
  return DG2_OK;
}

dg2_status batch_status(dg2_batch *b, unsigned *active, unsigned *flags) {
  BCHK(b, launch_batch_status(b->d_ctrls, (int)b->m.size(), b->d_status, b->stream), "status");
  BCHK(b, hipMemcpyAsync(b->h_status, b->d_status, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, b->stream),
       "status");
  BCHK(b, hipStreamSynchronize(b->stream), "status");
  *active = b->h_status[0];
  *flags = b->h_status[1];
  return DG2_OK;
}

dg2_status batch_setup(dg2_batch *b) {
  for (auto *c : b->m)
    if (c->stage_check > 0)
      return bfail(b, DG2_EINVAL, "the stage-1 Courant check is not available in batches");
  b->fused = true;
  for (auto *c : b->m) b->fused = b->fused && fused_active(c);
  if (b->fused && b->graph_steps > 1 && (b->graph_steps & 1)) b->graph_steps += 1;
  dg2_status st = b->f32 ? upload_scens<float>(b) : upload_scens<double>(b);
  if (st != DG2_OK) return st;
  if ((st = build_items(b)) != DG2_OK) return st;
  const int fx = b->consts.flux;
  if (b->fused) {
    b->blocksF = b->f32 ? batch_fused_blocks<float>(fx, b->wpb) : batch_fused_blocks<double>(fx, b->wpb);
    const int need = (b->nitems + b->wpb - 1) / b->wpb;
    if (b->blocksF > need) b->blocksF = need;
    if (b->blocksF < 1) b->blocksF = 1;
  }
  b->blocks1 = b->f32 ? batch_blocks<float>(1, b->variant, fx, b->wpb)
                      : batch_blocks<double>(1, b->variant, fx, b->wpb);
  b->blocks2 = b->f32 ? batch_blocks<float>(2, b->variant, fx, b->wpb)
                      : batch_blocks<double>(2, b->variant, fx, b->wpb);
  const int need = (b->nitems + b->wpb - 1) / b->wpb;
  if (b->blocks1 > need) b->blocks1 = need;
  if (b->blocks2 > need) b->blocks2 = need;
  if (b->blocks1 < 1) b->blocks1 = 1;
  if (b->blocks2 < 1) b->blocks2 = 1;
  return DG2_OK;
}

}  // namespace

extern "C" {

const char *dg2_batch_last_error(const dg2_batch *b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

void dg2_batch_destroy(dg2_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  void *bufs[] = {b->d_scens, b->d_items, b->d_ctrls, b->d_plan, b->d_status};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  if (b->h_status) (void)hipHostFree(b->h_status);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

dg2_status dg2_batch_create(dg2_ctx *const *members, int32_t n, void *hip_stream, dg2_batch **out) {
  if (!out) return bfail(nullptr, DG2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!members || n < 1) return bfail(nullptr, DG2_EINVAL, "need n >= 1 members");
  const dg2_ctx *c0 = members[0];
  for (int k = 0; k < n; ++k) {
    const dg2_ctx *c = members[k];
    if (!c) return bfail(nullptr, DG2_EINVAL, "NULL member");
    if (c->cfg.prec != c0->cfg.prec || c->cfg.variant != c0->cfg.variant ||
        c->cfg.flux != c0->cfg.flux || c->cfg.g != c0->cfg.g ||
        c->cfg.tol_dry != c0->cfg.tol_dry || c->cfg.ll_threshold != c0->cfg.ll_threshold ||
        c->partly_wet_flat != c0->partly_wet_flat)
      return bfail(nullptr, DG2_EINVAL,
                   "members differ in precision, variant, flux, g, tol_dry, threshold or partly-wet rule");
  }
  dg2_batch *b = new (std::nothrow) dg2_batch();
  if (!b) return bfail(nullptr, DG2_ENOMEM, "host allocation failed");
  auto bail = [&](dg2_status s) {
    g_batch_error = b->err;
    dg2_batch_destroy(b);
    return s;
  };
  b->m.assign(members, members + n);
  b->f32 = c0->f32;
  b->variant = c0->cfg.variant;
  b->consts = consts(c0);
  hipError_t e;
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(bhip(b, e, "stream"));
    b->own_stream = true;
  }
  for (auto *c : b->m) {
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(bhip(b, e, "member sync"));
  }
  const size_t ssz = b->f32 ? sizeof(Scen<float>) : sizeof(Scen<double>);
  if ((e = hipMalloc(&b->d_scens, 2 * n * ssz)) != hipSuccess) return bail(bhip(b, e, "scenarios"));
  if ((e = hipMalloc((void **)&b->d_ctrls, n * sizeof(Ctrl *))) != hipSuccess) return bail(bhip(b, e, "ctrls"));
  if ((e = hipMalloc((void **)&b->d_plan, n * sizeof(PlanArgs))) != hipSuccess) return bail(bhip(b, e, "plans"));
  if ((e = hipMalloc((void **)&b->d_status, 2 * sizeof(unsigned))) != hipSuccess) return bail(bhip(b, e, "status"));
  if ((e = hipHostMalloc((void **)&b->h_status, 2 * sizeof(unsigned), hipHostMallocDefault)) != hipSuccess)
    return bail(bhip(b, e, "status"));
  dg2_status st = batch_setup(b);
  if (st != DG2_OK) return bail(st);
  *out = b;
  return DG2_OK;
}

dg2_status dg2_batch_refresh(dg2_batch *b) {
  if (!b) return DG2_EINVAL;
  BCHK(b, hipStreamSynchronize(b->stream), "sync");
  for (auto *c : b->m) BCHK(b, hipStreamSynchronize(c->stream), "member sync");
  return batch_setup(b);
}

dg2_status dg2_batch_set_launch(dg2_batch *b, int32_t rows, int32_t wpb, int32_t graph_steps) {
  if (!b) return DG2_EINVAL;
  if (wpb != 1 && wpb != 2 && wpb != 4) return bfail(b, DG2_EINVAL, "waves per block must be 1, 2 or 4");
  BCHK(b, hipStreamSynchronize(b->stream), "sync");
  b->R_user = rows > 0 ? rows : 0;
  b->wpb = wpb;
  b->graph_steps = graph_steps > 1 ? graph_steps : 1;
  return batch_setup(b);
}

dg2_status dg2_batch_step(dg2_batch *b, int32_t nsteps) {
  if (!b) return DG2_EINVAL;
  if (nsteps < 0) return bfail(b, DG2_EINVAL, "nsteps must be >= 0");
  BCHK(b, batch_plan(b, kPlanOnly, std::numeric_limits<double>::infinity(), 1), "plan");
  return batch_queue_steps(b, nsteps);
}

dg2_status dg2_batch_sync(dg2_batch *b) {
  if (!b) return DG2_EINVAL;
  unsigned active = 0, flags = 0;
  dg2_status st = batch_status(b, &active, &flags);
  if (st != DG2_OK) return st;
  if (flags & kFlagNaN) return bfail(b, DG2_ENUMERIC, "NaN in a member's state");
  return DG2_OK;
}

dg2_status dg2_batch_run_to(dg2_batch *b, double T) {
  if (!b) return DG2_EINVAL;
  if (!std::isfinite(T)) return bfail(b, DG2_EINVAL, "T must be finite");
  BCHK(b, batch_plan(b, kPlanOnly, T, 1), "plan");
  const int chunk = b->graph_steps > 1 ? b->graph_steps : 32;
  for (long long guard = 0;; guard += chunk) {
    unsigned active = 0, flags = 0;
    dg2_status st = batch_status(b, &active, &flags);
    if (st != DG2_OK) return st;
    if (flags & kFlagNaN) return bfail(b, DG2_ENUMERIC, "NaN in a member's state");
    if (active == 0) break;
    if (guard > (1ll << 31)) return bfail(b, DG2_ESTATE, "run_to exceeded 2^31 steps");
    if ((st = batch_queue_steps(b, chunk)) != DG2_OK) return st;
  }
  // a member whose step collapsed to zero before T is a numerical failure
  for (auto *c : b->m) {
    Ctrl h;
    BCHK(b, hipMemcpy(&h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost), "ctrl");
    if (h.t < T) return bfail(b, DG2_ENUMERIC, "a member's time step collapsed before T");
  }
  return DG2_OK;
}

dg2_status dg2_batch_time_steps(dg2_batch *b, int32_t nsteps, double *ms) {
  if (!b) return DG2_EINVAL;
  if (nsteps < 1) return bfail(b, DG2_EINVAL, "nsteps must be >= 1");
  BCHK(b, batch_plan(b, kPlanOnly, std::numeric_limits<double>::infinity(), 1), "plan");
  dg2_status st = ensure_graph(b);
  if (st != DG2_OK) return st;
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0), "event");
  BCHK(b, hipEventCreate(&e1), "event");
  hipError_t e = hipEventRecord(e0, b->stream);
  if (e == hipSuccess) st = batch_queue_steps(b, nsteps);
  if (e == hipSuccess && st == DG2_OK) e = hipEventRecord(e1, b->stream);
  if (e == hipSuccess && st == DG2_OK) e = hipEventSynchronize(e1);
  float t = 0;
  if (e == hipSuccess && st == DG2_OK) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DG2_OK) return st;
  if (e != hipSuccess) return bhip(b, e, "timing");
  if (ms) *ms = t / nsteps;
  return dg2_batch_sync(b);
}

dg2_status dg2_batch_set_tune_cache(dg2_batch *b, const char *path) {
  if (!b) return DG2_EINVAL;
  b->tune_path = path ? path : "";
  return DG2_OK;
}

dg2_status dg2_batch_get_launch(const dg2_batch *b, int32_t *rows, int32_t *waves, int32_t *graph_steps,
                                int32_t *from_cache) {
  if (!b) return DG2_EINVAL;
  if (rows) *rows = batch_rows(b);
  if (waves) *waves = b->wpb;
  if (graph_steps) *graph_steps = b->graph_steps;
  if (from_cache) *from_cache = b->tuned_from_cache;
  return DG2_OK;
}

dg2_status dg2_batch_autotune(dg2_batch *b, double budget_ms, int32_t *rows) {
  if (!b) return DG2_EINVAL;
  if (!(budget_ms > 0)) return bfail(b, DG2_EINVAL, "budget must be > 0");
  BCHK(b, hipStreamSynchronize(b->stream), "sync");
  b->tuned_from_cache = 0;
  long long cells = 0;
  for (auto *c : b->m) cells += c->ncell;
  const dg2_ctx *c0 = b->m[0];
  char kb[256];
  std::snprintf(kb, sizeof(kb), "%s|batch|%s|%s|%s|%s|%zu members|%lld cells", device_arch().c_str(),
                b->f32 ? "fp32" : "fp64", b->variant == DG2_LL ? "LL" : "NL",
                c0->cfg.flux == DG2_FLUX_ROE ? "ROE" : "HLL", b->fused ? "fused" : "stages", b->m.size(),
                size_class(cells));
  const std::string key = kb;
  if (!b->tune_path.empty()) {
    const auto m = read_tune_cache(b->tune_path);
    const auto it = m.find(key);
    if (it != m.end() && it->second.rows >= 1 && it->second.graph_steps >= 1 &&
        (it->second.waves == 1 || it->second.waves == 2 || it->second.waves == 4)) {
      b->R_user = it->second.rows;
      b->wpb = it->second.waves;
      b->graph_steps = it->second.graph_steps;
      b->tuned_from_cache = 1;
      dg2_status st = batch_setup(b);
      if (rows) *rows = batch_rows(b);
      return st;
    }
  }
  // save every member's state and control block
  size_t total = 0;
  for (auto *c : b->m) total += 9 * (size_t)c->P * c->esz;
  void *save = nullptr;
  BCHK(b, hipMalloc(&save, total + b->m.size() * sizeof(Ctrl)), "autotune scratch");
  auto copy_all = [&](bool to_save) -> hipError_t {
    size_t off = 0;
    for (auto *c : b->m) {
      const size_t bytes = 9 * (size_t)c->P * c->esz;
      char *sv = (char *)save + off;
      hipError_t e = to_save ? hipMemcpyAsync(sv, c->U, bytes, hipMemcpyDeviceToDevice, b->stream)
                             : hipMemcpyAsync(c->U, sv, bytes, hipMemcpyDeviceToDevice, b->stream);
      if (e != hipSuccess) return e;
      off += bytes;
    }
    for (size_t k = 0; k < b->m.size(); ++k) {
      char *sv = (char *)save + total + k * sizeof(Ctrl);
      hipError_t e = to_save ? hipMemcpyAsync(sv, b->m[k]->ctrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, b->stream)
                             : hipMemcpyAsync(b->m[k]->ctrl, sv, sizeof(Ctrl), hipMemcpyDeviceToDevice, b->stream);
      if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(b->stream);
  };
  hipError_t e = copy_all(true);
  if (e != hipSuccess) {
    (void)hipFree(save);
    return bhip(b, e, "autotune save");
  }
  const int keepR = b->R_user, keepW = b->wpb, keepG = b->graph_steps;
  double best = 1e300, spent = 0;
  int bestR = batch_rows(b), bestW = b->wpb, bestG = b->graph_steps;
  dg2_status st = DG2_OK;
  // time one candidate over two graph replays, then restore the members
  auto trial = [&](int R, int W, int G) -> dg2_status {
    b->R_user = R;
    b->wpb = W;
    b->graph_steps = G;
    dg2_status s2 = batch_setup(b);
    if (s2 != DG2_OK) return s2;
    double ms = 0;
    s2 = dg2_batch_time_steps(b, 2 * G, &ms);
    e = copy_all(false);
    if (s2 != DG2_OK) return s2;
    if (e != hipSuccess) return bhip(b, e, "autotune restore");
    if (ms < best) {
      best = ms;
      bestR = R;
      bestW = W;
      bestG = G;
    }
    spent += (2 * G + 1) * ms;
    return DG2_OK;
  };
  // rows per wavefront x wavefronts per workgroup at the current graph
  // length, then the graph length at the best shape, while the budget lasts
  for (int W : {4, 2, 1}) {
    for (int R : {4, 8, 12, 16, 24, 32}) {
      if (spent > budget_ms || st != DG2_OK) break;
      st = trial(R, W, keepG);
    }
  }
  const int R1 = bestR, W1 = bestW;
  for (int G : {8, 16, 32}) {
    if (spent > budget_ms || st != DG2_OK) break;
    if (G != keepG) st = trial(R1, W1, G);
  }
  (void)hipFree(save);
  if (st != DG2_OK) {
    b->R_user = keepR;
    b->wpb = keepW;
    b->graph_steps = keepG;
    (void)batch_setup(b);
    return st;
  }
  b->R_user = bestR;
  b->wpb = bestW;
  b->graph_steps = bestG;
  st = batch_setup(b);
  if (st != DG2_OK) return st;
  if (rows) *rows = bestR;
  if (!b->tune_path.empty()) {
    TuneEntry te;
    te.rows = bestR;
    te.waves = bestW;
    te.graph_steps = bestG;
    te.ms = best;
    if (!write_tune_cache(b->tune_path, key, te))
      return bfail(b, DG2_EINVAL, "cannot write the tune cache " + b->tune_path);
  }
  return DG2_OK;
}

}  // extern "C"
