// Internal: the context object behind the C-ABI handle dg2_ctx and the
// per-context kernel arguments derived from it.  Shared by the runtime
// translation units; not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dg2.h"
#include "dg2_internal.h"

struct dg2_ctx {
  dg2_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int f32 = 0;
  size_t esz = 8;
  long long P = 0;  // plane stride (elements)
  long long ncell = 0;
  // U: the state, U1: the stage buffer (stage-kernel path) or the next state
  // (fused path, after which the two are swapped).  U_own and U1_own are the
  // library's two allocations behind them; U may instead be a caller's buffer
  // (dg2_bind_device_state), and then U1 is U1_own.
  void *U = nullptr, *U1 = nullptr, *W1 = nullptr, *z = nullptr, *n = nullptr;
  void *U_own = nullptr, *U1_own = nullptr;
  int fused_user = 1;  // dg2_set_step_kernel
  // stage-1 Courant check (dg2_set_stage_check): repeats allowed per step and
  // the repeat block (a Ctrl whose step the repeat stage-1 launches read)
  int stage_check = 0;
  dg2::Ctrl *ctrl2 = nullptr;
  // partly-wet rule (dg2_set_partly_wet_flat): 0 off (the paper's treatment)
  int partly_wet_flat = 0;
  bool has_ncell = false;
  double n_uniform = 0.0;
  dg2::Ctrl *ctrl = nullptr;
  dg2::Ctrl *hctrl = nullptr;  // pinned mirror
  // host copies used by setup
  std::vector<double> zc;  // corners
  std::vector<double> z0, z1x, z1y;
  // boundaries and hydrographs
  int seg_first[4] = {1, 1, 1, 1}, seg_last[4] = {0, 0, 0, 0};
  int bkind[4] = {0, 0, 0, 0};     // dg2_bc of each side's segment
  int hyd_kind[4] = {0, 0, 0, 0};  // what the side's table holds: DG2_BC_INFLOW_Q or DG2_BC_LEVEL
  double *hyd_t[4] = {nullptr, nullptr, nullptr, nullptr};
  double *hyd_Q[4] = {nullptr, nullptr, nullptr, nullptr};
  int nhyd[4] = {0, 0, 0, 0};
  double rain_rate = 0.0, rain_tb = 0.0, rain_te = 0.0;
  double fixed_dt = 0.0;
  // gauges
  int ng = 0, gcap = 0;
  int *g_cell = nullptr;
  void *g_xi = nullptr, *g_zeta = nullptr, *g_z = nullptr, *g_buf = nullptr;
  double *g_t = nullptr;
  long long g_read = 0;
  // diagnostics scratch
  double *diag_part = nullptr, *diag_out = nullptr;
  // launch shape
  int R_user = 0, wpb_user = 4;
  // autotuner cache file (dg2_set_tune_cache; empty: none) and whether the
  // current launch shape came from it
  std::string tune_path;
  int tuned_from_cache = 0;
  std::string err;
};

namespace dg2 {

// A side's hydrograph table drives its segment (inflow or level).
inline bool side_table_on(const dg2_ctx *c, int s) {
  return (c->bkind[s] == DG2_BC_INFLOW_Q || c->bkind[s] == DG2_BC_LEVEL) && c->nhyd[s] > 0 &&
         c->hyd_kind[s] == c->bkind[s];
}
// A side's segment is not a plain wall.
inline bool side_active(const dg2_ctx *c, int s) { return side_table_on(c, s) || c->bkind[s] == DG2_BC_OPEN; }

constexpr int kDiagBlocks = 1024;  // partial sums of the diagnostics reduction

inline char *plane(void *base, const dg2_ctx *c, int k) { return (char *)base + (size_t)k * c->P * c->esz; }

inline PlanArgs plan_args(const dg2_ctx *c) {
  PlanArgs p{};
  p.cfl = c->cfg.cfl;
  p.dt_max = c->cfg.dt_max;
  p.fixed_dt = c->fixed_dt;
  p.rain_rate = c->rain_rate;
  p.rain_tb = c->rain_tb;
  p.rain_te = c->rain_te;
  for (int s = 0; s < 4; ++s) {
    const bool on = side_table_on(c, s);
    p.nhyd[s] = on ? c->nhyd[s] : 0;
    p.hyd_t[s] = c->hyd_t[s];
    p.hyd_Q[s] = c->hyd_Q[s];
    const double d = (s == DG2_WEST || s == DG2_EAST) ? c->cfg.dy : c->cfg.dx;
    // inflow tables give Q, turned into a unit discharge; level tables give eta
    p.seg_len[s] = on && c->bkind[s] == DG2_BC_INFLOW_Q ? (c->seg_last[s] - c->seg_first[s] + 1) * d : 1.0;
  }
  p.ng = c->ng;
  p.gauge_cap = c->gcap > 0 ? c->gcap : 1;
  p.gauge_t = c->g_t;
  return p;
}

template <typename real>
inline Scen<real> scen(const dg2_ctx *c) {
  Scen<real> s{};
  s.U = (const real *)c->U;
  s.U1 = (real *)c->U1;
  s.W1 = (real *)c->W1;
  s.Uout = (real *)c->U;
  s.mask = nullptr;
  s.z = (const real *)c->z;
  s.n = c->has_ncell ? (const real *)c->n : nullptr;
  s.n_uniform = (real)c->n_uniform;
  s.ctrl = c->ctrl;
  s.nx = c->cfg.nx;
  s.ny = c->cfg.ny;
  s.P = c->P;
  s.dx = (real)c->cfg.dx;
  s.dy = (real)c->cfg.dy;
  s.idx = (real)(1.0 / c->cfg.dx);
  s.idy = (real)(1.0 / c->cfg.dy);
  for (int k = 0; k < 4; ++k) {
    const bool on = side_active(c, k);
    s.bkind[k] = on ? c->bkind[k] : (int)DG2_BC_WALL;
    s.seg_first[k] = on ? c->seg_first[k] : 1;
    s.seg_last[k] = on ? c->seg_last[k] : 0;
  }
  s.ng = c->ng;
  s.g_cell = c->g_cell;
  s.g_xi = (const real *)c->g_xi;
  s.g_zeta = (const real *)c->g_zeta;
  s.g_z = (const real *)c->g_z;
  s.g_buf = (real *)c->g_buf;
  s.g_cap = c->gcap > 0 ? c->gcap : 1;
  return s;
}

inline Consts consts(const dg2_ctx *c) {
  Consts k;
  k.g = c->cfg.g;
  k.tol = c->cfg.tol_dry;
  k.theta = c->cfg.ll_threshold;
  k.flux = c->cfg.flux;
  k.flat = c->partly_wet_flat;
  return k;
}

// Both RK stages in one kernel: DG2-NL with the state in library memory.
// FP32 runs three wavefronts per SIMD (168 VGPRs); FP64 one, whose 256 VGPRs
// and the accumulation registers hold the march without scratch.
inline bool fused_active(const dg2_ctx *c) {
  return c->fused_user && c->cfg.variant == DG2_NL &&
         (c->U == c->U_own || c->U == c->U1_own);
}

// Launch of the per-stage kernels, of the fused step kernel, and of whichever
// dg2_step uses.
inline Launch stage_launch_of(const dg2_ctx *c) {
  return make_launch(c->cfg.nx, c->cfg.ny, c->cfg.variant == DG2_LL ? kStripLL : kStripNL,
                     c->R_user, c->wpb_user, 34000);
}
// The fused kernel computes two halo rows of stage 1 per work item, so it
// takes longer items (about three rounds of its ~3k resident wavefronts).
// The fused kernel's built-in rows per wavefront: 48 at 4096^2 (about 5 900
// wavefronts); with the edge tiles' own marches, 48 rows ran 0.6 % faster
// than 32 and 24.
inline Launch fused_launch_of(const dg2_ctx *c) {
  return make_launch(c->cfg.nx, c->cfg.ny, kStripF, c->R_user, c->wpb_user, 5800, 48);
}
inline Launch launch_of(const dg2_ctx *c) {
  return fused_active(c) ? fused_launch_of(c) : stage_launch_of(c);
}

}  // namespace dg2
