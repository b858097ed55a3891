// Internal interface between the C-ABI runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "dg2_device.h"

namespace dg2 {

// Geometry and per-context constants of one scenario, as the stage kernels
// see it.  All device pointers index planes of ``P`` elements.
template <typename real>
struct Scen {
  const real *U;    // 9 planes: state at the start of the step
  real *U1;         // 9 planes: stage-1 result
  real *W1;         // 9 planes: limited stage-1 input (DG2-LL only)
  real *Uout;       // 9 planes: stage-2 result (== U: in place)
  unsigned char *mask;  // wet/dry code of each stage result (DG2-NL), or nullptr
  const real *z;    // 3 planes: z0, z1x, z1y
  const real *n;    // per-cell Manning or nullptr
  real n_uniform;
  Ctrl *ctrl;
  int nx, ny;
  long long P;
  real dx, dy, idx, idy;
  int bkind[4];                   // boundary kind of each side's segment (dg2_bc)
  int seg_first[4], seg_last[4];  // that segment (first > last: none)
  // gauges
  int ng;
  const int *g_cell;
  const real *g_xi, *g_zeta, *g_z;
  real *g_buf;
  int g_cap;
};

struct Consts {
  double g, tol, theta;
  int flux;  // kFluxHLL or kFluxRoe
  int flat;  // partly-wet elements drop their slope modes (an option; 0: off)
};

struct Launch {
  int R;        // rows per wavefront
  int wpb;      // wavefronts per workgroup
  int nstrips;  // ceil(nx / cols-per-strip)
  int nitems;   // nstrips * ceil(ny / R)
};

constexpr int kStripNL = 62;  // output columns per wavefront (halo 1)
constexpr int kStripLL = 60;  // output columns per wavefront (halo 2)
constexpr int kStripF = 60;   // fused NL step: output columns per wavefront (halo 2)

// Work items of a launch over strips of `cols` output columns; R <= 0 picks
// the built-in rows per wavefront, aiming at about `items` work items, with
// 4 <= R <= rmax.
Launch make_launch(int nx, int ny, int cols, int R, int wpb, int items, int rmax = 32);

template <typename real>
hipError_t launch_stage(int stage, int variant, const Scen<real> &s, const Consts &c,
                        const Launch &L, hipStream_t st);

// Both RK stages of a DG2-NL step in one launch; writes s.Uout,
// which must not alias s.U.
template <typename real>
hipError_t launch_fused(const Scen<real> &s, const Consts &c, const Launch &L, hipStream_t st,
                        bool check = false);

// Stage-1 Courant check with the fused kernel: begin (copy the pending step
// into the staging block and arm it) or check a trial (last: accept it).
hipError_t launch_fused_check(Ctrl *ctrl, Ctrl *rep, const PlanArgs &p, int begin, int last,
                              hipStream_t st);

hipError_t launch_plan(Ctrl *ctrl, const PlanArgs &p, int mode, double t_end, int set_tend,
                       hipStream_t st);

// Courant minimum of s.U into *bits (default: s.ctrl->minbits); skipped when
// gate is given and its step is idle.
template <typename real>
hipError_t launch_cfl(const Scen<real> &s, const Consts &c, hipStream_t st,
                      const Ctrl *gate = nullptr, unsigned long long *bits = nullptr);

// Stage-1 Courant check after stage 1 (first) or one of its repeats (last:
// no repeat follows); rep is the repeat block.
hipError_t launch_stage_check(Ctrl *ctrl, Ctrl *rep, const PlanArgs &p, int first, int last,
                              hipStream_t st);

// Mass, energy and minimum depth sums of s.U into out4 (4 doubles, mass
// scaled by sm and energy by se), via nblocks per-block records in partials.
template <typename real>
hipError_t launch_diag(const Scen<real> &s, const Consts &c, double *partials, int nblocks,
                       double *out4, hipStream_t st, double sm = 1.0, double se = 1.0);

// Records (4 doubles each) of the allocation-free diagnostics' scratch.
constexpr int kScratchRecords = 1024;
// Device address of that scratch on the current device (looked up once per
// device with hipGetSymbolAddress).
hipError_t scratch_records(double **ptr);

// Batched ensemble: items are (scenario, strip, segment, pad) int quadruples.
template <typename real>
hipError_t launch_batch_stage(int stage, int variant, const Scen<real> *scens, const void *items,
                              int nitems, const Consts &c, int R, int wpb, int blocks,
                              hipStream_t st);

hipError_t launch_plan_batch(Ctrl *const *ctrls, const PlanArgs *pa, int n, int mode, double t_end,
                             int set_tend, hipStream_t st);

hipError_t launch_batch_status(Ctrl *const *ctrls, int n, unsigned *out, hipStream_t st);

template <typename real>
int batch_blocks(int stage, int variant, int flux, int wpb);

// Fused step of a batch of DG2-NL scenarios of one precision (one launch
// per step); each table entry's Uout must not alias its U.
template <typename real>
hipError_t launch_batch_fused(const Scen<real> *scens, const void *items, int nitems, const Consts &c,
                              int R, int wpb, int blocks, hipStream_t st);
template <typename real>
int batch_fused_blocks(int flux, int wpb);

enum PlanMode { kPlanOnly = 0, kPlanFromMin = 1, kPlanFinishStep = 2 };

}  // namespace dg2
