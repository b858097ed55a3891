"""Benchmark of the DG2 time step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload urban|urban_fp64|urban_ll|floodplain|dambreak]

Also reported: a batched-ensemble leg (256 uneven FP32 scenarios advanced
together against the plain solver stepping them one by one) and an adjoint
leg (gradient of a gauge misfit on a 512 x 512 FP64 domain, 2000 steps,
against the plain forward run of those steps).

Default workload: the urban-like domain, 4096 x 4096 cells, dx = 0.5 m, from
dry under 50 mm/h rain, Manning 0.02 on streets and 0.05 elsewhere, FP32,
DG2-NL, 2000 steps: the configuration whose working set (>1 GB) exceeds the
256 MB Infinity Cache, so that its bandwidth is HBM bandwidth.

One step is one DG2 time step (two RK stages plus the device-side step
planner).  The workload is first advanced, untimed and with the per-stage
kernels, to a simulated time of --spinup-s seconds (40 s by default: the
rain film then covers every street and roof, so every wet-cell branch of
the step does its work), then W
warm-up steps run.  The timed region is the next K steps, queued back to
back on the library's stream.  The K steps after those are run with HIP
events around every kernel launch on that stream, for the per-kernel
roofline figures, and then the per-stage kernels take K timed steps and K
event-timed steps in turn.  Every figure therefore comes from the wet steady
state; `config` reports the wet fraction and the smallest mean depth at the
start of the timed region.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG2 element-stage updates/s + % HBM peak; batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4  # wave64 VALU instructions per ns: CUs x SIMDs x GHz / cycles

# Table 3 of the paper (Sec. 3.3): wall-clock seconds of DG2-NL and DG2-LL on
# one core of a desktop computer (model not given), at the industrial models'
# resolution.  Context only: the paper gives no cell or step counts for them.
PAPER_RUNTIMES = {
    "hardware": "one core of a desktop CPU (model not stated in the paper)",
    "source": "Table 3, Sec. 3.3",
    "DG2-NL_s": {"sloping topography, 20 h": 75, "multiple ponds, 48 h": 833,
                 "obstruction, 15 min": 5.5, "rural catchment, 30 h": 12297,
                 "oblique building, 2 min": 10363},
    "DG2-LL_s": {"sloping topography, 20 h": 166, "multiple ponds, 48 h": 1734,
                 "obstruction, 15 min": 12, "rural catchment, 30 h": 22260,
                 "oblique building, 2 min": 15337},
}


def kernel_source_hash() -> str:
    """Hash of the kernels' sources, launch shapes, buffer layout and build
    flags (traffic counters recorded for another hash are stale)."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2010_02003_amd")
    for f in ("csrc/dg2_device.h", "csrc/dg2_kernels.hip", "csrc/dg2_internal.h", "csrc/dg2_ctx.h",
              "csrc/dg2_api.hip", "build.py"):
        h.update(open(os.path.join(pkg, f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(sc, esz):
    """Bytes each stage kernel must move per cell: every plane read or written once.

    stage 1 reads 9 state planes, 2 bed-slope planes and the Manning plane and
    writes 9; stage 2 reads 9 stage-1 planes, 9 state planes, 2 bed slopes and
    the Manning plane and writes 9.  A uniform Manning value drops its plane.
    """
    nplane = 1 if isinstance(sc.manning, np.ndarray) else 0
    if sc.variant == "LL":
        # DG2-LL: stage 1 also reads z0 and writes the limited stage-1 input
        # W1 (9 planes); stage 2 reads U1, W1 and the 3 bed planes, no Manning
        return (9 + 3 + nplane + 18) * esz, (9 + 9 + 3 + 9) * esz
    s1 = (9 + 2 + nplane + 9) * esz
    s2 = (9 + 9 + 2 + nplane + 9) * esz
    return s1, s2


def fused_bytes(sc, esz):
    """Bytes the fused step kernel must move per cell: the 9 state planes, 2
    bed slopes and the Manning plane read once, the 9 new state planes
    written once."""
    nplane = 1 if isinstance(sc.manning, np.ndarray) else 0
    return (9 + 2 + nplane + 9) * esz


def make_workload(name):
    from paper_2010_02003_amd import workloads as WL

    if name == "urban":
        return WL.urban()
    if name == "urban_fp64":
        return WL.urban(precision="fp64")
    if name == "urban_ll":
        return WL.urban(variant="LL")
    if name == "floodplain":
        return WL.floodplain()
    if name == "dambreak":
        return WL.dambreak_bump()
    raise SystemExit("unknown workload " + name)


def cpu_baseline(sc, budget_s=15.0, single_core_s=8.0):
    """The FP64 oracle, as it stands, on a corner window of the same workload:
    with torch's default thread count (the host's cores), then on one core."""
    import torch

    from oracle import dg2_oracle as O

    w = min(512, sc.nx, sc.ny)
    sub = sc.__class__(**{**sc.__dict__})
    sub.nx = sub.ny = w
    sub.Z = sc.Z[: w + 1, : w + 1]
    sub.surface = sc.surface[: w + 1, : w + 1]
    if isinstance(sc.manning, np.ndarray):
        sub.manning = sc.manning[:w, :w]
    sub.inflows = [b for b in sc.inflows if (b.last < w)]
    U, bed, prm = O.setup(sub)

    def rate(budget, cap):
        t0 = time.perf_counter()
        r = O.run(U, bed, prm, steps=1)
        one = time.perf_counter() - t0
        steps = int(max(1, min(cap, budget / max(one, 1e-3))))
        t0 = time.perf_counter()
        O.run(r.U, bed, prm, steps=steps, t0=r.t)
        return w * w * 2 * steps / (time.perf_counter() - t0), steps

    cores = torch.get_num_threads()
    value, steps = rate(budget_s, 400)
    torch.set_num_threads(1)
    try:
        single, steps1 = rate(single_core_s, 100)
    finally:
        torch.set_num_threads(cores)
    return {"value": value, "unit": "element-stage updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%dx%d corner window of the %s workload, FP64 torch-CPU oracle, %d steps "
                      "after one warm-up step" % (w, w, sc.name, steps),
            "single_core": {"value": single, "cores": 1, "steps": steps1}}


def ensemble_leg(count=256, steps=200, plain_steps=100, warmup=5):
    """Batched ensemble against the plain per-scenario solver on the same GPU.

    The 256-member ensemble (uneven grids 64..512 x 64..256, dx = 2 m, FP32,
    each with its own device time step) is advanced by one persistent launch
    per stage replayed from a graph, then the same scenarios are stepped one
    after the other with the single-scenario path.  Both are reported as
    element-stage updates/s.
    """
    import torch

    from paper_2010_02003_amd import dg2
    from paper_2010_02003_amd import workloads as WL

    scs = WL.ensemble(count)
    cells = sum(sc.cells for sc in scs)
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    batch = dg2.Batch(sims)
    rows = batch.autotune(300.0)
    batch.step(warmup)
    batch.sync()
    ms = batch.time_steps(steps)
    batched = cells * 2 / (ms * 1e-3)
    batch.close()
    # plain: the same scenarios, one after the other, eager launches
    t0 = time.perf_counter()
    for s in sims:
        s.step(plain_steps)
    for s in sims:
        s.sync()
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t0
    plain = cells * 2 * plain_steps / plain_wall
    for s in sims:
        s.close()
    return {"scenarios": count, "cells": cells, "rows_per_wave": rows, "steps": steps,
            "ms_per_step": ms, "value": batched, "plain_value": plain,
            "plain_steps": plain_steps, "speedup_vs_plain": batched / plain,
            "unit": "element-stage updates/s", "dtype": "f32"}


def adjoint_leg():
    """Gradient of a gauge misfit on the 512 x 512 adjoint workload (FP64,
    DG2-NL, 2000 steps of 0.05 s, checkpoints every 100 steps) against the
    plain forward run of the same 2000 steps.

    The gradient evaluation is one forward run (gauge record and
    checkpoints) plus one backward run (segment recompute and the reverse
    steps); both are timed with HIP events inside the library.  The loss is
    the squared misfit to the gauge record of the target parameters.
    """
    import torch

    from paper_2010_02003_amd import dg2
    from paper_2010_02003_amd import workloads as WL

    c = WL.adjoint_case()
    n, nb, steps = c["n"], c["block"], c["steps"]
    man = np.kron(np.full_like(c["n_blocks_target"], c["n_model"]), np.ones((nb, nb)))
    man_t = np.kron(c["n_blocks_target"], np.ones((nb, nb)))
    Q = c["Q_target"] * c["model_scale"]

    def make_sim():
        s = dg2.Sim(n, n, c["dx"], c["dx"])
        s.set_dem_corners(c["Z"])
        s.set_manning(man)
        s.set_boundary(c["inflow_side"], dg2.BC_INFLOW_Q, c["inflow_first"], c["inflow_last"])
        s.set_inflow_hydrograph(c["inflow_side"], c["t_q"], Q)
        s.set_fixed_dt(c["dt"])
        s.set_initial_corners(c["eta"], True)
        s.set_gauges(c["gauges"], capacity=steps)
        return s

    plain = make_sim()
    rows = plain.autotune(300.0)
    plain.step(20)
    plain.sync()
    plain.set_initial_corners(c["eta"], True)
    _, _, ms_step = plain.time_kernels(steps)
    plain_ms = ms_step * steps
    plain.close()

    s = make_sim()
    s.set_launch(rows, 4)
    adj = dg2.Adjoint(s, steps, c["checkpoint_every"], c["inflow_side"], len(c["t_q"]))
    target = adj.forward(man_t, c["Q_target"])
    h = adj.forward(man, Q)
    adj.backward(2.0 * (h - target))  # warm-up
    h = adj.forward(man, Q)
    gn, gq = adj.backward(2.0 * (h - target))
    fwd_ms, bwd_ms = adj.timing()
    torch.cuda.synchronize()
    adj.close()
    # the same gradient with the whole trajectory kept in HBM (checkpoint
    # interval = step count: about 2 states per step, 76 GB here), so the
    # backward run recomputes nothing; bitwise the same gradient
    try:
        adj = dg2.Adjoint(s, steps, steps, c["inflow_side"], len(c["t_q"]))
        h2 = adj.forward(man, Q)
        adj.backward(2.0 * (h2 - target))  # warm-up
        h2 = adj.forward(man, Q)
        gn2, gq2 = adj.backward(2.0 * (h2 - target))
        kfwd_ms, kbwd_ms = adj.timing()
        torch.cuda.synchronize()
        adj.close()
        kept = None
    except dg2.DG2Error as e:  # e.g. not enough device memory for the whole trajectory
        kept = {"checkpoint_every": steps, "error": str(e)}
    s.close()
    cells = n * n
    grad_ms = fwd_ms + bwd_ms
    if kept is None:
        kept_ms = kfwd_ms + kbwd_ms
        kept = {"checkpoint_every": steps, "forward_ms": kfwd_ms, "backward_ms": kbwd_ms,
                "gradient_ms": kept_ms, "gradient_vs_plain": kept_ms / plain_ms,
                "same_gradient": bool(np.array_equal(gn2, gn) and np.array_equal(gq2, gq))}
    return {"workload": "adjoint_512x512", "cells": cells, "steps": steps,
            "checkpoint_every": c["checkpoint_every"], "dtype": "f64", "variant": "DG2-NL",
            "rows_per_wave": rows,
            "plain_ms": plain_ms, "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "gradient_ms": grad_ms, "gradient_vs_plain": grad_ms / plain_ms,
            "value": cells * 2 * steps / (grad_ms * 1e-3), "plain_value": cells * 2 * steps / (plain_ms * 1e-3),
            "unit": "element-stage updates/s (of the differentiated forward run)",
            "loss": float(((h - target) ** 2).sum()), "grad_n_max": float(np.abs(gn).max()),
            "grad_Q_max": float(np.abs(gq).max()),
            "trajectory_kept": kept}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--spinup-s", type=float, default=40.0,
                    help="simulated seconds to advance (untimed) before the warm-up steps")
    ap.add_argument("--workload", default="urban")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) leg")
    ap.add_argument("--leg", choices=["adjoint", "ensemble"], default=None,
                    help="run only this leg and print its JSON (for profiling)")
    ap.add_argument("--rows", type=int, default=0, help="rows per wavefront (0: built-in)")
    ap.add_argument("--step-kernel", choices=["fused", "stages"], default="fused",
                    help="both RK stages in one kernel (default) or one kernel per stage")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed region, copy this many MiB three times with a plain "
                         "device copy (reference reading for the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the DG2 step here runs on a single MI355X "
              "(multi-GPU sharding is not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2010_02003_amd import dg2

    assert torch.cuda.is_available(), "bench.py needs the MI355X"
    torch.cuda.set_device(0)
    if args.leg:
        print(json.dumps(adjoint_leg() if args.leg == "adjoint" else ensemble_leg()), flush=True)
        return
    sc = make_workload(args.workload)
    esz = 4 if sc.precision == "fp32" else 8
    sim = dg2.sim_from_scenario(sc, stream="torch")
    if args.rows:
        sim.set_launch(args.rows, 4)
    sim.set_step_kernel(args.step_kernel == "fused")

    # spin-up into the wet steady state, then warm-up steps; nothing is reset,
    # so every timed step below runs on a wet domain.  The spin-up runs on
    # the per-stage kernels (bitwise the same states as the fused kernel), so
    # that every launch of the fused step kernel in a profile of this command
    # belongs to the wet steady state.
    if args.spinup_s > 0:
        sim.set_step_kernel(False)
        t_mark = 0.0
        while t_mark < args.spinup_s:
            t_mark = min(args.spinup_s, t_mark + 5.0)
            sim.run_to(t_mark)
            sim.sync()
            print("spin-up: t = %.1f s, %d steps" % (t_mark, sim.time()[1]), file=sys.stderr, flush=True)
        sim.set_step_kernel(args.step_kernel == "fused")
    if args.warmup > 0:
        sim.step(args.warmup)
        sim.sync()
    state0, t_start, n_start, _ = sim.get_state()
    wet_fraction = float((state0[0] > sc.tol_dry).mean())
    min_h0_start = float(state0[0].min())
    del state0
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    sim.step(args.steps)  # K steps queued back to back on the library stream
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_sim, nstep, last_dt = sim.time()
    mass, energy, hmin = sim.diagnostics()
    # the next K steps with a HIP event pair around every kernel launch on
    # the library stream (the events add a little time per launch, so they
    # are kept out of the timed region)
    ms1, ms2, ms_step_ev = sim.time_kernels(args.steps)
    torch.cuda.synchronize()
    # the fused kernel ran iff there was no separate stage-2 launch (it
    # applies to DG2-NL; DG2-LL workloads use the stage kernels)
    fused = ms2 == 0.0

    cells = sc.nx * sc.ny
    value = cells * 2 * args.steps / wall
    b1, b2 = algorithmic_bytes(sc, esz)
    bf = fused_bytes(sc, esz)
    traffic = None
    valu_busy = None
    valu_insts = None
    copy_gbs = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    sname = "k_stage_ll" if sc.variant == "LL" else "k_stage_nl"
    kname = "k_step_nl" if fused else sname
    if os.path.exists(tfile):
        ent = json.load(open(tfile)).get(args.workload)
        if ent and ent.get("kernel_hash") == kernel_source_hash() and ent.get("kernel") == kname:
            traffic = ent.get("bytes_per_launch")
            valu_busy = ent.get("valu_busy")
            valu_insts = ent.get("valu_insts_per_launch")
            copy_gbs = ent.get("copy_bandwidth_gbs")
    real = "float" if esz == 4 else "double"
    if fused:
        ach = cells * bf / (ms1 * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "fused step (k_step_nl<%s, HLL>)" % real,
                "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": traffic, "bytes_per_cell": bf,
                "basis": "algorithmic bytes of one fused launch: per cell the 9 state planes, 2 bed "
                         "slopes and the Manning plane read once and the 9 new planes written once",
                "ms_per_launch": ms1,
                # the plain device-copy bandwidth measured on this machine with the counters
                "copy_ceiling": None if copy_gbs is None else {"GB/s": copy_gbs, "frac": ach / copy_gbs},
                "step_frac": cells * bf / (wall / args.steps) / 1e9 / HBM_PEAK_GBS,
                "ms_per_step_with_events": ms_step_ev,
                # the kernel is bound by vector-ALU issue, not HBM: the VALUBusy
                # counter of the profiled run of these sources, and the counted
                # VALU instructions per launch over this run's launch time
                # against the issue rate of 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
                "valu_busy": valu_busy,
                "valu_issue": None if valu_insts is None else {
                    "achieved": valu_insts / (ms1 * 1e-3) / 1e9, "peak": VALU_ISSUE_PEAK_G,
                    "unit": "G wave64 VALU instructions/s",
                    "frac": valu_insts / (ms1 * 1e-3) / 1e9 / VALU_ISSUE_PEAK_G}}
        # the per-stage kernels on the following steps, for comparison
        sim.set_step_kernel(False)
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.sync()
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t0
        s1, s2, _ = sim.time_kernels(args.steps)
        torch.cuda.synchronize()
        roof["stage_kernels"] = {
            "ms_per_step": wall_s * 1e3 / args.steps,
            "value": cells * 2 * args.steps / wall_s,
            "stage1": {"ms_per_launch": s1, "bytes_per_cell": b1,
                       "frac": cells * b1 / (s1 * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "stage2": {"ms_per_launch": s2, "bytes_per_cell": b2,
                       "frac": cells * b2 / (s2 * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "step_frac": cells * (b1 + b2) / (wall_s / args.steps) / 1e9 / HBM_PEAK_GBS}
    else:
        ach2 = cells * b2 / (ms2 * 1e-3) / 1e9
        ach1 = cells * b1 / (ms1 * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "stage 2 (%s<%s, 2, HLL>)" % (sname, real),
                "achieved": ach2, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach2 / HBM_PEAK_GBS,
                "traffic": traffic, "bytes_per_cell": b2, "ms_per_launch": ms2,
                "stage1": {"achieved": ach1, "frac": ach1 / HBM_PEAK_GBS, "bytes_per_cell": b1,
                           "ms_per_launch": ms1},
                "step_frac": cells * (b1 + b2) / (wall / args.steps) / 1e9 / HBM_PEAK_GBS,
                "ms_per_step_with_events": ms_step_ev}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "element-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if esz == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": sc.name, "nx": sc.nx, "ny": sc.ny, "dx": sc.dx, "variant": "DG2-" + sc.variant,
                   "precision": sc.precision, "cells": cells,
                   "end_of_stage": "partly-wet rule" if sc.partly_wet_flat else "paper (Sec. 2.1.3)",
                   "spinup_s": args.spinup_s, "timed_from_t_s": t_start, "timed_from_step": n_start,
                   "timed_to_t_s": t_sim, "mean_dt_s": (t_sim - t_start) / args.steps,
                   "wet_fraction": wet_fraction, "min_h0_at_start": min_h0_start,
                   "last_dt_s": last_dt, "mass_m3": mass, "min_h0": hmin,
                   "step_kernel": "fused" if fused else "stages"},
        "roofline": roof,
        "cpu_baseline": None,
        "paper_runtimes": PAPER_RUNTIMES,
    }
    if args.copy_mib > 0:
        # three plain device copies: the reference reading of the HBM traffic
        # counters, and the copy bandwidth this box attains (read + written
        # bytes over the HIP-event time of the second and third copy)
        n = args.copy_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 2
        out["copy_calibration_mib"] = args.copy_mib
        out["copy_bandwidth"] = {"GB/s": 2 * n * 4 / (ms * 1e-3) / 1e9, "ms_per_copy": ms,
                                 "frac": 2 * n * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if not args.no_ensemble:
        out["batched"] = ensemble_leg()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
