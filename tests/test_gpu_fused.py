"""The fused DG2-NL step kernel (both RK stages of Sec. 2.1.2 in one pass,
the stage-1 result kept in registers; FP32 and FP64) against the per-stage kernels,
through the C ABI: states, times, step sizes, gauge series and diagnostics
are bitwise equal, on ragged grids (strip and segment edges, single rows and
columns), with every boundary kind, inflows, rain and per-cell Manning, HLL
and Roe, at every launch shape; the state may be bound to caller memory or
shared with a batch.  The oracle comparisons of the other files (FP64 and
FP32 DG2-NL) run the fused kernel too, since it is the default."""
import numpy as np
import pytest
import torch

from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _pair(make):
    a, b = make(), make()
    b.set_step_kernel(False)
    return a, b


def _same(a, b, what):
    sa, ta, na, da = a.get_state()
    sb, tb, nb, db = b.get_state()
    assert (na, ta, da) == (nb, tb, db), what
    assert np.all(np.isfinite(sa)), what
    bad = np.argwhere(sa != sb)
    assert len(bad) == 0, "%s: %d values differ, first at %s" % (what, len(bad), bad[:3].tolist())


def _random_sim(nx, ny, prec, flux, seed, bcs=True):
    modes, Z = WL.random_modes(nx, ny, seed=seed, slope=1.2)
    man = np.random.default_rng(seed).uniform(0.0, 0.05, (ny, nx))

    def make():
        s = dg2.Sim(nx, ny, 2.0, 1.5, precision=prec, flux=flux)
        s.set_dem_corners(Z)
        s.set_manning(man)
        if bcs:
            s.set_boundary(dg2.WEST, dg2.BC_LEVEL, 0, ny - 1)
            s.set_level_hydrograph(dg2.WEST, [0.0, 1.0], [0.6, 0.9])
            s.set_boundary(dg2.EAST, dg2.BC_INFLOW_Q, 0, ny - 1)
            s.set_inflow_hydrograph(dg2.EAST, [0.0, 1.0], [0.5, 2.0])
            s.set_boundary(dg2.SOUTH, dg2.BC_OPEN, 0, nx - 1)
            s.set_boundary(dg2.NORTH, dg2.BC_INFLOW_Q, 0, nx - 1)
            s.set_inflow_hydrograph(dg2.NORTH, [0.0], [1.0])
            s.set_rainfall(1e-3, 0.0, 10.0)
        s.set_state(modes, 0.0)
        s.set_fixed_dt(1e-3)
        return s
    return make


# (250, 140) has interior tiles (halo inside the grid) in both the fused and
# the per-stage kernels, next to edge tiles with every boundary kind
SIZES = [(70, 45), (1, 5), (6, 1), (60, 7), (61, 3), (120, 9), (121, 130), (59, 61), (2, 2), (250, 140)]


@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("prec,flux", [("fp32", "HLL"), ("fp32", "ROE"), ("fp64", "HLL"), ("fp64", "ROE")])
def test_fused_step_equals_stage_kernels(nx, ny, prec, flux):
    _say("fused vs per-stage", nx, ny, prec, flux)
    a, b = _pair(_random_sim(nx, ny, prec, flux, seed=nx * 100 + ny))
    for k in (1, 2, 4):
        a.step(k)
        b.step(k)
        _same(a, b, "%dx%d %s %s after %d more steps" % (nx, ny, prec, flux, k))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("rows,wpb", [(1, 1), (2, 4), (3, 2), (5, 4), (8, 1), (13, 4), (200, 4)])
def test_fused_step_launch_shapes(rows, wpb, prec):
    make = _random_sim(125, 77, prec, "HLL", seed=3)
    a, b = _pair(make)
    a.set_launch(rows, wpb)
    a.step(3)
    b.step(3)
    _same(a, b, "rows %d wpb %d" % (rows, wpb))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fused_dam_break_and_floodplain_runs(prec):
    sc = WL.dambreak_bump()
    a, b = _pair(lambda: dg2.sim_from_scenario(sc, precision=prec))
    a.step(sc.steps)
    b.step(sc.steps)
    _same(a, b, "dam break 500 steps")
    sc = WL.floodplain()
    a, b = _pair(lambda: dg2.sim_from_scenario(sc, precision=prec))
    a.step(300)
    b.step(300)
    _same(a, b, "floodplain 300 steps")
    m1, m2 = a.diagnostics(), b.diagnostics()
    assert m1 == m2


def test_fused_urban_fp32_and_gauges():
    sc = WL.urban()
    a, b = _pair(lambda: dg2.sim_from_scenario(sc))
    gauges = [[100.3, 200.1], [1024.0, 1024.0], [2047.9, 1.2], [0.1, 2047.9]]
    for s in (a, b):
        s.set_gauges(gauges, capacity=64)
    a.step(41)
    b.step(41)
    _same(a, b, "urban 41 steps")
    ga, ta = a.read_gauges()
    gb, tb = b.read_gauges()
    assert len(ta) == 41 and np.array_equal(ta, tb) and np.array_equal(ga, gb)


def test_fused_run_to_and_time_kernels():
    make = _random_sim(90, 70, "fp32", "HLL", seed=8, bcs=False)

    def free():
        s = make()
        s.set_fixed_dt(0.0)
        return s
    a, b = _pair(free)
    a.run_to(0.37)
    b.run_to(0.37)
    _same(a, b, "run_to")
    assert a.time()[0] == 0.37
    ms1, ms2, ms = a.time_kernels(5)
    assert ms1 > 0 and ms2 == 0 and ms >= ms1
    ms1, ms2, ms = b.time_kernels(5)
    assert ms1 > 0 and ms2 > 0
    _same(a, b, "after time_kernels")


def test_fused_with_bound_state_and_unbind():
    make = _random_sim(64, 33, "fp32", "HLL", seed=4)
    a, b = _pair(make)
    a.step(3)  # odd: the state sits in the second buffer
    b.step(3)
    nbytes, P = a.state_layout()
    buf = torch.zeros(nbytes // 4 + 64, dtype=torch.float32, device="cuda")
    a.bind_device_state(buf.data_ptr(), buf.numel() * 4)
    torch.cuda.synchronize()
    a.step(2)  # per-stage kernels in place on the bound buffer
    b.step(2)
    _same(a, b, "bound")
    a.bind_device_state(None, 0)
    a.step(3)
    b.step(3)
    _same(a, b, "unbound again")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_after_a_member_was_stepped_alone(prec):
    scs = [WL.ensemble(3)[k] for k in range(3)]
    sims = [dg2.sim_from_scenario(sc, precision=prec) for sc in scs]
    plain = [dg2.sim_from_scenario(sc, precision=prec) for sc in scs]
    batch = dg2.Batch(sims)
    sims[1].step(1)  # fused: member 1's state moves to its other buffer
    plain[1].step(1)
    sims[1].sync()
    batch.step(5)
    batch.sync()
    for s in plain:
        s.step(5)
    for k in range(3):
        _same(sims[k], plain[k], "member %d" % k)
    batch.close()


def test_fp64_runs_the_fused_kernel_and_ll_the_stage_kernels():
    s = _random_sim(40, 30, "fp64", "HLL", seed=9)()
    ms1, ms2, _ = s.time_kernels(2)
    assert ms1 > 0 and ms2 == 0
    s.set_step_kernel(False)
    ms1, ms2, _ = s.time_kernels(2)
    assert ms1 > 0 and ms2 > 0
    sc = WL.dambreak_bump(variant="LL")
    s = dg2.sim_from_scenario(sc, precision="fp64")
    ms1, ms2, _ = s.time_kernels(2)
    assert ms1 > 0 and ms2 > 0


def test_step_kernel_switch_rejects_bad_values():
    s = dg2.Sim(8, 8, 1.0)
    with pytest.raises(dg2.DG2Error):
        s._check(s._lib.dg2_set_step_kernel(s._ctx, 2))


def test_fused_batch_parity_graphs_and_run_to():
    """A batch of FP32 members steps with the fused kernel too: every step
    switches each member between its two state buffers, so graph replays,
    eager remainders of odd length, an odd graph length and a run-to with
    members idling at the target must all leave each member equal to the
    member stepped alone."""
    scs = WL.ensemble(5)
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    plain = [dg2.sim_from_scenario(sc) for sc in scs]
    batch = dg2.Batch(sims)
    batch.set_launch(0, 4, 5)  # odd graph length: rounded up to 6
    for n in (7, 6, 1, 12, 3):
        batch.step(n)
        for p in plain:
            p.step(n)
        batch.sync()
        for k in range(len(scs)):
            _same(sims[k], plain[k], "member %d after %d more steps" % (k, n))
    T = max(s.time()[0] for s in sims) + 2.5
    batch.run_to(T)
    batch.sync()
    for p in plain:
        p.run_to(T)
    for k in range(len(scs)):
        assert sims[k].time()[0] == T
        _same(sims[k], plain[k], "member %d after run_to" % k)
    batch.close()
