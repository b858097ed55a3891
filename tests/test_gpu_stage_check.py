"""GPU parity of the stage-1 Courant check (an option, off by default)
against the oracle's step_checked: on the floodplain's inflow mouth, where
the plain step drives mean depths negative (after a few hundred steps with the
paper's end-of-stage treatment, within 30 with the optional partly-wet
rule), the checked run
matches the oracle step for step (sizes, times, states) over 100 steps and
keeps every mean depth non-negative over 200; run-to targets are still met
exactly; in FP32 the fused step kernel's trials of the whole step give the
per-stage kernels' result bit for bit; a fixed step size turns the check off;
batches refuse members that use it.  The thin films of this case amplify round-off: the oracle itself,
with the inflow changed by one part in 1e14, agrees with itself to 7e-16
after 100 steps but only to 1e-3 after 200, so parity is taken at 100."""
import numpy as np
import pytest

from oracle import dg2_oracle as O
from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _close(gpu, ref, rtol, what):
    scale = np.maximum(np.abs(ref).reshape(9, -1).max(axis=1), 1.0)
    err = (np.abs(gpu - ref).reshape(9, -1).max(axis=1) / scale).max()
    assert np.all(np.isfinite(gpu)) and err <= rtol, "%s: %.3e" % (what, err)
    return err


@pytest.mark.parametrize("variant,flux", [("NL", "HLL"), ("LL", "HLL"), ("NL", "ROE")])
def test_checked_steps_match_oracle_and_stay_positive(variant, flux):
    sc = WL.floodplain_mouth(stage_check=3)
    sc.variant, sc.flux = variant, flux
    s = dg2.sim_from_scenario(sc)
    s.step(100)
    gpu, t, steps, _ = s.get_state()
    U, bed, prm = O.setup(sc)
    r = O.run(U, bed, prm, steps=100)
    ref = O.to_planes(r.U)
    e = _close(gpu, ref, 1e-10, "checked run")
    _say("stage check %s %s, mouth 40 x 40, 100 steps: t gpu %.12f oracle %.12f, max rel err %.2e, "
         "min h0 %.2e" % (variant, flux, t, r.t, e, gpu[0].min()))
    assert steps == 100 and abs(t - r.t) <= 1e-12 * r.t
    assert gpu[0].min() >= 0.0 and ref[0].min() >= 0.0
    hmin = gpu[0].min()
    for _ in range(100):
        s.step(1)
        hmin = min(hmin, s.diagnostics()[2])
    assert hmin >= 0.0
    # the plain step goes negative on the same case
    plain = WL.floodplain_mouth(stage_check=0)
    plain.variant, plain.flux = variant, flux
    p = dg2.sim_from_scenario(plain)
    pmin = 0.0
    for _ in range(300):
        p.step(5)
        pmin = min(pmin, p.diagnostics()[2])
    _say("plain step, same case, 1500 steps: min h0 %.2e" % pmin)
    assert pmin < 0.0


def test_checked_run_to_lands_on_target():
    sc = WL.floodplain_mouth(stage_check=2)
    s = dg2.sim_from_scenario(sc)
    s.run_to(5.0)
    gpu, t, steps, _ = s.get_state()
    U, bed, prm = O.setup(sc)
    r = O.run(U, bed, prm, t_end=5.0)
    _say("checked run_to(5 s): %d steps (oracle %d)" % (steps, r.steps))
    assert t == 5.0 and steps == r.steps and steps < 400
    _close(gpu, O.to_planes(r.U), 1e-10, "checked run_to")


def test_checked_fp32():
    sc = WL.floodplain_mouth(stage_check=3, precision="fp32")
    s = dg2.sim_from_scenario(sc)
    s.step(200)
    st = s.get_state()[0]
    ref = dg2.sim_from_scenario(WL.floodplain_mouth(stage_check=3))
    ref.step(200)
    r64 = ref.get_state()[0]
    _say("stage check FP32: min h0 %.2e, max |h0 - FP64| %.2e" % (st[0].min(), np.abs(st[0] - r64[0]).max()))
    assert st[0].min() >= -1e-6
    assert np.abs(st[0] - r64[0]).max() < 1e-2


@pytest.mark.parametrize("flux,nx,ny,row0,prec", [("HLL", 40, 40, 236, "fp32"), ("ROE", 40, 40, 236, "fp32"),
                                                  ("HLL", 200, 100, 200, "fp32"),
                                                  ("HLL", 200, 100, 200, "fp64")])
def test_checked_fused_step_kernel_matches_per_stage_kernels(flux, nx, ny, row0, prec):
    """With the fused step kernel (the default) the check tries the
    whole step; each trial computes stage 1 as the matching repeat of the
    per-stage check does, so both paths take the same step sizes and give
    the same states, bit for bit.  The 200 x 100 corner has interior tiles
    (halo inside the grid) beside the inflow mouth."""
    sc = WL.floodplain_mouth(nx=nx, ny=ny, row0=row0, stage_check=3, precision=prec)
    sc.flux = flux
    a = dg2.sim_from_scenario(sc)
    b = dg2.sim_from_scenario(sc)
    b.set_step_kernel(False)
    # gauges next to the inflow segment (rows 15..24 of the west side), recorded every step
    xy = [(sc.x0 + (i + 0.5) * sc.dx, sc.y0 + (j + 0.5) * sc.dy) for i, j in ((0, 19), (3, 20), (8, 17))]
    for s in (a, b):
        s.set_gauges(xy, capacity=4096)
    hmin = 0.0
    for n in range(4):
        for s in (a, b):
            s.step(50)
        sa, ta, na, da = a.get_state()
        sb, tb, nb, db = b.get_state()
        assert na == nb == 50 * (n + 1)
        assert ta == tb and da == db, (n, ta, tb, da, db)
        assert np.array_equal(sa, sb), (n, np.abs(sa - sb).max())
        hmin = min(hmin, float(sa[0].min()))
    _say("stage check, fused vs per-stage kernels, %s %s, %d x %d, 200 steps: t %.9f, min h0 %.2e"
         % (prec, flux, nx, ny, ta, hmin))
    assert hmin >= -1e-6
    # run-to with trials: the target is still met exactly, in the same steps
    T = float(np.ceil(ta)) + 5.0
    for s in (a, b):
        s.run_to(T)
    sa, ta, na, _ = a.get_state()
    sb, tb, nb, _ = b.get_state()
    assert ta == tb == T and na == nb and np.array_equal(sa, sb)
    ga, tga = a.read_gauges()
    gb, tgb = b.read_gauges()
    assert len(tga) == na and np.array_equal(tga, tgb) and np.array_equal(ga, gb)


def test_fixed_step_turns_the_check_off():
    sc = WL.floodplain_mouth(stage_check=3)
    a = dg2.sim_from_scenario(sc)
    b = dg2.sim_from_scenario(WL.floodplain_mouth(stage_check=0))
    for s in (a, b):
        s.set_fixed_dt(0.01)
        s.step(50)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])


def test_invalid_use():
    s = dg2.sim_from_scenario(WL.floodplain_mouth(stage_check=1))
    with pytest.raises(dg2.DG2Error):
        s.set_stage_check(9)
    with pytest.raises(dg2.DG2Error):
        dg2.Batch([s])
