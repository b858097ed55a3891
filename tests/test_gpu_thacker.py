"""Thacker's curved oscillatory flow in a frictionless parabolic bowl (the
long-run test of Sec. 2.3), on the GPU.

* parity with the oracle over half a period (80 m cells, FP64), with the
  mass and energy histories (Eq. 11-12) at every eighth of the period;
* the sign of the energy error.  The paper reports energy lost by its DG2
  (about 1 % over 30 periods).  With the paper's end-of-stage treatment (the
  default) the run loses energy over the first period, as the paper's does;
  with the optional partly-wet rule (partly wet elements drop their slope
  modes after each stage; not in the paper) it gains energy instead.
* the paper's long run on 40 m cells, 30 periods.  With the paper's
  treatment the films at the moving shoreline carry fictitious speeds
  (hundreds of m/s at mean depths just above the drying tolerance), mean
  depths reach -2.1 m by 7.5 periods and the Courant step collapses after
  about 26 periods, so the long run uses the partly-wet option: depth
  against the exact solution at the maximally wet (7 tau/2) and maximally
  dry (8 tau) times the paper plots, mass to round-off, and total energy,
  which this option gains (+0.8 % after 30 periods).  The paper's sign
  (energy lost) is asserted as an expected failure for this run, strict, so
  the discrepancy stays visible; the gain shrinks at second order with the
  cell size (the last test).
"""
import numpy as np
import pytest

from oracle import dg2_oracle as O
from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu
TAU = 1756.2


def _say(*a):
    print(*a, flush=True)


def test_thacker_matches_oracle_over_half_a_period():
    sc = WL.thacker_bowl(dx=80.0)
    s = dg2.sim_from_scenario(sc)
    times = [TAU / 8, TAU / 4, 3 * TAU / 8, TAU / 2]
    hist = s.history(times)
    gpu, t, step, _ = s.get_state()
    U, bed, prm = O.setup(sc)
    t0, n = 0.0, 0
    for k, T in enumerate(times):
        r = O.run(U, bed, prm, t_end=T, t0=t0)
        U, t0, n = r.U, r.t, n + r.steps
        # mass and energy histories (Eq. 11-12) against the oracle's
        assert hist[k, 0] == T
        assert hist[k, 1] == pytest.approx(O.mass(U, prm), rel=1e-13)
        assert hist[k, 2] == pytest.approx(O.energy(U, bed, prm), rel=1e-12)
        assert hist[k, 3] == pytest.approx(float(U[0, 0].min()), abs=1e-12)
    dh = np.abs(gpu[0] - U[0, 0].numpy()).max()
    _say("Thacker 80 m, tau/2: steps gpu %d oracle %d, max |dh0| %.2e, energy / initial %.6f"
         % (step, n, dh, hist[-1, 2] / hist[0, 2]))
    assert t == TAU / 2 and step == n
    ref = O.to_planes(U)
    scale = np.maximum(np.abs(ref).reshape(9, -1).max(axis=1), 1.0)
    assert (np.abs(gpu - ref).reshape(9, -1).max(axis=1) / scale).max() <= 1e-10


def _energy_after(dx, T, flat):
    sc = WL.thacker_bowl(dx=dx)
    sc.partly_wet_flat = flat
    s = dg2.sim_from_scenario(sc)
    m0, e0, _ = s.diagnostics()
    s.run_to(T)
    m, e, hmin = s.diagnostics()
    steps = s.time()[1]
    s.close()
    return e / e0, (m - m0) / m0, hmin, steps


def test_thacker_energy_sign_over_one_period():
    """Paper's treatment: energy lost (the paper's sign); partly-wet option:
    energy gained.  40 m cells, one period."""
    e_paper, dm_paper, hmin, n_paper = _energy_after(40.0, TAU, False)
    e_flat, dm_flat, _, n_flat = _energy_after(40.0, TAU, True)
    _say("Thacker 40 m, one period: E/E0 - 1 = %+.3e (paper's treatment, %d steps, min h0 %.2e), "
         "%+.3e (partly-wet option, %d steps)" % (e_paper - 1, n_paper, hmin, e_flat - 1, n_flat))
    assert abs(dm_paper) < 1e-12 and abs(dm_flat) < 1e-12
    assert 0.98 < e_paper < 1.0
    assert 1.0 < e_flat < 1.01


@pytest.fixture(scope="module")
def long_runs():
    dx = 40.0
    out = {}
    for variant in ("NL", "LL"):
        sc = WL.thacker_bowl(dx=dx, variant=variant)
        sc.partly_wet_flat = True
        s = dg2.sim_from_scenario(sc)
        m0, e0, _ = s.diagnostics()
        XC, YC = WL.cell_xy(sc.nx, sc.ny, dx, dx, sc.x0, sc.y0)
        res = {}
        for name, T in (("wet 7tau/2", 3.5 * TAU), ("dry 8tau", 8.0 * TAU), ("30tau", 30.0 * TAU)):
            s.run_to(T)
            st, t, step, _ = s.get_state()
            m, e, hmin = s.diagnostics()
            he, _, _ = WL.thacker_exact(XC, YC, T)
            l1 = float(np.abs(st[0] - he).mean())
            res[name] = (l1, (m - m0) / m0, e / e0, step)
            _say("Thacker %s (partly-wet option) %s: steps %d, L1(h) %.3e m, mass error %.2e, "
                 "energy / initial %.5f, min h0 %.1e" % (variant, name, step, l1, (m - m0) / m0, e / e0, hmin))
        s.close()
        out[variant] = res
    return out


@pytest.mark.parametrize("variant", ["NL", "LL"])
def test_thacker_long_run_30_periods(long_runs, variant):
    out = long_runs[variant]
    for name, (l1, dm, er, _) in out.items():
        assert abs(dm) < 1e-11, name
    # depth stays close to the exact profiles the paper plots after 7 periods
    assert out["wet 7tau/2"][0] < 2e-2 and out["dry 8tau"][0] < 2e-2
    # the total energy stays within 1.5 % of its initial value over 30 periods
    assert abs(out["30tau"][2] - 1.0) < 1.5e-2


@pytest.mark.xfail(strict=True, reason="the partly-wet option gains energy over 30 periods (+0.8 %); "
                                       "the paper reports about 1 % lost (Sec. 2.3)")
@pytest.mark.parametrize("variant", ["NL", "LL"])
def test_thacker_long_run_loses_energy_as_the_paper_reports(long_runs, variant):
    er = long_runs[variant]["30tau"][2]
    assert 0.98 < er < 1.0


def test_thacker_energy_error_shrinks_with_the_cell_size():
    """The partly-wet option's energy gain falls at second order with dx."""
    drift = {}
    for dx in (80.0, 40.0):
        er, _, _, _ = _energy_after(dx, 8.0 * TAU, True)
        drift[dx] = abs(er - 1.0)
        _say("Thacker %g m (partly-wet option): |E/E0 - 1| after 8 tau = %.3e" % (dx, drift[dx]))
    assert drift[40.0] < drift[80.0] / 2.5
