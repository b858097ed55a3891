"""Thacker's curved oscillatory flow in a frictionless parabolic bowl (the
long-run test of Sec. 2.3), on the GPU.

* parity with the oracle over half a period (80 m cells, FP64), with the
  mass and energy histories (Eq. 11-12) at every eighth of the period;
* the paper's long run on 40 m cells: depth against the exact solution at
  the maximally wet (7 tau/2) and maximally dry (8 tau) times the paper
  plots, and mass and total energy (Eq. 11-12) over 30 periods: mass to
  round-off, total energy within 1.5 % of its initial value (the paper
  reports about 1 % lost for its DG2; here the front treatment gains a
  little energy instead, an error that shrinks at second order with the
  cell size, which the last test checks).
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


@pytest.mark.parametrize("variant", ["NL", "LL"])
def test_thacker_long_run_30_periods(variant):
    dx = 40.0
    sc = WL.thacker_bowl(dx=dx, variant=variant)
    s = dg2.sim_from_scenario(sc)
    m0, e0, _ = s.diagnostics()
    XC, YC = WL.cell_xy(sc.nx, sc.ny, dx, dx, sc.x0, sc.y0)
    out = {}
    for name, T in (("wet 7tau/2", 3.5 * TAU), ("dry 8tau", 8.0 * TAU), ("30tau", 30.0 * TAU)):
        s.run_to(T)
        st, t, step, _ = s.get_state()
        m, e, hmin = s.diagnostics()
        he, _, _ = WL.thacker_exact(XC, YC, T)
        l1 = float(np.abs(st[0] - he).mean())
        out[name] = (l1, (m - m0) / m0, e / e0, step)
        _say("Thacker %s %s: steps %d, L1(h) %.3e m, mass error %.2e, energy / initial %.5f, "
             "min h0 %.1e" % (variant, name, step, l1, (m - m0) / m0, e / e0, hmin))
    for name, (l1, dm, er, _) in out.items():
        assert abs(dm) < 1e-11, name
    # depth stays close to the exact profiles the paper plots after 7 periods
    assert out["wet 7tau/2"][0] < 2e-2 and out["dry 8tau"][0] < 2e-2
    # total energy stays within 1.5 % over 30 periods
    assert abs(out["30tau"][2] - 1.0) < 1.5e-2


def test_thacker_energy_error_shrinks_with_the_cell_size():
    drift = {}
    for dx in (80.0, 40.0):
        sc = WL.thacker_bowl(dx=dx)
        s = dg2.sim_from_scenario(sc)
        _, e0, _ = s.diagnostics()
        s.run_to(8.0 * TAU)
        _, e, _ = s.diagnostics()
        drift[dx] = abs(e / e0 - 1.0)
        _say("Thacker %g m: |E/E0 - 1| after 8 tau = %.3e" % (dx, drift[dx]))
    assert drift[40.0] < drift[80.0] / 2.5
