"""Batched ensemble (one persistent launch per stage for many scenarios of
uneven size, each with its own device-resident time step) against the plain
per-scenario solver: the same device arithmetic on the same inputs, so the
results must be bitwise equal, with or without graph replay."""
import numpy as np
import pytest

from oracle import dg2_oracle as O
from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _members(k, precision="fp32", variant="NL", shrink=4):
    """k ensemble scenarios (uneven sizes) at 1/shrink of their side lengths."""
    out = []
    for m in range(k):
        sc = WL.ensemble_member(m)
        nx, ny = max(8, sc.nx // shrink), max(8, sc.ny // shrink)
        sc.nx, sc.ny = nx, ny
        sc.Z = sc.Z[: ny + 1, : nx + 1]
        sc.surface = sc.surface[: ny + 1, : nx + 1]
        b = sc.inflows[0]
        mid = ny // 2
        sc.inflows = [WL.Inflow(b.side, max(0, mid - 5), min(ny - 1, mid + 4), b.t, 40.0 * b.Q)]
        sc.precision = precision
        sc.variant = variant
        out.append(sc)
    return out


@pytest.mark.parametrize("precision,variant,graph", [("fp32", "NL", 16), ("fp32", "NL", 1),
                                                     ("fp64", "NL", 8), ("fp64", "NL", 1),
                                                     ("fp32", "LL", 4)])
def test_batch_equals_plain_runs(precision, variant, graph):
    scs = _members(7, precision, variant)
    _say("batch of", len(scs), precision, variant, "graph steps", graph, [(s.nx, s.ny) for s in scs])
    plain = []
    for sc in scs:
        s = dg2.sim_from_scenario(sc)
        s.step(40)
        plain.append(s.get_state())
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    b = dg2.Batch(sims)
    b.set_launch(0, 4, graph)
    b.step(40)
    b.sync()
    for k, s in enumerate(sims):
        m, t, step, ldt = s.get_state()
        assert step == 40 == plain[k][2]
        assert t == plain[k][1] and ldt == plain[k][3], k
        assert np.array_equal(m, plain[k][0]), k
    b.close()


def test_batch_run_to_and_per_scenario_dt():
    scs = _members(5, "fp64", "NL")
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    b = dg2.Batch(sims)
    b.run_to(12.5)
    dts = []
    for k, s in enumerate(sims):
        m, t, step, ldt = s.get_state()
        assert t == 12.5
        U, bed, prm = O.setup(scs[k])
        r = O.run(U, bed, prm, t_end=12.5)
        assert step == r.steps
        np.testing.assert_allclose(m, O.to_planes(r.U), rtol=0, atol=1e-10)
        dts.append(r.steps)
    assert len(set(dts)) > 1  # scenarios really took different step sizes


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_autotune_keeps_results(precision):
    scs = _members(6, precision, "NL")
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    b = dg2.Batch(sims)
    b.step(10)
    b.sync()
    before = [s.get_state() for s in sims]
    rows = b.autotune(200.0)
    _say("autotuned rows per wavefront:", rows)
    assert rows >= 1
    after = [s.get_state() for s in sims]
    for x, y in zip(before, after):
        assert np.array_equal(x[0], y[0]) and x[1] == y[1] and x[2] == y[2]
    b.step(10)
    b.sync()
    ref = []
    for sc in scs:
        s = dg2.sim_from_scenario(sc)
        s.step(20)
        ref.append(s.get_state()[0])
    for s, r in zip(sims, ref):
        assert np.array_equal(s.get_state()[0], r)
