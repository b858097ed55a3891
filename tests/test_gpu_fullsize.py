"""GPU parity at the full workload sizes, in the launch configuration that
bench.py times (built-in rows per wavefront, four wavefronts per workgroup).

A whole-grid oracle run is out of reach at these sizes, but one step of a
cell depends only on the cells within two of it (one per RK stage).  So the
GPU runs the workload for a while, then one more step; the oracle takes the
GPU's state before that step on sampled windows with a two-cell margin
(the margin's mirror ghosts at interior window edges are wrong, the cells
two or more inside are exact) and must reproduce the GPU's step on every
window cell more than two cells from an interior window edge.  Windows cover
domain corners (two walls), the inflow mouth, wall edges and the interior.
"""
import numpy as np
import pytest

from oracle import dg2_oracle as O
from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu

MARGIN = 2


def _say(*a):
    print(*a, flush=True)


def _window_params(sc, J0, J1, I0, I1):
    man = sc.manning
    man = O._t(man[J0:J1, I0:I1]) if isinstance(man, np.ndarray) else float(man)
    inflows = []
    for b in sc.inflows:
        if b.side in (O.WEST, O.EAST):
            on_edge = (I0 == 0) if b.side == O.WEST else (I1 == sc.nx)
            lo, hi = max(b.first, J0), min(b.last, J1 - 1)
            off = J0
        else:
            on_edge = (J0 == 0) if b.side == O.SOUTH else (J1 == sc.ny)
            lo, hi = max(b.first, I0), min(b.last, I1 - 1)
            off = I0
        if on_edge and lo <= hi:
            # the unit discharge is Q / (full segment length): rescale Q to the window's part
            frac = (hi - lo + 1) / (b.last - b.first + 1)
            inflows.append(O.InflowBC(b.side, lo - off, hi - off, O._t(b.t), O._t(b.Q) * frac))
    return O.Params(nx=I1 - I0, ny=J1 - J0, dx=sc.dx, dy=sc.dy, g=sc.g, tol=sc.tol_dry, cfl=sc.cfl,
                    dt_max=sc.dt_max, theta=sc.theta, variant=sc.variant, manning=man,
                    inflows=inflows, rain=sc.rain, flux=sc.flux)


def _check_window(sc, before, after, t, dt, j0, j1, i0, i1, rtol, atol, margin=MARGIN):
    J0, J1 = max(0, j0 - margin), min(sc.ny, j1 + margin)
    I0, I1 = max(0, i0 - margin), min(sc.nx, i1 + margin)
    prm = _window_params(sc, J0, J1, I0, I1)
    bed = O.bed_from_corners(sc.Z[J0:J1 + 1, I0:I1 + 1])
    U = O.from_planes(before[:, J0:J1, I0:I1])
    ref = O.to_planes(O.step(U, t, bed, prm, dt))[:, j0 - J0:j1 - J0, i0 - I0:i1 - I0]
    gpu = after[:, j0:j1, i0:i1]
    scale = np.maximum(np.abs(ref).reshape(9, -1).max(axis=1), atol / max(rtol, 1e-300))
    err = np.abs(gpu - ref).reshape(9, -1).max(axis=1) / scale
    assert np.all(np.isfinite(gpu))
    assert err.max() <= rtol, "window %s: plane errors %s" % ((j0, j1, i0, i1), err)
    return err.max(), float((before[0, j0:j1, i0:i1] > sc.tol_dry).mean())


def _run(sc, steps, t_end=None):
    s = dg2.sim_from_scenario(sc)
    if t_end is not None:
        s.run_to(t_end)
    else:
        s.step(steps)
    before, t, n, _ = s.get_state()
    s.step(1)
    after, t1, n1, dt = s.get_state()
    assert n1 == n + 1 and t1 == pytest.approx(t + dt, rel=0, abs=1e-12)
    s.close()
    return before, after, t, dt


def _windows(sc, rng, extra):
    w = 40
    wins = [(0, w, 0, w), (sc.ny - w, sc.ny, sc.nx - w, sc.nx),  # two corners
            (sc.ny // 2 - w // 2, sc.ny // 2 + w // 2, sc.nx - w, sc.nx)]  # east wall
    wins += extra
    for _ in range(3):
        j = int(rng.integers(MARGIN, sc.ny - w - MARGIN))
        i = int(rng.integers(MARGIN, sc.nx - w - MARGIN))
        wins.append((j, j + w, i, i + w))
    return wins


def _around(sc, j, i, w=40):
    j0 = int(np.clip(j - w // 2, 0, sc.ny - w))
    i0 = int(np.clip(i - w // 2, 0, sc.nx - w))
    return (j0, j0 + w, i0, i0 + w)


def test_floodplain_full_size_fp64_windows():
    sc = WL.floodplain()
    _say("floodplain 1024 x 512 FP64: run to 900 s, then one step on sampled windows")
    before, after, t, dt = _run(sc, 0, t_end=900.0)
    b = sc.inflows[0]
    mouth = (max(0, b.first - 15), min(sc.ny, b.last + 16), 0, 40)
    rng = np.random.default_rng(21)
    # windows on wet cells and on the wetting front (wet cells next to dry ones)
    wet = before[0] > sc.tol_dry
    front = wet & ~(np.roll(wet, 1, 0) & np.roll(wet, -1, 0) & np.roll(wet, 1, 1) & np.roll(wet, -1, 1))
    extra = [mouth]
    for mask in (wet, wet, front, front):
        cells = np.argwhere(mask)
        if len(cells):
            j, i = cells[int(rng.integers(len(cells)))]
            extra.append(_around(sc, j, i))
    _say("  t = %.1f s, wet cells %d, front cells %d" % (t, int(wet.sum()), int(front.sum())))
    wet_seen = 0.0
    for win in _windows(sc, rng, extra):
        e, wf = _check_window(sc, before, after, t, dt, *win, rtol=1e-12, atol=1e-12)
        wet_seen = max(wet_seen, wf)
        _say("  window", win, "max rel err %.2e" % e, "wet fraction %.2f" % wf)
    assert wet_seen > 0.2  # the inflow mouth is flooded


@pytest.mark.parametrize("flux", ["HLL", "ROE"])
def test_urban_full_size_fp32_windows(flux):
    sc = WL.urban()
    sc.flux = flux
    _say("urban 4096 x 4096 FP32 %s: 400 steps, then one step on sampled windows" % flux)
    before, after, t, dt = _run(sc, 400)
    rng = np.random.default_rng(22)
    # a window on a block edge: find a cell whose bed jumps by the block height
    Z = sc.Z
    jump = np.argwhere(np.abs(np.diff(Z[1000:1200, 1000:1200], axis=1)) > 5.0)
    j, i = (int(jump[0][0]) + 1000, int(jump[0][1]) + 1000) if len(jump) else (2000, 2000)
    block = (j - 20, j + 20, i - 20, i + 20)
    for win in _windows(sc, rng, [block]):
        # FP32 state and arithmetic against the FP64 oracle on the same input:
        # one step's rounding, relative to each plane's magnitude
        e, wet = _check_window(sc, before, after, t, dt, *win, rtol=2e-5, atol=1e-9)
        _say("  window", win, "max rel err %.2e" % e, "wet fraction %.2f" % wet)


def test_urban_full_size_fp64_windows():
    """The urban grid with an FP64 state (the per-stage kernels): the oracle's
    own precision, so the windows must match to round-off."""
    sc = WL.urban(precision="fp64")
    _say("urban 4096 x 4096 FP64: 400 steps, then one step on sampled windows")
    before, after, t, dt = _run(sc, 400)
    rng = np.random.default_rng(23)
    Z = sc.Z
    jump = np.argwhere(np.abs(np.diff(Z[2000:2200, 2000:2200], axis=0)) > 5.0)
    j, i = (int(jump[0][0]) + 2000, int(jump[0][1]) + 2000) if len(jump) else (2100, 2100)
    block = (j - 20, j + 20, i - 20, i + 20)
    for win in _windows(sc, rng, [block]):
        e, wet = _check_window(sc, before, after, t, dt, *win, rtol=1e-12, atol=1e-12)
        _say("  window", win, "max rel err %.2e" % e, "wet fraction %.2f" % wet)


def test_urban_full_size_ll_fp64_windows():
    """DG2-LL on the urban grid (FP64 state, the oracle's precision), with
    the minmod limiter (Eq. 7) on every element: the limiter of a stage reads
    two cells on each side, so a cell's step depends on the cells within four
    of it and the windows carry a margin of four."""
    sc = WL.urban(precision="fp64", variant="LL")
    # threshold 0: every element is limited (a smooth rain film never trips
    # the detector at the default threshold, which would leave DG2-NL)
    sc.theta = 0.0
    _say("urban 4096 x 4096 FP64 DG2-LL (always limited): 400 steps, then one step on sampled windows")
    before, after, t, dt = _run(sc, 400)
    rng = np.random.default_rng(24)
    Z = sc.Z
    jump = np.argwhere(np.abs(np.diff(Z[3000:3200, 1000:1200], axis=1)) > 5.0)
    j, i = (int(jump[0][0]) + 3000, int(jump[0][1]) + 1000) if len(jump) else (3100, 1100)
    block = (j - 20, j + 20, i - 20, i + 20)
    for win in _windows(sc, rng, [block]):
        e, wet = _check_window(sc, before, after, t, dt, *win, rtol=1e-12, atol=1e-12, margin=4)
        _say("  window", win, "max rel err %.2e" % e, "wet fraction %.2f" % wet)


def test_ensemble_full_size_batch_equals_plain():
    """The 256-member ensemble as bench.py runs it (autotuned rows, graph
    replay): every member's state after 200 steps equals, bit for bit, the
    member stepped alone by the single-scenario path."""
    scs = WL.ensemble(256)
    _say("ensemble 256 members, %d cells: 200 batched steps vs plain" % sum(sc.cells for sc in scs))
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    batch = dg2.Batch(sims)
    rows = batch.autotune(300.0)
    batch.step(200)
    batch.sync()
    _say("  autotuned rows per wavefront", rows)
    plain = [dg2.sim_from_scenario(sc) for sc in scs]
    for s in plain:
        s.step(200)
    moved = 0
    for k, (a, b) in enumerate(zip(sims, plain)):
        sa, ta, na, _ = a.get_state()
        sb, tb, nb, _ = b.get_state()
        assert na == nb == 200 and ta == tb, k
        assert np.array_equal(sa, sb), "member %d differs" % k
        moved += int(np.abs(sa[3]).max() > 0)
        b.close()
    batch.close()
    for s in sims:
        s.close()
    assert moved > 200  # water is flowing in most members
