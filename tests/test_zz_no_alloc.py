"""The allocation-free diagnostics entry point (dg2_diagnostics_noalloc)
against the context's dg2_diagnostics, through the C ABI, on two calls in a
row (the second on a smaller grid), in FP64 and FP32.

Both reduce the same device state; the bed planes given to the
allocation-free call are the oracle's bed modes of the same corner DEM
(Eq. 3), so the energy may differ from the context's by rounding only."""
import numpy as np
import pytest
import torch

from oracle import dg2_oracle as O
from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _case(nx, ny, precision, steps):
    sc = WL.dambreak_bump(nx=nx, ny=ny, precision=precision)
    sim = dg2.sim_from_scenario(sc)
    nbytes, P = sim.state_layout()
    dt = torch.float32 if precision == "fp32" else torch.float64
    esz = 4 if precision == "fp32" else 8
    state = torch.zeros(nbytes // esz, dtype=dt, device="cuda")
    sim.bind_device_state(state.data_ptr(), nbytes)
    sim.step(steps)
    sim.sync()
    bed = torch.zeros(3 * P, dtype=dt, device="cuda")
    z = O.bed_from_corners(sc.Z).z.reshape(3, -1).to(dt)
    for k in range(3):
        bed[k * P:k * P + nx * ny] = z[k].to("cuda")
    return sc, sim, state, bed, P


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_diagnostics_match_the_context_two_calls(precision):
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    out = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    for nx, ny, steps in ((150, 130, 40), (40, 34, 25)):  # second call: smaller input
        sc, sim, state, bed, P = _case(nx, ny, precision, steps)
        mass, energy, hmin = sim.diagnostics()
        torch.cuda.synchronize()
        dg2.diagnostics_noalloc(state.data_ptr(), bed.data_ptr(), nx, ny, P, precision, sc.dx, sc.dy,
                                sc.g, sc.tol_dry, out.data_ptr(), stream.cuda_stream)
        stream.synchronize()
        got = out.cpu().numpy()
        _say("%s %dx%d: noalloc %s, context mass %.15g energy %.15g min h %.6g"
             % (precision, nx, ny, got, mass, energy, hmin))
        assert got[0] == pytest.approx(mass, rel=1e-14, abs=0)
        assert got[2] == hmin
        assert got[3] == 0.0
        etol = 1e-12 if precision == "fp64" else 1e-6
        assert got[1] == pytest.approx(energy, rel=etol)
        sim.bind_device_state(None, 0)
        sim.close()


def test_noalloc_diagnostics_reject_bad_arguments():
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    a = torch.zeros(9 * 64, dtype=torch.float64, device="cuda")
    with pytest.raises(dg2.DG2Error) as e:
        dg2.diagnostics_noalloc(a.data_ptr(), a.data_ptr(), 8, 8, 63, "fp64", 1.0, 1.0, 9.81, 1e-5,
                                out.data_ptr())
    assert e.value.status == -1
    with pytest.raises(dg2.DG2Error):
        dg2.diagnostics_noalloc(0, a.data_ptr(), 8, 8, 64, "fp64", 1.0, 1.0, 9.81, 1e-5, out.data_ptr())
    with pytest.raises(dg2.DG2Error):
        dg2.diagnostics_noalloc(a.data_ptr(), a.data_ptr(), 8, 8, 64, "fp64", 0.0, 1.0, 9.81, 1e-5,
                                out.data_ptr())
