"""The reverse-mode building blocks of the adjoint step (csrc/dg2_vjp.h),
compiled for the host and checked against fourth-order central differences
of their own forward functions: HLL flux in every wave regime (both wet,
supercritical either way, one side dry), physical flux at Gauss points with
the dummy limit, the prescribed-discharge inflow flux (critical depth and
inner depth branches) and the friction split of a planar element, including
the derivative with respect to the Manning coefficient."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2010_02003_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
def test_vjp_building_blocks_vs_central_differences(tmp_path):
    exe = str(tmp_path / "vjp_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "vjp_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout


# ---------------------------------------------------------------------------
# Operator adjoint over a grid vs reverse-mode differentiation of the oracle
# ---------------------------------------------------------------------------

import ctypes

import numpy as np
import torch

from oracle import dg2_oracle as O


class _SqrtZeroAtZero(torch.autograd.Function):
    """sqrt whose derivative is taken as 0 at 0 (the adjoint's convention for
    the wave celerity sqrt(g h) of a dry side); torch's own gives inf * 0."""

    @staticmethod
    def forward(ctx, x):
        y = _TORCH_SQRT(x)
        ctx.save_for_backward(y)
        return y

    @staticmethod
    def backward(ctx, gy):
        (y,) = ctx.saved_tensors
        pos = y > 0
        return torch.where(pos, gy / (2.0 * torch.where(pos, y, torch.ones_like(y))), torch.zeros_like(y))


_TORCH_SQRT = torch.sqrt


@pytest.fixture(scope="module")
def adj_host_lib(tmp_path_factory):
    if not (shutil.which(HIPCC) or os.path.exists(HIPCC)):
        pytest.skip("hipcc not found")
    so = str(tmp_path_factory.mktemp("adjhost") / "adj_host.so")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC",
                    "-shared", "-I", CSRC, os.path.join(HERE, "adj_host.cpp"), "-o", so], check=True)
    lib = ctypes.CDLL(so)
    P = ctypes.POINTER
    d, i = ctypes.c_double, ctypes.c_int
    lib.op_vjp_grid.argtypes = [P(d), P(d), P(ctypes.c_uint8), P(d), i, i, d, d, d, d, P(i), P(i),
                                P(d), P(d), P(d)]
    return lib


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _random_state(rng, nx, ny, tol):
    X = np.zeros((9, ny, nx))
    h0 = rng.uniform(0.05, 2.0, (ny, nx))
    dry = rng.random((ny, nx)) < 0.2
    h0[dry] = rng.uniform(0.0, tol, dry.sum())
    X[0] = h0
    # slopes up to 1.3 h0: some face limits go negative (wall-revised bed, h* = 0)
    X[1] = rng.uniform(-1.3, 1.3, (ny, nx)) * h0
    X[2] = rng.uniform(-1.3, 1.3, (ny, nx)) * h0
    X[3:] = rng.uniform(-1.0, 1.0, (6, ny, nx))
    X[3:][:, dry] = 0.0
    return X


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_operator_adjoint_vs_oracle_autograd(adj_host_lib, monkeypatch, seed):
    rng = np.random.default_rng(seed)
    nx, ny, dx, dy, g, tol = 9, 7, 1.5, 2.0, 9.81, 1e-5
    Z = rng.uniform(0.0, 0.8, (ny + 1, nx + 1))
    bed = O.bed_from_corners(Z)
    X = _random_state(rng, nx, ny, tol)
    lam = rng.uniform(-1.0, 1.0, (9, ny, nx))
    mask = rng.integers(0, 3, (ny, nx)).astype(np.uint8)
    # inflow on the west (rows 2..4) and south (columns 3..7); north segment
    # with zero discharge (a wall); east wall
    segs = {O.WEST: (2, 4, 0.7), O.SOUTH: (3, 7, 0.4), O.NORTH: (1, 5, 0.0)}

    # host build of the library's operator adjoint
    first = np.array([segs.get(s, (1, 0, 0))[0] for s in range(4)], dtype=np.int32)
    last = np.array([segs.get(s, (1, 0, 0))[1] for s in range(4)], dtype=np.int32)
    q = np.array([segs.get(s, (1, 0, 0.0))[2] for s in range(4)])
    zc = np.ascontiguousarray(bed.z.numpy().reshape(3, ny, nx))
    Xc, lc, mc = np.ascontiguousarray(X), np.ascontiguousarray(lam), np.ascontiguousarray(mask)
    JT = np.zeros((9, ny, nx))
    lq = np.zeros(4)
    adj_host_lib.op_vjp_grid(_ptr(Xc), _ptr(lc), _ptr(mc, ctypes.c_uint8), _ptr(zc), nx, ny, dx, dy,
                             g, tol, _ptr(first, ctypes.c_int), _ptr(last, ctypes.c_int), _ptr(q),
                             _ptr(JT), _ptr(lq))

    # reverse mode through the oracle's operator
    monkeypatch.setattr(torch, "sqrt", _SqrtZeroAtZero.apply)
    Xt = torch.tensor(X.reshape(3, 3, ny, nx), requires_grad=True)
    prm = O.Params(nx=nx, ny=ny, dx=dx, dy=dy, g=g, tol=tol)
    Qs = {}
    for side, (a, b, qv) in segs.items():
        width = (b - a + 1) * (dy if side in (O.WEST, O.EAST) else dx)
        Qs[side] = (torch.tensor(qv * width, dtype=torch.float64, requires_grad=True), width)
        prm.inflows.append(O.InflowBC(side, a, b, torch.tensor([0.0, 1.0], dtype=torch.float64),
                                      torch.stack([Qs[side][0], Qs[side][0]])))
    L = O.spatial_operator(Xt, bed, prm, 0.0).reshape(9, ny, nx)
    mu = torch.tensor(lam)
    dry = torch.tensor(mask == 1)
    part = torch.tensor(mask == 2)
    for k in range(3, 9):
        mu[k] = torch.where(dry, 0.0, mu[k])
    for k in (1, 2, 4, 5, 7, 8):
        mu[k] = torch.where(part, 0.0, mu[k])
    loss = (mu * L).sum()
    grads = torch.autograd.grad(loss, [Xt] + [Qs[s][0] for s in segs], allow_unused=True)
    grads = [torch.zeros((), dtype=torch.float64) if gr is None else gr for gr in grads]
    ref = grads[0].reshape(9, ny, nx).numpy()
    scale = np.abs(ref).max()
    assert np.isfinite(ref).all()
    np.testing.assert_allclose(JT, ref, rtol=0, atol=1e-12 * scale)
    for (side, (qt, width)), gq in zip(Qs.items(), grads[1:]):
        want = float(gq) * width
        if segs[side][2] == 0.0:
            assert lq[side] == 0.0 and want == 0.0
        else:
            assert lq[side] == pytest.approx(want, rel=1e-12, abs=1e-13 * scale)
