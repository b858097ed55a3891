"""Pins of the oracle's reverse-mode reference (gauge-misfit gradients).

The reference differentiates the oracle step with torch autograd; here its
gradients are checked against central differences of the plain forward
oracle, which shares nothing with the reverse pass.  The case is fully wet
(depth 1 m over an fBm bed with a bump), has a west inflow segment whose
hydrograph rises and falls within the run, per-cell Manning values, and
three gauges with an arbitrary target depth.
"""
import numpy as np
import pytest
import torch

from oracle import dg2_oracle as O
from paper_2010_02003_amd import workloads as WL

N, DX, DT, STEPS = 14, 2.0, 0.06, 14
TQ = torch.tensor([0.0, 0.3, 0.6, 0.9], dtype=torch.float64)
GAUGES = np.array([[4.0, 14.0], [17.0, 11.0], [23.0, 23.0]])


def _case():
    X, Y = WL.corner_xy(N, N, DX, DX)
    Z = WL.fbm_surface((N + 1, N + 1), 0.7, 2.0, 5) + 1.0 * np.exp(-((X - 14) ** 2 + (Y - 14) ** 2) / 30)
    eta = np.full_like(Z, Z.max() + 1.0)
    U0 = O.initial_state(Z, eta, True)
    bed = O.bed_from_corners(Z)
    prm = O.Params(nx=N, ny=N, dx=DX, dy=DX)
    rng = np.random.default_rng(11)
    man = torch.tensor(rng.uniform(0.02, 0.06, (N, N)), dtype=torch.float64)
    Q = torch.tensor([0.0, 3.0, 6.0, 2.0], dtype=torch.float64)
    target = torch.full((STEPS, len(GAUGES)), 1.2, dtype=torch.float64)
    return U0, bed, prm, man, Q, target


def _loss(U0, bed, prm, man, Q, target):
    p = O.Params(**{**prm.__dict__})
    p.manning = man
    p.inflows = [O.InflowBC(O.WEST, 5, 8, TQ, Q)]
    p.fixed_dt = DT
    U, t, J = U0.clone(), 0.0, 0.0
    for k in range(STEPS):
        U = O.step(U, t, bed, p, DT)
        t += DT
        h = O.sample_gauges(U, bed, p, GAUGES)[:, 0]
        J += float(((h - target[k]) ** 2).sum())
    return J


@pytest.fixture(scope="module")
def reference():
    U0, bed, prm, man, Q, target = _case()
    J, gn, gq = O.gauge_misfit_reference(U0, bed, prm, man, O.WEST, 5, 8, TQ, Q, DT, STEPS, GAUGES,
                                         target)
    return (U0, bed, prm, man, Q, target), J, gn, gq


def test_loss_matches_forward(reference):
    case, J, _, _ = reference
    assert float(J) == pytest.approx(_loss(*case), rel=1e-14)


def test_hydrograph_gradient_vs_central_differences(reference):
    (U0, bed, prm, man, Q, target), _, _, gq = reference
    eps = 1e-4
    for k in range(1, len(Q)):
        Qp, Qm = Q.clone(), Q.clone()
        Qp[k] += eps
        Qm[k] -= eps
        fd = (_loss(U0, bed, prm, man, Qp, target) - _loss(U0, bed, prm, man, Qm, target)) / (2 * eps)
        assert float(gq[k]) == pytest.approx(fd, rel=2e-5, abs=1e-12), k
    # Q[0] = 0 is left out: at t = 0 a zero discharge switches the inflow
    # face to a wall, so the loss is not differentiable in Q[0] there.


def test_manning_gradient_vs_central_differences(reference):
    (U0, bed, prm, man, Q, target), _, gn, _ = reference
    eps = 1e-5
    # cells next to the inflow, next to a gauge, and far from both
    for (j, i) in [(6, 0), (6, 1), (5, 8), (12, 12), (1, 12)]:
        mp, mm = man.clone(), man.clone()
        mp[j, i] += eps
        mm[j, i] -= eps
        fd = (_loss(U0, bed, prm, mp, Q, target) - _loss(U0, bed, prm, mm, Q, target)) / (2 * eps)
        scale = float(gn.abs().max())
        assert abs(float(gn[j, i]) - fd) <= 1e-4 * scale + 1e-12, (j, i, float(gn[j, i]), fd)
