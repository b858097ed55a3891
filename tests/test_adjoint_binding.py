"""Host logic of the torch binding of the adjoint (paper_2010_02003_amd.adjoint).

The library keeps the checkpoints of its last forward run only.  Two nodes
made with one Adjoint (two losses in one graph) must still each get the
gradient at their own parameters.  A stand-in Adjoint with the library's
calling convention checks this on the CPU: its backward returns the
gradient of a known function at the parameters of its *last* forward run,
so a binding that forgot to repeat a node's forward run returns the other
node's gradient.
"""
import numpy as np
import torch

from paper_2010_02003_amd.adjoint import DG2Loss, GaugeDepths


class FakeAdjoint:
    """h[k, g] = (k + 1) * sum(n) * (g + 1) + sum(Q); backward at the last forward's (n, Q)."""

    def __init__(self, steps=3, ng=2, shape=(4, 6), nq=5):
        self.steps, self.ng, self.shape, self.nq = steps, ng, shape, nq
        self.generation = 0
        self.forwards = 0
        self._last = None

    def forward(self, n, q):
        n = np.array(n, dtype=np.float64)
        q = np.zeros(self.nq) if q is None else np.array(q, dtype=np.float64)
        self._last = (n, q)
        self.generation += 1
        self.forwards += 1
        k = np.arange(1, self.steps + 1)[:, None]
        g = np.arange(1, self.ng + 1)[None, :]
        return k * g * n.sum() + q.sum() + 0.0 * k * g

    def backward(self, dL_dh):
        n, q = self._last
        k = np.arange(1, self.steps + 1)[:, None]
        g = np.arange(1, self.ng + 1)[None, :]
        # dh/dn_cell = k g (every cell alike), dh/dQ_i = 1; plus a term that depends on
        # the parameters of the last run, so a stale run gives a wrong gradient
        gn = np.full(self.shape, float((dL_dh * k * g).sum())) + n
        gq = np.full(self.nq, float(dL_dh.sum())) + q
        return gn, gq


def _expected(fake, n, q, dL_dh):
    k = np.arange(1, fake.steps + 1)[:, None]
    g = np.arange(1, fake.ng + 1)[None, :]
    return (np.full(fake.shape, float((dL_dh * k * g).sum())) + n,
            np.full(fake.nq, float(dL_dh.sum())) + q)


def test_two_gauge_depth_nodes_each_get_their_own_gradient():
    fake = FakeAdjoint()
    rng = np.random.default_rng(0)
    n1 = torch.tensor(rng.uniform(0.02, 0.06, fake.shape), requires_grad=True)
    n2 = torch.tensor(rng.uniform(0.02, 0.06, fake.shape), requires_grad=True)
    q1 = torch.tensor(rng.uniform(0, 5, fake.nq), requires_grad=True)
    q2 = torch.tensor(rng.uniform(0, 5, fake.nq), requires_grad=True)
    h1 = GaugeDepths.apply(n1, q1, fake)
    h2 = GaugeDepths.apply(n2, q2, fake)  # the library now holds run 2
    w1 = torch.tensor(rng.normal(size=h1.shape))
    w2 = torch.tensor(rng.normal(size=h2.shape))
    ((h1 * w1).sum() + (h2 * w2).sum()).backward()
    e1n, e1q = _expected(fake, n1.detach().numpy(), q1.detach().numpy(), w1.numpy())
    e2n, e2q = _expected(fake, n2.detach().numpy(), q2.detach().numpy(), w2.numpy())
    # each parameter got its own node's gradient (order of the backward calls is torch's)
    assert np.allclose(n1.grad.numpy(), e1n) and np.allclose(q1.grad.numpy(), e1q)
    assert np.allclose(n2.grad.numpy(), e2n) and np.allclose(q2.grad.numpy(), e2q)
    assert fake.forwards >= 3  # at least one repeated forward run


def test_single_node_does_not_repeat_its_forward_run():
    fake = FakeAdjoint()
    n = torch.full(fake.shape, 0.03, dtype=torch.float64, requires_grad=True)
    q = torch.ones(fake.nq, dtype=torch.float64, requires_grad=True)
    GaugeDepths.apply(n, q, fake).sum().backward()
    assert fake.forwards == 1


def test_dg2_loss_after_a_validation_forward_run():
    fake = FakeAdjoint(shape=(4, 4))
    nb = torch.tensor([[0.03, 0.05], [0.04, 0.02]], dtype=torch.float64, requires_grad=True)
    q = torch.ones(fake.nq, dtype=torch.float64, requires_grad=True)
    target = np.zeros((fake.steps, fake.ng))
    J = DG2Loss.apply(nb, q, fake, target, 2)  # blocks of 2 x 2 cells
    n_cell = np.kron(nb.detach().numpy(), np.ones((2, 2)))
    h = fake.forward(n_cell, q.detach().numpy())  # what the node's forward run gave
    fake.forward(np.full((4, 4), 0.09), np.zeros(fake.nq))  # a validation run in between
    J.backward()
    en, eq = _expected(fake, n_cell, q.detach().numpy(), 2.0 * (h - target))
    assert np.allclose(nb.grad.numpy(), en.reshape(2, 2, 2, 2).sum(axis=(1, 3)))
    assert np.allclose(q.grad.numpy(), eq)
