"""Adjoint and autograd of the HIP periodic-DMK path against the FP64 Ewald oracle.

For a loss l with g = dl/dPhi the kernel's symmetry makes the adjoint one more
evaluation with the roles of sources and targets swapped (Psi = potential of
the charges g at the targets, with a uniform background when sum g != 0):
dq = Psi(y), dy = q grad Psi(y) (+ g grad Phi(y) when targets are sources),
dx = g grad Phi(x).  Every reference below is built from oracle potentials and
gradients only; gradient accuracy is not stated by the method, so positions
are held to 10 eps (relative l2) and potentials to eps.
"""
import os

import numpy as np
import pytest

from oracle import ewald
from paper_2606_28608_amd import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def pdmk():
    from paper_2606_28608_amd import pdmk as m
    m.lib()
    return m


def _t(torch_dev, a):
    torch, dev = torch_dev
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("dim", [3, 2])
def test_adjoint_targets_are_sources(pdmk, torch_dev, dim):
    eps = 1e-6
    if dim == 3:
        L, src, q = workloads.clustered3d(3000, seed=21)
        over = dict(kappa=2.0, n_s=60)
    else:
        L, src, q = workloads.oblique2d(2000, seed=22)
        over = dict(n_s=20)
    g = np.random.default_rng(23).standard_normal(len(q))   # not neutral
    phi, gphi = ewald.ewald(L, src, q, grad=True)
    psi, gpsi = ewald.ewald(L, src, g, grad=True)
    plan = pdmk.Plan(L, eps=eps, grad=True, **over)
    S, Q, G = _t(torch_dev, src), _t(torch_dev, q), _t(torch_dev, g)
    pot, grad = plan.eval(S, Q, want_grad=True)
    assert ewald.rel_l2(pot.cpu().numpy(), phi) <= eps
    dq, ds, _ = plan.adjoint(S, Q, G, grad_phi=grad)
    assert ewald.rel_l2(dq.cpu().numpy(), psi) <= eps
    ref = g[:, None] * gphi + q[:, None] * gpsi
    assert ewald.rel_l2(ds.cpu().numpy(), ref) <= 10 * eps


def test_adjoint_separate_targets(pdmk, torch_dev):
    eps = 1e-6
    L, src, q = workloads.clustered3d(2000, seed=24)
    trg = np.random.default_rng(25).random((700, 3)) @ L.T
    g = np.random.default_rng(26).standard_normal(700)
    phi, gphi = ewald.ewald(L, src, q, trg=trg, grad=True)
    # Psi at the sources: charges g at the targets
    psi, gpsi = ewald.ewald(L, trg, g, trg=src, grad=True)
    plan = pdmk.Plan(L, eps=eps, grad=True, kappa=2.0, n_s=60)
    S, Q, T, G = (_t(torch_dev, a) for a in (src, q, trg, g))
    pot, grad = plan.eval(S, Q, trg=T, want_grad=True)
    assert ewald.rel_l2(pot.cpu().numpy(), phi) <= eps
    dq, ds, dt = plan.adjoint(S, Q, G, trg=T, grad_phi=grad, want_dtrg=True)
    assert ewald.rel_l2(dq.cpu().numpy(), psi) <= eps
    assert ewald.rel_l2(ds.cpu().numpy(), q[:, None] * gpsi) <= 10 * eps
    assert ewald.rel_l2(dt.cpu().numpy(), g[:, None] * gphi) <= 10 * eps


def test_autograd_function(pdmk, torch_dev):
    """torch.autograd through periodic_potential equals the adjoint formulas
    built from oracle values, and reciprocity sum g Phi = sum q Psi holds."""
    torch, dev = torch_dev
    eps = 1e-6
    L, src, q = workloads.clustered3d(2500, seed=27)
    w = np.random.default_rng(28).standard_normal(len(q))
    phi, gphi = ewald.ewald(L, src, q, grad=True)
    psi, gpsi = ewald.ewald(L, src, w, grad=True)
    plan = pdmk.Plan(L, eps=eps, grad=True, kappa=2.0, n_s=60)
    S = _t(torch_dev, src).requires_grad_(True)
    Q = _t(torch_dev, q).requires_grad_(True)
    W = _t(torch_dev, w)
    pot = pdmk.periodic_potential(plan, S, Q)
    loss = (W * pot).sum()
    loss.backward()
    assert ewald.rel_l2(pot.detach().cpu().numpy(), phi) <= eps
    assert ewald.rel_l2(Q.grad.cpu().numpy(), psi) <= eps
    ref = w[:, None] * gphi + q[:, None] * gpsi
    assert ewald.rel_l2(S.grad.cpu().numpy(), ref) <= 10 * eps
    # reciprocity of the two evaluations (exact for the operator, eps for the method)
    lhs = float(loss.detach().cpu())
    rhs = float(np.dot(q, Q.grad.cpu().numpy()))
    assert abs(lhs - rhs) <= 10 * eps * np.linalg.norm(w) * np.linalg.norm(phi)
    # only charges need gradients: the forward skips grad Phi
    Q2 = _t(torch_dev, q).requires_grad_(True)
    pot2 = pdmk.periodic_potential(plan, _t(torch_dev, src), Q2)
    (W * pot2).sum().backward()
    assert ewald.rel_l2(Q2.grad.cpu().numpy(), psi) <= eps


def test_forces_full_size_golden(pdmk, torch_dev):
    """C2/C4 workload at N=1e6 (clustered triclinic): potential and gradient at
    64 sampled sources against stored oracle values."""
    path = os.path.join(HERE, "golden", "clustered3d_n1e6_seed2_grad.txt")
    if not os.path.exists(path):
        pytest.skip("stored oracle gradients not generated")
    data = np.loadtxt(path)
    idx = data[:, 0].astype(np.int64)
    L, src, q = workloads.clustered3d(1_000_000, seed=2)
    plan = pdmk.Plan(L, eps=1e-6, grad=True, kappa=7.0)
    pot, grad = plan.eval(_t(torch_dev, src), _t(torch_dev, q))
    assert ewald.rel_l2(pot.cpu().numpy()[idx], data[:, 1]) <= 1e-6
    assert ewald.rel_l2(grad.cpu().numpy()[idx], data[:, 2:5]) <= 1e-5


def test_adjoint_argument_errors(pdmk, torch_dev):
    L, src, q = workloads.clustered3d(200, seed=29)
    plan = pdmk.Plan(L, eps=1e-3)
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    with pytest.raises(pdmk.PdmkError) as e:
        plan.adjoint(S, Q, Q, grad_phi=None, want_dsrc=True)   # needs grad_phi
    assert e.value.code == -1
    with pytest.raises(ValueError):
        plan.adjoint(S, Q, Q[:10])


def test_autograd_positions_against_finite_differences(pdmk, torch_dev):
    """d(sum w Phi)/dy from the adjoint against central differences of the
    GPU forward itself (FP64, eps = 1e-9), for 12 coordinates.  A tree
    change between the two shifted evaluations moves the result by at most
    eps |Phi|, i.e. eps |Phi| / h in the difference quotient."""
    torch, dev = torch_dev
    eps, h = 1e-9, 1e-5
    L, src, q = workloads.clustered3d(3000, seed=31)
    w = np.random.default_rng(32).standard_normal(len(q))
    plan = pdmk.Plan(L, eps=eps, grad=True, kappa=2.0, n_s=60)
    W = _t(torch_dev, w)
    S = _t(torch_dev, src).requires_grad_(True)
    loss = (W * pdmk.periodic_potential(plan, S, _t(torch_dev, q))).sum()
    loss.backward()
    g = S.grad.cpu().numpy()

    def f(x):
        pot = plan.eval(_t(torch_dev, x), _t(torch_dev, q), want_grad=False)
        return float(np.dot(w, pot.cpu().numpy()))

    rng = np.random.default_rng(33)
    for i in rng.choice(len(q), 4, replace=False):
        for a in range(3):
            xp, xm = src.copy(), src.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = (f(xp) - f(xm)) / (2 * h)
            assert abs(fd - g[i, a]) <= 1e-4 * np.abs(g).max(), (i, a, fd, g[i, a])
