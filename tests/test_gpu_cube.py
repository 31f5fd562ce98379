"""The cube-cell construction of rem:cube (PDMK_VIRTUAL_IMAGES): the root
cubes tile the cell, colleagues across a face are the boxes of the other side
shifted by L n, and no image point exists.

* cubes at kappa = 4 (the paper's r_c = side / 4) and 3, eps = 1e-3 .. 1e-12,
  clustered and uniform sources, against the oracle;
* kappa = 1 and 2 (one or two root cubes per axis: a box is its own
  colleague under several shifts);
* commensurate rectangular cells in 3D and 2D, separate targets, gradients,
  mixed precision, a kept tree with displaced positions, deterministic mode;
* the image count equals N (no halo) and the result agrees with the
  physical-image path on the same cell.
"""
import numpy as np
import pytest

from oracle import ewald
from paper_2606_28608_amd import workloads

pytestmark = pytest.mark.gpu


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


def _uniform(L, n, seed):
    rng = np.random.default_rng(seed)
    d = L.shape[0]
    q = rng.standard_normal(n)
    return (rng.random((n, d)) @ L.T), q - q.mean()


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9, 1e-12])
@pytest.mark.parametrize("kappa", [4.0, 3.0])
def test_cube_clustered(pdmk, torch_dev, eps, kappa):
    L, src, q = workloads.clustered3d(6000, seed=91, cell="cubic")
    plan = pdmk.Plan(L, eps=eps, kappa=kappa, n_s=60, virtual_images=True)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    st = plan.stats()
    assert st["n_images"] == len(q)
    err = ewald.rel_l2(pot, ewald.ewald(L, src, q))
    print("cube kappa=%g eps=%g E_rel=%.3e levels=%d" % (kappa, eps, err, st["n_levels"]))
    assert err <= eps
    ref = pdmk.Plan(L, eps=eps, kappa=kappa, n_s=60).eval(_t(torch_dev, src),
                                                          _t(torch_dev, q)).cpu().numpy()
    assert ewald.rel_l2(pot, ref) <= eps


@pytest.mark.parametrize("kappa", [1.0, 2.0])
def test_cube_few_roots(pdmk, torch_dev, kappa):
    L = 1.7 * np.eye(3)
    src, q = _uniform(L, 3000, seed=92)
    plan = pdmk.Plan(L, eps=1e-6, kappa=kappa, n_s=50, virtual_images=True)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    assert ewald.rel_l2(pot, ewald.ewald(L, src, q)) <= 1e-6


@pytest.mark.parametrize("dim", [3, 2])
def test_rectangular_commensurate(pdmk, torch_dev, dim):
    L = np.diag([1.0, 2.0, 3.0]) if dim == 3 else np.diag([1.0, 3.0])
    src, q = _uniform(L, 4000, seed=93)
    trg = np.random.default_rng(94).random((500, dim)) @ L.T - 0.3
    plan = pdmk.Plan(L, eps=1e-9, kappa=3.0, n_s=50, virtual_images=True)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    assert ewald.rel_l2(pot, ewald.ewald(L, src, q)) <= 1e-9
    pt = plan.eval(_t(torch_dev, src), _t(torch_dev, q), trg=_t(torch_dev, trg)).cpu().numpy()
    assert ewald.rel_l2(pt, ewald.ewald(L, src, q, trg=trg)) <= 1e-9


def test_cube_gradient_mixed_kept(pdmk, torch_dev):
    L, src, q = workloads.clustered3d(5000, seed=95, cell="cubic")
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    ref, gref = ewald.ewald(L, src, q, grad=True)
    plan = pdmk.Plan(L, eps=1e-6, grad=True, kappa=4.0, n_s=60, virtual_images=True)
    pot, g = plan.eval(S, Q)
    assert ewald.rel_l2(pot.cpu().numpy(), ref) <= 1e-6
    assert ewald.rel_l2(g.cpu().numpy(), gref) <= 1e-5
    pm = pdmk.Plan(L, eps=1e-6, precision="mixed", kappa=4.0, n_s=60,
                   virtual_images=True).eval(S, Q).cpu().numpy()
    assert ewald.rel_l2(pm, ref) <= 1e-6
    kept = pdmk.Plan(L, eps=1e-6, kappa=4.0, n_s=60, virtual_images=True)
    kept.bind(S, Q)
    moved = src + 1e-4 * np.random.default_rng(96).standard_normal(src.shape)
    got = kept.execute(Q, src=_t(torch_dev, moved)).cpu().numpy()
    kept.status()
    assert ewald.rel_l2(got, ewald.ewald(L, moved, q)) <= 1e-6


def test_cube_deterministic(pdmk, torch_dev):
    L, src, q = workloads.clustered3d(8000, seed=97, cell="cubic")
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    plan = pdmk.Plan(L, eps=1e-6, kappa=4.0, n_s=60, virtual_images=True, deterministic=True)
    a = plan.eval(S, Q).cpu().numpy()
    b = plan.eval(S, Q).cpu().numpy()
    assert np.array_equal(a, b)
    assert ewald.rel_l2(a, ewald.ewald(L, src, q)) <= 1e-6


def test_cube_large_sampled(pdmk, torch_dev):
    """N = 1e6 clustered in the unit cube, kappa = 4, eps = 1e-6: the image
    count is N, and 48 sampled sources meet eps."""
    L, src, q = workloads.clustered3d(1_000_000, seed=98, cell="cubic")
    plan = pdmk.Plan(L, eps=1e-6, kappa=4.0, virtual_images=True)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    assert plan.stats()["n_images"] == len(q)
    idx = np.random.default_rng(99).choice(len(q), 48, replace=False)
    assert ewald.rel_l2(pot[idx], ewald.ewald_sampled(L, src, q, idx)) <= 1e-6
