"""Parity of the large-input path, on which a call runs the far field on a
second stream beside the tree, lists and near field (inputs of 2^18 points
and more), against the FP64 Ewald oracle at seeded samples of the targets:
separate targets with gradients, 2D, mixed precision, and a plan reused
across the size at which the second stream is taken."""
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
    return torch.tensor(a, device=dev)


def test_separate_targets_with_gradients(pdmk, torch_dev):
    L, src, q = workloads.clustered3d(200_000, seed=21)
    rng = np.random.default_rng(22)
    trg = rng.random((80_000, 3)) @ L.T            # 280,000 points in all
    pot, g = pdmk.pdmk_eval(L, _t(torch_dev, src), _t(torch_dev, q), trg=_t(torch_dev, trg),
                            eps=1e-6, grad=True, kappa=4.0)
    pot, g = pot.cpu().numpy(), g.cpu().numpy()
    idx = rng.choice(len(trg), 48, replace=False)
    ref, gref = ewald.ewald(L, src, q, trg=trg[idx], grad=True)
    assert ewald.rel_l2(pot[idx], ref) <= 1e-6
    assert ewald.rel_l2(g[idx], gref) <= 1e-5


def test_oblique_2d_large(pdmk, torch_dev):
    L, src, q = workloads.oblique2d(300_000, seed=23)
    pot = pdmk.pdmk_eval(L, _t(torch_dev, src), _t(torch_dev, q), eps=1e-6).cpu().numpy()
    idx = np.random.default_rng(24).choice(len(q), 48, replace=False)
    assert ewald.rel_l2(pot[idx], ewald.ewald_sampled(L, src, q, idx)) <= 1e-6


def test_mixed_large(pdmk, torch_dev):
    L, src, q = workloads.shell3d(400_000, seed=25)
    pot = pdmk.pdmk_eval(L, _t(torch_dev, src), _t(torch_dev, q), eps=1e-6,
                         precision="mixed").cpu().numpy()
    idx = np.random.default_rng(26).choice(len(q), 48, replace=False)
    assert ewald.rel_l2(pot[idx], ewald.ewald_sampled(L, src, q, idx)) <= 1e-6


def test_plan_reused_across_stream_threshold(pdmk, torch_dev):
    """One plan: small (one stream), large (two), small again; each result
    matches the oracle, and the large one is unchanged by the small calls."""
    rng = np.random.default_rng(27)
    L = workloads.shell3d(10, seed=28)[0]
    plan = pdmk.Plan(L, eps=1e-6)
    out = []
    for n in (5_000, 300_000, 5_000):
        src = rng.random((n, 3)) @ L.T
        q = rng.choice([-1.0, 1.0], n)
        q -= q.mean()
        pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
        idx = rng.choice(n, 32, replace=False)
        assert ewald.rel_l2(pot[idx], ewald.ewald_sampled(L, src, q, idx)) <= 1e-6
        out.append((src, q, pot))
    src, q, pot = out[1]
    again = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    assert np.abs(again - pot).max() <= 1e-12 * np.abs(pot).max()
