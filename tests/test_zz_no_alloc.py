"""The allocation-free entry point pdmk_plan_eval_noalloc (the library's
fixed device scratch as workspace) against pdmk_plan_eval on the same plan and
input: bitwise equal under PDMK_DETERMINISTIC (same kernels, same order), on
two calls in a row, the second with a smaller input; both within eps of the
oracle.  An input too large for the scratch is rejected with
PDMK_ERR_SCRATCH and the outputs stay unwritten."""
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_eval(pdmk, torch_dev, precision):
    torch, dev = torch_dev
    plan = pdmk.Plan(workloads.TRICLINIC3D_L, eps=1e-6, precision=precision, grad=True,
                     deterministic=True)
    for n, seed in ((8000, 71), (2000, 72)):   # second call: smaller input
        L, src, q = workloads.clustered3d(n, seed=seed)
        S, Q = _t(torch_dev, src), _t(torch_dev, q)
        pot = torch.full((n,), 7.0, dtype=torch.float64, device=dev)
        grad = torch.full((n, 3), 7.0, dtype=torch.float64, device=dev)
        plan.eval_noalloc(S, Q, pot, grad)
        pe, ge = plan.eval(S, Q)
        assert np.array_equal(pot.cpu().numpy(), pe.cpu().numpy())
        assert np.array_equal(grad.cpu().numpy(), ge.cpu().numpy())
        ref, gref = ewald.ewald(L, src, q, grad=True)
        assert ewald.rel_l2(pot.cpu().numpy(), ref) <= 1e-6
        assert ewald.rel_l2(grad.cpu().numpy(), gref) <= 1e-5


def test_noalloc_separate_targets_and_2d(pdmk, torch_dev):
    torch, dev = torch_dev
    L, src, q = workloads.clustered3d(4000, seed=73)
    trg = np.random.default_rng(74).random((900, 3)) @ L.T
    plan = pdmk.Plan(L, eps=1e-6, deterministic=True)
    pot = torch.empty(900, dtype=torch.float64, device=dev)
    plan.eval_noalloc(_t(torch_dev, src), _t(torch_dev, q), pot, trg=_t(torch_dev, trg))
    pe = plan.eval(_t(torch_dev, src), _t(torch_dev, q), trg=_t(torch_dev, trg))
    assert np.array_equal(pot.cpu().numpy(), pe.cpu().numpy())
    L2, s2, q2 = workloads.oblique2d(2000, seed=75)
    plan2 = pdmk.Plan(L2, eps=1e-6, deterministic=True)
    pot2 = torch.empty(2000, dtype=torch.float64, device=dev)
    plan2.eval_noalloc(_t(torch_dev, s2), _t(torch_dev, q2), pot2)
    assert ewald.rel_l2(pot2.cpu().numpy(), ewald.ewald(L2, s2, q2)) <= 1e-6


def test_noalloc_rejects_inputs_beyond_the_scratch(pdmk, torch_dev):
    torch, dev = torch_dev
    for n in (2_000_000, 200_000):   # host pre-check, and a failure inside the pipeline
        L, src, q = workloads.clustered3d(n, seed=76)
        plan = pdmk.Plan(L, eps=1e-6)
        pot = torch.full((n,), 7.0, dtype=torch.float64, device=dev)
        with pytest.raises(pdmk.PdmkError) as e:
            plan.eval_noalloc(_t(torch_dev, src), _t(torch_dev, q), pot)
        assert e.value.code == -10
        assert bool((pot == 7.0).all())
    # the scratch still serves a small input afterwards
    L, src, q = workloads.clustered3d(2000, seed=77)
    plan = pdmk.Plan(L, eps=1e-6)
    pot = torch.empty(2000, dtype=torch.float64, device=dev)
    plan.eval_noalloc(_t(torch_dev, src), _t(torch_dev, q), pot)
    assert ewald.rel_l2(pot.cpu().numpy(), ewald.ewald(L, src, q)) <= 1e-6
