"""Each half of the split on its own (pdmk_plan_eval_parts) against the
oracle's halves (oracle/split.py): the near field against the finite sum of
G - W_0 over every image within r_c minus the self terms W_0(0) q, the far
field against the direct Fourier sum of eq:W0p over the modes of eq:Mi.
Both halves depend on the split's bandwidth c (only their sum does not), so
the oracle evaluates the split at the plan's c; its own calibration of c
(psi(1)/psi(0) = eps, pinned in test_oracle_split.py) must agree with it, and
so must r_c and the eq:Mi grid.  A compensating error between the stages
would show here and not in the end-to-end tests.  Errors are measured
against the norm of the whole potential: ||part - part_ref|| <= eps ||Phi||."""
import numpy as np
import pytest

from oracle import ewald, split
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


CASES = [("triclinic", 1e-6, "fp64"), ("triclinic", 1e-9, "fp64"), ("cubic", 1e-6, "fp64"),
         ("triclinic", 1e-6, "mixed"), ("oblique2d", 1e-6, "fp64")]


@pytest.mark.parametrize("cell,eps,precision", CASES)
def test_near_and_far_halves(pdmk, torch_dev, cell, eps, precision):
    if cell == "oblique2d":
        L, src, q = workloads.oblique2d(600, seed=81)
        kappa, n_s = 7.0, 2
    else:
        L, src, q = workloads.clustered3d(600, seed=82, cell=cell)
        kappa, n_s = 3.0, 20
    d = L.shape[0]
    plan = pdmk.Plan(L, eps=eps, precision=precision, kappa=kappa, n_s=n_s)
    g = plan.geometry()
    assert abs(g.rc - split.root_side(L, kappa)) <= 1e-13 * g.rc
    assert abs(g.c - split.calibrate(eps).c) <= 1e-6 * g.c
    assert sorted(split.fourier_grid(L, g.c, g.rc)) == sorted(list(g.fgrid_paper)[:d])
    near, far = plan.eval_parts(_t(torch_dev, src), _t(torch_dev, q))
    near, far = near.cpu().numpy(), far.cpu().numpy()
    near_ref = split.near_part(L, src, q, eps, kappa, c=g.c)
    far_ref = split.far_part(L, src, q, eps, kappa, c=g.c)
    tot = ewald.ewald(L, src, q)
    scale = np.linalg.norm(tot)
    e_near = np.linalg.norm(near - near_ref) / scale
    e_far = np.linalg.norm(far - far_ref) / scale
    print("%s eps=%g %s: near %.3e far %.3e" % (cell, eps, precision, e_near, e_far))
    assert e_near <= eps
    assert e_far <= eps
    assert ewald.rel_l2(near + far, tot) <= eps
    # the tree had several levels (plane waves took part in the near half)
    assert plan.stats()["n_levels"] >= 3
