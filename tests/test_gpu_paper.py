"""The paper's test cells and source distributions (Section 6): 2D oblique
(pi/3) cells of aspect ratio 1, 10, 100 with the wavy ring, 3D rectangular and
triclinic base cells (edges 1, sqrt2, sqrt3) in the isotropic, rod and slab
scalings with the wavy sphere, at eps = 1e-3, 1e-6, 1e-9, 1e-12 (FP64, the
default plan), against the Ewald oracle on sampled sources.

* N = 2e5 per cell, 32 sampled sources (the oracle takes about a second);
* N = 1e7 per cell at eps = 1e-6 and 1e-12 against the stored oracle values
  (tests/golden/paper_*, written by make_golden.py from the oracle only);
* Fourier axes longer than one LDS line (four-step transforms): the aspect-100
  cell below eps = 1e-3 (one long axis), and a small cell with a large kappa
  (both axes long).
"""
import functools
import os

import numpy as np
import pytest

from oracle import ewald
from paper_2606_28608_amd import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NAMES = list(workloads.PAPER_SYSTEMS)
EPS = [1e-3, 1e-6, 1e-9, 1e-12]


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


@functools.lru_cache(maxsize=None)
def _system(name, n):
    L, src, q = workloads.paper_system(name, n)
    idx = np.random.default_rng(5).choice(n, 32, replace=False)
    return L, src, q, idx, ewald.ewald_sampled(L, src, q, idx)


@pytest.mark.parametrize("eps", EPS)
@pytest.mark.parametrize("name", NAMES)
def test_paper_cells(pdmk, torch_dev, name, eps):
    L, src, q, idx, ref = _system(name, 200_000)
    plan = pdmk.Plan(L, eps=eps)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    err = ewald.rel_l2(pot[idx], ref)
    print("%s eps=%g E_rel=%.3e fgrid=%s" % (name, eps, err, list(plan.geometry().fgrid)))
    assert err <= eps


@pytest.mark.parametrize("eps", [1e-6, 1e-12])
@pytest.mark.parametrize("name", NAMES)
def test_paper_cells_full_size(pdmk, torch_dev, name, eps):
    path = os.path.join(HERE, "golden", "paper_%s_n1e7_seed8.txt" % name)
    if not os.path.exists(path):
        pytest.skip("stored oracle values not written")
    data = np.loadtxt(path)
    idx, ref = data[:, 0].astype(np.int64), data[:, 1]
    L, src, q = workloads.paper_system(name, 10_000_000)
    plan = pdmk.Plan(L, eps=eps)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    err = ewald.rel_l2(pot[idx], ref)
    print("%s N=1e7 eps=%g E_rel=%.3e" % (name, eps, err))
    assert err <= eps


def test_long_axis_is_split(pdmk):
    g = pdmk.geometry(workloads.oblique_pi3(100.0), eps=1e-12)
    assert max(g.fgrid[:2]) > 4096


def test_two_long_axes(pdmk, torch_dev):
    """kappa = 800 on an oblique cell of aspect 1: both Fourier axes exceed
    4096 points, so both (the contiguous and the strided one) take the
    four-step transform."""
    L, src, q = workloads.oblique2d(2000, seed=71)
    g = pdmk.geometry(L, eps=1e-6, kappa=800.0)
    assert min(g.fgrid[:2]) > 4096
    plan = pdmk.Plan(L, eps=1e-6, kappa=800.0, n_s=40)
    pot = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    err = ewald.rel_l2(pot, ewald.ewald(L, src, q))
    print("two long axes fgrid=%s E_rel=%.3e" % (list(g.fgrid[:2]), err))
    assert err <= 1e-6
