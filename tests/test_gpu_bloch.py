"""Quasi-periodic (Bloch) evaluation, pdmk_plan_eval_bloch (Section 4.1),
against the Bloch Ewald oracle (oracle/bloch.c, pinned in
test_oracle_bloch.py).

* triclinic / cubic 3D and oblique 2D cells, eps = 1e-3, 1e-6, 1e-9, FP64
  and mixed arithmetic, non-neutral charges (no neutrality is needed);
* sources and targets given outside the cell (literal positions: the phase
  of each wrap is carried), so quasi-periodicity is checked on the device;
* a Bloch vector comparable to c / r_c (the enlarged far-field grid);
* N = 3e5 clustered triclinic on 48 sampled sources;
* empty inputs and the entry points that reject Bloch plans.

E_rel = ||Phi - Phi_ref|| / ||Phi_ref|| over complex values.
"""
import numpy as np
import pytest

from oracle import ewald
from paper_2606_28608_amd import workloads

pytestmark = pytest.mark.gpu

BETA3 = np.array([0.7, -1.1, 0.4])
BETA2 = np.array([1.3, -0.6])


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


def _crel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(dim, cell, n, seed):
    if dim == 3:
        L, src, _ = workloads.clustered3d(n, seed=seed, cell=cell)
        beta = BETA3
    else:
        L, src, _ = workloads.oblique2d(n, seed=seed)
        beta = BETA2
    q = np.random.default_rng(seed + 100).standard_normal(n)   # not neutral
    return L, src, q, beta


# (dim, cell, eps, precision)
CASES = [(3, "triclinic", 1e-6, "fp64"), (3, "triclinic", 1e-9, "fp64"),
         (3, "triclinic", 1e-3, "fp64"), (3, "triclinic", 1e-6, "mixed"),
         (3, "cubic", 1e-6, "fp64"), (2, "oblique", 1e-6, "fp64"),
         (2, "oblique", 1e-9, "fp64"), (2, "oblique", 1e-6, "mixed")]


@pytest.mark.parametrize("dim,cell,eps,precision", CASES)
def test_bloch_matches_oracle(pdmk, torch_dev, dim, cell, eps, precision):
    L, src, q, beta = _case(dim, cell, 3000, seed=61)
    plan = pdmk.Plan(L, eps=eps, precision=precision, bloch=beta, kappa=3.0, n_s=60)
    got = plan.eval_bloch(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    ref = ewald.ewald_bloch(L, src, q, beta)
    err = _crel(got, ref)
    print("Bloch %dD %s eps=%g %s E_rel=%.3e" % (dim, cell, eps, precision, err))
    assert err <= eps


@pytest.mark.parametrize("dim", [3, 2])
def test_bloch_points_outside_the_cell(pdmk, torch_dev, dim):
    """Sources moved by whole lattice vectors and targets inside and outside
    the cell: every wrap carries its phase."""
    L, src, q, beta = _case(dim, "triclinic", 2500, seed=62)
    rng = np.random.default_rng(63)
    moved = src + rng.integers(-2, 3, size=src.shape) @ L.T
    trg = rng.random((600, dim)) @ L.T
    trg[::2] += rng.integers(-3, 4, size=(300, dim)) @ L.T
    plan = pdmk.Plan(L, eps=1e-6, bloch=beta, kappa=3.0, n_s=60)
    got = plan.eval_bloch(_t(torch_dev, moved), _t(torch_dev, q),
                          trg=_t(torch_dev, trg)).cpu().numpy()
    ref = ewald.ewald_bloch(L, moved, q, beta, trg=trg)
    assert _crel(got, ref) <= 1e-6
    # quasi-periodicity of the device result itself
    n = np.array([1, -2, 1][:dim], dtype=float)
    shifted = plan.eval_bloch(_t(torch_dev, moved), _t(torch_dev, q),
                              trg=_t(torch_dev, trg + L @ n)).cpu().numpy()
    assert _crel(shifted, np.exp(1j * beta @ (L @ n)) * got) <= 1e-9


def test_bloch_large_vector(pdmk, torch_dev):
    """|beta| comparable to c / r_c: the far-field grid of Section 4.1 grows
    and the result still meets eps."""
    L, src, q, _ = _case(3, "triclinic", 2000, seed=64)
    g = pdmk.geometry(L, eps=1e-6, kappa=3.0)
    beta = BETA3 / np.linalg.norm(BETA3) * 0.5 * g.c / g.rc
    plan = pdmk.Plan(L, eps=1e-6, bloch=beta, kappa=3.0, n_s=60)
    gb = pdmk.geometry(L, eps=1e-6, kappa=3.0, bloch=beta)
    assert all(gb.fgrid_paper[i] > g.fgrid_paper[i] for i in range(3))
    got = plan.eval_bloch(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    ref = ewald.ewald_bloch(L, src, q, beta)
    assert _crel(got, ref) <= 1e-6


def test_bloch_sampled_large(pdmk, torch_dev):
    L, src, q, beta = _case(3, "triclinic", 300_000, seed=65)
    plan = pdmk.Plan(L, eps=1e-6, bloch=beta)
    got = plan.eval_bloch(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    idx = np.random.default_rng(66).choice(len(q), 48, replace=False)
    ref = ewald.ewald_bloch_sampled(L, src, q, beta, idx)
    err = _crel(got[idx], ref)
    print("Bloch N=3e5 E_rel=%.3e" % err)
    assert err <= 1e-6


def test_bloch_empty_and_rejections(pdmk, torch_dev):
    torch, dev = torch_dev
    L, src, q, beta = _case(3, "triclinic", 500, seed=67)
    plan = pdmk.Plan(L, eps=1e-6, bloch=beta)
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    z = plan.eval_bloch(S[:0], Q[:0], trg=S[:5])
    assert z.shape == (5,) and bool((z == 0).all())
    assert plan.eval_bloch(S, Q, trg=S[:0]).shape == (0,)
    with pytest.raises(pdmk.PdmkError) as e:
        plan.eval(S, Q - Q.mean())   # the periodic entry point
    assert e.value.code == -9
    with pytest.raises(pdmk.PdmkError) as e:
        plan.bind(S, Q - Q.mean())
    assert e.value.code == -9
    per = pdmk.Plan(L, eps=1e-6)
    with pytest.raises(pdmk.PdmkError) as e:
        per.eval_bloch(S, Q)
    assert e.value.code == -1
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.Plan(L, eps=1e-6, bloch=beta, grad=True)
    assert e.value.code == -9
    bad = q.copy()
    bad[3] = np.inf
    with pytest.raises(pdmk.PdmkError) as e:
        plan.eval_bloch(S, _t(torch_dev, bad))
    assert e.value.code == -5
