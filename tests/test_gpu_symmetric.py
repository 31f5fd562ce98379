"""Residual pairs evaluated once (targets = sources, no gradients): the pair
kernel R_h depends on |x - y| alone, so a pair of points in two different
leaves is summed by the leaf that comes first in source order and added to
both ends; PDMK_ALL_PAIRS evaluates every pair from both ends.

* the two agree to rounding and both meet eps against the oracle: triclinic
  cells with image halos (default kappa; halo copies stay one-way), the cube
  construction (virtual colleagues: the mirror pair under the opposite
  shift), 2D, leaves with few targets (several lanes per target), mixed
  precision, Bloch conditions;
* the once-only lists hold about half the pairs;
* modes that keep both-way lists (gradients, deterministic, separate
  targets, kept trees) give the same results as before.
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


def _both(pdmk, torch_dev, L, src, q, **kw):
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    once = pdmk.Plan(L, **kw)
    a = once.eval(S, Q).cpu().numpy()
    sa = once.stats()
    both = pdmk.Plan(L, all_pairs=True, **kw)
    b = both.eval(S, Q).cpu().numpy()
    sb = both.stats()
    return a, b, sa, sb


CASES = [
    # (name, workload, plan options)
    ("triclinic-halo", lambda: workloads.clustered3d(20000, seed=201), dict(eps=1e-6)),
    ("triclinic-halo-1e-9", lambda: workloads.clustered3d(12000, seed=202), dict(eps=1e-9)),
    ("cube-virtual", lambda: workloads.clustered3d(12000, seed=203, cell="cubic"),
     dict(eps=1e-6, kappa=4.0, n_s=60, virtual_images=True)),
    ("few-targets", lambda: workloads.clustered3d(15000, seed=204),
     dict(eps=1e-6, n_s=12)),
    ("oblique-2d", lambda: workloads.oblique2d(6000, seed=205), dict(eps=1e-9)),
    ("oblique-2d-few", lambda: workloads.oblique2d(6000, seed=206), dict(eps=1e-6, n_s=10)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make,opts", CASES, ids=[c[0] for c in CASES])
def test_once_matches_both_ways_and_oracle(pdmk, torch_dev, name, make, opts, precision):
    if precision == "mixed" and opts["eps"] < 1e-8:
        pytest.skip("mixed plans compute in FP64 below eps 1e-8")
    L, src, q = make()
    a, b, sa, sb = _both(pdmk, torch_dev, L, src, q, precision=precision, **opts)
    ref = ewald.ewald(L, src, q)
    ea, eb = ewald.rel_l2(a, ref), ewald.rel_l2(b, ref)
    diff = ewald.rel_l2(a, b)
    print("%s %s: once %.3e both %.3e diff %.3e pairs %d / %d" % (
        name, precision, ea, eb, diff, sa["n_direct_pairs"], sb["n_direct_pairs"]))
    assert ea <= opts["eps"] and eb <= opts["eps"]
    # the same sums in another order: FP64 rounding; in mixed mode each side
    # carries its own FP32 residual error (a few 1e-7 at eps = 1e-6)
    assert diff <= (1e-13 if precision == "fp64" else opts["eps"])
    # the once-only lists hold the leaves' own boxes plus half of the rest
    assert sa["n_direct_pairs"] < 0.7 * sb["n_direct_pairs"]
    assert sa["n_images"] == sb["n_images"]


def test_shell_tuned_plan_golden(pdmk, torch_dev):
    """The benchmark's shell (N = 1e7, eps = 1e-6) at the planned kappa = 6,
    n_s = 300 / 400: once-only evaluation against the stored oracle values,
    both precisions."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "shell3d_n1e7_seed3.txt")
    data = np.loadtxt(path)
    idx, refv = data[:, 0].astype(np.int64), data[:, 1]
    L, src, q = workloads.shell3d()
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    for prec, ns in (("mixed", 300), ("mixed", 400), ("fp64", 400)):
        plan = pdmk.Plan(L, eps=1e-6, precision=prec, kappa=6.0, n_s=ns)
        pot = plan.eval(S, Q).cpu().numpy()
        err = ewald.rel_l2(pot[idx], refv)
        st = plan.stats()
        print("shell %s n_s=%d E_rel=%.3e pairs %d in support %d" % (
            prec, ns, err, st["n_direct_pairs"], st["n_support_pairs"]))
        assert err <= 1e-6


def test_both_way_modes_unchanged(pdmk, torch_dev):
    """Gradients, deterministic mode, separate targets and kept trees keep the
    both-way lists; their results agree with the once-only evaluation."""
    L, src, q = workloads.clustered3d(8000, seed=207)
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    once = pdmk.Plan(L, eps=1e-9).eval(S, Q).cpu().numpy()
    pg, _ = pdmk.Plan(L, eps=1e-9, grad=True).eval(S, Q)
    det = pdmk.Plan(L, eps=1e-9, deterministic=True).eval(S, Q).cpu().numpy()
    kept = pdmk.Plan(L, eps=1e-9)
    kept.bind(S, Q)
    kv = kept.execute(Q).cpu().numpy()
    for other in (pg.cpu().numpy(), det, kv):
        assert ewald.rel_l2(once, other) <= 1e-9
    assert ewald.rel_l2(once, ewald.ewald(L, src, q)) <= 1e-9
    # separate targets (off the sources: a target on a source keeps that
    # source's smooth self term) sum one way
    trg = src + 1e-3 * np.random.default_rng(208).standard_normal(src.shape)
    sep = pdmk.Plan(L, eps=1e-9).eval(S, Q, trg=_t(torch_dev, trg)).cpu().numpy()
    assert ewald.rel_l2(sep, ewald.ewald(L, src, q, trg=trg)) <= 1e-9


@pytest.mark.parametrize("dim,precision", [(3, "fp64"), (3, "mixed"), (2, "fp64")])
def test_bloch_once_matches_both_ways_and_oracle(pdmk, torch_dev, dim, precision):
    """Bloch conditions: each near pass is a plain sum over the phased image
    charges, so the pairs of two unshifted points are evaluated once there
    too, the source end taking its own image's charge in each pass."""
    rng = np.random.default_rng(209)
    if dim == 3:
        L, src, _ = workloads.clustered3d(6000, seed=209)
        beta = np.array([0.7, -1.1, 0.4])
    else:
        L, src, _ = workloads.oblique2d(4000, seed=209)
        beta = np.array([0.9, -0.6])
    q = rng.standard_normal(len(src))
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    opts = dict(eps=1e-6, precision=precision, bloch=beta, kappa=3.0, n_s=60)
    once = pdmk.Plan(L, **opts)
    a = once.eval_bloch(S, Q).cpu().numpy()
    assert once.stats()["pairs_once"] == 1
    both = pdmk.Plan(L, all_pairs=True, **opts)
    b = both.eval_bloch(S, Q).cpu().numpy()
    assert both.stats()["pairs_once"] == 0
    ref = ewald.ewald_bloch(L, src, q, beta)
    rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
    print("Bloch %dD %s: once %.3e both %.3e diff %.3e" % (dim, precision, rel(a, ref),
                                                           rel(b, ref), rel(a, b)))
    assert rel(a, ref) <= 1e-6 and rel(b, ref) <= 1e-6
    assert rel(a, b) <= (1e-13 if precision == "fp64" else 1e-6)


def test_kept_tree_pairs_once(pdmk, torch_dev):
    """A kept tree of a plan without gradients keeps the once-only lists: its
    executes (new charges, displaced points) match the one-shot evaluation and
    the oracle; an execute asking for gradients is rejected; a plan made with
    gradients keeps both-way lists and executes with them."""
    L, src, q = workloads.clustered3d(8000, seed=210)
    S, Q = _t(torch_dev, src), _t(torch_dev, q)
    q2 = np.random.default_rng(211).standard_normal(len(q))
    q2 -= q2.mean()
    plan = pdmk.Plan(L, eps=1e-9)
    plan.bind(S, Q)
    assert plan.stats()["pairs_once"] == 1
    got = plan.execute(_t(torch_dev, q2)).cpu().numpy()
    plan.status()
    ref = ewald.ewald(L, src, q2)
    assert ewald.rel_l2(got, ref) <= 1e-9
    one = pdmk.Plan(L, eps=1e-9).eval(S, _t(torch_dev, q2)).cpu().numpy()
    assert ewald.rel_l2(got, one) <= 1e-10   # kept executes use the hand-written axis kernels
    moved = src + 1e-5 * np.random.default_rng(212).standard_normal(src.shape)
    gm = plan.execute(_t(torch_dev, q2), src=_t(torch_dev, moved)).cpu().numpy()
    plan.status()
    assert ewald.rel_l2(gm, ewald.ewald(L, moved, q2)) <= 1e-9
    with pytest.raises(pdmk.PdmkError) as e:
        plan.execute(_t(torch_dev, q2), want_grad=True)
    assert e.value.code == -9
    gp = pdmk.Plan(L, eps=1e-9, grad=True)
    gp.bind(S, Q)
    assert gp.stats()["pairs_once"] == 0
    pot, g = gp.execute(_t(torch_dev, q2))
    gp.status()
    rp, rg = ewald.ewald(L, src, q2, grad=True)
    assert ewald.rel_l2(pot.cpu().numpy(), rp) <= 1e-9
    assert ewald.rel_l2(g.cpu().numpy(), rg) <= 1e-8
