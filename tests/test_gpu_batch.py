"""Batched evaluation (many independent cells in one call) against the FP64
Ewald oracle, system by system."""
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


def _pack(systems):
    offs = np.cumsum([0] + [len(s[2]) for s in systems]).astype(np.int64)
    src = np.vstack([s[1] for s in systems])
    q = np.concatenate([s[2] for s in systems])
    Ls = np.stack([s[0] for s in systems])
    return Ls, offs, src, q


@pytest.fixture(scope="module")
def systems():
    sy = workloads.batch_cells(n_sys=7, seed=5, n_min=200, n_max=2500)
    refs = [ewald.ewald(L, src, q) for L, src, q in sy]
    return sy, refs


@pytest.mark.parametrize("precision,eps", [("fp64", 1e-6), ("mixed", 1e-6), ("fp64", 1e-3)])
def test_batch_matches_oracle(pdmk, torch_dev, systems, precision, eps):
    torch, dev = torch_dev
    sy, refs = systems
    Ls, offs, src, q = _pack(sy)
    B = pdmk.Batch(Ls, eps=eps, precision=precision, workers=4)
    pot = B.eval(offs, torch.tensor(src, device=dev), torch.tensor(q, device=dev)).cpu().numpy()
    for s, ref in enumerate(refs):
        got = pot[offs[s]:offs[s + 1]]
        assert ewald.rel_l2(got, ref) <= eps, (s, ewald.rel_l2(got, ref))
        assert B.stats(s)["n_src"] == offs[s + 1] - offs[s]


def test_batch_workers_and_gradients(pdmk, torch_dev, systems):
    """One worker or several give the same values; gradients per system match
    the oracle's."""
    torch, dev = torch_dev
    sy, _ = systems
    sy = sy[:4]
    Ls, offs, src, q = _pack(sy)
    S, Q = torch.tensor(src, device=dev), torch.tensor(q, device=dev)
    a, ga = pdmk.Batch(Ls, eps=1e-6, grad=True, workers=1).eval(offs, S, Q)
    b, gb = pdmk.Batch(Ls, eps=1e-6, grad=True, workers=3).eval(offs, S, Q)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    ga = ga.cpu().numpy()
    for s, (L, x, qq) in enumerate(sy):
        _, gref = ewald.ewald(L, x, qq, grad=True)
        assert ewald.rel_l2(ga[offs[s]:offs[s + 1]], gref) <= 1e-5


def test_batch_errors_and_empty(pdmk, torch_dev, systems):
    torch, dev = torch_dev
    sy, _ = systems
    Ls, offs, src, q = _pack(sy[:3])
    B = pdmk.Batch(Ls, eps=1e-3)
    q2 = q.copy()
    q2[offs[1]] += 1.0                  # system 1 no longer neutral
    with pytest.raises(pdmk.PdmkError) as e:
        B.eval(offs, torch.tensor(src, device=dev), torch.tensor(q2, device=dev))
    assert e.value.code == -3
    # an empty system in the middle
    offs_e = np.array([0, offs[1], offs[1], offs[2]], dtype=np.int64)
    Ls_e = np.stack([Ls[0], Ls[1], Ls[1]])
    Be = pdmk.Batch(Ls_e, eps=1e-3)
    n = int(offs[2])
    pot = Be.eval(offs_e, torch.tensor(src[:n], device=dev), torch.tensor(q[:n], device=dev))
    assert pot.shape == (n,)
    with pytest.raises(ValueError):
        B.eval(offs[:-1], torch.tensor(src, device=dev), torch.tensor(q, device=dev))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_tune_matches_oracle(pdmk, torch_dev, systems, precision):
    """The batch autotuner re-plans each size class with its fastest (kappa,
    n_s) among the candidates; every tuned system still meets eps against the
    oracle, and the reported parameters are among the candidates."""
    torch, dev = torch_dev
    sy, refs = systems
    Ls, offs, src, q = _pack(sy)
    B = pdmk.Batch(Ls, eps=1e-6, precision=precision, workers=3)
    s_d, q_d = torch.tensor(src, device=dev), torch.tensor(q, device=dev)
    cands = [(1.0, 60), (2.0, 30), (3.0, 400)]
    k, n = B.tune(offs, s_d, q_d, candidates=cands, trials=1)
    assert set(zip(k.tolist(), n.tolist())) <= set(cands)
    pot = B.eval(offs, s_d, q_d).cpu().numpy()
    for s, ref in enumerate(refs):
        got = pot[offs[s]:offs[s + 1]]
        assert ewald.rel_l2(got, ref) <= 1e-6, (s, k[s], n[s], ewald.rel_l2(got, ref))


def test_batch_tune_gradients_and_empty_system(pdmk, torch_dev, systems):
    """Tuning a gradient batch that holds a system without sources: the empty
    system keeps its plan, the others' gradients still match the oracle's."""
    torch, dev = torch_dev
    sy, _ = systems
    sy = [sy[0], (sy[1][0], sy[1][1][:0], sy[1][2][:0]), sy[2]]
    Ls, offs, src, q = _pack(sy)
    B = pdmk.Batch(Ls, eps=1e-6, grad=True, workers=2)
    s_d, q_d = torch.tensor(src, device=dev), torch.tensor(q, device=dev)
    k, n = B.tune(offs, s_d, q_d, candidates=[(2.0, 30), (1.0, 200)], trials=1)
    base = pdmk.default_opts(3, 1e-6)
    assert (k[1], n[1]) == (base.kappa, base.n_s)
    pot, g = B.eval(offs, s_d, q_d)
    pot, g = pot.cpu().numpy(), g.cpu().numpy()
    for s in (0, 2):
        L, x, qq = sy[s]
        ref_p, ref_g = ewald.ewald(L, x, qq, grad=True)
        assert ewald.rel_l2(pot[offs[s]:offs[s + 1]], ref_p) <= 1e-6
        assert ewald.rel_l2(g[offs[s]:offs[s + 1]], ref_g) <= 1e-5, s


def test_batch_tune_default_candidates(pdmk, torch_dev, systems):
    """The default candidate set of the autotuner (leaf capacities up to 512
    times the default, whole root cubes as leaves) still meets eps against
    the oracle on every system, in both precisions."""
    torch, dev = torch_dev
    sy, refs = systems
    Ls, offs, src, q = _pack(sy)
    s_d, q_d = torch.tensor(src, device=dev), torch.tensor(q, device=dev)
    for precision in ("fp64", "mixed"):
        B = pdmk.Batch(Ls, eps=1e-6, precision=precision, workers=4)
        k, n = B.tune(offs, s_d, q_d, trials=1)
        pot = B.eval(offs, s_d, q_d).cpu().numpy()
        for s, ref in enumerate(refs):
            err = ewald.rel_l2(pot[offs[s]:offs[s + 1]], ref)
            assert err <= 1e-6, (precision, s, k[s], n[s], err)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_single_leaves_sampled(pdmk, torch_dev, precision):
    """A clustered cell of 40000 sources in a batch planned with a leaf
    capacity above N (the shallow trees the autotuner picks for small cells:
    leaves of tens of thousands of sources, many target groups and source
    segments per leaf) against the oracle at 48 sampled sources."""
    torch, dev = torch_dev
    L, src, q = workloads.batch_cells(n_sys=2, seed=7, n_min=40_000, n_max=40_000)[1]
    offs = np.array([0, len(q)], dtype=np.int64)
    B = pdmk.Batch(L[None], eps=1e-6, precision=precision, workers=1, kappa=3.0, n_s=102400)
    pot = B.eval(offs, torch.tensor(src, device=dev), torch.tensor(q, device=dev)).cpu().numpy()
    st = B.stats(0)
    assert st["n_levels"] == 1 and st["n_leaves"] >= 1
    idx = np.random.default_rng(3).choice(len(q), 48, replace=False)
    assert ewald.rel_l2(pot[idx], ewald.ewald_sampled(L, src, q, idx)) <= 1e-6


def test_batch_kept_trees_and_captured_graph(pdmk, torch_dev, systems):
    """pdmk_batch_bind / pdmk_batch_execute: new charges on every system's
    kept tree equal a fresh batch evaluation of them and the oracle; the
    execute of the whole batch is captured into one graph and replayed three
    times with new charges, eager work and synchronisations in between, each
    replay equal to the eager execute."""
    torch, dev = torch_dev
    sy, refs = systems
    Ls, offs, src, q = _pack(sy)
    S = torch.tensor(src, device=dev)
    B = pdmk.Batch(Ls, eps=1e-6, workers=3)
    p0 = B.bind(offs, S, torch.tensor(q, device=dev)).cpu().numpy()
    for s, ref in enumerate(refs):
        assert ewald.rel_l2(p0[offs[s]:offs[s + 1]], ref) <= 1e-6
    rng = np.random.default_rng(31)

    def new_charges():
        qn = rng.standard_normal(len(q))
        for s in range(len(sy)):
            qn[offs[s]:offs[s + 1]] -= qn[offs[s]:offs[s + 1]].mean()
        return qn

    q2 = new_charges()
    got = B.execute(torch.tensor(q2, device=dev))
    B.status()
    fresh = B.eval(offs, S, torch.tensor(q2, device=dev)).cpu().numpy()
    got = got.cpu().numpy()
    assert ewald.rel_l2(got, fresh) <= 1e-12
    for s in (0, 3):
        ref = ewald.ewald(sy[s][0], sy[s][1], q2[offs[s]:offs[s + 1]])
        assert ewald.rel_l2(got[offs[s]:offs[s + 1]], ref) <= 1e-6
    # one graph for the whole batch
    q_in = torch.tensor(q2, device=dev)
    out = torch.empty(len(q), dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.execute(q_in, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        B.execute(q_in, out=out)
    for r in range(3):
        qr = new_charges()
        q_in.copy_(torch.tensor(qr, device=dev))
        g.replay()
        torch.cuda.synchronize()
        replayed = out.clone()
        eager = B.execute(torch.tensor(qr, device=dev))
        B.status()
        assert ewald.rel_l2(replayed.cpu().numpy(), eager.cpu().numpy()) <= 1e-12, r
        _ = (eager * 2.0).sum().item()
    # a bad charge is reported by the status and leaves the others' values
    bad = new_charges()
    bad[offs[2] + 1] = np.nan
    B.execute(torch.tensor(bad, device=dev))
    with pytest.raises(pdmk.PdmkError) as e:
        B.status()
    assert e.value.code == -5
