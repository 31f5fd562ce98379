"""Kept trees (pdmk_plan_bind / pdmk_plan_execute / pdmk_plan_status).

* execute with new charges on the bound positions equals a fresh evaluation
  of those charges (same tree: equal to rounding) and the oracle (to eps);
* execute with displaced positions on the frozen tree matches the oracle at
  the displaced positions to eps;
* device-detected input errors are reported by pdmk_plan_status and leave
  the outputs unwritten;
* an execute captured into a HIP graph replays correctly, with eager work
  between the replays;
* C4: forces from the adjoint (autograd) at N = 1e6 clustered against
  central finite differences (h = 1e-5) of the energy on the frozen tree, on
  100 sampled particles x 3 axes.
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_execute_new_charges(pdmk, torch_dev, precision):
    L, src, q = workloads.clustered3d(5000, seed=41)
    q2 = np.random.default_rng(42).standard_normal(len(q))
    q2 -= q2.mean()
    plan = pdmk.Plan(L, eps=1e-6, precision=precision, kappa=3.0, n_s=60)
    S = _t(torch_dev, src)
    p1 = plan.bind(S, _t(torch_dev, q)).cpu().numpy()
    assert ewald.rel_l2(p1, ewald.ewald(L, src, q)) <= 1e-6
    got = plan.execute(_t(torch_dev, q2))
    plan.status()
    got = got.cpu().numpy()
    fresh = plan.eval(S, _t(torch_dev, q2)).cpu().numpy()
    # same tree and arithmetic; atomics reorder sums (FP32 ones in the mixed
    # proxy transfers), so equal to the rounding of the arithmetic type
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert ewald.rel_l2(got, fresh) <= tol
    assert ewald.rel_l2(got, ewald.ewald(L, src, q2)) <= 1e-6
    # the bound charges again: the first result
    again = plan.execute(_t(torch_dev, q)).cpu().numpy()
    plan.status()
    assert ewald.rel_l2(again, p1) <= tol


def test_execute_separate_targets_and_gradient(pdmk, torch_dev):
    L, src, q = workloads.clustered3d(3000, seed=43)
    trg = np.random.default_rng(44).random((700, 3)) @ L.T
    plan = pdmk.Plan(L, eps=1e-6, grad=True, kappa=2.0, n_s=60)
    plan.bind(_t(torch_dev, src), _t(torch_dev, q), trg=_t(torch_dev, trg))
    q2 = np.random.default_rng(45).standard_normal(len(q))
    q2 -= q2.mean()
    pot, g = plan.execute(_t(torch_dev, q2))
    plan.status()
    ref, gref = ewald.ewald(L, src, q2, trg=trg, grad=True)
    assert ewald.rel_l2(pot.cpu().numpy(), ref) <= 1e-6
    assert ewald.rel_l2(g.cpu().numpy(), gref) <= 1e-5


@pytest.mark.parametrize("n", [4000, 300_000])
def test_execute_displaced_positions(pdmk, torch_dev, n):
    """Small displacements on the frozen tree (the far field runs on the
    plan's second stream for the larger case)."""
    L, src, q = workloads.clustered3d(n, seed=46)
    plan = pdmk.Plan(L, eps=1e-6, kappa=3.0, n_s=100)
    plan.bind(_t(torch_dev, src), _t(torch_dev, q))
    rng = np.random.default_rng(47)
    moved = src + 1e-4 * rng.standard_normal(src.shape)
    got = plan.execute(_t(torch_dev, q), src=_t(torch_dev, moved)).cpu().numpy()
    plan.status()
    if n <= 5000:
        ref = ewald.ewald(L, moved, q)
        assert ewald.rel_l2(got, ref) <= 1e-6
    else:
        idx = rng.choice(n, 48, replace=False)
        ref = ewald.ewald_sampled(L, moved, q, idx)
        assert ewald.rel_l2(got[idx], ref) <= 1e-6
    # back to the bound positions
    back = plan.execute(_t(torch_dev, q)).cpu().numpy()
    plan.status()
    fresh = plan.eval(_t(torch_dev, src), _t(torch_dev, q)).cpu().numpy()
    assert ewald.rel_l2(back, fresh) <= 1e-12


def test_status_reports_device_errors(pdmk, torch_dev):
    torch, dev = torch_dev
    L, src, q = workloads.clustered3d(2000, seed=48)
    plan = pdmk.Plan(L, eps=1e-6, kappa=2.0, n_s=60)
    plan.bind(_t(torch_dev, src), _t(torch_dev, q))
    out = torch.full((len(q),), 7.0, dtype=torch.float64, device=dev)
    plan.execute(_t(torch_dev, q + 0.05), out=out)
    with pytest.raises(pdmk.PdmkError) as e:
        plan.status()
    assert e.value.code == -3
    assert bool((out == 7.0).all())
    bad = q.copy()
    bad[7] = np.nan
    plan.execute(_t(torch_dev, bad), out=out)
    with pytest.raises(pdmk.PdmkError) as e:
        plan.status()
    assert e.value.code == -5
    assert bool((out == 7.0).all())
    # the error is cleared; a valid execute works
    plan.execute(_t(torch_dev, q), out=out)
    plan.status()
    assert ewald.rel_l2(out.cpu().numpy(), ewald.ewald(L, src, q)) <= 1e-6


def test_execute_in_captured_graph(pdmk, torch_dev):
    """Capture one execute into a graph, replay it three times with new
    charges copied into the captured input, with eager work and
    synchronisations between the replays; every replay equals the eager
    execute of the same charges."""
    torch, dev = torch_dev
    L, src, q = workloads.clustered3d(6000, seed=49)
    plan = pdmk.Plan(L, eps=1e-6, kappa=3.0, n_s=80)
    plan.bind(_t(torch_dev, src), _t(torch_dev, q))
    q_in = _t(torch_dev, q)
    out = torch.empty(len(q), dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(q_in, out=out)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        plan.execute(q_in, out=out)
    rng = np.random.default_rng(50)
    for r in range(3):
        qr = rng.standard_normal(len(q))
        qr -= qr.mean()
        q_in.copy_(_t(torch_dev, qr))
        g.replay()
        torch.cuda.synchronize()
        replayed = out.clone()
        eager = plan.execute(_t(torch_dev, qr))
        plan.status()
        assert ewald.rel_l2(replayed.cpu().numpy(), eager.cpu().numpy()) <= 1e-12, r
        _ = (eager * 2.0).sum().item()   # eager work between replays
    ref = ewald.ewald(L, src, qr)
    assert ewald.rel_l2(replayed.cpu().numpy(), ref) <= 1e-6


def test_c4_forces_against_finite_differences(pdmk, torch_dev):
    """C4: N = 1e6 clustered triclinic, eps = 1e-6, FP64.  The energy
    U = 1/2 sum_i q_i Phi(y_i) has dU/dy_j = q_j grad Phi(y_j) (minus the
    force on j), here from the adjoint through torch.autograd.  Central
    differences of U with h = 1e-5 on the frozen tree (pdmk_plan_execute with
    displaced positions), for 100 seeded particles x 3 axes.

    A central difference carries a truncation error ~ (h / r)^2 of the
    derivative from the closest pair terms (r ~ 1e-4 in this cluster: about
    1e-2 at h = 1e-5), which says nothing about the method.  The differences
    at h, h/2 and h/4 are therefore combined by Romberg extrapolation
    (error ~ (h / r)^6), held to 1e-6 per component relative to the largest
    component of the sample; the raw h = 1e-5 differences are held to their
    own truncation estimate."""
    torch, dev = torch_dev
    L, src, q = workloads.clustered3d(1_000_000, seed=2)
    plan = pdmk.Plan(L, eps=1e-6, grad=True, kappa=7.0)
    S = _t(torch_dev, src).requires_grad_(True)
    Q = _t(torch_dev, q)
    pot = pdmk.periodic_potential(plan, S, Q)
    (0.5 * (Q * pot).sum()).backward()
    dU = S.grad.cpu().numpy()
    plan.bind(_t(torch_dev, src), Q, want_grad=False)
    idx = np.random.default_rng(51).choice(len(q), 100, replace=False)
    base = _t(torch_dev, src)
    moved = base.clone()

    def energy_diff(i, a, h):
        moved[i, a] = base[i, a] + h
        up = plan.execute(Q, src=moved, want_grad=False)
        moved[i, a] = base[i, a] - h
        dn = plan.execute(Q, src=moved, want_grad=False)
        moved[i, a] = base[i, a]
        return float((0.5 * Q * (up - dn)).sum().item()) / (2.0 * h)

    h = 1e-5
    D = np.zeros((3, len(idx), 3))   # central differences at h, h/2, h/4
    for k, i in enumerate(idx):
        for a in range(3):
            for lv in range(3):
                D[lv, k, a] = energy_diff(int(i), a, h / 2 ** lv)
    plan.status()
    ref = dU[idx]
    scale = np.abs(ref).max()
    r1 = (4.0 * D[1] - D[0]) / 3.0
    r1b = (4.0 * D[2] - D[1]) / 3.0
    romberg = (16.0 * r1b - r1) / 15.0
    err_rom = np.abs(romberg - ref).max() / scale
    err_raw = np.abs(D[0] - ref).max() / scale
    trunc = np.abs(D[0] - D[1]).max() * 4.0 / 3.0 / scale
    l2 = np.linalg.norm(romberg - ref) / np.linalg.norm(ref)
    print("C4 FD: h=1e-5 max rel %.3e (truncation estimate %.3e); Romberg max rel %.3e, "
          "l2 rel %.3e" % (err_raw, trunc, err_rom, l2))
    assert err_rom <= 1e-6
    assert err_raw <= 2.0 * trunc + 1e-6
