"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
validates arguments, and its host-side planning matches the closed forms the
paper gives (orientation eq:Ltri, bounding box and root cubes eq:mi, Fourier
grid eq:Mi with eq:anorms, shift bounds eq:shift_bounds, the PSWF
calibration of Section 2.2 and the kernel split eq:pswf_split / eq:W0hat).
No compute call touches a device here."""
import math
import os
import re

import numpy as np
import pytest

from paper_2606_28608_amd import pdmk, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pdmk.LIB_PATH):
        from paper_2606_28608_amd import build
        build.build()
    return pdmk.lib()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "pdmk.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(pdmk_\w+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 12
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_default_opts_and_validation(lib):
    o = pdmk.default_opts(3, 1e-6)
    assert o.dim == 3 and o.n_s > 0 and o.porder > 0 and o.npw > 0
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.default_opts(4, 1e-6)
    assert e.value.code == -1
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.default_opts(3, 1e-14)
    assert e.value.code == -4
    assert lib.pdmk_status_string(-3) == b"charges are not neutral"


def test_unknown_flags_and_stage_bits_rejected(lib):
    L = workloads.TRICLINIC3D_L
    pdmk.geometry(L, eps=1e-6, deterministic=True, vector_plane_waves=True, fp32_stages=15)
    for over in (dict(flags=512), dict(fp32_stages=16)):
        with pytest.raises(pdmk.PdmkError) as e:
            pdmk.geometry(L, eps=1e-6, **over)
        assert e.value.code == -1


def test_singular_lattice_rejected(lib):
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.geometry(np.array([[1.0, 2.0, 0], [0, 0, 0], [0, 0, 1.0]]), eps=1e-6)
    assert e.value.code == -2
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.geometry(np.array([[1.0, np.nan], [0, 1.0]]), eps=1e-6)


def test_pswf_calibration(lib):
    # psi(1)/psi(0) = eps (Section 2.2): What_0(k) k^2 = psi~(k rc / c) = eps at k = c / rc
    for eps in (1e-3, 1e-6, 1e-9, 1e-12):
        ki = pdmk.kernel_info(3, eps)
        v = pdmk.w0hat(3, eps, 1.0, np.array([ki.c]))[0] * ki.c ** 2
        assert abs(v / eps - 1) < 1e-4
        # lambda0 psi(0) = int psi = 2 c0 (eq:pswf_eig at x = 0)
        assert abs(ki.lambda0 - 2 * ki.c0_over_psi0) < 1e-12
    # c grows like log(1/eps) (eq:c_log_eps): slope of c against ln(1/eps) near 1
    cs = [pdmk.kernel_info(3, e).c for e in (1e-3, 1e-6, 1e-9, 1e-12)]
    slopes = np.diff(cs) / math.log(1e3)
    assert np.all((slopes > 0.9) & (slopes < 1.2))


def test_w0_zero_closed_form(lib):
    # eq:W0zero: W_0(0) = psi(0) / (4 pi c0 rc); the residual table must reach
    # it as r -> 0: W_h(r) = 1/(4 pi r) - R_h(r) -> W_0(0) / h
    h = 0.37
    for eps in (1e-3, 1e-6, 1e-9):
        ki = pdmk.kernel_info(3, eps)
        w0 = 1.0 / (4 * math.pi * ki.c0_over_psi0)
        assert abs(ki.w0_zero - w0) < 1e-14
        r = 1e-6 * h
        lim = 1.0 / (4 * math.pi * r) - pdmk.residual(3, eps, h, np.array([r]))[0]
        assert abs(lim * h - w0) < max(1e-3 * eps, 1e-10) * w0


@pytest.mark.parametrize("dim", [3, 2])
@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_residual_is_fourier_pair_of_split(lib, dim, eps):
    """R_h = G - W_h in physical space (eq:pswf_split; 2D by the projection of
    the 3D residual) has the radial Fourier transform 1/k^2 - What_h(k) of
    eq:W0hat: checked by quadrature of the physical kernel."""
    from scipy.special import j0
    h = 0.7
    nq = 4000
    x, w = np.polynomial.legendre.leggauss(nq)
    # substitute r = h t^2 to resolve the singularity at 0
    t = 0.5 * (x + 1)
    r = h * t * t
    dr = 0.5 * w * 2 * h * t
    R = pdmk.residual(dim, eps, h, r)
    assert np.all(pdmk.residual(dim, eps, h, np.array([h, 1.5 * h])) == 0)
    for k in (0.5, 3.0, 9.0, 20.0):
        if dim == 3:
            ft = np.sum(4 * math.pi * R * r * np.sin(k * r) / k * dr)
        else:
            ft = np.sum(2 * math.pi * R * j0(k * r) * r * dr)
        want = 1.0 / k ** 2 - pdmk.w0hat(dim, eps, h, np.array([k]))[0]
        assert abs(ft - want) < max(1e-3 * eps, 5e-11) / k ** 2, (k, ft, want)


def test_orientation_and_root_grid_closed_forms(lib):
    L = workloads.SHELL3D_L
    g = pdmk.geometry(L, eps=1e-6)
    Lo = np.array(g.L_oriented).reshape(3, 3, order="F")
    Q = np.array(g.Q).reshape(3, 3, order="F")
    # upper triangular with positive diagonal, L11 = |a_1| the longest (eq:Ltri)
    assert np.allclose(np.tril(Lo, -1), 0)
    assert np.all(np.diag(Lo) > 0)
    lens = np.linalg.norm(L, axis=0)
    assert abs(Lo[0, 0] - lens.max()) < 1e-12
    # Q^T maps the permuted input basis to the oriented one; metric preserved
    perm = list(g.perm)
    assert np.allclose(Q.T @ L[:, perm], Lo, atol=1e-12)
    assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-13)
    assert abs(g.volume - abs(np.linalg.det(L))) < 1e-10
    # eq:w1/eq:w2/eq:mi with rc = Lmin / kappa
    rc = np.diag(Lo).min() / g.kappa
    assert abs(g.rc - rc) < 1e-14
    w = [Lo[0, 0] + abs(Lo[0, 1]) + abs(Lo[0, 2]), Lo[1, 1] + abs(Lo[1, 2]), Lo[2, 2]]
    assert list(g.nroot) == [math.ceil(wi / rc) for wi in w]
    xlo = [min(0, Lo[0, 1]) + min(0, Lo[0, 2]), min(0, Lo[1, 2]), 0.0]
    assert np.allclose(np.array(g.origin), np.array(xlo) - rc)
    # eq:Mi with eq:anorms
    an = [Lo[0, 0], math.hypot(Lo[0, 1], Lo[1, 1]), np.linalg.norm(Lo[:, 2])]
    M = [2 * math.ceil(g.c * a / (2 * math.pi * rc)) for a in an]
    assert list(g.fgrid_paper) == M
    assert all(f >= m for f, m in zip(g.fgrid, M))


def test_shift_bounds_cover_brute_force(lib):
    """Every lattice shift that places some point of the cell inside the
    extended domain passes the bounds of eq:shift_bounds (checked against a
    brute-force search over a much wider box of shifts)."""
    rng = np.random.default_rng(3)
    for L in (workloads.SHELL3D_L, workloads.TRICLINIC3D_L, workloads.triclinic_base((1, 10, 10))):
        g = pdmk.geometry(L, eps=1e-3)
        Lo = np.array(g.L_oriented).reshape(3, 3, order="F")
        u = rng.random((4000, 3))
        corners = np.array(np.meshgrid([0, 1], [0, 1], [0, 1], indexing="ij")).reshape(3, -1).T
        x = np.vstack([u, corners * (1 - 1e-12)]) @ Lo.T
        lo = np.array(g.origin)
        hi = lo + (np.array(g.nroot) + 2) * g.rc
        need = set()
        R = 12
        for n in np.array(np.meshgrid(*[np.arange(-R, R + 1)] * 3, indexing="ij")).reshape(3, -1).T:
            y = x + Lo @ n
            if np.any(np.all((y >= lo) & (y < hi), axis=1)):
                need.add(tuple(n))
        # the bounds of eq:shift_bounds, recomputed
        m = np.array(g.nroot)
        allowed = set()
        for n3 in range(-50, 51):
            b3 = math.ceil((m[2] + 1) * g.rc / Lo[2, 2])
            if abs(n3) > b3:
                continue
            b2 = math.ceil(((m[1] + 1) * g.rc + abs(Lo[1, 2] * n3)) / Lo[1, 1])
            for n2 in range(-b2, b2 + 1):
                b1 = math.ceil(((m[0] + 1) * g.rc + abs(Lo[0, 1] * n2 + Lo[0, 2] * n3)) / Lo[0, 0])
                for n1 in range(-b1, b1 + 1):
                    allowed.add((n1, n2, n3))
        assert need <= allowed
        assert g.n_shifts == len(allowed)


def test_image_count_bound_orthogonal(lib):
    """eq:Nbound: N'/N <= prod(floor((m_i+2) rc / L_i) + 1) for orthogonal cells,
    checked by counting images of random points with the plan's geometry."""
    rng = np.random.default_rng(5)
    for Ls, kappa in (((1.0, 1.5, 2.5), 1.0), ((1.0, 1.0, 10.0), 5.0), ((1.0, 10.0, 10.0), 1.0)):
        L = np.diag(Ls)
        g = pdmk.geometry(L, eps=1e-3, kappa=kappa)
        Lo = np.array(g.L_oriented).reshape(3, 3, order="F")
        x = rng.random((3000, 3)) @ Lo.T
        lo = np.array(g.origin)
        hi = lo + (np.array(g.nroot) + 2) * g.rc
        cnt = 0
        R = 4
        for n in np.array(np.meshgrid(*[np.arange(-R, R + 1)] * 3, indexing="ij")).reshape(3, -1).T:
            y = x + Lo @ n
            cnt += np.sum(np.all((y >= lo) & (y < hi), axis=1))
        bound = np.prod([math.floor((mi + 2) * g.rc / Li) + 1
                         for mi, Li in zip(g.nroot, np.diag(Lo))])
        assert cnt / len(x) <= bound


def test_geometry_2d(lib):
    g = pdmk.geometry(workloads.OBLIQUE2D_L, eps=1e-6)
    Lo = np.array(g.L_oriented)[:4].reshape(2, 2, order="F")
    assert abs(Lo[1, 0]) < 1e-15 and Lo[0, 0] > 0 and Lo[1, 1] > 0
    assert g.kappa == 7.0
    assert list(g.fgrid_paper)[:2] == [2 * math.ceil(g.c * a / (2 * math.pi * g.rc))
                                       for a in (Lo[0, 0], math.hypot(Lo[0, 1], Lo[1, 1]))]


def test_plan_tune_argument_errors(lib):
    """pdmk_plan_tune rejects bad arguments before touching a device."""
    import ctypes
    from paper_2606_28608_amd import pdmk
    o = pdmk.Opts()
    assert lib.pdmk_default_opts(3, ctypes.c_double(1e-6), ctypes.byref(o)) == 0
    L = np.eye(3).ravel(order="F").copy()
    kap = np.array([3.0])
    ns = (ctypes.c_int * 1)(200)
    bk, bn = ctypes.c_double(0), ctypes.c_int(0)
    dp = ctypes.POINTER(ctypes.c_double)
    for n_cand, trials in ((0, 1), (1, 0)):
        st = lib.pdmk_plan_tune(ctypes.byref(o), L.ctypes.data_as(dp), n_cand,
                                kap.ctypes.data_as(dp), ns, trials, 10, None, None, 10, None,
                                None, None, None, ctypes.byref(bk), ctypes.byref(bn))
        assert st == -1


def test_batch_tune_argument_errors(lib):
    """pdmk_batch_tune rejects a null batch, no candidates or no trials before
    touching a device."""
    import ctypes
    off = np.array([0, 10], dtype=np.int64)
    kap = np.array([3.0])
    ns = (ctypes.c_int * 1)(200)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    for n_cand, trials in ((1, 1), (0, 1), (1, 0)):
        st = lib.pdmk_batch_tune(None, off.ctypes.data_as(ip), None, None, n_cand,
                                 kap.ctypes.data_as(dp), ns, trials, None, None, None)
        assert st == -1
    assert b"null argument" in lib.pdmk_last_error()


def test_bloch_grid_and_reciprocal_lattice():
    """Bloch plans (Section 4.1): the far-field grid grows to
    M_i = 2 ceil((c / r_c + |beta|) |a_i| / 2 pi); a Bloch vector in the
    reciprocal lattice (the periodic case) is rejected; the vector needs one
    component per dimension."""
    L = workloads.TRICLINIC3D_L
    beta = np.array([0.7, -1.1, 0.4])
    g0 = pdmk.geometry(L, eps=1e-6)
    g1 = pdmk.geometry(L, eps=1e-6, bloch=beta)
    bn = float(np.linalg.norm(beta))
    Lo = np.asarray(g1.L_oriented[:9]).reshape(3, 3)   # row a = oriented column a
    for i in range(3):
        an = float(np.linalg.norm(Lo[i]))
        assert g1.fgrid_paper[i] == 2 * math.ceil((g1.c / g1.rc + bn) * an / (2 * math.pi))
        assert g1.fgrid_paper[i] >= g0.fgrid_paper[i]
    # a Bloch vector comparable to c / r_c enlarges every axis
    big = pdmk.geometry(L, eps=1e-6, bloch=beta * (g1.c / g1.rc) / bn)
    assert all(big.fgrid_paper[i] > g0.fgrid_paper[i] for i in range(3))
    recip = 2.0 * math.pi * np.linalg.solve(L.T, np.array([1.0, 0.0, -2.0]))
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.geometry(L, eps=1e-6, bloch=recip)
    assert e.value.code == -1
    with pytest.raises(ValueError):
        pdmk.geometry(L, eps=1e-6, bloch=[0.1, 0.2])
    # flags that Bloch plans do not support
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.geometry(L, eps=1e-6, bloch=beta, deterministic=True)
    assert e.value.code == -9


def test_virtual_image_geometry():
    """rem:cube: a cube with integer kappa tiles into kappa^3 root cubes with
    no halo and no shifts; commensurate rectangular cells tile likewise; other
    cells, and Bloch conditions, are rejected."""
    g = pdmk.geometry(np.eye(3) * 2.0, eps=1e-6, kappa=4.0, virtual_images=True)
    assert list(g.nroot) == [4, 4, 4]
    assert g.n_shifts == 1 and abs(g.rc - 0.5) < 1e-15
    assert list(g.origin) == [0.0, 0.0, 0.0]
    g = pdmk.geometry(np.diag([1.0, 2.0, 3.0]), eps=1e-6, kappa=3.0, virtual_images=True)
    assert sorted(g.nroot) == [3, 6, 9]
    g2 = pdmk.geometry(np.diag([1.0, 2.0]), eps=1e-6, kappa=2.0, virtual_images=True)
    assert sorted(list(g2.nroot)[:2]) == [2, 4]
    # a rotated cube is a cube
    th = 0.3
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    g = pdmk.geometry(R @ np.eye(3), eps=1e-6, kappa=3.0, virtual_images=True)
    assert list(g.nroot) == [3, 3, 3]
    for L in (workloads.rectangular_base(), workloads.TRICLINIC3D_L):
        with pytest.raises(pdmk.PdmkError) as e:
            pdmk.geometry(L, eps=1e-6, kappa=3.0, virtual_images=True)
        assert e.value.code == -9
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.geometry(np.eye(3), eps=1e-6, kappa=3.5, virtual_images=True)
    assert e.value.code == -9
    with pytest.raises(pdmk.PdmkError) as e:
        pdmk.geometry(np.eye(3), eps=1e-6, virtual_images=True, bloch=[0.1, 0.2, 0.3])
    assert e.value.code == -9
