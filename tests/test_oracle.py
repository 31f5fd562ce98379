"""Pins of the Ewald oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
textbook Madelung constants, a closed form (Jacobi theta function for the 2D
periodic Green's function), brute-force image sums over balls of cells with
the macroscopic polarisation term, invariances the lattice sum must have
(splitting parameter, unimodular change of basis, rigid motions, supercells),
finite differences and reciprocity.  A dropped term, a wrong sign or a
transposed lattice matrix in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest


def _neutral(rng, n, scale=1.0):
    q = rng.standard_normal(n) * scale
    return q - q.mean()


TRI3 = np.array([[1.0, 0.4, 0.3], [0.0, 1.2, 0.5], [0.0, 0.0, 2.0]])   # columns a1, a2, a3
OBL2 = np.array([[1.0, 0.3], [0.0, 1.0]])


def test_expint_e1_against_scipy(oracle):
    from scipy.special import exp1
    xs = np.concatenate([np.geomspace(1e-8, 0.999, 40), [1.0], np.geomspace(1.001, 60.0, 40)])
    for x in xs:
        assert abs(oracle.expint_e1(x) - exp1(x)) <= 2e-15 * max(1.0, abs(exp1(x)))


# Textbook Madelung constants (referred to the nearest-neighbour distance r0):
# Phi(cation) = -M / (4 pi r0) with unit charges and G = 1/(4 pi r).
M_NACL = 1.747564594633182
M_CSCL = 1.762674773070988


def test_madelung_nacl_conventional(oracle):
    L = np.eye(3)
    na = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    cl = np.array([[.5, 0, 0], [0, .5, 0], [0, 0, .5], [.5, .5, .5]])
    src = np.vstack([na, cl])
    q = np.r_[np.ones(4), -np.ones(4)]
    pot = oracle.ewald(L, src, q)
    np.testing.assert_allclose(pot[:4], -M_NACL / (4 * math.pi * 0.5), rtol=1e-12)
    np.testing.assert_allclose(pot[4:], +M_NACL / (4 * math.pi * 0.5), rtol=1e-12)


def test_madelung_nacl_primitive_triclinic(oracle):
    # fcc primitive cell: a 60-degree triclinic cell, Na at 0, Cl at (1/2,1/2,1/2)
    L = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
    src = np.array([[0, 0, 0], [.5, .5, .5]])
    q = np.array([1.0, -1.0])
    pot = oracle.ewald(L, src, q)
    np.testing.assert_allclose(pot, [-M_NACL / (2 * math.pi), M_NACL / (2 * math.pi)], rtol=1e-12)


def test_madelung_cscl(oracle):
    src = np.array([[0, 0, 0], [.5, .5, .5]])
    q = np.array([1.0, -1.0])
    r0 = math.sqrt(3) / 2
    pot = oracle.ewald(np.eye(3), src, q)
    np.testing.assert_allclose(pot, [-M_CSCL / (4 * math.pi * r0), M_CSCL / (4 * math.pi * r0)],
                               rtol=1e-12)


def _jtheta_green_2d(tau, z):
    """Zero-mean periodic Green's function of -Delta on C / (Z + tau Z), up to a
    constant: -(1/2pi) log|theta_1(pi z | tau)| + (Im z)^2 / (2 Im tau)."""
    import mpmath as mp
    nome = mp.exp(1j * mp.pi * tau)
    zc = mp.mpc(float(z[0]), float(z[1]))
    return -mp.log(abs(mp.jtheta(1, mp.pi * zc, nome))) / (2 * mp.pi) + float(z[1]) ** 2 / (2 * tau.imag)


def test_2d_theta_closed_form(oracle):
    import mpmath as mp
    rng = np.random.default_rng(11)
    L = OBL2
    tau = mp.mpc(L[0, 1], L[1, 1])
    src = rng.random((7, 2)) @ L.T
    q = _neutral(rng, 7)
    trg = rng.random((5, 2)) @ L.T
    ref = [float(sum(q[j] * _jtheta_green_2d(tau, trg[i] - src[j]) for j in range(7)))
           for i in range(5)]
    np.testing.assert_allclose(oracle.ewald(L, src, q, trg=trg), ref, rtol=0, atol=1e-13)
    # targets = sources: regular part of G at 0 is -(1/2pi) log|pi theta_1'(0)|
    th1p = mp.jtheta(1, 0, mp.exp(1j * mp.pi * tau), 1)
    reg0 = float(-mp.log(abs(mp.pi * th1p)) / (2 * mp.pi))
    ref_self = [float(sum(q[j] * _jtheta_green_2d(tau, src[i] - src[j]) for j in range(7) if j != i))
                + q[i] * reg0 for i in range(7)]
    np.testing.assert_allclose(oracle.ewald(L, src, q), ref_self, rtol=0, atol=1e-13)


@pytest.mark.parametrize("L", [TRI3, OBL2], ids=["3d", "2d"])
def test_alpha_independence(oracle, L):
    rng = np.random.default_rng(3)
    d = L.shape[0]
    src = rng.random((40, d)) @ L.T
    q = _neutral(rng, 40)
    a0 = oracle.choose_alpha(L, 40, 40)
    ref, gref = oracle.ewald(L, src, q, grad=True, alpha=a0)
    for f in (0.5, 0.7, 1.4, 2.0):
        p, g = oracle.ewald(L, src, q, grad=True, alpha=a0 * f)
        assert np.abs(p - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(g - gref).max() <= 1e-12 * np.abs(gref).max()


@pytest.mark.parametrize("L", [TRI3, OBL2], ids=["3d", "2d"])
def test_alpha_independence_nonneutral(oracle, L):
    # pins the uniform-background (k = 0) term for non-neutral charges
    rng = np.random.default_rng(5)
    d = L.shape[0]
    src = rng.random((15, d)) @ L.T
    q = rng.standard_normal(15) + 0.3
    a0 = oracle.choose_alpha(L, 15, 15)
    ref = oracle.ewald(L, src, q, alpha=a0)
    for f in (0.5, 2.0):
        p = oracle.ewald(L, src, q, alpha=a0 * f)
        assert np.abs(p - ref).max() <= 1e-13 * np.abs(ref).max()


def _wrap(L, pts):
    u = np.linalg.solve(L, pts.T).T
    u -= np.floor(u)
    return u @ L.T


@pytest.mark.parametrize("L,U", [
    (TRI3, np.array([[1, 1, 0], [0, 1, 0], [2, 0, 1]])),
    (OBL2, np.array([[1, 3], [0, 1]])),
], ids=["3d", "2d"])
def test_unimodular_basis_change(oracle, L, U):
    assert round(abs(np.linalg.det(U))) == 1
    rng = np.random.default_rng(7)
    d = L.shape[0]
    src = rng.random((25, d)) @ L.T
    q = _neutral(rng, 25)
    trg = rng.random((9, d)) @ L.T
    ref = oracle.ewald(L, src, q, trg=trg)
    L2 = L @ U
    got = oracle.ewald(L2, _wrap(L2, src), q, trg=_wrap(L2, trg))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("L", [TRI3, OBL2], ids=["3d", "2d"])
def test_rigid_motions(oracle, L):
    rng = np.random.default_rng(9)
    d = L.shape[0]
    src = rng.random((20, d)) @ L.T
    q = _neutral(rng, 20)
    trg = rng.random((6, d)) @ L.T
    ref, gref = oracle.ewald(L, src, q, trg=trg, grad=True)
    # translation
    t = rng.standard_normal(d) * 3.0
    got = oracle.ewald(L, src + t, q, trg=trg + t)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # rotation composed with a reflection (Q in O(d), det -1)
    Qm, _ = np.linalg.qr(rng.standard_normal((d, d)))
    if np.linalg.det(Qm) > 0:
        Qm[:, 0] *= -1
    got, g = oracle.ewald(Qm @ L, src @ Qm.T, q, trg=trg @ Qm.T, grad=True)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    np.testing.assert_allclose(g, gref @ Qm.T, rtol=0, atol=1e-12 * np.abs(gref).max())


@pytest.mark.parametrize("L", [TRI3, OBL2], ids=["3d", "2d"])
def test_supercell(oracle, L):
    rng = np.random.default_rng(13)
    d = L.shape[0]
    src = rng.random((12, d)) @ L.T
    q = _neutral(rng, 12)
    trg = rng.random((5, d)) @ L.T
    ref = oracle.ewald(L, src, q, trg=trg)
    L2 = L.copy()
    L2[:, 1] *= 2.0          # double a2: the same crystal with a doubled cell
    src2 = np.vstack([src, src + L[:, 1]])
    got = oracle.ewald(L2, src2, np.r_[q, q], trg=trg)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("d", [3, 2])
def test_ball_sum_is_ewald_plus_polarisation(oracle, d):
    """Brute-force sums over whole cells in a growing ball converge to the
    Ewald (tin-foil) value plus the potential of the uniformly polarised
    sphere (disc): slope D/(dV) with D = sum q_j y_j, constant
    -sum q_j |y_j|^2 / (2 d V)."""
    rng = np.random.default_rng(21)
    L = TRI3 / 2.0 if d == 3 else np.array([[1.0, 0.3], [0.0, 1.2]])
    V = abs(np.linalg.det(L))
    src = rng.random((4, d)) @ L.T
    q = np.array([1.0, -1.0, 0.7, -0.7])
    trg = rng.random((6, d)) @ L.T
    pe = oracle.ewald(L, src, q, trg=trg)
    # average a few radii: whole-cell counting makes the constant fluctuate ~1/R
    radii = (36.0, 40.0, 44.0) if d == 3 else (900.0, 1000.0, 1100.0)
    diff = np.mean([oracle.ball_sum(L, src, q, trg, R) for R in radii], axis=0) - pe
    A = np.c_[np.ones(len(trg)), trg]
    coef = np.linalg.lstsq(A, diff, rcond=None)[0]
    D = (q[:, None] * src).sum(0)
    Q2 = (q * (src ** 2).sum(1)).sum()
    assert np.abs(diff - A @ coef).max() < 1e-6 * np.abs(pe).max()      # affine
    np.testing.assert_allclose(coef[1:], D / (d * V), rtol=2e-3, atol=2e-4 * np.abs(D).max())
    np.testing.assert_allclose(coef[0], -Q2 / (2 * d * V), rtol=0.1)


@pytest.mark.parametrize("L", [TRI3, OBL2], ids=["3d", "2d"])
def test_gradient_finite_difference(oracle, L):
    rng = np.random.default_rng(17)
    d = L.shape[0]
    src = rng.random((15, d)) @ L.T
    q = _neutral(rng, 15)
    trg = rng.random((4, d)) @ L.T
    _, g = oracle.ewald(L, src, q, trg=trg, grad=True)
    h = 1e-5
    for ax in range(d):
        e = np.zeros(d)
        e[ax] = h
        fd = (oracle.ewald(L, src, q, trg=trg + e) - oracle.ewald(L, src, q, trg=trg - e)) / (2 * h)
        np.testing.assert_allclose(g[:, ax], fd, rtol=1e-7, atol=1e-7 * np.abs(g).max())


@pytest.mark.parametrize("L", [TRI3, OBL2], ids=["3d", "2d"])
def test_reciprocity(oracle, L):
    rng = np.random.default_rng(19)
    d = L.shape[0]
    ys = rng.random((10, d)) @ L.T
    xs = rng.random((8, d)) @ L.T
    qy = _neutral(rng, 10)
    gx = _neutral(rng, 8)
    a = np.dot(gx, oracle.ewald(L, ys, qy, trg=xs))
    b = np.dot(qy, oracle.ewald(L, xs, gx, trg=ys))
    assert abs(a - b) <= 1e-13 * max(abs(a), 1e-3)


def test_zero_cell_mean(oracle):
    """Tin-foil: the potential has zero mean over the cell (midpoint rule on a
    fine fractional grid; the integrable 1/r singularities limit the accuracy)."""
    rng = np.random.default_rng(23)
    L = TRI3
    src = rng.random((6, 3)) @ L.T
    q = _neutral(rng, 6)
    n = 24
    g = (np.arange(n) + 0.5) / n
    U = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pot = oracle.ewald(L, src, q, trg=U @ L.T)
    assert abs(pot.mean()) < 2e-3 * np.abs(pot).mean()


def test_empty_and_sampled(oracle):
    rng = np.random.default_rng(29)
    L = TRI3
    src = rng.random((30, 3)) @ L.T
    q = _neutral(rng, 30)
    full = oracle.ewald(L, src, q)
    idx = np.array([3, 17, 29])
    np.testing.assert_allclose(oracle.ewald_sampled(L, src, q, idx), full[idx], rtol=1e-13)
    assert oracle.ewald(L, src, q, trg=np.zeros((0, 3))).shape == (0,)
