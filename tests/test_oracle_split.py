"""Pins of oracle/split.py (the two halves of the kernel split, each on its
own) against facts outside it: the PSWF eigen-equation (eq:pswf_eig) and
its calibration psi(1)/psi(0) = eps (Section 2.2); the Fourier pair of the
physical residual and its Fourier multiplier (eq:pswf_split against
eq:W0hat) in 3D and 2D by numerical radial transforms; the limit W_0(0)
(eq:W0zero, and its 2D analogue) from the kernel itself; and the split
reassembling the Ewald oracle's potential, a pinned independent summation
(near half + far half over the eq:Mi modes = Ewald to the tolerance the
split is built for)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import special

from oracle import ewald, split
from paper_2606_28608_amd import workloads


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_prolate_eigen_equation_and_calibration(eps):
    P = split.calibrate(eps)
    xs = np.linspace(-1.0, 1.0, 41)
    assert P.eig_residual(xs) <= 1e-12 * P.lam0 * P.psi0
    assert abs(P.psi1 / P.psi0 - eps) <= 1e-5 * eps
    # psit continues psi / psi(0) (eq:npsi) through the eigen-equation
    assert np.allclose(P.psit(xs), P.psi(xs) / P.psi0, rtol=0, atol=1e-13)
    assert abs(P.phi(1.0) - 1.0) <= 1e-15


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_residual_3d_is_the_fourier_pair_of_its_multiplier(eps):
    """(4 pi / k) int_0^h r R(r) sin(k r) dr = (1 - psit(k h / c)) / k^2."""
    P = split.calibrate(eps)
    h = 0.7
    x, w = npleg.leggauss(400)
    r = 0.5 * h * (x + 1.0)
    w = 0.5 * h * w
    rR = r * split.near_kernel(3, P, r, h)
    for k in (0.3, 2.0, 9.0, 31.0, 70.0):
        lhs = 4.0 * math.pi / k * np.sum(w * rR * np.sin(k * r))
        rhs = (1.0 - P.psit(k * h / P.c)[0]) / k ** 2
        assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1.0 / k ** 2), k


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_residual_2d_is_the_fourier_pair_of_its_multiplier(eps):
    """2 pi int_0^h r R_2(r) J_0(k r) dr = (1 - psit(k h / c)) / k^2 (the
    logarithmic singularity at r = 0 is removed by r = h t^2)."""
    P = split.calibrate(eps)
    h = 0.45
    x, w = npleg.leggauss(600)
    t = 0.5 * (x + 1.0)
    w = 0.5 * w
    r = h * t * t
    jac = 2.0 * h * t
    rR = r * split.near_kernel(2, P, r, h)
    for k in (0.5, 3.0, 15.0, 60.0):
        lhs = 2.0 * math.pi * np.sum(w * jac * rR * special.j0(k * r))
        rhs = (1.0 - P.psit(k * h / P.c)[0]) / k ** 2
        assert abs(lhs - rhs) <= 1e-10 * max(abs(rhs), 1.0 / k ** 2), k


@pytest.mark.parametrize("dim", [3, 2])
def test_w0_zero_is_the_limit_of_the_smooth_kernel(dim):
    P = split.calibrate(1e-6)
    h = 0.37
    r = 1e-6 * h
    G = 1.0 / (4.0 * math.pi * r) if dim == 3 else -math.log(r) / (2.0 * math.pi)
    w0 = G - split.near_kernel(dim, P, np.array([r]), h)[0]
    assert abs(w0 - split.w0_zero(dim, P, h)) <= 1e-9 * abs(split.w0_zero(dim, P, h))
    if dim == 3:
        # eq:W0zero: psi(0) / (4 pi c_0 r_c)
        assert split.w0_zero(3, P, h) == pytest.approx(P.psi0 / (4 * math.pi * P.c0 * h),
                                                      rel=1e-15)


def test_kernel_vanishes_beyond_the_root_side():
    P = split.calibrate(1e-6)
    r = np.array([0.999999, 1.0, 1.3]) * 0.5
    v3 = split.near_kernel(3, P, r, 0.5)
    v2 = split.near_kernel(2, P, r, 0.5)
    assert v3[1] == 0 and v3[2] == 0 and v2[1] == 0 and v2[2] == 0
    assert abs(v3[0]) < 1e-10 and abs(v2[0]) < 1e-10   # continuous at the edge


@pytest.mark.parametrize("eps,kappa", [(1e-12, 3.0), (1e-9, 2.0)])
def test_halves_reassemble_the_ewald_potential_3d(eps, kappa):
    L = workloads.TRICLINIC3D_L
    rng = np.random.default_rng(5)
    src = rng.random((14, 3)) @ L.T
    q = rng.standard_normal(14)
    q -= q.mean()
    ref = ewald.ewald(L, src, q)
    tot = split.near_part(L, src, q, eps, kappa) + split.far_part(L, src, q, eps, kappa)
    assert ewald.rel_l2(tot, ref) <= 10 * eps


def test_halves_reassemble_the_ewald_potential_2d():
    L = workloads.OBLIQUE2D_L
    rng = np.random.default_rng(6)
    src = rng.random((20, 2)) @ L.T
    q = rng.standard_normal(20)
    q -= q.mean()
    ref = ewald.ewald(L, src, q)
    eps = 1e-12
    tot = split.near_part(L, src, q, eps, 3.0) + split.far_part(L, src, q, eps, 3.0)
    assert ewald.rel_l2(tot, ref) <= 10 * eps


def test_orientation_and_grid():
    """eq:Ltri keeps the metric up to the permutation; eq:Mi on a cubic cell."""
    L = workloads.TRICLINIC3D_L
    R = split.oriented(L)
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)
    order = sorted(range(3), key=lambda i: -np.linalg.norm(L[:, i]))
    assert np.allclose(R.T @ R, L[:, order].T @ L[:, order])
    c = 16.0
    assert split.fourier_grid(np.eye(3), c, 0.25) == [2 * math.ceil(c / (2 * math.pi * 0.25))] * 3
