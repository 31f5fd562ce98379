"""Pins of the quasi-periodic (Bloch) Ewald oracle (oracle/bloch.c) against
facts outside it (Section 4.1, eq:qp_def): independence of the Ewald
splitting parameter (the real-space image phases and the shifted reciprocal
modes must agree for every split), invariance under a unimodular change of
lattice basis (the same lattice, other n) and under a shift of beta by a
reciprocal lattice vector (the image phases are unchanged), quasi-periodicity
Phi(x + L n) = e^{i beta.L n} Phi(x), complex conjugation Phi_{-beta} =
conj(Phi_beta) for real charges, reciprocity K_beta(x, y) = K_{-beta}(y, x),
the literal-position convention (a source moved by L m equals the original
with its charge times e^{-i beta.L m}), and the small-beta limit: without its
m = 0 term the Bloch potential tends to the tin-foil periodic potential of
the pinned periodic oracle."""
import math

import numpy as np
import pytest

from oracle import ewald
from paper_2606_28608_amd import workloads


def _case(d, n=12, seed=5):
    rng = np.random.default_rng(seed)
    if d == 3:
        L = workloads.TRICLINIC3D_L
        beta = np.array([0.7, -1.1, 0.4])
    else:
        L = workloads.OBLIQUE2D_L
        beta = np.array([1.3, -0.6])
    src = rng.random((n, d)) @ L.T
    q = rng.standard_normal(n)
    return L, src, q, beta


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("d", [3, 2])
def test_alpha_independence(d):
    L, src, q, beta = _case(d)
    ref = ewald.ewald_bloch(L, src, q, beta, alpha=2.0)
    for a in (1.0, 4.0):
        assert _rel(ewald.ewald_bloch(L, src, q, beta, alpha=a), ref) <= 1e-13


@pytest.mark.parametrize("d", [3, 2])
def test_unimodular_basis_and_reciprocal_shift(d):
    L, src, q, beta = _case(d)
    ref = ewald.ewald_bloch(L, src, q, beta)
    U = np.array([[1, 1, 0], [0, 1, 0], [1, 0, 1]]) if d == 3 else np.array([[2, 1], [1, 1]])
    assert _rel(ewald.ewald_bloch(L @ U, src, q, beta), ref) <= 1e-12
    g = np.array([1, -2, 1][:d], dtype=float)
    beta2 = beta + 2.0 * math.pi * np.linalg.solve(L.T, g)
    assert _rel(ewald.ewald_bloch(L, src, q, beta2), ref) <= 1e-12


@pytest.mark.parametrize("d", [3, 2])
def test_quasi_periodicity_and_conjugation(d):
    L, src, q, beta = _case(d)
    rng = np.random.default_rng(9)
    trg = rng.random((6, d)) @ L.T
    n = np.array([2, -1, 1][:d], dtype=float)
    shift = L @ n
    a = ewald.ewald_bloch(L, src, q, beta, trg=trg)
    b = ewald.ewald_bloch(L, src, q, beta, trg=trg + shift)
    assert _rel(b, np.exp(1j * beta @ shift) * a) <= 1e-12
    c = ewald.ewald_bloch(L, src, q, -beta, trg=trg)
    assert _rel(c, np.conj(a)) <= 1e-12


def test_reciprocity():
    """sum_i g_i Phi^beta_q(x_i) = sum_j q_j Phi^{-beta}_g(y_j)."""
    L, src, q, beta = _case(3)
    rng = np.random.default_rng(10)
    trg = rng.random((7, 3)) @ L.T
    g = rng.standard_normal(7)
    lhs = np.dot(g, ewald.ewald_bloch(L, src, q, beta, trg=trg))
    rhs = np.dot(q, ewald.ewald_bloch(L, trg, g, -beta, trg=src))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_moved_source_carries_the_bloch_phase():
    L, src, q, beta = _case(3)
    rng = np.random.default_rng(11)
    trg = rng.random((5, 3)) @ L.T
    m = np.array([1.0, -2.0, 1.0])
    moved = src.copy()
    moved[3] += L @ m
    got = ewald.ewald_bloch(L, moved, q, beta, trg=trg)
    only = np.zeros_like(q)
    only[3] = q[3]
    ref = ewald.ewald_bloch(L, src, q, beta, trg=trg) + \
        (np.exp(-1j * beta @ (L @ m)) - 1.0) * ewald.ewald_bloch(L, src, only, beta, trg=trg)
    assert _rel(got, ref) <= 1e-12


@pytest.mark.parametrize("d", [3, 2])
def test_small_beta_limit_is_the_periodic_potential(d):
    """Phi_beta minus its m = 0 term, (1/V) |beta|^-2 sum_j q_j
    e^{i beta.(x - y_j)}, tends to the tin-foil potential as beta -> 0."""
    L, src, q, _ = _case(d, n=10, seed=7)
    q = q - q.mean()
    per = ewald.ewald(L, src, q)
    V = abs(np.linalg.det(L))
    errs = []
    for s in (1e-3, 1e-4):
        beta = s * np.array([0.6, -0.8, 0.3][:d])
        b2 = beta @ beta
        m0 = np.array([np.sum(q * np.exp(1j * beta @ (x - src).T)) for x in src]) / (V * b2)
        errs.append(_rel(ewald.ewald_bloch(L, src, q, beta) - m0, per))
    assert errs[1] <= 2e-3 and errs[1] < 0.3 * errs[0]   # converges like O(|beta|)


def test_reciprocal_lattice_beta_rejected():
    L, src, q, _ = _case(3)
    beta = 2.0 * math.pi * np.linalg.solve(L.T, np.array([1.0, 0.0, -1.0]))
    with pytest.raises(ValueError):
        ewald.ewald_bloch(L, src, q, beta)
