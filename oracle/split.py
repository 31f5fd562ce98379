"""Reference for the two halves of the periodic DMK split, each on its own.

TEST INFRASTRUCTURE ONLY (like ewald.py): plain FP64 numpy, written from the
paper, sharing no code with the GPU library.  Only ``tests/`` may import it.

The method splits the Laplace kernel as G = (G - W_0) + W_0 (Section 2.3,
eq:tele / eq:W0hat / eq:pswf_split): the near part G - W_0 vanishes for
r >= r_c (the root-cube side h_0), the far part W_0 is smooth and is summed
over the lattice in Fourier space (Section 3.6, eq:W0p, eq:diag) on the modes
of the grid of eq:Mi.  For targets that are the sources (self pair removed)
the method's result is

    Phi = Phi_near + Phi_far,
    Phi_far(x_i)  = (1/V) sum_{m != 0} What_0(|k_m|) Re[e^{i k_m.x_i} S(m)],
                    S(m) = sum_j q_j e^{-i k_m.y_j}      (self pair included)
    Phi_near(x_i) = sum'_{j,n} q_j (G - W_0)(|x_i - y_j - L n|) - q_i W_0(0)

(the far sum includes the self pair's W_0(0); Section 3.8 removes it).

Pieces, each following the paper:
  * ``Prolate(c)``: psi_0^c of eq:pswf_eig, the even eigenfunction of the
    prolate differential operator -d/dx (1 - x^2) d/dx + c^2 x^2 (which
    commutes with the integral operator of eq:pswf_eig), expanded in
    normalised Legendre polynomials: the operator is diagonal (k (k+1)) on
    them plus c^2 times the square of the matrix of multiplication by x,
    whose entries follow from the three-term Legendre recurrence.
  * ``calibrate(eps)``: c with psi(1) / psi(0) = eps (Section 2.2, by
    bisection; psi(1)/psi(0) decreases with c).
  * ``phi(t)`` of eq:Phic (psi zero outside [-1, 1], so phi = 1 for t >= 1),
    the 3D W_0 and residual of eq:pswf_split, W_0(0) of eq:W0zero.
  * ``psit(x)``: the normalised prolate of eq:npsi continued to x > 1 by its
    integral representation (eq:pswf_eig holds for every real x), as the
    Fourier multiplier What_0(k) = psit(k r_c / c) / k^2 of eq:W0hat needs.
  * 2D: no closed form is printed (Section 2.3 obtains it by a radial
    Fourier transform).  A function of (x, y) that is the integral over z of
    a function g(x, y, z) has the 2D transform g^(k_x, k_y, 0); the 3D
    residual's transform (1 - psit(|k| h / c)) / |k|^2 is the 2D residual's
    too, so the 2D residual is the line integral of the 3D one:
    R_2(r) = int R_3(sqrt(r^2 + z^2)) dz = (1 / 2pi) int_0^{acosh(h/r)}
    (1 - phi((r / h) cosh s)) ds (substituting z = r sinh s), a smooth
    integrand; r -> 0 gives W_0(0) = (int_0^1 phi(t) / t dt - log 2h) / 2pi.
  * ``oriented(L)``: eq:Ltri (lattice vectors by decreasing length, then QR
    with a positive diagonal), for r_c = L_min / kappa (Section 5) and the
    lattice vector lengths of eq:anorms used by eq:Mi.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy import special


class Prolate:
    """psi_0^c on [-1, 1] in normalised Legendre polynomials."""

    def __init__(self, c: float):
        self.c = float(c)
        n = int(2 * self.c + 60)
        n += n % 2
        k = np.arange(n, dtype=np.float64)
        # multiplication by x: x Pbar_k = b_{k+1} Pbar_{k+1} + b_k Pbar_{k-1},
        # b_k = k / sqrt(4 k^2 - 1) (normalised Legendre recurrence)
        b = k[1:] / np.sqrt(4.0 * k[1:] ** 2 - 1.0)
        X = np.diag(b, 1) + np.diag(b, -1)
        A = np.diag(k * (k + 1.0)) + self.c ** 2 * (X @ X)
        # even functions only: the even-indexed block
        ev = np.arange(0, n, 2)
        Ae = A[np.ix_(ev, ev)]
        w, V = np.linalg.eigh(Ae)
        v = V[:, 0]
        coef = np.zeros(n)
        coef[ev] = v
        # plain Legendre coefficients (Pbar_k = sqrt(k + 1/2) P_k); psi(0) > 0
        self.leg = coef * np.sqrt(k + 0.5)
        if npleg.legval(0.0, self.leg) < 0:
            self.leg = -self.leg
        self.psi0 = float(npleg.legval(0.0, self.leg))
        self.psi1 = float(npleg.legval(1.0, self.leg))
        self._int = npleg.legint(self.leg, lbnd=0.0)   # int_0^x psi
        self.c0 = float(npleg.legval(1.0, self._int))  # eq:Phic
        # eigenvalue of eq:pswf_eig from x = 0: lambda_0 psi(0) = int psi
        self.lam0 = 2.0 * self.c0 / self.psi0
        nq = int(self.c * 4 + 80)
        self._gx, self._gw = npleg.leggauss(nq)
        self._gpsi = npleg.legval(self._gx, self.leg)

    def psi(self, x):
        x = np.asarray(x, dtype=np.float64)
        out = npleg.legval(np.clip(x, -1.0, 1.0), self.leg)
        return np.where(np.abs(x) <= 1.0, out, 0.0)

    def phi(self, t):
        """eq:Phic: (1 / c_0) int_0^t psi, equal to 1 for t >= 1."""
        t = np.asarray(t, dtype=np.float64)
        v = npleg.legval(np.clip(t, 0.0, 1.0), self._int) / self.c0
        return np.where(t >= 1.0, 1.0, v)

    def psit(self, x):
        """eq:npsi for any real x: int psi(t) cos(c x t) dt / int psi(t) dt."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        out = np.empty_like(x)
        for s in range(0, x.size, 4096):
            xs = x.flat[s:s + 4096]
            out.flat[s:s + 4096] = (np.cos(self.c * np.outer(xs, self._gx)) @
                                    (self._gw * self._gpsi)) / (2.0 * self.c0)
        return out

    def eig_residual(self, xs):
        """max |int psi(t) e^{i c x t} dt - lambda_0 psi(x)| over xs (eq:pswf_eig)."""
        lhs = (np.cos(self.c * np.outer(xs, self._gx)) @ (self._gw * self._gpsi))
        return float(np.max(np.abs(lhs - self.lam0 * self.psi(xs))))


_CACHE: dict = {}


def calibrate(eps: float) -> Prolate:
    """The prolate whose c gives psi(1) / psi(0) = eps (bisection on c)."""
    key = float(eps)
    if key in _CACHE:
        return _CACHE[key]
    lo, hi = 1.0, 80.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        r = Prolate(mid)
        if r.psi1 / r.psi0 > eps:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-13 * hi:
            break
    P = Prolate(0.5 * (lo + hi))
    _CACHE[key] = P
    return P


def oriented(L):
    """eq:Ltri: lattice vectors (columns) sorted by decreasing length (stable),
    then QR with a positive diagonal.  Returns the upper-triangular R."""
    L = np.asarray(L, dtype=np.float64)
    order = sorted(range(L.shape[1]), key=lambda i: -np.linalg.norm(L[:, i]))
    _, R = np.linalg.qr(L[:, order])
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return R * sgn[:, None]


def root_side(L, kappa: float) -> float:
    """r_c = L_min / kappa, L_min = min_i L_ii of the oriented cell."""
    return float(np.min(np.diag(oriented(L))) / kappa)


def fourier_grid(L, c: float, rc: float):
    """eq:Mi, M_i = 2 ceil(c |a_i| / (2 pi r_c)), for each lattice vector a_i
    in the order of the columns of L (eq:anorms gives the same lengths from
    the oriented cell, whose columns are these vectors sorted by length)."""
    L = np.asarray(L, dtype=np.float64)
    return [2 * int(math.ceil(c * np.linalg.norm(L[:, i]) / (2.0 * math.pi * rc)))
            for i in range(L.shape[1])]


_GS, _GW = npleg.leggauss(96)


def near_kernel(dim: int, P: Prolate, r, h: float):
    """(G - W_0)(r) for root side h: zero for r >= h; r > 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    m = r < h
    rr = r[m]
    if dim == 3:
        out[m] = (1.0 - P.phi(rr / h)) / (4.0 * math.pi * rr)
    else:
        # (1 / 2pi) int_0^S (1 - phi((r/h) cosh s)) ds, S = acosh(h / r)
        S = np.arccosh(h / rr)
        sv = 0.5 * S[:, None] * (_GS[None, :] + 1.0)
        f = 1.0 - P.phi((rr / h)[:, None] * np.cosh(sv))
        out[m] = 0.5 * S * (f @ _GW) / (2.0 * math.pi)
    return out


def w0_zero(dim: int, P: Prolate, h: float) -> float:
    """W_0(0): eq:W0zero in 3D; in 2D the limit r -> 0 of G(r) - R_2(r)."""
    if dim == 3:
        return P.psi0 / (4.0 * math.pi * P.c0 * h)
    t = 0.5 * (_GS + 1.0)
    # int_a^1 (1 - phi) / sqrt(t^2 - a^2) dt = acosh(1/a) - int_a^1 phi / sqrt(...)
    # -> log(2 / a) - int_0^1 phi(t) / t dt as a = r / h -> 0
    return float((0.5 * np.sum(_GW * P.phi(t) / t) - math.log(2.0 * h)) / (2.0 * math.pi))


def _shifts(L, rmax):
    """Lattice shifts n with |L n| possibly below rmax + cell diameter."""
    L = np.asarray(L, dtype=np.float64)
    d = L.shape[0]
    diam = np.sum(np.linalg.norm(L, axis=0))
    # |n_i| <= (rmax + diam) |row i of L^{-1}|
    Li = np.linalg.inv(L)
    b = [int(math.ceil((rmax + diam) * np.linalg.norm(Li[i]))) for i in range(d)]
    rng = [np.arange(-bi, bi + 1) for bi in b]
    g = np.meshgrid(*rng, indexing="ij")
    n = np.stack([x.ravel() for x in g], axis=1).astype(np.float64)
    # a pair of points of the cell is at most diam apart
    return n[np.linalg.norm(n @ L.T, axis=1) <= rmax + diam]


def wrap(L, x):
    """Positions wrapped into the cell (u = L^{-1} x mod 1)."""
    L = np.asarray(L, dtype=np.float64)
    u = np.linalg.solve(L, np.asarray(x, dtype=np.float64).T).T
    u -= np.floor(u)
    return u @ L.T


def prolate_for(eps: float, c=None) -> Prolate:
    """The calibrated prolate of eps, or the prolate of a given bandwidth c
    (the split is defined for any c; to compare one half of it with an
    evaluation, both must use the same c)."""
    return calibrate(eps) if c is None else Prolate(c)


def near_part(L, src, q, eps: float, kappa: float, c=None):
    """Phi_near at the sources (targets = sources, self pair removed): the
    finite sum of (G - W_0) over all images within r_c, minus q_i W_0(0)."""
    L = np.asarray(L, dtype=np.float64)
    d = L.shape[0]
    P = prolate_for(eps, c)
    h = root_side(L, kappa)
    x = wrap(L, src)
    q = np.asarray(q, dtype=np.float64)
    n = len(q)
    S = _shifts(L, h) @ L.T
    out = np.zeros(n)
    for i in range(n):
        dv = x[i][None, None, :] - x[None, :, :] - S[:, None, :]
        r = np.sqrt(np.sum(dv * dv, axis=2))
        r[np.abs(r) == 0.0] = np.inf   # the self pair (n = 0, j = i)
        m = r < h
        if np.any(m):
            rr = r[m]
            qq = np.broadcast_to(q[None, :], r.shape)[m]
            out[i] = np.sum(qq * near_kernel(d, P, rr, h))
    return out - q * w0_zero(d, P, h)


def far_part(L, src, q, eps: float, kappa: float, grid=None, c=None):
    """Phi_far at the sources: (1/V) sum over modes m != 0 of the box
    |m_a| < M_a / 2 (M = eq:Mi unless grid is given) of
    psit(|k_m| r_c / c) / |k_m|^2 Re[e^{i k_m.x_i} S(m)]."""
    L = np.asarray(L, dtype=np.float64)
    d = L.shape[0]
    P = prolate_for(eps, c)
    h = root_side(L, kappa)
    M = fourier_grid(L, P.c, h) if grid is None else list(grid)
    u = np.linalg.solve(L, np.asarray(src, dtype=np.float64).T).T
    q = np.asarray(q, dtype=np.float64)
    V = abs(np.linalg.det(L))
    rng = [np.arange(-(Ma // 2) + 1, Ma // 2) if Ma % 2 == 0 else
           np.arange(-(Ma // 2), Ma // 2 + 1) for Ma in M]
    g = np.meshgrid(*rng, indexing="ij")
    modes = np.stack([x.ravel() for x in g], axis=1).astype(np.float64)
    modes = modes[np.any(modes != 0, axis=1)]
    K = 2.0 * math.pi * np.linalg.solve(L.T, modes.T).T   # k_m = 2 pi L^{-T} m
    k2 = np.sum(K * K, axis=1)
    wt = P.psit(np.sqrt(k2) * h / P.c) / k2 / V
    out = np.zeros(len(q))
    for s in range(0, len(modes), 2048):
        ph = 2.0 * math.pi * (u @ modes[s:s + 2048].T)        # (n, nm)
        c, si = np.cos(ph), np.sin(ph)
        Sr = q @ c          # S(m) = sum q e^{-i phase}: real part, and -imag
        Si = q @ si
        # Re[e^{i ph_i} S(m)] = cos ph_i Sr + sin ph_i Si
        out += c @ (wt[s:s + 2048] * Sr) + si @ (wt[s:s + 2048] * Si)
    return out
