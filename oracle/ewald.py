"""Python side of the reference Ewald oracle.

TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle the GPU library is
checked against.  Only ``tests/``, the smoke check and the CPU-baseline leg of
the benchmark may import it.  It shares no code with the library.

It evaluates the tin-foil periodic Laplace potential of Introduction
eq:potential / eq:greens (self pair removed, k = 0 mode zero) by classical
Ewald summation; the C implementation (``ewald.c``) documents the split.

Public functions
----------------
``ewald(L, src, q, trg=None, grad=False, alpha=None, tol=1e-16)``
    potential (and gradient) at targets; ``trg=None`` means targets are the
    sources with the self pair removed.
``ewald_sampled(L, src, q, idx, grad=False)``
    the same at the sources ``idx`` only (targets = sources, self removed);
    the structure factor still runs over all sources, so the values are
    exact for the whole system.
``ball_sum(L, src, q, trg, R)``
    brute-force image sum over whole cells inside a ball of radius R (used
    only to pin the Ewald code).
``ewald_bloch(L, src, q, beta, trg=None)``
    the quasi-periodic (Bloch) potential of Section 4.1 (complex), bloch.c.
``expint_e1(x)``
    the exponential integral used by the 2D real-space kernel.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ewald.c")
_SRCS = [_SRC, os.path.join(_HERE, "bloch.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ewald.c and bloch.c into liboracle.so with gcc (OpenMP, -O2)."""
    newest = max(os.path.getmtime(f) for f in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99"] +
                              _SRCS + ["-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.oracle_ewald.argtypes = [ctypes.c_int, dp, ctypes.c_long, dp, dp, ctypes.c_long,
                                     dp, lp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, dp]
        lib.oracle_ewald.restype = ctypes.c_int
        lib.oracle_ewald_nmodes.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double]
        lib.oracle_ewald_nmodes.restype = ctypes.c_long
        lib.oracle_ball_sum.argtypes = [ctypes.c_int, dp, ctypes.c_long, dp, dp, ctypes.c_long,
                                        dp, lp, ctypes.c_double, dp]
        lib.oracle_ball_sum.restype = ctypes.c_int
        lib.oracle_expint_e1.argtypes = [ctypes.c_double]
        lib.oracle_expint_e1.restype = ctypes.c_double
        lib.oracle_ewald_bloch.argtypes = [ctypes.c_int, dp, dp, ctypes.c_long, dp, dp,
                                           ctypes.c_long, dp, lp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, dp, dp]
        lib.oracle_ewald_bloch.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def _lattice(L):
    L = np.asarray(L, dtype=np.float64)
    d = L.shape[0]
    if L.shape != (d, d) or d not in (2, 3):
        raise ValueError("L must be 2x2 or 3x3 with lattice vectors as columns")
    return np.asfortranarray(L), d


def expint_e1(x: float) -> float:
    return _load().oracle_expint_e1(float(x))


# erfc(s) ~ 1e-18 and E1(s^2) ~ 1e-18 at s = 6.3: both truncations are far
# below the 1e-13 accuracy the oracle is meant to carry.
_S = 6.3


def choose_alpha(L, n_src: int, n_trg: int) -> float:
    """Splitting parameter that balances the real-space and reciprocal work
    (cost model only; the result does not depend on it, which the tests pin)."""
    L, d = _lattice(L)
    Li = np.linalg.inv(L)
    V = abs(np.linalg.det(L))
    rows = np.sqrt((Li ** 2).sum(axis=1))
    unit = V ** (1.0 / d)
    best = None
    for a in unit ** -1 * np.geomspace(0.5, 200.0, 120):
        rcut = _S / a
        kcut = 2.0 * a * _S
        cand = np.prod(2.0 * rows * rcut + 1.0)
        ball = (math.pi * kcut ** 2) if d == 2 else (4.0 / 3.0 * math.pi * kcut ** 3)
        nk = 0.5 * ball * V / (2 * math.pi) ** d
        cost = n_trg * n_src * cand * 1.0 + (n_src + n_trg) * nk * 4.0 * d
        if best is None or cost < best[0]:
            best = (cost, a)
    return float(best[1])


def ewald(L, src, q, trg=None, grad=False, alpha=None, self_idx=None, tol_s=_S):
    """Tin-foil periodic potential (and gradient) by Ewald summation, FP64.

    L: d x d lattice, columns = lattice vectors.  src: (N, d).  q: (N,).
    trg: (M, d) or None (targets = sources, self pair removed).
    self_idx: optional (M,) int array naming the coincident source of each
    target (-1 = none) when trg is given explicitly.
    Returns pot (M,) or (pot, grad (M, d)).
    """
    L, d = _lattice(L)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, d)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    if trg is None:
        trg = src
        self_idx = np.arange(src.shape[0], dtype=np.int64)
    trg = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, d)
    if self_idx is not None:
        self_idx = np.ascontiguousarray(self_idx, dtype=np.int64)
    if alpha is None:
        alpha = choose_alpha(L, src.shape[0], trg.shape[0])
    rcut = tol_s / alpha
    kcut = 2.0 * alpha * tol_s
    pot = np.zeros(trg.shape[0])
    g = np.zeros((trg.shape[0], d)) if grad else None
    rc = _load().oracle_ewald(d, _dp(L), src.shape[0], _dp(src), _dp(q), trg.shape[0],
                              _dp(trg), _lp(self_idx), alpha, rcut, kcut, _dp(pot),
                              _dp(g) if grad else None)
    if rc != 0:
        raise ValueError("oracle_ewald failed with code %d" % rc)
    return (pot, g) if grad else pot


def ewald_sampled(L, src, q, idx, grad=False, alpha=None):
    """Ewald values at the sources listed in idx (targets = sources, self removed)."""
    L, d = _lattice(L)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, d)
    idx = np.asarray(idx, dtype=np.int64)
    return ewald(L, src, q, trg=src[idx], grad=grad, alpha=alpha, self_idx=idx)


def ewald_bloch(L, src, q, beta, trg=None, alpha=None, self_idx=None, tol_s=_S):
    """Quasi-periodic (Bloch) potential of Section 4.1 by Ewald summation
    (bloch.c): sum_n sum_j q_j e^{i beta.L n} G(x - y_j - L n), self pair
    removed, positions taken literally (not wrapped).  Returns a complex
    array (M,).  trg=None: targets are the sources."""
    L, d = _lattice(L)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, d)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(d)
    if trg is None:
        trg = src
        self_idx = np.arange(src.shape[0], dtype=np.int64)
    trg = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, d)
    if self_idx is not None:
        self_idx = np.ascontiguousarray(self_idx, dtype=np.int64)
    if alpha is None:
        alpha = choose_alpha(L, src.shape[0], trg.shape[0])
    re = np.zeros(trg.shape[0])
    im = np.zeros(trg.shape[0])
    rc = _load().oracle_ewald_bloch(d, _dp(L), _dp(beta), src.shape[0], _dp(src), _dp(q),
                                    trg.shape[0], _dp(trg), _lp(self_idx), alpha,
                                    tol_s / alpha, 2.0 * alpha * tol_s, _dp(re), _dp(im))
    if rc == -2:
        raise ValueError("beta is in the reciprocal lattice (the periodic case)")
    if rc != 0:
        raise ValueError("oracle_ewald_bloch failed with code %d" % rc)
    return re + 1j * im


def ewald_bloch_sampled(L, src, q, beta, idx, alpha=None):
    """Bloch values at the sources listed in idx (self pair removed)."""
    L, d = _lattice(L)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, d)
    idx = np.asarray(idx, dtype=np.int64)
    return ewald_bloch(L, src, q, beta, trg=src[idx], alpha=alpha, self_idx=idx)


def nmodes(L, alpha, tol_s=_S):
    L, d = _lattice(L)
    return _load().oracle_ewald_nmodes(d, _dp(L), alpha, 2.0 * alpha * tol_s)


def ball_sum(L, src, q, trg, R, self_idx=None):
    """Plain image sum over whole cells with |L n| <= R."""
    L, d = _lattice(L)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, d)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    trg = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, d)
    if self_idx is not None:
        self_idx = np.ascontiguousarray(self_idx, dtype=np.int64)
    pot = np.zeros(trg.shape[0])
    _load().oracle_ball_sum(d, _dp(L), src.shape[0], _dp(src), _dp(q), trg.shape[0],
                            _dp(trg), _lp(self_idx), float(R), _dp(pot))
    return pot


def threads() -> int:
    """OpenMP threads the oracle's sums use."""
    return int(_load().oracle_threads())


def rel_l2(approx, ref) -> float:
    """Relative l2 error ||approx - ref|| / ||ref||."""
    approx = np.asarray(approx, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(approx - ref) / np.linalg.norm(ref))
