"""Seeded synthetic inputs (lattice, sources, charges) for tests and benchmarks.

This module holds no arithmetic of the method: it only draws positions and
charges.  Both the oracle-side tests and the GPU-side tests call it, so the two
sides see identical inputs.  Every generator uses numpy's PCG64 with an
explicit seed; positions are drawn in fractional coordinates u in [0,1)^d and
returned in Cartesian form x = L u.  L has the lattice vectors as columns.

Workloads
---------
``oblique2d``   2D cell a1=(1,0), a2=(0.3,1); uniform sources; +-1 charges.
``clustered3d`` 3D cubic or triclinic cell (a1=(1,0,0), a2=(0.4,1.2,0),
                a3=(0.3,0.5,2)); 90% of points in a Gaussian cluster
                (sigma 0.02 per fractional axis, centre 0.5, wrapped), 10%
                uniform; N(0,1) charges shifted to zero mean.
``shell3d``     triclinic cell a1=(1,0,0), a2=(0.5,4,0), a3=(0.3,0.7,17)
                (edge ratio ~17); points on a thin spherical shell in
                fractional coordinates (centre 0.5, radius uniform in
                [0.2995, 0.3005], direction uniform on the sphere); +-1 charges.
``wavy3d``      the paper's wavy-sphere distribution (Section 6, source
                distributions: r = r0 + A sin(k theta) + eta) in the triclinic
                (all angles pi/3) or rectangular base cell with edges
                (1, sqrt2, sqrt3), optionally scaled; zero-mean N(0,1) charges.
``wavy2d``      the paper's wavy-ring distribution in the oblique cell
                a1 = (1, 0), a2 = A (cos pi/3, sin pi/3) of aspect ratio A.
``paper_system`` the nine cells of the paper's tables (2D A = 1, 10, 100;
                3D rectangular / triclinic x isotropic / rod / slab) with
                their wavy distributions.
``batch_cells`` random triclinic cells and sizes for batched evaluation.
"""
from __future__ import annotations

import math

import numpy as np

OBLIQUE2D_L = np.array([[1.0, 0.3], [0.0, 1.0]])
CUBIC3D_L = np.eye(3)
TRICLINIC3D_L = np.array([[1.0, 0.4, 0.3], [0.0, 1.2, 0.5], [0.0, 0.0, 2.0]])
SHELL3D_L = np.array([[1.0, 0.5, 0.3], [0.0, 4.0, 0.7], [0.0, 0.0, 17.0]])


def _pm_charges(rng, n):
    """n/2 charges +1 and n/2 charges -1 (n even), shuffled: exactly neutral."""
    if n % 2:
        raise ValueError("+-1 neutral charges need an even count")
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    rng.shuffle(q)
    return q


def _zero_mean_normal(rng, n):
    q = rng.standard_normal(n)
    return q - q.mean()


def oblique2d(n=2000, seed=1):
    rng = np.random.default_rng(seed)
    u = rng.random((n, 2))
    return OBLIQUE2D_L.copy(), u @ OBLIQUE2D_L.T, _pm_charges(rng, n)


def clustered3d(n=1_000_000, seed=2, cell="triclinic", frac_cluster=0.9, sigma=0.02):
    L = TRICLINIC3D_L.copy() if cell == "triclinic" else CUBIC3D_L.copy()
    rng = np.random.default_rng(seed)
    nc = int(round(frac_cluster * n))
    uc = 0.5 + sigma * rng.standard_normal((nc, 3))
    uu = rng.random((n - nc, 3))
    u = np.vstack([uc, uu])
    u -= np.floor(u)
    perm = rng.permutation(n)
    u = u[perm]
    return L, u @ L.T, _zero_mean_normal(rng, n)


def shell3d(n=10_000_000, seed=3, radius=0.3, width=1e-3):
    rng = np.random.default_rng(seed)
    dirs = rng.standard_normal((n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = radius + width * (rng.random(n) - 0.5)
    u = 0.5 + dirs * r[:, None]
    u -= np.floor(u)
    return SHELL3D_L.copy(), u @ SHELL3D_L.T, _pm_charges(rng, n)


def triclinic_base(scale=(1, 1, 1)):
    """Edges (1, sqrt2, sqrt3) pairwise at angle pi/3, each scaled by scale[i]."""
    lens = np.array([1.0, math.sqrt(2.0), math.sqrt(3.0)]) * np.asarray(scale, float)
    c = math.cos(math.pi / 3)
    a1 = np.array([1.0, 0.0, 0.0])
    a2 = np.array([c, math.sqrt(1 - c * c), 0.0])
    # a3 with a3.a1 = c, a3.a2 = c
    x = c
    y = (c - a2[0] * x) / a2[1]
    a3 = np.array([x, y, math.sqrt(1 - x * x - y * y)])
    return np.stack([a1 * lens[0], a2 * lens[1], a3 * lens[2]], axis=1)


def rectangular_base(scale=(1, 1, 1)):
    """Edges (1, sqrt2, sqrt3) at right angles, each scaled by scale[i]."""
    lens = np.array([1.0, math.sqrt(2.0), math.sqrt(3.0)]) * np.asarray(scale, float)
    return np.diag(lens)


def wavy3d(n=1_000_000, seed=6, scale=(1, 1, 1), r0=0.4, amp=0.05, k=32, sigma=0.01,
           cell="triclinic"):
    L = triclinic_base(scale) if cell == "triclinic" else rectangular_base(scale)
    rng = np.random.default_rng(seed)
    dirs = rng.standard_normal((n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    theta = np.arctan2(dirs[:, 1], dirs[:, 0])
    r = r0 + amp * np.sin(k * theta) + sigma * rng.standard_normal(n)
    u = 0.5 + dirs * r[:, None]
    u -= np.floor(u)
    return L, u @ L.T, _zero_mean_normal(rng, n)


def oblique_pi3(aspect=1.0):
    """a1 = (1, 0), a2 = aspect (cos pi/3, sin pi/3) as columns."""
    return np.array([[1.0, 0.5 * aspect], [0.0, 0.5 * math.sqrt(3.0) * aspect]])


def wavy2d(n=1_000_000, seed=7, aspect=1.0, r0=0.4, amp=0.05, k=32, sigma=0.01):
    """Ring of fractional radius r0 + amp sin(k theta) + N(0, sigma^2) about
    the cell centre, theta uniform on [0, 2 pi)."""
    L = oblique_pi3(aspect)
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, n)
    r = r0 + amp * np.sin(k * theta) + sigma * rng.standard_normal(n)
    u = 0.5 + np.stack([np.cos(theta), np.sin(theta)], axis=1) * r[:, None]
    u -= np.floor(u)
    return L, u @ L.T, _zero_mean_normal(rng, n)


# the cells of the paper's tables: 2D aspect ratios, 3D base cell x scaling
PAPER_SYSTEMS = {
    "2d-A1": ("2d", 1.0), "2d-A10": ("2d", 10.0), "2d-A100": ("2d", 100.0),
    "rect-iso": ("rect", (1, 1, 1)), "rect-rod": ("rect", (1, 1, 10)),
    "rect-slab": ("rect", (1, 10, 10)),
    "tri-iso": ("triclinic", (1, 1, 1)), "tri-rod": ("triclinic", (1, 1, 10)),
    "tri-slab": ("triclinic", (1, 10, 10)),
}


def paper_system(name, n, seed=8):
    """(L, src, q) of one of PAPER_SYSTEMS with n wavy sources."""
    kind, arg = PAPER_SYSTEMS[name]
    if kind == "2d":
        return wavy2d(n, seed=seed, aspect=arg)
    return wavy3d(n, seed=seed, scale=arg, cell=kind)


def random_triclinic_cell(rng):
    """Edge lengths 1, U[1,8], U[1,8]; angles U[60,120] degrees; rejected unless
    the cell is not too flat (Gram determinant > 0.05 * prod |a_i|^2)."""
    while True:
        lens = np.array([1.0, rng.uniform(1, 8), rng.uniform(1, 8)])
        al, be, ga = np.radians(rng.uniform(60, 120, 3))
        G = np.array([[1, math.cos(ga), math.cos(be)],
                      [math.cos(ga), 1, math.cos(al)],
                      [math.cos(be), math.cos(al), 1]]) * np.outer(lens, lens)
        if np.linalg.det(G) <= 0.05 * np.prod(lens ** 2):
            continue
        # lower-triangular Cholesky G = R^T R with R upper triangular
        R = np.linalg.cholesky(G).T
        return R


def batch_cells(n_sys=512, seed=5, n_min=500, n_max=50_000):
    """List of (L, src, q) systems: random triclinic cells, log-uniform sizes,
    even systems uniform and odd systems clustered, +-1 neutral charges."""
    out = []
    for s in range(n_sys):
        rng = np.random.default_rng(seed * 1000 + s)
        L = random_triclinic_cell(rng)
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) / 2)) * 2
        if s % 2 == 0:
            u = rng.random((n, 3))
        else:
            u = 0.5 + 0.02 * rng.standard_normal((n, 3))
            u -= np.floor(u)
        out.append((L, u @ L.T, _pm_charges(rng, n)))
    return out
