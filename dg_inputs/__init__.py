"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no part of the discontinuous Galerkin arithmetic: it only
draws meshes, field noise and problem mixes from seeds, and evaluates a
closed-form initial condition at coordinates that the caller supplies.  Both
the FP64 CPU oracle and the HIP library receive exactly these arrays, so the
two implementations never share a line of the method itself.

Mesh recipe (the paper leaves its Maxwell test meshes unspecified beyond
being large, three-dimensional and made of face-conforming tetrahedra,
Sections 2 and 5): the unit cube [0,1]^3 cut into
k^3 hexahedra, each split into the six Kuhn tetrahedra that share the main
diagonal, interior vertices jittered uniformly by up to 10% of h = 1/k.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "kuhn_cube",
    "cavity_mode",
    "cavity_omega",
    "field_noise",
    "batch_draws",
    "k_for_dofs",
    "FACE_VERTS",
    "cube_face_bc",
    "random_face_bc",
]

#: local vertices of face f of a tetrahedron, in the face numbering of the
#: library's interface (face_bc[k][f] refers to face f of element k)
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))

# The six axis permutations; tetrahedron p of a cube walks the cube corners
# v0 -> v0+e[p0] -> v0+e[p0]+e[p1] -> v0+(1,1,1).
_KUHN_PERMS = tuple(itertools.permutations(range(3)))


def kuhn_cube(k: int, jitter: float = 0.1, seed: int = 0):
    """Jittered Kuhn mesh of the unit cube.

    Returns ``(VX, EToV)``: VX is (Nv, 3) float64 vertex coordinates and EToV is
    (6 k^3, 4) int32 vertex indices, 0-based, every element positively
    oriented (det[v1-v0, v2-v0, v3-v0] > 0).

    Vertex (i, j, l) sits at (i, j, l) * h with index (i*(k+1) + j)*(k+1) + l.
    Jitter: one draw of shape (Nv, 3) from U(-jitter*h, jitter*h) with
    ``numpy.random.default_rng(seed)``, applied to interior vertices only, in
    vertex-index order.  Boundary vertices stay on the cube faces.
    """
    if k < 1:
        raise ValueError("k must be >= 1")
    h = 1.0 / k
    n1 = k + 1
    ii, jj, ll = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    lattice = np.stack([ii.ravel(), jj.ravel(), ll.ravel()], axis=1)
    VX = lattice.astype(np.float64) * h
    rng = np.random.default_rng(seed)
    draw = rng.uniform(-jitter * h, jitter * h, size=VX.shape)
    interior = np.all((lattice > 0) & (lattice < k), axis=1)
    VX[interior] += draw[interior]

    def vid(i, j, l):
        return (i * n1 + j) * n1 + l

    cubes = np.stack(np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij"), axis=-1).reshape(-1, 3)
    elems = []
    eye = np.eye(3, dtype=np.int64)
    for c in cubes:
        for p in _KUHN_PERMS:
            a = c
            b = a + eye[p[0]]
            d = b + eye[p[1]]
            e = c + 1
            elems.append([vid(*a), vid(*b), vid(*d), vid(*e)])
    EToV = np.asarray(elems, dtype=np.int64)
    # Orientation fix: swap the last two vertices where the signed volume is negative.
    x0 = VX[EToV[:, 0]]
    m = np.stack([VX[EToV[:, 1]] - x0, VX[EToV[:, 2]] - x0, VX[EToV[:, 3]] - x0], axis=2)
    neg = np.linalg.det(m) < 0.0
    EToV[neg, 2], EToV[neg, 3] = EToV[neg, 3].copy(), EToV[neg, 2].copy()
    return VX, EToV.astype(np.int32)


def cavity_omega() -> float:
    """Angular frequency of the (1,1,0) mode of the unit PEC cube: pi*sqrt(2)."""
    return math.pi * math.sqrt(2.0)


def cavity_mode(x, y, z, t: float = 0.0):
    """Closed-form PEC-cavity eigenmode of the unit cube (eps = mu = 1).

    E = (0, 0, sin(pi x) sin(pi y) cos(w t)),
    H = (-(pi/w) sin(pi x) cos(pi y) sin(w t), (pi/w) cos(pi x) sin(pi y) sin(w t), 0),
    w = pi*sqrt(2).  It solves dE/dt = curl H, dH/dt = -curl E with n x E = 0
    on all six walls.  Returns an array of shape (6,) + x.shape in the field
    order (Ex, Ey, Ez, Hx, Hy, Hz).
    """
    w = cavity_omega()
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sx, cx = np.sin(np.pi * x), np.cos(np.pi * x)
    sy, cy = np.sin(np.pi * y), np.cos(np.pi * y)
    zero = np.zeros_like(x)
    ez = sx * sy * math.cos(w * t)
    hx = -(math.pi / w) * sx * cy * math.sin(w * t)
    hy = (math.pi / w) * cx * sy * math.sin(w * t)
    return np.stack([zero, zero, ez, hx, hy, zero.copy()])


def field_noise(shape, sigma: float = 1e-3, seed: int = 1):
    """Seeded N(0, sigma^2) noise, one draw per degree of freedom."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=shape)


def batch_draws(n: int = 64, seed: int = 2, k_range=(4, 20), n_range=(2, 7)):
    """Problem mix for batched solves: per problem (k, N, mesh_seed).

    k ~ U{k_range}, N ~ U{n_range} (both inclusive), mesh seed 1000 + p.
    """
    rng = np.random.default_rng(seed)
    ks = rng.integers(k_range[0], k_range[1] + 1, size=n)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n)
    return [(int(ks[p]), int(ns[p]), 1000 + p) for p in range(n)]


def k_for_dofs(N: int, dofs_per_field: float = 1e7) -> int:
    """Cube resolution k with 6 k^3 elements giving about ``dofs_per_field``
    nodal values per field at order N."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    return int(round((dofs_per_field / (6 * Np)) ** (1.0 / 3.0)))


def cube_face_bc(VX, EToV, sides):
    """Boundary-condition codes per (element, face) for a mesh of the unit cube.

    ``sides`` maps a cube side name ("x0", "x1", "y0", "y1", "z0", "z1": the
    plane x = 0, x = 1, ...) to a code; a face whose three vertices lie on that
    plane gets it, every other face 0.  Returns (K, 4) int8.
    """
    VX = np.asarray(VX, dtype=np.float64)
    EToV = np.asarray(EToV)
    out = np.zeros((EToV.shape[0], 4), dtype=np.int8)
    for f, fv in enumerate(FACE_VERTS):
        pts = VX[EToV[:, list(fv)]]                       # (K, 3, 3)
        for name, code in sides.items():
            axis, val = "xyz".index(name[0]), float(name[1])
            on = np.all(np.abs(pts[:, :, axis] - val) < 1e-12, axis=1)
            out[on, f] = code
    return out


def random_face_bc(K: int, seed: int, codes=(0, 1, 2)):
    """Seeded uniform draw of a code per (element, face): (K, 4) int8."""
    rng = np.random.default_rng(seed)
    return np.asarray(codes, dtype=np.int8)[rng.integers(0, len(codes), size=(K, 4))]
