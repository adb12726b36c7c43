"""Affine geometry and connectivity for the DG oracle (FP64, NumPy).  Test infrastructure only.

Geometry follows the reference-matrix form for affine simplices (Section 2.1
of the paper): the map from the reference tetrahedron is
x(r,s,t) = -(1+r+s+t)/2 x0 + (1+r)/2 x1 + (1+s)/2 x2 + (1+t)/2 x3, so the
Jacobian matrix, J_k = det and the inverse metric (rx .. tz) are constant per
element.  Face normals and face Jacobians are taken from the physical
vertices directly (cross product, outward by a centroid test), a different
route from the library's inverse-metric formula; sJ = face area / 2 (2 is the
area of the reference triangle the face mass matrix integrates over) and
Fscale = sJ / J.

Connectivity (the "flux gather" of Section 2.1 picks facial nodes of the
neighbour): faces are matched by their sorted vertex triple, face nodes by
physical coordinates (nearest node; tolerance 1e-10 of the smallest edge).
Unmatched faces are boundary faces.  Each boundary face carries a condition
code (the boundary data of Section 2 on the domain boundary; the paper leaves
the condition open): 0 perfectly conducting wall (the default), 1 perfectly
magnetic-conducting wall, 2 absorbing face (zero exterior state).  The codes
are read from ``face_bc[k, f]`` for unmatched faces and ignored elsewhere.

Parity: pinned by tests/test_oracle_mesh.py (cube volume, boundary area,
J = h^3/8 on the unjittered mesh, outward normals, coordinate equality of
matched traces, boundary-face count 12 k^2).
"""
from __future__ import annotations

import numpy as np

from .refelem import FACE_VERTS, ref_element


class Mesh:
    """Mesh data at order N.

    x, y, z        (K, Np) node coordinates
    rx .. tz       (K,) inverse metric terms; J (K,)
    nx, ny, nz     (K, 4) outward unit normals; sJ, Fscale (K, 4)
    EToE, EToF     (K, 4) neighbour element / face, -1 on the boundary
    vmapP          (K, 4, Nfp) flat index k*Np + i of the neighbour trace node,
                   -1 on boundary faces
    bc             (K, 4) boundary condition code of boundary faces (0, 1, 2),
                   -1 on interior faces
    eps, mu        (K,) permittivity and permeability, constant per element
                   (default 1); Z = sqrt(mu / eps) the impedance
    """

    def __init__(self, N: int, VX, EToV, face_bc=None, eps=None, mu=None):
        re = ref_element(N)
        self.re = re
        self.N, self.Np, self.Nfp = N, re.Np, re.Nfp
        VX = np.asarray(VX, dtype=np.float64)
        EToV = np.asarray(EToV, dtype=np.int64)
        self.K = K = EToV.shape[0]
        self.VX, self.EToV = VX, EToV
        v = VX[EToV]  # (K, 4, 3)
        # Node coordinates.
        lam = np.stack([-(1 + re.r + re.s + re.t) / 2, (1 + re.r) / 2, (1 + re.s) / 2, (1 + re.t) / 2], axis=1)
        X = np.einsum("iv,kvd->kid", lam, v)
        self.x, self.y, self.z = X[..., 0], X[..., 1], X[..., 2]
        # Metric.
        A = 0.5 * np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)  # (K, xyz, rst)
        self.J = np.linalg.det(A)
        if np.any(self.J <= 0):
            raise ValueError("non-positive Jacobian in element %d" % int(np.argmin(self.J)))
        Ainv = np.linalg.inv(A)  # rows: r, s, t; cols: x, y, z
        self.rx, self.ry, self.rz = Ainv[:, 0, 0], Ainv[:, 0, 1], Ainv[:, 0, 2]
        self.sx, self.sy, self.sz = Ainv[:, 1, 0], Ainv[:, 1, 1], Ainv[:, 1, 2]
        self.tx, self.ty, self.tz = Ainv[:, 2, 0], Ainv[:, 2, 1], Ainv[:, 2, 2]
        # Faces.
        cen = v.mean(axis=1)
        n = np.zeros((K, 4, 3))
        area = np.zeros((K, 4))
        for f, (a, b, c) in enumerate(FACE_VERTS):
            cr = np.cross(v[:, b] - v[:, a], v[:, c] - v[:, a])
            nr = np.linalg.norm(cr, axis=1)
            out = np.einsum("kd,kd->k", cr, (v[:, a] + v[:, b] + v[:, c]) / 3 - cen)
            sign = np.where(out > 0, 1.0, -1.0)
            n[:, f] = sign[:, None] * cr / nr[:, None]
            area[:, f] = 0.5 * nr
        self.nx, self.ny, self.nz = n[..., 0], n[..., 1], n[..., 2]
        self.sJ = area / 2.0
        self.Fscale = self.sJ / self.J[:, None]
        self._connect(X, v)
        codes = np.zeros((K, 4), dtype=np.int64) if face_bc is None else np.asarray(face_bc, dtype=np.int64)
        if codes.shape != (K, 4):
            raise ValueError("face_bc must have shape (K, 4)")
        bnd = self.EToE < 0
        if np.any((codes[bnd] < 0) | (codes[bnd] > 2)):
            raise ValueError("boundary condition codes must be 0, 1 or 2")
        self.bc = np.where(bnd, codes, -1)
        self.eps = np.ones(K) if eps is None else np.asarray(eps, dtype=np.float64).reshape(K)
        self.mu = np.ones(K) if mu is None else np.asarray(mu, dtype=np.float64).reshape(K)
        if not (np.all(np.isfinite(self.eps)) and np.all(self.eps > 0) and np.all(np.isfinite(self.mu))
                and np.all(self.mu > 0)):
            raise ValueError("eps and mu must be finite and positive")
        self.Z = np.sqrt(self.mu / self.eps)

    def _connect(self, X, v):
        K, Np, Nfp = self.K, self.Np, self.Nfp
        Fmask = self.re.Fmask
        keys = {}
        self.EToE = -np.ones((K, 4), dtype=np.int64)
        self.EToF = -np.ones((K, 4), dtype=np.int64)
        ev = self.EToV
        for k in range(K):
            for f, fv in enumerate(FACE_VERTS):
                key = tuple(sorted(int(ev[k, i]) for i in fv))
                if key in keys:
                    k2, f2 = keys.pop(key)
                    self.EToE[k, f], self.EToF[k, f] = k2, f2
                    self.EToE[k2, f2], self.EToF[k2, f2] = k, f
                else:
                    keys[key] = (k, f)
        # Coordinate matching of face nodes.
        edges = [np.linalg.norm(v[:, i] - v[:, j], axis=1) for i in range(4) for j in range(i + 1, 4)]
        hmin = float(np.min(edges))
        tol = 1e-10 * hmin
        self.vmapP = -np.ones((K, 4, Nfp), dtype=np.int64)
        self.max_match_dist = 0.0
        chunk = 4096
        for k0 in range(0, K, chunk):
            ks = np.arange(k0, min(K, k0 + chunk))
            for f in range(4):
                nb = self.EToE[ks, f]
                inner = nb >= 0
                if not np.any(inner):
                    continue
                kk, nbk = ks[inner], nb[inner]
                nbf = self.EToF[kk, f]
                own = X[kk][:, Fmask[f], :]                          # (n, Nfp, 3)
                oth = X[nbk[:, None], Fmask[nbf], :]                 # (n, Nfp, 3)
                d = np.linalg.norm(own[:, :, None, :] - oth[:, None, :, :], axis=3)
                j = np.argmin(d, axis=2)
                dmin = np.take_along_axis(d, j[:, :, None], axis=2)[..., 0]
                self.max_match_dist = max(self.max_match_dist, float(dmin.max()))
                if dmin.max() > tol:
                    raise ValueError("face nodes do not match within tolerance")
                nbnode = np.take_along_axis(Fmask[nbf], j, axis=1)
                self.vmapP[kk, f, :] = nbk[:, None] * Np + nbnode
        self.n_boundary_faces = int(np.sum(self.EToE < 0))
