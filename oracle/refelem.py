"""Reference tetrahedron for the nodal DG oracle (FP64, NumPy).  Test infrastructure only.

Follows Section 2 of the paper: a nodal Lagrange basis of P_N on a set of
interpolation nodes (the warp-and-blend family the paper cites), the mass,
stiffness and differentiation matrices of the global-matrix definitions,
D = M^-1 S, the face mass matrices M^A, and the lifting matrix L built as in
the figure on its construction (face masses embedded, then M^-1).  The
reference-matrix form for affine simplices (Section 2.1) means only these
reference matrices are needed.

Readings where the paper is silent (each listed in the design notes):
  * reference tetrahedron with vertices v0=(-1,-1,-1), v1=(1,-1,-1),
    v2=(-1,1,-1), v3=(-1,-1,1); faces 0: t=-1 (v0 v1 v2), 1: s=-1 (v0 v1 v3),
    2: r+s+t=-1 (v1 v2 v3), 3: r=-1 (v0 v2 v3);
  * nodes: Warburton's explicit warp & blend construction on a regular
    tetrahedron of edge length 2 with the optimised blend parameters alpha(N)
    of that construction; node order: t index outermost, then s, then r;
  * operators from an orthonormal (collapsed-coordinate Jacobi) basis:
    V = psi(nodes), Dr = Vr V^-1, M = (V V^T)^-1, LIFT = V V^T E.

Parity: every function is pinned by tests/test_oracle_refelem.py against
quadrature, exact differentiation of monomials, the discrete divergence
theorem (SBP identity), symmetry of the node set and library GLL points.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import roots_jacobi

# Optimised warp & blend parameters alpha(N), N = 1..15 (warp & blend paper);
# N above 15 uses 1.
_ALPHA_OPT = (0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603,
              1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655)

# Reference vertices and faces (vertex ids) -- see module docstring.
REF_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
# Two reference coordinates (indices into (r, s, t)) that parametrise each face
# as the 2D reference triangle {(-1,-1), (1,-1), (-1,1)}.
FACE_PARAM = ((0, 1), (0, 2), (1, 2), (1, 2))


def n_p(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_fp(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def alpha_opt(N: int) -> float:
    return _ALPHA_OPT[N - 1] if 1 <= N <= len(_ALPHA_OPT) else 1.0


# ----------------------------------------------------------------------------
# Orthonormal Jacobi polynomials (weight (1-x)^a (1+x)^b on [-1, 1])
# ----------------------------------------------------------------------------
def jacobi_p(x, a: float, b: float, n: int):
    """Orthonormal Jacobi polynomial P_n^(a,b)(x) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    g0 = 2.0 ** (a + b + 1) / (a + b + 1) * math.gamma(a + 1) * math.gamma(b + 1) / math.gamma(a + b + 1)
    p_prev = np.full_like(x, 1.0 / math.sqrt(g0))
    if n == 0:
        return p_prev
    g1 = (a + 1) * (b + 1) / (a + b + 3) * g0
    p_cur = ((a + b + 2) * x / 2 + (a - b) / 2) / math.sqrt(g1)
    if n == 1:
        return p_cur
    a_old = 2.0 / (2 + a + b) * math.sqrt((a + 1) * (b + 1) / (a + b + 3))
    for i in range(1, n):
        h = 2 * i + a + b
        a_new = 2.0 / (h + 2) * math.sqrt((i + 1) * (i + 1 + a + b) * (i + 1 + a) * (i + 1 + b) / ((h + 1) * (h + 3)))
        b_new = -(a * a - b * b) / (h * (h + 2))
        p_next = (-a_old * p_prev + (x - b_new) * p_cur) / a_new
        p_prev, p_cur = p_cur, p_next
        a_old = a_new
    return p_cur


def grad_jacobi_p(x, a: float, b: float, n: int):
    """d/dx of the orthonormal P_n^(a,b): sqrt(n (n+a+b+1)) P_{n-1}^(a+1,b+1)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return math.sqrt(n * (n + a + b + 1)) * jacobi_p(x, a + 1, b + 1, n - 1)


def gll_points(N: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points on [-1, 1], ascending: -1, roots of P_N', 1.

    The interior points are the Gauss-Jacobi(1,1) points of degree N-1
    (library routine)."""
    if N == 1:
        return np.array([-1.0, 1.0])
    xi, _ = roots_jacobi(N - 1, 1.0, 1.0)
    return np.concatenate([[-1.0], np.sort(xi), [1.0]])


# ----------------------------------------------------------------------------
# Warp & blend nodes
# ----------------------------------------------------------------------------
def lattice(N: int) -> np.ndarray:
    """Integer barycentric lattice (l0, l1, l2, l3), sum N, in node order.

    l1, l2, l3 are the r, s, t lattice indices; t index outermost, r innermost."""
    out = []
    for n in range(N + 1):
        for m in range(N + 1 - n):
            for q in range(N + 1 - n - m):
                out.append((N - q - m - n, q, m, n))
    return np.asarray(out, dtype=np.int64)


def warp_over_bubble(N: int, x):
    """1D warp divided by (1 - x^2).

    The warp interpolates, with the equispaced Lagrange basis, the displacement
    from the N+1 equispaced points to the GLL points; both end displacements
    vanish, so dividing by (1 - x^2) leaves a polynomial, evaluated here as
    sum_i d_i prod_{j interior, j != i} (x - e_j)/(e_i - e_j) / (1 - e_i^2).
    """
    x = np.asarray(x, dtype=np.float64)
    e = -1.0 + 2.0 * np.arange(N + 1) / N
    d = gll_points(N) - e
    out = np.zeros_like(x)
    for i in range(1, N):
        term = np.full_like(x, d[i] / (1.0 - e[i] * e[i]))
        for j in range(1, N):
            if j != i:
                term = term * (x - e[j]) / (e[i] - e[j])
        out = out + term
    return out


def _equilateral_vertices():
    """Regular tetrahedron of edge length 2; vertex i stands for reference vertex i."""
    return np.array([[-1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
                     [1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
                     [0.0, 2.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
                     [0.0, 0.0, 3.0 / math.sqrt(6.0)]])


def _face_warp(N, alpha, P, lam, face):
    """Warp of face ``face`` (vertex ids) at barycentrics ``lam`` (n, 4): for each
    edge (i, j) of the face with third face vertex k, the edge warp blended by
    4 l_i l_j (1 + (alpha l_k)^2), directed from vertex i to vertex j."""
    b, c, d = face
    out = np.zeros((lam.shape[0], 3))
    for (i, j, k) in ((b, c, d), (c, d, b), (d, b, c)):
        direction = (P[j] - P[i]) / np.linalg.norm(P[j] - P[i])
        amp = 4.0 * lam[:, i] * lam[:, j] * warp_over_bubble(N, lam[:, j] - lam[:, i]) * (1.0 + (alpha * lam[:, k]) ** 2)
        out += amp[:, None] * direction[None, :]
    return out


@lru_cache(maxsize=None)
def nodes(N: int):
    """Warp & blend interpolation nodes (r, s, t) on the reference tetrahedron.

    Interior lattice points take the sum over the four faces of the face warp
    times the volume blend l_b l_c l_d (1 + (alpha l_a)^2) / prod(l_x + l_a/2)
    (l_a: barycentric of the vertex opposite the face); face-interior points
    take their face's warp; edge points the 1D edge warp; vertices stay.
    """
    if N < 1:
        raise ValueError("N >= 1")
    alpha = alpha_opt(N)
    L = lattice(N)
    lam = L.astype(np.float64) / N
    P = _equilateral_vertices()
    X = lam @ P
    shift = np.zeros_like(X)
    zeros = (L == 0).sum(axis=1)
    opposite = {0: 3, 1: 2, 2: 0, 3: 1}
    for f, face in enumerate(FACE_VERTS):
        a = opposite[f]
        fw = _face_warp(N, alpha, P, lam, face)
        lb, lc, ld = lam[:, face[0]], lam[:, face[1]], lam[:, face[2]]
        la = lam[:, a]
        denom = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la)
        blend = np.zeros_like(la)
        ok = zeros == 0
        blend[ok] = lb[ok] * lc[ok] * ld[ok] * (1.0 + (alpha * la[ok]) ** 2) / denom[ok]
        shift[ok] += blend[ok, None] * fw[ok]
        on_face = (zeros == 1) & (L[:, a] == 0)
        shift[on_face] = fw[on_face]
    # Edge points: the 1D warp along the edge.
    for i in range(4):
        for j in range(i + 1, 4):
            sel = (zeros == 2) & (L[:, i] > 0) & (L[:, j] > 0)
            if np.any(sel):
                direction = (P[j] - P[i]) / np.linalg.norm(P[j] - P[i])
                amp = 4.0 * lam[sel, i] * lam[sel, j] * warp_over_bubble(N, lam[sel, j] - lam[sel, i])
                shift[sel] = amp[:, None] * direction[None, :]
    X = X + shift
    A = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)
    rst = 2.0 * np.linalg.solve(A, (X - P[0]).T) - 1.0
    return rst[0].copy(), rst[1].copy(), rst[2].copy()


# ----------------------------------------------------------------------------
# Orthonormal basis on the tetrahedron (collapsed coordinates)
# ----------------------------------------------------------------------------
def collapse(r, s, t):
    """(r, s, t) -> (a, b, c) with a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t;
    the degenerate edge/vertex take a = -1 / b = -1."""
    r, s, t = (np.asarray(v, dtype=np.float64) for v in (r, s, t))
    a = np.full_like(r, -1.0)
    b = np.full_like(r, -1.0)
    den = -(s + t)
    nz = den != 0.0
    a[nz] = 2.0 * (1.0 + r[nz]) / den[nz] - 1.0
    nz = t != 1.0
    b[nz] = 2.0 * (1.0 + s[nz]) / (1.0 - t[nz]) - 1.0
    return a, b, t.copy()


def modes(N: int):
    return [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i) for k in range(N + 1 - i - j)]


def basis(r, s, t, i, j, k):
    """psi_ijk = 2 sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i P_k^(2i+2j+2,0)(c) (1-c)^(i+j)."""
    a, b, c = collapse(r, s, t)
    return (2.0 * math.sqrt(2.0) * jacobi_p(a, 0, 0, i) * jacobi_p(b, 2 * i + 1, 0, j) * (1 - b) ** i
            * jacobi_p(c, 2 * i + 2 * j + 2, 0, k) * (1 - c) ** (i + j))


def grad_basis(r, s, t, i, j, k):
    """(d/dr, d/ds, d/dt) psi_ijk by the chain rule through (a, b, c), with the
    (1-b), (1-c) powers reduced analytically so no 0/0 appears."""
    a, b, c = collapse(r, s, t)
    f, df = jacobi_p(a, 0, 0, i), grad_jacobi_p(a, 0, 0, i)
    g, dg = jacobi_p(b, 2 * i + 1, 0, j), grad_jacobi_p(b, 2 * i + 1, 0, j)
    h, dh = jacobi_p(c, 2 * i + 2 * j + 2, 0, k), grad_jacobi_p(c, 2 * i + 2 * j + 2, 0, k)
    nrm = 2.0 * math.sqrt(2.0)
    # d psi / d r
    if i > 0:
        dr = nrm * 4.0 * df * g * (1 - b) ** (i - 1) * h * (1 - c) ** (i + j - 1)
    else:
        dr = np.zeros_like(a)
    # d/db [g (1-b)^i]
    dgb = dg * (1 - b) ** i
    if i > 0:
        dgb = dgb - i * g * (1 - b) ** (i - 1)
    if i + j > 0:
        hc_red = h * (1 - c) ** (i + j - 1)
    else:
        hc_red = np.zeros_like(c)  # multiplies dgb, which is 0 when i = j = 0
    ds = 0.5 * (1 + a) * dr + nrm * f * dgb * 2.0 * hc_red
    dhc = dh * (1 - c) ** (i + j)
    if i + j > 0:
        dhc = dhc - (i + j) * h * (1 - c) ** (i + j - 1)
    dt = 0.5 * (1 + a) * dr + nrm * f * dgb * (1 + b) * hc_red + nrm * f * g * (1 - b) ** i * dhc
    return dr, ds, dt


def vandermonde(N, r, s, t):
    return np.stack([basis(r, s, t, *m) for m in modes(N)], axis=1)


def grad_vandermonde(N, r, s, t):
    g = [grad_basis(r, s, t, *m) for m in modes(N)]
    return tuple(np.stack([x[d] for x in g], axis=1) for d in range(3))


def basis2d(r, s, i, j):
    """Orthonormal basis on the reference triangle: sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i,
    a = 2(1+r)/(1-s) - 1 (a = -1 at s = 1), b = s."""
    r, s = np.asarray(r, dtype=np.float64), np.asarray(s, dtype=np.float64)
    a = np.full_like(r, -1.0)
    nz = s != 1.0
    a[nz] = 2.0 * (1.0 + r[nz]) / (1.0 - s[nz]) - 1.0
    return math.sqrt(2.0) * jacobi_p(a, 0, 0, i) * jacobi_p(s, 2 * i + 1, 0, j) * (1 - s) ** i


def vandermonde2d(N, r, s):
    return np.stack([basis2d(r, s, i, j) for i in range(N + 1) for j in range(N + 1 - i)], axis=1)


# ----------------------------------------------------------------------------
# Reference element
# ----------------------------------------------------------------------------
class RefElement:
    """All reference-element data at order N (FP64).

    Attributes: N, Np, Nfp, r, s, t, V, Vr, Vs, Vt, Dr, Ds, Dt, M, Fmask (4, Nfp),
    Mf (4, Nfp, Nfp) face mass matrices in each face's own node order,
    Emat (Np, 4 Nfp), LIFT (Np, 4 Nfp).
    """

    def __init__(self, N: int):
        if not 1 <= N <= 15:
            raise ValueError("N must be in 1..15")
        self.N, self.Np, self.Nfp = N, n_p(N), n_fp(N)
        self.r, self.s, self.t = nodes(N)
        self.V = vandermonde(N, self.r, self.s, self.t)
        self.Vr, self.Vs, self.Vt = grad_vandermonde(N, self.r, self.s, self.t)
        Vinv = np.linalg.inv(self.V)
        self.Dr, self.Ds, self.Dt = self.Vr @ Vinv, self.Vs @ Vinv, self.Vt @ Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)
        self.Fmask = self._fmask()
        rst = (self.r, self.s, self.t)
        self.Mf = np.zeros((4, self.Nfp, self.Nfp))
        self.Emat = np.zeros((self.Np, 4 * self.Nfp))
        for f in range(4):
            p, q = FACE_PARAM[f]
            idx = self.Fmask[f]
            V2 = vandermonde2d(N, rst[p][idx], rst[q][idx])
            self.Mf[f] = np.linalg.inv(V2 @ V2.T)
            self.Emat[idx, f * self.Nfp:(f + 1) * self.Nfp] = self.Mf[f]
        self.LIFT = self.V @ (self.V.T @ self.Emat)

    def _fmask(self):
        """Face node lists (ascending node index) by coordinate test, tolerance 1e-7."""
        r, s, t = self.r, self.s, self.t
        tol = 1e-7
        tests = (np.abs(1 + t) < tol, np.abs(1 + s) < tol, np.abs(1 + r + s + t) < tol, np.abs(1 + r) < tol)
        fm = [np.nonzero(m)[0] for m in tests]
        for m in fm:
            if len(m) != self.Nfp:
                raise RuntimeError("face node count mismatch")
        return np.stack(fm)


@lru_cache(maxsize=None)
def ref_element(N: int) -> RefElement:
    return RefElement(N)


# ----------------------------------------------------------------------------
# Quadrature (used to pin M and S against their integral definitions)
# ----------------------------------------------------------------------------
def tet_quadrature(q: int):
    """Collapsed Gauss-Jacobi rule with q points per direction, exact to degree 2q-1.

    r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c,
    dr ds dt = (1-b)(1-c)^2/8 da db dc; the (1-b) and (1-c)^2 factors are the
    Jacobi weights of the b and c rules (library routine)."""
    xa, wa = roots_jacobi(q, 0.0, 0.0)
    xb, wb = roots_jacobi(q, 1.0, 0.0)
    xc, wc = roots_jacobi(q, 2.0, 0.0)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    W = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]) / 8.0
    r = (1 + A) * (1 - B) * (1 - C) / 4.0 - 1.0
    s = (1 + B) * (1 - C) / 2.0 - 1.0
    return r.ravel(), s.ravel(), C.ravel(), W.ravel()


def quadrature_mass_stiffness(N: int):
    """M_ij = int l_i l_j and S^nu_ij = int l_i d_nu l_j over the reference
    tetrahedron, by a rule exact to degree 2N+1 (definitions of Section 2)."""
    re = ref_element(N)
    rq, sq, tq, wq = tet_quadrature(N + 1)
    Vinv = np.linalg.inv(re.V)
    Lq = vandermonde(N, rq, sq, tq) @ Vinv
    dLq = [G @ Vinv for G in grad_vandermonde(N, rq, sq, tq)]
    M = Lq.T @ (wq[:, None] * Lq)
    S = [Lq.T @ (wq[:, None] * d) for d in dLq]
    return M, S
