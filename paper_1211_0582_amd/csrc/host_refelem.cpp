// Reference tetrahedron of the nodal DG method (host, binary64).
//
// Section 2 of the paper: nodal Lagrange basis of P_N on interpolation nodes
// of the warp & blend family, differentiation matrices D = M^-1 S, face mass
// matrices, and the lifting matrix L = M^-1 [embedded face masses] of the
// figure on its construction.  Operators are formed through an orthonormal
// collapsed-coordinate (Proriol-Koornwinder-Dubiner) basis psi:
// V = psi(nodes), Dr = (d psi/dr)(nodes) V^-1, M^-1 = V V^T, LIFT = V V^T E.
//
// Nodes: Warburton's explicit warp & blend construction, evaluated on a
// regular tetrahedron of edge length 2: the 1D warp (equispaced -> Gauss-
// Lobatto-Legendre displacement) is blended along the edges into each face
// and the face warps into the volume with the optimised parameter alpha(N).
// Every node keeps its integer barycentric lattice point, which gives exact
// face membership (Fmask) and the face-node permutations between neighbours.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>

#include "host_common.hpp"

namespace dgh {

const int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
const int kFaceOpposite[4] = {3, 2, 0, 1};
const int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

namespace {

// Optimised blend parameter of the warp & blend construction, N = 1..15.
const double kAlphaOpt[15] = {0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577,
                              1.1603, 1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655};

// ---------------------------------------------------------------------------
// Orthonormal Jacobi polynomials, weight (1-x)^a (1+x)^b on [-1, 1].
// p_{n+1} = ((x - b_n) p_n - a_n p_{n-1}) / a_{n+1} with the normalised
// recurrence coefficients a_n, b_n.
double jacobi(double x, double a, double b, int n) {
  const double g0 = std::pow(2.0, a + b + 1) / (a + b + 1) * std::tgamma(a + 1) * std::tgamma(b + 1) /
                    std::tgamma(a + b + 1);
  double pm = 1.0 / std::sqrt(g0);
  if (n == 0) return pm;
  const double g1 = (a + 1) * (b + 1) / (a + b + 3) * g0;
  double pc = ((a + b + 2) * x * 0.5 + (a - b) * 0.5) / std::sqrt(g1);
  if (n == 1) return pc;
  double aold = 2.0 / (2 + a + b) * std::sqrt((a + 1) * (b + 1) / (a + b + 3));
  for (int i = 1; i < n; ++i) {
    const double h = 2.0 * i + a + b;
    const double anew = 2.0 / (h + 2) *
                        std::sqrt((i + 1) * (i + 1 + a + b) * (i + 1 + a) * (i + 1 + b) / ((h + 1) * (h + 3)));
    const double bnew = -(a * a - b * b) / (h * (h + 2));
    const double pn = (-aold * pm + (x - bnew) * pc) / anew;
    pm = pc;
    pc = pn;
    aold = anew;
  }
  return pc;
}

// d/dx of the orthonormal P_n^(a,b) = sqrt(n (n+a+b+1)) P_{n-1}^(a+1,b+1).
double djacobi(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + a + b + 1)) * jacobi(x, a + 1, b + 1, n - 1);
}

// Gauss-Lobatto-Legendre points, ascending: -1, zeros of P_N', +1.
// Newton on P_N' from the Chebyshev-Lobatto guesses, with
// (1-x^2) P'' = 2x P' - N(N+1) P.
std::vector<double> gll(int N) {
  std::vector<double> x(N + 1);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double z = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // Legendre P_0, P_1
      for (int k = 2; k <= N; ++k) {
        const double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_N, p0 = P_{N-1}
      const double dp = N * (p0 - z * p1) / (1.0 - z * z);
      const double d2p = (2.0 * z * dp - N * (N + 1.0) * p1) / (1.0 - z * z);
      const double dz = dp / d2p;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  std::sort(x.begin(), x.end());
  return x;
}

// The 1D warp divided by (1 - x^2): sum over interior equispaced points e_i of
// (gll_i - e_i) * prod_{j interior, j != i} (x - e_j)/(e_i - e_j) / (1 - e_i^2).
struct Warp {
  int N;
  std::vector<double> e, d;
  explicit Warp(int n) : N(n), e(n + 1), d(n + 1) {
    const std::vector<double> g = gll(n);
    for (int i = 0; i <= n; ++i) {
      e[i] = -1.0 + 2.0 * i / n;
      d[i] = g[i] - e[i];
    }
  }
  double operator()(double x) const {
    double w = 0.0;
    for (int i = 1; i < N; ++i) {
      double term = d[i] / (1.0 - e[i] * e[i]);
      for (int j = 1; j < N; ++j)
        if (j != i) term *= (x - e[j]) / (e[i] - e[j]);
      w += term;
    }
    return w;
  }
};

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 scal(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline double norm(V3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

void build_nodes(RefElement& re) {
  const int N = re.N;
  const double alpha = N <= 15 ? kAlphaOpt[N - 1] : 1.0;
  const Warp warp(N);
  const double s3 = std::sqrt(3.0), s6 = std::sqrt(6.0);
  const V3 P[4] = {{-1.0, -1.0 / s3, -1.0 / s6}, {1.0, -1.0 / s3, -1.0 / s6}, {0.0, 2.0 / s3, -1.0 / s6},
                   {0.0, 0.0, 3.0 / s6}};
  auto unit = [&](int i, int j) {
    V3 d = sub(P[j], P[i]);
    return scal(1.0 / norm(d), d);
  };
  // Affine map back to (r, s, t): X - P0 = A ((1+r)/2, (1+s)/2, (1+t)/2).
  const V3 c0 = sub(P[1], P[0]), c1 = sub(P[2], P[0]), c2 = sub(P[3], P[0]);
  const double det = c0.x * (c1.y * c2.z - c1.z * c2.y) - c1.x * (c0.y * c2.z - c0.z * c2.y) +
                     c2.x * (c0.y * c1.z - c0.z * c1.y);
  // Rows of A^-1 (cofactor form).
  const V3 i0 = scal(1.0 / det, {c1.y * c2.z - c1.z * c2.y, c1.z * c2.x - c1.x * c2.z, c1.x * c2.y - c1.y * c2.x});
  const V3 i1 = scal(1.0 / det, {c2.y * c0.z - c2.z * c0.y, c2.z * c0.x - c2.x * c0.z, c2.x * c0.y - c2.y * c0.x});
  const V3 i2 = scal(1.0 / det, {c0.y * c1.z - c0.z * c1.y, c0.z * c1.x - c0.x * c1.z, c0.x * c1.y - c0.y * c1.x});

  re.lat.clear();
  for (int n = 0; n <= N; ++n)
    for (int m = 0; m <= N - n; ++m)
      for (int q = 0; q <= N - n - m; ++q) re.lat.push_back({N - q - m - n, q, m, n});
  const int Np = int(re.lat.size());
  re.r.resize(Np);
  re.s.resize(Np);
  re.t.resize(Np);
  for (int p = 0; p < Np; ++p) {
    double lam[4];
    int zeros = 0;
    for (int v = 0; v < 4; ++v) {
      lam[v] = double(re.lat[p][v]) / N;
      zeros += re.lat[p][v] == 0;
    }
    V3 X = {0, 0, 0};
    for (int v = 0; v < 4; ++v) X = add(X, scal(lam[v], P[v]));
    auto face_warp = [&](int f) {
      const int b = kFaceVerts[f][0], c = kFaceVerts[f][1], d = kFaceVerts[f][2];
      const int tri[3][3] = {{b, c, d}, {c, d, b}, {d, b, c}};
      V3 w = {0, 0, 0};
      for (auto& e : tri) {
        const int i = e[0], j = e[1], k = e[2];
        const double amp = 4.0 * lam[i] * lam[j] * warp(lam[j] - lam[i]) * (1.0 + (alpha * lam[k]) * (alpha * lam[k]));
        w = add(w, scal(amp, unit(i, j)));
      }
      return w;
    };
    V3 shift = {0, 0, 0};
    if (zeros == 0) {
      for (int f = 0; f < 4; ++f) {
        const int a = kFaceOpposite[f];
        const double lb = lam[kFaceVerts[f][0]], lc = lam[kFaceVerts[f][1]], ld = lam[kFaceVerts[f][2]];
        const double la = lam[a];
        const double denom = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la);
        const double blend = lb * lc * ld * (1.0 + (alpha * la) * (alpha * la)) / denom;
        shift = add(shift, scal(blend, face_warp(f)));
      }
    } else if (zeros == 1) {
      for (int f = 0; f < 4; ++f)
        if (re.lat[p][kFaceOpposite[f]] == 0) shift = face_warp(f);
    } else if (zeros == 2) {
      int i = -1, j = -1;
      for (int v = 0; v < 4; ++v)
        if (re.lat[p][v] > 0) (i < 0 ? i : j) = v;
      shift = scal(4.0 * lam[i] * lam[j] * warp(lam[j] - lam[i]), unit(i, j));
    }
    X = add(X, shift);
    const V3 y = sub(X, P[0]);
    re.r[p] = 2.0 * (i0.x * y.x + i0.y * y.y + i0.z * y.z) - 1.0;
    re.s[p] = 2.0 * (i1.x * y.x + i1.y * y.y + i1.z * y.z) - 1.0;
    re.t[p] = 2.0 * (i2.x * y.x + i2.y * y.y + i2.z * y.z) - 1.0;
  }
}

// Orthonormal basis on the tetrahedron and its gradient at one point.
// Collapsed coordinates a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t;
// psi_ijk = 2 sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i P_k^(2i+2j+2,0)(c) (1-c)^(i+j).
// The gradient follows the chain rule through (a, b, c) with the powers of
// (1-b), (1-c) reduced by hand so the collapsed vertex gives no 0/0.
void basis_and_grad(double r, double s, double t, int i, int j, int k, double* psi, double* g) {
  const double a = (-(s + t) != 0.0) ? 2.0 * (1.0 + r) / (-(s + t)) - 1.0 : -1.0;
  const double b = (t != 1.0) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
  const double c = t;
  const double fa = jacobi(a, 0, 0, i), dfa = djacobi(a, 0, 0, i);
  const double gb = jacobi(b, 2 * i + 1, 0, j), dgb = djacobi(b, 2 * i + 1, 0, j);
  const double hc = jacobi(c, 2 * i + 2 * j + 2, 0, k), dhc = djacobi(c, 2 * i + 2 * j + 2, 0, k);
  const double nrm = 2.0 * std::sqrt(2.0);
  const double omb = 1.0 - b, omc = 1.0 - c;
  if (psi) *psi = nrm * fa * gb * std::pow(omb, i) * hc * std::pow(omc, i + j);
  if (!g) return;
  const double dr = (i > 0) ? nrm * 4.0 * dfa * gb * std::pow(omb, i - 1) * hc * std::pow(omc, i + j - 1) : 0.0;
  // d/db [gb (1-b)^i]
  double dgbb = dgb * std::pow(omb, i);
  if (i > 0) dgbb -= i * gb * std::pow(omb, i - 1);
  const double hred = (i + j > 0) ? hc * std::pow(omc, i + j - 1) : 0.0;
  double dhcc = dhc * std::pow(omc, i + j);
  if (i + j > 0) dhcc -= (i + j) * hc * std::pow(omc, i + j - 1);
  g[0] = dr;
  g[1] = 0.5 * (1.0 + a) * dr + nrm * fa * dgbb * 2.0 * hred;
  g[2] = 0.5 * (1.0 + a) * dr + nrm * fa * dgbb * (1.0 + b) * hred + nrm * fa * gb * std::pow(omb, i) * dhcc;
}

// Orthonormal basis on the reference triangle: sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i,
// a = 2(1+x)/(1-y) - 1, b = y.
double basis2d(double x, double y, int i, int j) {
  const double a = (y != 1.0) ? 2.0 * (1.0 + x) / (1.0 - y) - 1.0 : -1.0;
  return std::sqrt(2.0) * jacobi(a, 0, 0, i) * jacobi(y, 2 * i + 1, 0, j) * std::pow(1.0 - y, i);
}

std::unique_ptr<RefElement> build(int N) {
  auto re = std::make_unique<RefElement>();
  re->N = N;
  re->Np = n_p(N);
  re->Nfp = n_fp(N);
  const int Np = re->Np, Nfp = re->Nfp;
  build_nodes(*re);

  // Vandermonde and gradient Vandermonde.
  Mat V(Np, Np), Vr(Np, Np), Vs(Np, Np), Vt(Np, Np);
  int col = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++col)
        for (int p = 0; p < Np; ++p) {
          double psi, g[3];
          basis_and_grad(re->r[p], re->s[p], re->t[p], i, j, k, &psi, g);
          V(p, col) = psi;
          Vr(p, col) = g[0];
          Vs(p, col) = g[1];
          Vt(p, col) = g[2];
        }
  Mat Vinv;
  if (!invert(V, Vinv)) return nullptr;
  re->V = V;
  re->Dr = matmul(Vr, Vinv);
  re->Ds = matmul(Vs, Vinv);
  re->Dt = matmul(Vt, Vinv);

  // Face membership from the lattice: face f holds the nodes whose lattice
  // coordinate of the opposite vertex is zero, in ascending node order.
  re->fmask.assign(4 * Nfp, -1);
  for (int f = 0; f < 4; ++f) {
    int j = 0;
    for (int p = 0; p < Np; ++p)
      if (re->lat[p][kFaceOpposite[f]] == 0) re->fmask[f * Nfp + j++] = p;
    if (j != Nfp) return nullptr;
  }

  // Face mass matrices (each face parametrised by two reference coordinates
  // as the triangle {(-1,-1),(1,-1),(-1,1)}) and the embedding E.
  const int param[4][2] = {{0, 1}, {0, 2}, {1, 2}, {1, 2}};
  const std::vector<double>* rst[3] = {&re->r, &re->s, &re->t};
  re->Mf.assign(4 * Nfp * Nfp, 0.0);
  Mat E(Np, 4 * Nfp);
  for (int f = 0; f < 4; ++f) {
    Mat V2(Nfp, Nfp);
    for (int q = 0; q < Nfp; ++q) {
      const int p = re->fmask[f * Nfp + q];
      const double x = (*rst[param[f][0]])[p], y = (*rst[param[f][1]])[p];
      int m = 0;
      for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j, ++m) V2(q, m) = basis2d(x, y, i, j);
    }
    Mat VVt = matmul(V2, transpose(V2)), Mface;
    if (!invert(VVt, Mface)) return nullptr;
    for (int a = 0; a < Nfp; ++a)
      for (int b = 0; b < Nfp; ++b) {
        re->Mf[(f * Nfp + a) * Nfp + b] = Mface(a, b);
        E(re->fmask[f * Nfp + a], f * Nfp + b) = Mface(a, b);
      }
  }
  re->LIFT = matmul(V, matmul(transpose(V), E));

  // Neighbour node table.  Own face f, slot i holds local vertex
  // kFaceVerts[f][i]; orientation o says that this vertex is slot
  // kPerm3[o][i] of the neighbour face nf.  A face node is the lattice point
  // with the same barycentric weights on the shared vertices.
  std::map<std::array<int, 4>, int> lookup;
  for (int p = 0; p < Np; ++p) lookup[re->lat[p]] = p;
  re->nbr_node.assign(4 * 24 * Nfp, 0);
  for (int f = 0; f < 4; ++f)
    for (int nf = 0; nf < 4; ++nf)
      for (int o = 0; o < 6; ++o)
        for (int j = 0; j < Nfp; ++j) {
          const auto& L = re->lat[re->fmask[f * Nfp + j]];
          std::array<int, 4> Ln = {0, 0, 0, 0};
          for (int i = 0; i < 3; ++i) Ln[kFaceVerts[nf][kPerm3[o][i]]] = L[kFaceVerts[f][i]];
          auto it = lookup.find(Ln);
          if (it == lookup.end()) return nullptr;
          re->nbr_node[(f * 24 + nf * 6 + o) * Nfp + j] = uint8_t(it->second);
        }
  return re;
}

}  // namespace

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.rows, B.cols);
  for (int i = 0; i < A.rows; ++i)
    for (int k = 0; k < A.cols; ++k) {
      const double a = A(i, k);
      if (a == 0.0) continue;
      for (int j = 0; j < B.cols; ++j) C(i, j) += a * B(k, j);
    }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T(A.cols, A.rows);
  for (int i = 0; i < A.rows; ++i)
    for (int j = 0; j < A.cols; ++j) T(j, i) = A(i, j);
  return T;
}

bool invert(const Mat& A, Mat& Ainv) {
  const int n = A.rows;
  Mat LU = A;
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(LU(i, k)) > std::fabs(LU(p, k))) p = i;
    if (LU(p, k) == 0.0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(LU(k, j), LU(p, j));
      std::swap(piv[k], piv[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      LU(i, k) /= LU(k, k);
      const double l = LU(i, k);
      for (int j = k + 1; j < n; ++j) LU(i, j) -= l * LU(k, j);
    }
  }
  Ainv = Mat(n, n);
  std::vector<double> x(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) x[i] = (piv[i] == c) ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) x[i] -= LU(i, j) * x[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) x[i] -= LU(i, j) * x[j];
      x[i] /= LU(i, i);
    }
    for (int i = 0; i < n; ++i) Ainv(i, c) = x[i];
  }
  return true;
}

const RefElement* ref_element(int N) {
  static std::mutex mu;
  static std::unique_ptr<RefElement> cache[kMaxOrder + 1];
  if (N < 1 || N > kMaxOrder) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!cache[N]) cache[N] = build(N);
  return cache[N].get();
}

}  // namespace dgh
