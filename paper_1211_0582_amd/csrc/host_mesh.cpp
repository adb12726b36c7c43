// Affine geometry and face connectivity of a tetrahedral mesh (host).
//
// Section 2.1 of the paper: for straight-sided simplices the map from the
// reference element is affine, so the metric terms (rx .. tz), the Jacobian
// J and, per face, the unit normal and sJ are constants per element.  Normals
// come from the inverse metric applied to the reference face normals
// (Nanson's formula): face 0 -(t_x), face 1 -(s_x), face 2 r_x+s_x+t_x,
// face 3 -(r_x); sJ = J |A^-T n_ref| (area over the reference triangle's 2),
// Fscale = sJ / J.
//
// Connectivity: faces are keyed by their sorted global vertex triple and
// matched by sorting.  A matched face stores the neighbour element, its local
// face and the orientation code (which of the six slot permutations maps our
// face's vertices to the neighbour's), all the flux gather needs to find u+.
// An unmatched face is a boundary face and stores -1 - b, b its boundary
// condition code (the boundary data of Section 2 on the domain boundary):
// 0 perfectly conducting, 1 perfectly magnetic-conducting, 2 absorbing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "host_common.hpp"

namespace dgh {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
dg_status fail(dg_status s, const std::string& msg) {
  g_error = msg;
  return s;
}

dg_status build_mesh(int N, int64_t Nv, const double* VX, int64_t K, const int32_t* EToV, const int8_t* face_bc,
                     HostMesh& out) {
  if (!VX || !EToV) return fail(DG_EINVAL, "VX and EToV must be non-null");
  if (Nv < 4 || K < 1) return fail(DG_EINVAL, "need Nv >= 4 and K >= 1");
  if (N < 1 || N > kMaxOrder) return fail(DG_EUNSUPPORTED, "order N must be in 1..9");
  if (K >= (int64_t(1) << 26)) return fail(DG_EUNSUPPORTED, "K must be below 2^26");
  for (int64_t i = 0; i < 4 * K; ++i)
    if (EToV[i] < 0 || int64_t(EToV[i]) >= Nv)
      return fail(DG_EMESH, "element " + std::to_string(i / 4) + " has a vertex id out of range");
  for (int64_t i = 0; i < 3 * Nv; ++i)
    if (!std::isfinite(VX[i])) return fail(DG_EMESH, "vertex " + std::to_string(i / 3) + " is not finite");

  out.N = N;
  out.K = K;
  out.metric.assign(size_t(K) * 9, 0.0);
  out.J.assign(size_t(K), 0.0);
  out.face.assign(size_t(K) * 16, 0.0);
  out.sJ.assign(size_t(K) * 4, 0.0);
  out.conn.assign(size_t(K) * 4, -1);
  double maxfs = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double* X[4];
    for (int v = 0; v < 4; ++v) X[v] = VX + 3 * int64_t(EToV[4 * k + v]);
    // Columns of A = d x / d (r, s, t).
    double A[3][3];
    for (int d = 0; d < 3; ++d) {
      A[d][0] = 0.5 * (X[1][d] - X[0][d]);
      A[d][1] = 0.5 * (X[2][d] - X[0][d]);
      A[d][2] = 0.5 * (X[3][d] - X[0][d]);
    }
    const double J = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(J > 0.0)) return fail(DG_EMESH, "element " + std::to_string(k) + " has non-positive Jacobian");
    // Inverse: row r = (rx, ry, rz) etc.
    double I[3][3];
    I[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / J;
    I[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / J;
    I[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / J;
    I[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / J;
    I[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / J;
    I[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / J;
    I[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / J;
    I[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / J;
    I[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / J;
    double* g = &out.metric[size_t(k) * 9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) g[3 * a + b] = I[a][b];
    out.J[k] = J;
    const double n_ref[4][3] = {{0, 0, -1}, {0, -1, 0}, {1, 1, 1}, {-1, 0, 0}};
    for (int f = 0; f < 4; ++f) {
      double n[3];
      for (int d = 0; d < 3; ++d) n[d] = I[0][d] * n_ref[f][0] + I[1][d] * n_ref[f][1] + I[2][d] * n_ref[f][2];
      const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      double* fo = &out.face[(size_t(k) * 4 + f) * 4];
      fo[0] = n[0] / len;
      fo[1] = n[1] / len;
      fo[2] = n[2] / len;
      fo[3] = len;  // Fscale = sJ / J = |A^-T n_ref|
      out.sJ[size_t(k) * 4 + f] = len * J;
      maxfs = std::max(maxfs, len);
    }
  }
  out.max_fscale = maxfs;

  // Face matching by sorted vertex triples.
  struct FaceKey {
    int32_t v[3];
    int32_t elem_face;  // k * 4 + f
  };
  std::vector<FaceKey> keys(size_t(K) * 4);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      FaceKey fk;
      for (int i = 0; i < 3; ++i) fk.v[i] = EToV[4 * k + kFaceVerts[f][i]];
      std::sort(fk.v, fk.v + 3);
      fk.elem_face = int32_t(k * 4 + f);
      keys[size_t(k) * 4 + f] = fk;
    }
  std::sort(keys.begin(), keys.end(), [](const FaceKey& a, const FaceKey& b) {
    if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
    if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
    if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
    return a.elem_face < b.elem_face;
  });
  auto same = [](const FaceKey& a, const FaceKey& b) {
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
  };
  int64_t nb = 0;
  for (size_t i = 0; i < keys.size();) {
    size_t j = i + 1;
    while (j < keys.size() && same(keys[i], keys[j])) ++j;
    if (j - i > 2)
      return fail(DG_EMESH, "a face of element " + std::to_string(keys[i].elem_face / 4) +
                                " is shared by more than two elements");
    if (keys[i].v[0] == keys[i].v[1] || keys[i].v[1] == keys[i].v[2])
      return fail(DG_EMESH, "element " + std::to_string(keys[i].elem_face / 4) + " has a degenerate face");
    if (j - i == 2) {
      const int ka = keys[i].elem_face / 4, fa = keys[i].elem_face % 4;
      const int kb = keys[i + 1].elem_face / 4, fb = keys[i + 1].elem_face % 4;
      for (int side = 0; side < 2; ++side) {
        const int k1 = side ? kb : ka, f1 = side ? fb : fa;
        const int k2 = side ? ka : kb, f2 = side ? fa : fb;
        int g[3], h[3];
        for (int s = 0; s < 3; ++s) {
          g[s] = EToV[4 * int64_t(k1) + kFaceVerts[f1][s]];
          h[s] = EToV[4 * int64_t(k2) + kFaceVerts[f2][s]];
        }
        int code = -1;
        for (int o = 0; o < 6 && code < 0; ++o)
          if (h[kPerm3[o][0]] == g[0] && h[kPerm3[o][1]] == g[1] && h[kPerm3[o][2]] == g[2]) code = o;
        if (code < 0) return fail(DG_EMESH, "face orientation not found");
        out.conn[size_t(k1) * 4 + f1] = k2 * 32 + f2 * 6 + code;
      }
    } else {
      const int k1 = keys[i].elem_face / 4, f1 = keys[i].elem_face % 4;
      const int b = face_bc ? int(face_bc[size_t(k1) * 4 + f1]) : kBcConducting;
      if (b < kBcConducting || b > kBcAbsorbing)
        return fail(DG_EINVAL, "boundary face " + std::to_string(f1) + " of element " + std::to_string(k1) +
                                   " has condition code " + std::to_string(b) + " (must be 0, 1 or 2)");
      out.conn[size_t(k1) * 4 + f1] = -1 - b;
      ++nb;
    }
    i = j;
  }
  out.n_boundary = nb;
  return DG_OK;
}

const char* error_text() { return g_error.c_str(); }

}  // namespace dgh
