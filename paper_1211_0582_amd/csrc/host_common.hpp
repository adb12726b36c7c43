// Host-side shared declarations of the DG library (no device code).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dgh {

// Thread-local error text behind dg_last_error().
void set_error(const std::string& msg);
void clear_error();
dg_status fail(dg_status s, const std::string& msg);
const char* error_text();

constexpr int kMaxOrder = 9;

// Boundary condition codes of dg_mesh_desc.face_bc.
constexpr int kBcConducting = 0, kBcMagnetic = 1, kBcAbsorbing = 2;

inline int n_p(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
inline int n_fp(int N) { return (N + 1) * (N + 2) / 2; }

// Local vertex ids of the four faces of the reference tetrahedron
// v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1), v3=(-1,-1,1):
// face 0: t=-1, face 1: s=-1, face 2: r+s+t=-1, face 3: r=-1.
extern const int kFaceVerts[4][3];
// Vertex opposite each face.
extern const int kFaceOpposite[4];
// The six permutations of three face slots, indexed by orientation code.
extern const int kPerm3[6][3];

// Row-major dense matrix helper.
struct Mat {
  int rows = 0, cols = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int r, int c) : rows(r), cols(c), a(size_t(r) * c, 0.0) {}
  double& operator()(int i, int j) { return a[size_t(i) * cols + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * cols + j]; }
};

Mat matmul(const Mat& A, const Mat& B);
Mat transpose(const Mat& A);
// Inverse by LU with partial pivoting; returns false if singular.
bool invert(const Mat& A, Mat& Ainv);

// Reference element at order N (binary64).
struct RefElement {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> r, s, t;                 // nodes
  std::vector<std::array<int, 4>> lat;         // integer barycentric lattice per node
  Mat V, Dr, Ds, Dt, LIFT;                     // LIFT: Np x 4Nfp
  std::vector<int> fmask;                      // 4 x Nfp
  std::vector<double> Mf;                      // 4 x Nfp x Nfp
  // Neighbour node table: for own face f, packed code = nbr_face*6 + orient,
  // and own face node j -> the neighbour's volume node id.  4 x 24 x Nfp.
  std::vector<uint8_t> nbr_node;
};

// Builds (and caches) the reference element; nullptr if N is out of range.
const RefElement* ref_element(int N);

// Per-mesh host data.
struct HostMesh {
  int N = 0;
  int64_t K = 0;
  std::vector<double> metric;   // K x 9
  std::vector<double> J;        // K
  std::vector<double> face;     // K x 4 x 4 (nx, ny, nz, Fscale)
  std::vector<double> sJ;       // K x 4
  std::vector<int32_t> conn;    // K x 4: nbr*32 + nbr_face*6 + orient, or -1 - bc on a boundary face
  double max_fscale = 0.0;
  int64_t n_boundary = 0;
};

// face_bc: K x 4 condition codes read on boundary faces only (NULL: all 0).
dg_status build_mesh(int N, int64_t Nv, const double* VX, int64_t K, const int32_t* EToV,
                     const int8_t* face_bc, HostMesh& out);

}  // namespace dgh
