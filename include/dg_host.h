/*
 * dg_host.h -- host-side setup of the DG library, callable without a GPU.
 *
 * These are the host computations dg_setup_mesh performs before it uploads
 * anything: the reference element of Section 2 of the paper (nodal basis on
 * warp & blend nodes, differentiation matrices D = M^-1 S, face mass matrices
 * and the lifting matrix L of the figure on its construction), the affine
 * geometry of Section 2.1 (constant metric, face normals and Fscale = sJ/J),
 * and the face connectivity used by the flux gather.  They are exported so
 * that the setup can be checked on a machine without a GPU.
 *
 * All arrays are host pointers owned by the caller, row-major, binary64
 * unless stated.  Every function returns dg_status (see dg.h) and leaves
 * outputs unspecified on error.  N must be in 1..9.
 */
#ifndef DG_HOST_H_
#define DG_HOST_H_

#include <stdint.h>

#include "dg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Reference nodes: r, s, t each of length Np = (N+1)(N+2)(N+3)/6.
 * Errors: DG_EINVAL (null), DG_EUNSUPPORTED (N). */
dg_status dg_host_ref_nodes(int32_t N, double* r, double* s, double* t);

/* Reference operators: Dr, Ds, Dt (Np x Np), LIFT (Np x 4 Nfp, face-major
 * columns f*Nfp + j), Fmask (4 x Nfp int32, ascending node ids of each face),
 * Mf (4 x Nfp x Nfp face mass matrices in each face's Fmask order).
 * Any output pointer may be NULL to skip it.  Errors: DG_EUNSUPPORTED (N). */
dg_status dg_host_ref_operators(int32_t N, double* Dr, double* Ds, double* Dt,
                                double* LIFT, int32_t* Fmask, double* Mf);

/* Geometry and connectivity of a mesh (Section 2.1; same validation as
 * dg_setup_mesh; face_bc as dg_mesh_desc.face_bc, may be NULL):
 *   metric   K x 9   (rx, ry, rz, sx, sy, sz, tx, ty, tz)
 *   J        K
 *   face     K x 4 x 4 (nx, ny, nz, Fscale) per face
 *   sJ       K x 4
 *   vmapP    K x 4 x Nfp int64: k'*Np + i' of the neighbour node matching
 *            face node j of face f of element k, -1 on a wall face
 *   conn     K x 4 int32 packed neighbour code as used on the device:
 *            nbr_elem * 32 + nbr_face * 6 + orient on an interior face, where
 *            orient in 0..5 names how the shared face's vertices permute;
 *            -1 - b on a boundary face with condition code b (DG_BC_*)
 * Any output pointer may be NULL.  Errors: as dg_setup_mesh. */
dg_status dg_host_mesh(int32_t N, int64_t Nv, const double* VX, int64_t K,
                       const int32_t* EToV, const int8_t* face_bc, double* metric, double* J,
                       double* face, double* sJ, int64_t* vmapP, int32_t* conn);

#ifdef __cplusplus
}
#endif

#endif /* DG_HOST_H_ */
