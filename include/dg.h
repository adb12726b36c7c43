/*
 * dg.h -- C ABI of the MI355X (gfx950) nodal discontinuous Galerkin library
 * for the 3D Maxwell equations on straight-sided tetrahedra.
 *
 * What is computed.  The semi-discrete scheme of Kloeckner, Warburton and
 * Hesthaven, "High-Order Discontinuous Galerkin Methods by GPU
 * Metaprogramming", Section 2 (strong form and the semi-discrete equation),
 * for the linear Maxwell system with field order u = (Ex, Ey, Ez, Hx, Hy, Hz)
 * and a permittivity eps and permeability mu constant per element:
 *
 *     du/dt = -sum_nu D^nu F(u) + L [ n.F - (n.F)* ],
 *
 * i.e. eps dE/dt = curl H + LIFT(Fscale fE), mu dH/dt = -curl E + LIFT(Fscale fH)
 * with the upwind flux of the results section (Section 5, Maxwell flux
 * figure, part a; H part by duality), dE = E- - E+, dH = H- - H+, and the
 * impedances Z = sqrt(mu / eps), Y = 1 / Z of the own (-) and neighbour (+)
 * element:
 *     fE = [ -Z+ n x dH + alpha (n (n.dE) - dE) ] / (Z- + Z+)
 *     fH = [  Y+ n x dE + alpha (n (n.dH) - dH) ] / (Y- + Y+),
 * which for eps = mu = 1 is 1/2 [ -n x dH + alpha (n (n.dE) - dE) ] and
 * 1/2 [ n x dE + alpha (n (n.dH) - dH) ].  A boundary face takes the
 * exterior state E+ = a_E E-, H+ = a_H H- of its condition code (the boundary
 * data of Section 2 on the domain boundary): (a_E, a_H) = (-1, 1) perfectly
 * conducting, (1, -1) perfectly magnetic-conducting, (0, 0) absorbing; its
 * exterior has the element's own material.  Time stepping is the
 * five-stage fourth-order low-storage Runge-Kutta scheme of Carpenter and
 * Kennedy (the paper times whole steps with their Runge-Kutta update
 * included, Section 5).
 *
 * Reference element: nodal Lagrange basis of P_N on warp & blend nodes,
 * operators built from an orthonormal basis; reference tetrahedron
 * v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1), v3=(-1,-1,1); element map
 * x = -(1+r+s+t)/2 X0 + (1+r)/2 X1 + (1+s)/2 X2 + (1+t)/2 X3 with X_i the
 * vertices EToV[k][i].  Node order: t lattice index outermost, then s, then r.
 * Face f of an element has the local vertices {0,1,2}, {0,1,3}, {1,2,3},
 * {0,2,3} for f = 0..3.
 *
 * Conventions for every call:
 *   - every function returns dg_status (0 = DG_OK, negative = error); nothing
 *     throws across the ABI; dg_last_error() gives a thread-local message;
 *   - invalid arguments are rejected before any device work is queued;
 *   - "device pointer" arguments are HIP device allocations owned by the
 *     caller, "host pointer" arguments are ordinary host memory;
 *   - stream arguments are hipStream_t values passed as void* (NULL = the
 *     null stream) of the problem's device; calls that take a stream are
 *     asynchronous on it and neither allocate nor synchronise;
 *   - a call on a problem makes the problem's device current for its
 *     duration and restores the caller's current device before returning.
 */
#ifndef DG_H_
#define DG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument (null pointer, size, enum value)        */
  DG_EMESH = -2,         /* invalid mesh: J <= 0, bad vertex index, a face shared
                            by more than two elements; the message names it    */
  DG_EHIP = -3,          /* a HIP runtime call failed; the message has its text  */
  DG_ENOMEM = -4,        /* device or host allocation failed                     */
  DG_EUNSUPPORTED = -5   /* valid request this build does not support (order,
                            precision, size limits)                             */
} dg_status;

/* Arithmetic of the right-hand side and of the state arrays.
 *   DG_FP64: state, geometry, operators and all arithmetic in binary64.
 *   DG_FP32: state, geometry, operators and all arithmetic in binary32.
 *   The others keep the state, geometry, fluxes and the Runge-Kutta update
 *   in binary32 and run the two dense contractions (Dr/Ds/Dt and LIFT) on
 *   16-bit matrix cores with binary32 accumulation.  Each operand a is split
 *   as a = a_hi + a_lo, a_hi = round16(a), a_lo = round16(a - a_hi):
 *   DG_BF16 / DG_F16:      a_hi b_hi                        (one product)
 *   DG_BF16X2 / DG_F16X2:  a_hi b_hi + a_lo b_hi            (operator split)
 *   DG_BF16X3 / DG_F16X3:  a_hi b_hi + a_lo b_hi + a_hi b_lo (both split)
 *   where a is the operator and b the fields or fluxes; BF16 = bfloat16,
 *   F16 = IEEE binary16.  These have only the matrix-core variants.         */
typedef enum {
  DG_FP64 = 0, DG_FP32 = 1, DG_BF16X3 = 2, DG_F16X3 = 3,
  DG_BF16 = 4, DG_F16 = 5, DG_BF16X2 = 6, DG_F16X2 = 7
} dg_precision;

typedef struct dg_problem_s* dg_problem;  /* opaque; owns all mesh-derived device data */

/* Boundary condition codes of dg_mesh_desc.face_bc (Section 2: boundary data
 * on the domain boundary; the exterior state of a boundary face is built from
 * the interior trace, see the header comment). */
enum { DG_BC_CONDUCTING = 0, DG_BC_MAGNETIC = 1, DG_BC_ABSORBING = 2 };

/* Mesh and discretisation (inputs of dg_setup_mesh): the tetrahedral mesh,
 * polynomial space and flux of Section 2.  Host pointers; the library copies
 * what it needs, the caller keeps ownership. */
typedef struct {
  int32_t N;             /* polynomial order, 1..9                                */
  int32_t precision;     /* dg_precision                                          */
  double alpha;          /* flux parameter: 1 = upwind, 0 = central; finite      */
  int64_t Nv;            /* number of vertices                                    */
  const double* VX;      /* host, Nv x 3 row-major (x, y, z)                      */
  int64_t K;             /* number of tetrahedra, 1 .. 2^26-1                     */
  const int32_t* EToV;   /* host, K x 4 row-major, 0-based vertex ids; every
                            element must be positively oriented (J > 0)          */
  const int8_t* face_bc; /* host, K x 4 (element, face) condition codes, read on
                            boundary faces only (DG_BC_*); NULL: every boundary
                            face is DG_BC_CONDUCTING                              */
  const double* eps;     /* host, K permittivities (finite, > 0); NULL: all 1     */
  const double* mu;      /* host, K permeabilities (finite, > 0); NULL: all 1     */
  int32_t device;        /* HIP device ordinal the problem lives on; -1: the
                            device current at dg_setup_mesh                       */
} dg_mesh_desc;

/* Layout of device state arrays (u, rhs, res).  A state array holds the
 * nfields fields (six for Maxwell) one after the other, field c starting at
 * element offset c * field_stride; inside a field, element k's Np nodal
 * values are contiguous at offset k * Np.  Entries between K*Np and
 * field_stride are padding: never read as data.  state_elems =
 * nfields * field_stride scalars of elem_bytes bytes each.  State arrays
 * passed to the library must start on a 16-byte boundary (hipMalloc gives
 * 256); the kernels write them with 16-byte stores. */
typedef struct {
  int32_t N, Np, Nfp, precision;
  int64_t K;
  int64_t field_stride;  /* scalars                                               */
  int64_t state_elems;   /* scalars in one state array                            */
  int32_t elem_bytes;    /* 8 (DG_FP64) or 4 (every other precision)              */
  int32_t tile_elems;    /* elements per workgroup of the RHS kernel              */
  double dt_cfl1;        /* 2 / ((N+1)^2 max Fscale): dt at CFL number 1          */
  double alpha;
  int64_t n_boundary_faces;
  int32_t variant;       /* kernel variant in use (dg_variant_name); a compiled
                            system reports dg_variant_count()                     */
  int32_t nfields;       /* fields per state array: 6, or a compiled system's M   */
} dg_info;

/* Builds the reference element (Section 2: nodal basis, D = M^-1 S, face mass
 * matrices, the lifting matrix L), the affine geometry and the face
 * connectivity of Section 2.1, and uploads them to the problem's device.
 * Synchronous.  *out receives a new handle on success and is left untouched
 * on error.  Elements whose eps or mu differ from 1 select the material form
 * of the kernels (FP64 and FP32 only).
 * Errors: DG_EINVAL (null pointer, K or Nv < 1, alpha not finite, precision
 * out of range, a boundary face code outside 0..2, eps or mu not finite and
 * positive, device out of range), DG_EUNSUPPORTED (N outside 1..9,
 * K >= 2^26, one state array -- 6 fields of K * Np values, each padded to
 * 256 bytes -- of 2 GiB or more: the kernels use 32-bit buffer offsets; eps
 * or mu other than 1 with a split 16-bit precision), DG_EMESH (vertex id out
 * of range, J <= 0, face multiplicity > 2), DG_EHIP/DG_ENOMEM. */
dg_status dg_setup_mesh(const dg_mesh_desc* desc, dg_problem* out);

/* Sizes and layout of a problem.  Errors: DG_EINVAL on null arguments. */
dg_status dg_info_get(dg_problem p, dg_info* info);

/* rhs <- du/dt evaluated at u: the semi-discrete equation of Section 2, split
 * as in Section 2.1 into local differentiation, flux gather and flux lifting
 * (flux and boundary states as in the header comment).  u, rhs: device pointers to state arrays in the
 * problem's precision and layout; they must not overlap.  Asynchronous on
 * stream.  Only the K*Np entries of each field of rhs are written.
 * Errors: DG_EINVAL (null pointer, u == rhs, or a pointer not 16-byte
 * aligned), DG_EHIP (launch failure). */
dg_status dg_rhs(dg_problem p, const void* u, void* rhs, void* stream);

/* Kernel variants of the right-hand side, all computing the same operator
 * (the paper tunes its kernels by timing generated variants, Section 4):
 *   0 "valu":            one workgroup per element tile on the vector ALUs
 *                        (FP64 / FP32);
 *   1 "mfma":            one workgroup (2 or 4 waves) per tile of 16
 *                        elements, the contraction with [Dr|Ds|Dt|LIFT] on the
 *                        matrix cores, Runge-Kutta stage fused into its
 *                        epilogue, choices by built-in heuristics;
 *   2 "mfma_waves":      the other number of waves per tile (2 <-> 4);
 *   3 "mfma_prefetch":   the other operator-fragment prefetch depth;
 *   4 "mfma_occupancy":  registers allocated for the occupancy the tile's LDS
 *                        allows;
 *   5 "mfma_interleave": flux work interleaved with the volume contraction
 *                        or not, the other way round (FP64 / FP32);
 *   6 "mfma_lift":       the lift in two halves or not, the other way round
 *                        (FP64 / FP32);
 *   7 "mfma_tail":       the last row block on the 4-row matrix-core form or
 *                        not, the other way round (FP64 / FP32, where that
 *                        block holds at most 4 nodes).
 * Variants 2..7 exist where they give a different kernel (FP64, FP32 and the
 * x3 split forms, vacuum flux); batches use "mfma".  dg_setup_mesh picks
 * the variant the library's tuning table (the autotuner's measurements on
 * gfx950, compiled in) records for (precision, N, K below or from 20000
 * elements) where it is built, else "mfma" where built, else "valu".
 * dg_variant_name returns NULL outside 0 .. dg_variant_count()-1.
 * dg_set_variant: DG_EINVAL (null p, v out of range), DG_EUNSUPPORTED (not
 * built for this order, precision and flux form; the problem keeps its
 * variant). */
int32_t dg_variant_count(void);
const char* dg_variant_name(int32_t v);
dg_status dg_set_variant(dg_problem p, int32_t v);

/* Order in which the matrix-core kernels take the 16-element tiles (the
 * paper's tuning of the element blocks the flux gather works on, Section 4):
 * enable != 0 (the default) walks the tiles in the Morton order of their
 * centroids, so the tiles an XCD holds at one time are spatial neighbours
 * and their neighbour-trace reads hit its L2; 0 walks them in element order.
 * Results are bitwise identical either way.  Errors: DG_EINVAL (null p). */
dg_status dg_set_tile_order(dg_problem p, int32_t enable);

/* Timing core of the autotuner (the paper's automated tuning, Section 4):
 * runs dg_rhs(p, u, rhs) `warmup` times, then `reps` times between two HIP
 * events on stream, waits for the second event and stores the mean time of
 * one evaluation in *ms.  Synchronous.  Errors: DG_EINVAL (null pointers,
 * reps < 1, warmup < 0), DG_EHIP. */
dg_status dg_time_rhs(dg_problem p, const void* u, void* rhs, int32_t warmup, int32_t reps,
                      void* stream, double* ms);

/* nsteps steps of the 5-stage low-storage RK4 scheme (the time stepping
 * that the paper's Section 5 times together with the operator), in place:
 *   for each stage s: res <- A_s res + dt du/dt(u);  u <- u + B_s res.
 * A_1 = 0 and the first stage of every step does not read res: its
 * contents on entry, NaN or Inf bit patterns included, never enter the
 * result.  u, res: device state arrays.
 * t is the start time; the perfectly conducting cavity has no time-dependent
 * data, so the stage times t + C_s dt do not enter the arithmetic.
 * Uses library-owned scratch allocated at setup; asynchronous on stream.
 * Where the fused stage kernel exists, each stage reads one state buffer
 * (u or the scratch) and writes the other, so a call whose 5 * nsteps stages
 * are odd in number ends with one device copy of the state back into u:
 * step many times per call rather than once per call.
 * Errors: DG_EINVAL (null pointer, u == res, a pointer not 16-byte aligned,
 * nsteps < 0, dt not finite). */
dg_status dg_rk_step(dg_problem p, void* u, void* res, double t, double dt,
                     int32_t nsteps, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_rk_step
 * whose second state buffer is a library-static device array of
 * DG_NOALLOC_SCRATCH_BYTES per device instead of the problem's own scratch.
 * It calls no allocating routine.  The array is shared by every call on a
 * device and keeps the last call's contents: calls that overlap on one
 * device (other streams, other threads) race on it.  Results equal
 * dg_rk_step's bit for bit.  Errors: as dg_rk_step, DG_EUNSUPPORTED when one
 * state array (state_elems * elem_bytes) exceeds DG_NOALLOC_SCRATCH_BYTES. */
#define DG_NOALLOC_SCRATCH_BYTES (256ll << 20)
dg_status dg_rk_step_noalloc(dg_problem p, void* u, void* res, double t, double dt,
                             int32_t nsteps, void* stream);

/* ---- Run-time compiled systems (Section 4, run-time code generation) -----
 * A hyperbolic system other than the built-in Maxwell one, given as C++
 * source that defines `struct System` (M fields; volume flux, numerical flux
 * n.F - (n.F)* and boundary exterior states as __device__ templates; the
 * contract is spelled out in the library's rtc_kernel.hpp and produced by the
 * Python front end paper_1211_0582_amd/systems.py).  The library puts it in
 * front of its matrix-core kernel template and compiles it with hipRTC for
 * the problem's order, precision and device, so the system's zero flux
 * entries, N, Np and Nfp are all compile-time constants of the kernel.
 *
 * dg_system_compile: compiles only (no device needed) for the architecture
 * `arch` (e.g. "gfx950"); the compiler log goes to log[0 .. log_size-1]
 * (NUL-terminated; may be NULL).  Errors: DG_EINVAL (null source or arch,
 * nfields outside 1..12, source that does not compile), DG_EUNSUPPORTED
 * (N outside 1..9, precision other than FP64/FP32).
 *
 * dg_setup_system: as dg_setup_mesh for the system: state arrays hold
 * nfields fields (dg_info.nfields); face_bc codes are passed to
 * System::exterior; eps and mu must be NULL (or all 1).  dg_rhs, dg_rk_step
 * (right-hand side plus the update kernel), dg_rk_step_noalloc, dg_energy
 * (sum_k J_k u^T M u / 2 over all fields), dg_pack/dg_unpack ([nfields][K][Np]),
 * dg_time_rhs and dg_destroy apply; batches and dg_set_variant do not.  The
 * compiled module is cached for the process (per device, architecture,
 * order, precision and source).  Errors: as dg_setup_mesh and
 * dg_system_compile, DG_EHIP (module load). */
dg_status dg_system_compile(const char* system_source, int32_t nfields, int32_t N, int32_t precision,
                            const char* arch, char* log, int64_t log_size);
dg_status dg_setup_system(const dg_mesh_desc* desc, const char* system_source, int32_t nfields,
                          dg_problem* out);

/* ---- Batches of independent problems -------------------------------------
 * A batch owns n problems (any mix of orders and sizes, one precision) and
 * steps them together: problems are grouped by order N and each Runge-Kutta
 * stage is one launch per group over all of its (problem, element tile)
 * pairs.  The paper notes (Section 4) that the host's launch rate only
 * suffices when each launch carries enough work; batching many small problems
 * restores that. */
typedef struct dg_batch_s* dg_batch;

/* Sets up descs[0..n-1] (host array) as one batch: each problem as by
 * dg_setup_mesh (Section 2's mesh, space and flux).  All problems must share
 * one precision and one device, have eps = mu = 1 and have a batched kernel
 * (the "mfma" variant is built for their order and precision).  Errors: as
 * dg_setup_mesh (the message names the problem), DG_EINVAL (n < 1, mixed
 * precisions or devices), DG_EUNSUPPORTED (materials, no batched kernel). */
dg_status dg_setup_batch(int32_t n, const dg_mesh_desc* descs, dg_batch* out);

/* Borrowed handle of problem i (for dg_info_get, dg_pack, dg_unpack,
 * dg_nodes, dg_rhs); it stays owned by the batch: never dg_destroy it. */
dg_status dg_batch_problem(dg_batch b, int32_t i, dg_problem* p);

/* nsteps LSERK steps (as dg_rk_step, res not read at the first stage) of
 * every problem, in place.  u, res, dt: host arrays of n device pointers /
 * time steps; u[i], res[i] are state arrays of problem i.  mode 0: each step replays a graph of (5 stages x order groups) kernel
 * launches, captured on the first call; mode 1: the same launches issued
 * directly; mode 2: one launch per problem and stage (dg_rk_step per
 * problem).  All modes give bitwise identical results.  Asynchronous on
 * stream; the descriptor upload (when pointers or dt change) is staged
 * before the call returns.  Errors: DG_EINVAL (null, aliasing or not
 * 16-byte aligned pointers, nsteps < 0, dt not finite, mode), DG_EHIP. */
dg_status dg_rk_step_batch(dg_batch b, void* const* u, void* const* res, const double* dt,
                           int32_t nsteps, int32_t mode, void* stream);

/* Releases the batch and its problems; NULL is a no-op. */
void dg_destroy_batch(dg_batch b);

/* On-device diagnostics: the discrete energy of u - ref in the mass-matrix
 * norm of Section 2 (M^k = J_k M on affine elements, Section 2.1), weighted
 * by the material,
 *   *dev_out = 1/2 sum_k J_k [ eps_k dE^T M dE + mu_k dH^T M dH ],
 * dE = E - E_ref, dH = H - H_ref, accumulated in binary64 in a fixed order
 * (bitwise reproducible).  ref NULL gives the energy of u, which the upwind
 * flux never increases; with ref the interpolated exact solution,
 * sqrt(2 *dev_out) is the L2 error.  u, ref: device state arrays of the
 * problem; dev_out: device pointer to one double.  Asynchronous on stream;
 * uses a partial-sum buffer owned by the problem, so calls on one problem
 * must not overlap.  Errors: DG_EINVAL (null p, u or dev_out), DG_EHIP. */
dg_status dg_energy(dg_problem p, const void* u, const void* ref, double* dev_out, void* stream);

/* Host <-> device conversion between the canonical host layout
 * [6][K][Np] binary64 (host pointer) and a device state array (layout above,
 * problem precision).  dg_pack zeroes the padding.  Both block until the copy
 * has finished on stream.  Errors: DG_EINVAL, DG_EHIP, DG_ENOMEM. */
dg_status dg_pack(dg_problem p, const double* host_u, void* dev_u, void* stream);
dg_status dg_unpack(dg_problem p, const void* dev_u, double* host_u, void* stream);

/* Physical node coordinates, host pointer K x Np x 3 (x, y, z) binary64. */
dg_status dg_nodes(dg_problem p, double* host_xyz);

/* Releases every device and host resource of p; NULL is a no-op.  The caller
 * must ensure no queued work still uses p. */
void dg_destroy(dg_problem p);

/* Thread-local text of the last error ("" if none). */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DG_H_ */
