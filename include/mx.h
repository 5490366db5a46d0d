/*
 * mx.h -- C ABI of the MI355X (gfx950) Schwarz-preconditioned GMRES solver (one- and two-level
 * AS, RAS and ORAS; standard or weighted GMRES) for the lowest- and second-order Nedelec
 * discretisations of  curl curl E - (k^2 + i xi) E = F  (Bonazzoli, Dolean, Graham, Spence,
 * Tournier, "Domain decomposition preconditioning for the high-frequency time-harmonic Maxwell
 * equations with absorption", arXiv:1711.03789).
 *
 * Conventions for every entry point:
 *   - return value: MX_OK (0) or a negative MX_E* code; mx_last_error() gives a message for the
 *     calling thread.  No C++ exception crosses this boundary.
 *   - handles (mx_mesh, mx_matrix, mx_partition, mx_precond, mx_ctx) are created and destroyed
 *     by the library; destroy functions accept NULL.
 *   - "host" pointers are caller-owned CPU memory, borrowed for the duration of the call;
 *     "dev" pointers are caller-owned device memory on the context's GPU (for instance the
 *     data_ptr of a torch tensor), also borrowed.  Device results are written asynchronously on
 *     the given stream (a hipStream_t passed as void*, NULL = the null stream) unless stated.
 *   - complex vectors are interleaved (re, im) pairs: complex128 = 2 doubles, complex64 =
 *     2 floats per entry (the C99 _Complex layout).
 *   - a context is used by one host thread at a time.
 *   - where no "Errors:" line is given: MX_EINVAL for a NULL handle or pointer that is required,
 *     a size or index out of range or a handle of the wrong state, MX_EDEVICE for a failing HIP
 *     call; destroy functions return nothing.
 */
#ifndef MX_H
#define MX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------- */
#define MX_OK 0
#define MX_EINVAL (-1)    /* bad argument (sizes, kinds, NULL where not allowed)              */
#define MX_ENOMEM (-2)    /* host or device allocation failed                                  */
#define MX_EDEVICE (-3)   /* HIP runtime error or no usable gfx950 device                      */
#define MX_EPIVOT (-4)    /* zero or non-finite pivot in a local LDL^T factorisation           */
#define MX_ENAN (-5)      /* non-finite residual norm in GMRES                                 */
#define MX_ESTALL (-6)    /* a bounded device-side wait expired (dependency never satisfied)   */
#define MX_EHBM (-7)      /* a server request whose footprint can never fit the HBM budget      */
#define MX_ETIMEOUT (-8)  /* a server request is not finished within the given time             */

/* ---- enums -------------------------------------------------------------------------------- */
#define MX_BC_PEC 0        /* E x n = 0 on the boundary (eq:PECcond)                          */
#define MX_BC_IMPEDANCE 1  /* first-order impedance condition (eq:imp)                        */

#define MX_AS 0    /* additive Schwarz, PEC local minors, no partition of unity (eq:defAS)     */
#define MX_RAS 1   /* restricted AS: PEC local minors, Boolean partition of unity (Sec. 6.3)   */
#define MX_ORAS 2  /* ImpRAS: impedance local problems, Boolean partition of unity (Sec. 6.3)  */

#define MX_C128 0  /* complex double factors                                                   */
#define MX_C64 1   /* complex float factors (FP32 matrix-core updates, FP32 accumulation)      */

typedef struct mx_ctx mx_ctx;
typedef struct mx_mesh mx_mesh;
typedef struct mx_matrix mx_matrix;
typedef struct mx_partition mx_partition;
typedef struct mx_precond mx_precond;
typedef struct mx_server mx_server;

const char *mx_last_error(void);
int mx_version(void);

/* ---- context ------------------------------------------------------------------------------ */
/* Binds HIP device `device` (must be gfx950).  Large device blocks (64 MiB and up: factor tiles,
 * trimmed factors) freed by the library stay mapped in a process-wide cache and are reused by
 * later setups (remapping tens of GB costs seconds); mx_ctx_destroy waits for the device and
 * returns the cached blocks and the stream-ordered pool's unused memory to HIP.  Objects must
 * not be destroyed while work that uses them is still queued.  Errors: MX_EDEVICE. */
int mx_ctx_create(int device, mx_ctx **out);
void mx_ctx_destroy(mx_ctx *ctx);

/* ---- mesh and edge numbering (host only; Sec. 2.2, Sec. 6.1) ------------------------------ */
/* Box [0,lx]x[0,ly]x[0,lz] of nx*ny*nz cubes, each split into the 6 Kuhn tetrahedra (path
 * o -> o+e_s0 -> o+e_s0+e_s1 -> o+(1,1,1) for the axis permutations s in lexicographic order).
 * vertex (i,j,k) = i + (nx+1)(j + (ny+1)k); tet = 6*cube + permutation rank, cube x-fastest;
 * edges = all vertex pairs of tetrahedra oriented lo -> hi, sorted by (lo, hi); the DOF of an
 * edge is the tangential line integral along that orientation (lowest-order duality).
 * Errors: MX_EINVAL (n < 1, length <= 0, more than 2^31-1 edges), MX_ENOMEM. */
int mx_mesh_box(int nx, int ny, int nz, double lx, double ly, double lz, mx_mesh **out);
int mx_mesh_sizes(const mx_mesh *m, int64_t *n_vert, int64_t *n_tet, int64_t *n_edge,
                  int64_t *n_bface);
/* Copies into caller buffers of sizes tet_vert[4T], edge_vert[2E], tet_edge[6T],
 * tet_edge_sign[6T] (+1 when the tetrahedron's local edge a->b runs lo -> hi), bface_vert[3F]
 * (boundary triangles, vertices ascending).  Any pointer may be NULL to skip that array. */
int mx_mesh_export(const mx_mesh *m, int32_t *tet_vert, int32_t *edge_vert, int32_t *tet_edge,
                   int8_t *tet_edge_sign, int32_t *bface_vert);
void mx_mesh_destroy(mx_mesh *m);

/* ---- Galerkin matrix and load (Sec. 2.2, eq:Helmholtzvf_intro, eq:imp) -------------------- */
/* A = K - (k^2 + i xi) M - i sign(xi) k M_b (impedance; sign(0) = +1) or, for PEC, K - (k^2 +
 * i xi) M with identity rows/columns on boundary edges.  Whitney element matrices in closed
 * form.  The CSR (int64 row pointers, int32 columns sorted ascending, complex128 values, plus a
 * complex64 copy of the values) is built on the host and kept on the context's device.
 * Errors: MX_EINVAL, MX_ENOMEM, MX_EDEVICE. */
/* ctx may be NULL: the matrix is then host-only until mx_matrix_upload. */
int mx_matrix_assemble(mx_ctx *ctx, const mx_mesh *m, double k, double xi, int bc,
                       mx_matrix **out);
/* D_k of eq:ip: the Gram matrix of the wavenumber-weighted inner product of eq:weight,
 * (v, w)_{curl,k} = (curl v, curl w) + k^2 (v, w), in the edge basis: D = K + k^2 M (real
 * symmetric positive definite, stored like a Galerkin matrix with zero imaginary parts; no
 * boundary term; PEC: identity rows and columns on boundary edges).  For mx_gmres_weighted.
 * ctx may be NULL (host-only until mx_matrix_upload).  Errors: MX_EINVAL, MX_ENOMEM, MX_EDEVICE. */
int mx_weight_assemble(mx_ctx *ctx, const mx_mesh *m, double k, int bc, mx_matrix **out);
/* The same operator on the Nedelec space of order `order` (Sec. 2.2: order m; the paper's
 * second-order runs are Tables tab:theoryDeltamin and tab:6bis).  order 1 is mx_matrix_assemble.
 * order 2: the hierarchical basis of the first-family space, 20 functions per tetrahedron, with
 * l the barycentric coordinates and vertices taken in ascending global id: per edge i -> j the
 * Whitney function l_i grad l_j - l_j grad l_i and grad(l_i l_j); per face i < j < k the two
 * functions l_k w_ij and l_j w_ik.  DOF numbering: the E Whitney functions (the edge numbering,
 * so the lowest-order space is the leading block), then the E edge gradients, then two per face
 * (faces sorted by their ascending vertex triples; mx_mesh_order2_export).  Element integrals
 * are exact (polynomial moments of barycentric coordinates).  PEC: identity rows and columns on
 * every DOF of a boundary edge or face.  The matrix keeps its order: preconditioners built from
 * it use the order-2 local spaces.  ctx may be NULL.  Errors: MX_EINVAL (order not 1 or 2, more
 * than 2^31-1 DOFs), MX_ENOMEM, MX_EDEVICE. */
int mx_matrix_assemble_order(mx_ctx *ctx, const mx_mesh *m, int order, double k, double xi, int bc,
                             mx_matrix **out);
/* D_k = K + k^2 M of mx_weight_assemble on the Nedelec space of order `order` (1 or 2; order 2 in
 * the basis and numbering of mx_matrix_assemble_order), for mx_gmres_weighted with a matrix of
 * the same order.  ctx may be NULL.  Errors: MX_EINVAL, MX_ENOMEM, MX_EDEVICE. */
int mx_weight_assemble_order(mx_ctx *ctx, const mx_mesh *m, int order, double k, int bc,
                             mx_matrix **out);
/* Order-2 sizes: faces F (interior and boundary) and DOFs N = 2E + 2F.  The order-2 topology is
 * built on the mesh's first order-2 call (thread safe) and kept with the mesh. */
int mx_mesh_order2_sizes(const mx_mesh *m, int64_t *n_face, int64_t *n_dof);
/* face_vert[3F] (ascending triples, sorted), tet_face[4T] (face ids of the local faces (1,2,3),
 * (0,2,3), (0,1,3), (0,1,2) of each tetrahedron), dof_boundary[N] (1: the DOF's edge or face
 * lies on the box boundary).  Any pointer may be NULL. */
int mx_mesh_order2_export(const mx_mesh *m, int32_t *face_vert, int32_t *tet_face,
                          uint8_t *dof_boundary);
/* Order-2 local DOF sets (eq:restriction1 for the order-2 space) and the Boolean owner of every
 * DOF (eq:algebPartUnity).  MX_AS / MX_RAS: the Whitney and gradient DOFs of the lowest-order
 * AS set's edges and the two DOFs of every face whose tetrahedra all lie in the subdomain;
 * MX_ORAS: every DOF of the subdomain's tetrahedra; sorted ascending.  owner = least
 * non-overlapping part holding a tetrahedron of the DOF's edge or face.  offsets[n_sub+1]
 * (required), loc2glob[offsets[n_sub]], owner[N] (either may be NULL; call with loc2glob NULL
 * for the sizes).  Errors: MX_EINVAL. */
int mx_partition_order2_export(const mx_mesh *m, const mx_partition *p, int kind, int64_t *offsets,
                               int32_t *loc2glob, int32_t *owner);
/* Device copy of a host-only matrix (assembled with ctx = NULL).  The copies run on a private
 * stream that does not wait for other streams, and the call returns when they are done, so
 * another host thread may upload the next matrix while the device works.  Errors: MX_EINVAL
 * (already on a device), MX_ENOMEM, MX_EDEVICE. */
int mx_matrix_upload(mx_ctx *ctx, mx_matrix *A);
int mx_matrix_sizes(const mx_matrix *A, int64_t *n, int64_t *nnz);
/* Host copies: rowptr[n+1], col[nnz], val[2*nnz] (complex128).  Any may be NULL. */
int mx_matrix_export(const mx_matrix *A, int64_t *rowptr, int32_t *col, double *val);
void mx_matrix_destroy(mx_matrix *A);
/* y = A x on the device; x_dev, y_dev complex128[n], must not overlap. */
int mx_spmv(mx_ctx *ctx, const mx_matrix *A, const void *x_dev, void *y_dev, void *stream);
/* Load f_e = int F . w_e for F = pol * exp(-|x - c|^2 / (2 sigma^2)) with the 4-point degree-2
 * tetrahedron rule; zero on PEC boundary edges.  f_host: complex128[E] (host). */
int mx_rhs_gaussian(const mx_mesh *m, int bc, const double center[3], const double pol[3],
                    double sigma, double *f_host);

/* ---- partition with overlap (Sec. 3.1, Sec. 6.1, eq:restriction1, eq:algebPartUnity) ----- */
/* px*py*pz boxes of cubes cut at cx[0..px] (cx[0] = 0, cx[px] = nx, strictly increasing; NULL =
 * even cuts floor(i*nx/px)), likewise cy, cz; subdomain l = bx + px(by + py bz).  `layers`
 * sweeps each add every tetrahedron sharing a vertex with the current set.  AS/RAS local DOFs:
 * edges all of whose tetrahedra lie in the subdomain; ORAS: all edges of its tetrahedra; both
 * sorted by global edge id.  owner(e) = least non-overlapping part holding a tetrahedron of e.
 * Errors: MX_EINVAL, MX_ENOMEM. */
int mx_partition_box(const mx_mesh *m, int px, int py, int pz, const int32_t *cx,
                     const int32_t *cy, const int32_t *cz, int layers, mx_partition **out);
/* n_sub = px*py*pz; total = sum of local sizes for `kind` (MX_AS and MX_RAS share sets). */
int mx_partition_sizes(const mx_partition *p, int kind, int32_t *n_sub, int64_t *total);
/* offsets[n_sub+1] (int64), loc2glob[total] (local DOFs of subdomain l at offsets[l]..),
 * owner[E], n_tet_local[n_sub] (tetrahedra per subdomain).  Any may be NULL. */
int mx_partition_export(const mx_partition *p, int kind, int64_t *offsets, int32_t *loc2glob,
                        int32_t *owner, int64_t *n_tet_local);
void mx_partition_destroy(mx_partition *p);

/* ---- one-level Schwarz preconditioner (eq:defAS, eq:minor, RAS_1, ImpRAS_1 of Sec. 6.3) --- */
typedef struct {
  int kind;        /* MX_AS | MX_RAS | MX_ORAS                                                */
  double xi_prec;  /* absorption of the local problems (ORAS local assembly; AS/RAS use A's)  */
                   /* A problem at another xi (xi_prob != xi_prec, e.g. 0) is preconditioned  */
                   /* by setting up from a matrix assembled at xi_prec and passing the       */
                   /* problem's matrix to mx_gmres (Sec. 1.2, eq. key_intro)                 */
  int precision;   /* MX_C128 | MX_C64 (local factors and local solves)                       */
  int sweep_grid;  /* workgroups of the persistent sweep kernels; 0 = one per compute unit      */
  int sub_begin;   /* resident share: build only subdomains [sub_begin, sub_end) (both 0 = all); */
  int sub_end;     /* the application then returns the share's part of the sum (zero elsewhere)*/
  int64_t pool_limit; /* bytes of full factor tiles held at a time: the subdomains are factored in */
                      /* consecutive groups that fit (0 = as many as free device memory allows)  */
  int32_t factor_schedule; /* MX_FACTOR_*: order of the blocked factorisation's launches; every */
                           /* schedule computes the same LDL^T up to rounding (0 = automatic)   */
  int32_t factor_width;    /* look-ahead: block columns applied per pass of the trailing update */
                           /* (1 .. 4; 0 = 4 for MX_C128, 3 for MX_C64)                        */
} mx_precond_opts;

/* factor_schedule values.  ONE_STREAM: diagonal tile, panel and trailing update of one block
 * column after another on one stream (the automatic choice when steps are a few tiles per CU).
 * LOOKAHEAD: two streams; the next block columns are updated and factored on one while the rest
 * of the trailing update runs on the other, factor_width block columns per pass over each tile
 * (the automatic choice otherwise). */
enum { MX_FACTOR_AUTO = 0, MX_FACTOR_ONE_STREAM = 1, MX_FACTOR_LOOKAHEAD = 2 };

/* Host-only view of one local problem, as mx_precond_setup builds it (for inspection and
 * tests): A^l in local numbering (local DOFs sorted by global id) as CSR rowptr[n+1],
 * col[nnz], val[2*nnz], and its reverse Cuthill-McKee order perm[n] (new -> old; key (degree,
 * index), George-Liu pseudo-peripheral start per component, neighbours by increasing key) with
 * the envelope start first[n] of each permuted row.  Call once with rowptr == NULL to get *n and
 * *nnz, then with buffers of those sizes (any array may be NULL).  An order-2 matrix gives the
 * order-2 local problem on the sets of mx_partition_order2_export.  Errors: MX_EINVAL. */
int mx_local_problem(const mx_mesh *m, const mx_matrix *A, const mx_partition *p,
                     const mx_precond_opts *opts, int l, int64_t *n, int64_t *nnz, int64_t *rowptr,
                     int32_t *col, double *val, int32_t *perm, int32_t *first);

typedef struct {
  int32_t n_sub, tile;          /* subdomains, tile edge of the block-skyline storage         */
  int64_t n_local_total;        /* sum of local sizes                                          */
  int64_t max_local, max_blocks;
  int64_t tiles;                /* stored tiles (tile x tile complex each)                     */
  int64_t factor_bytes;         /* device bytes of the factor tiles (held during the factorisation)*/
  int64_t env_entries;          /* sum over subdomains of the exact lower envelope (diag incl.)*/
  double env_flops;             /* 8 * sum_i w_i^2 / 2 real flops (envelope LDL^T)             */
  double tile_flops;            /* real flops of the blocked factorisation as executed         */
  int64_t apply_bytes;          /* algorithmic bytes of one application (see mx_precond_apply)*/
  int64_t sweep_bytes;          /* algorithmic bytes of one block-sweep launch (either direction):*/
                                /* the envelope factor read once and three local-vector passes   */
  double t_host_setup, t_upload, t_factor; /* seconds of the last mx_precond_setup phases      */
  int64_t pack_bytes;           /* device bytes of the trimmed tiles read by the sweeps (the tile */
                                /* rows that meet the envelope; diagonal tiles in full)          */
  double t_pack;                /* seconds spent trimming the tiles and freeing the full ones    */
  int32_t factor_groups;        /* consecutive subdomain groups the factorisation ran in         */
} mx_precond_info;

/* Builds the local matrices (AS/RAS: minors of A, so the matrix's k, xi and bc are used; ORAS:
 * impedance local problems assembled with xi_prec, impedance coefficient k on the subdomain
 * boundary), orders each by reverse Cuthill-McKee, stores it in block-skyline tiles and
 * factors all subdomains together on the device (pivot-free complex-symmetric LDL^T, which
 * exists for xi != 0 by the coercivity lemma).  Synchronous.  For a matrix of order 2
 * (mx_matrix_assemble_order) the local spaces, owners and ORAS problems are those of the order-2
 * space (mx_partition_order2_export); vectors then have the order-2 DOF count.
 * Errors: MX_EINVAL, MX_ENOMEM, MX_EDEVICE, MX_EPIVOT. */
int mx_precond_setup(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                     const mx_precond_opts *opts, mx_precond **out);
/* The two halves of mx_precond_setup, so that the host half of one preconditioner can run on
 * another host thread while the device works on an earlier one.  mx_precond_plan does all host
 * work (local matrices, orderings, tile layout, schedules; no device work, A needs no device
 * copy; ctx may be NULL, and the device is then bound by stage or materialize) and returns the
 * exact peak device bytes that materialising it will allocate;
 * mx_precond_materialize uploads and factors on `stream` (NULL = null stream) and returns when
 * done.  A planned, not yet materialised preconditioner may only be materialised or destroyed.
 * Device buffers of P are allocated on `stream` and released on it by mx_precond_destroy, so a
 * stream passed here must outlive P (the null stream always does).
 * Errors: as mx_precond_setup. */
int mx_precond_plan(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                    const mx_precond_opts *opts, mx_precond **out, uint64_t *device_bytes);
int mx_precond_materialize(mx_ctx *ctx, mx_precond *P, void *stream);
/* Optional, between plan and materialize: copies everything the device half reads from the
 * host (tile layout, schedules, gather maps, the local matrices' entries) to the device and
 * returns when done.  The copies run on a private stream that does not wait for other streams,
 * so another host thread can stage the next preconditioner while the device works;
 * mx_precond_materialize then only zeroes, scatters, factors and trims.  The staged entries are
 * freed by mx_precond_materialize.  Errors: MX_EINVAL (materialised or staged already, or
 * planned for another device), MX_ENOMEM, MX_EDEVICE. */
int mx_precond_stage(mx_ctx *ctx, mx_precond *P);
/* z = sum_l R_l^T D_l (A^l)^-1 R_l v (D_l = I for AS); v_dev, z_dev complex128[E], distinct.
 * Enqueued on `stream`; device-side failures surface at the next synchronising call.
 * apply_bytes = factors read twice (forward and backward sweep) + local vectors + gathers.
 * With a coarse level, the two-level form (mx_precond_add_coarse).  Errors: MX_EINVAL (planned
 * but not materialised, a planned coarse level not built), MX_EPIVOT / MX_ESTALL (a failure
 * already reported for P), MX_EDEVICE. */
int mx_precond_apply(mx_ctx *ctx, mx_precond *P, const void *v_dev, void *z_dev, void *stream);
int mx_precond_get_info(const mx_precond *P, mx_precond_info *info);
/* For subdomain l: perm[n_l] (new -> old local index, RCM) and first[n_l] (envelope start of
 * each permuted row).  Either may be NULL.  n is the caller's buffer length and must equal n_l
 * (MX_EINVAL otherwise; nothing is written).  Available once planned. */
int mx_precond_export_perm(const mx_precond *P, int l, int64_t n, int32_t *perm, int32_t *first);
/* Host copy of the factored diagonal D of subdomain l (complex128[n_l], permuted order); n as
 * for mx_precond_export_perm.  Needs a materialised preconditioner. */
int mx_precond_export_diag(const mx_precond *P, int l, int64_t n, double *d);
/* Per-launch timing of the two block-sweep kernels (forward and backward; together the dominant
 * work of an application) with HIP events recorded on the launch stream around each launch.
 * enable = 1 clears earlier records and starts recording; enable = 0 stops, waits for the
 * recorded events and returns the number of timed applications and the summed durations of the
 * forward and of the backward launches, in milliseconds.  Errors: MX_EINVAL, MX_EDEVICE. */
int mx_precond_sweep_timing(mx_precond *P, int enable, int64_t *launches, double *ms_forward,
                            double *ms_backward);
/* Launch-shape tuner: times the application with several sweep grid sizes (fractions and
 * multiples of the CU count) on `stream`, keeps the fastest in P and returns it (best_grid,
 * best_ms per application).  Synchronous; allocates two temporary E-vectors.
 * Errors: MX_EINVAL, MX_ENOMEM, MX_EDEVICE, MX_ESTALL. */
int mx_precond_autotune(mx_ctx *ctx, mx_precond *P, void *stream, int32_t *best_grid,
                        double *best_ms);
/* ---- two-level preconditioners (Sec. 3.2, Sec. 3.3, Sec. 6.3) ------------------------------ */
#define MX_COARSE_ADDITIVE 0   /* B = B1 + G: AS_2 (eq:defAS), RAS_2 (eq:RAS2), ImpRAS_2            */
#define MX_COARSE_HYBRID 1     /* B = (I - G A) B1 (I - A G) + G: HRAS, ImpHRAS (eq:HRAS)           */
#define MX_COARSE_DEFLATION 2  /* B = B1 (I - A G) + G: ADEF1-RAS, ADEF1-ImpRAS (eq:ADEF1ras)       */
/* Adds a coarse level to the materialised one-level preconditioner P (B1: AS, RAS or ORAS =
 * ImpRAS), which was built from A on mesh m (all subdomains, not a resident share).  Coarse
 * mesh: the box of m with `ratio` times fewer cubes on every axis (ratio must divide each
 * count; the two meshes are then nested).  Coarse basis: the Whitney functions of the coarse
 * edges (PEC: those with zero tangential trace).  R^0 (eq:restriction): (R^0)_pj = fine DOF j of
 * coarse basis function p (line integral along fine edge j); with an order-2 A the coarse basis
 * stays the lowest-order one, which lies in the fine order-2 space with Whitney coefficients
 * only, so R^0 has zero columns for the gradient and face DOFs; A^0 = R^0 A R^0^T (eq:minor),
 * factored on the device like a local problem; G = R^0^T (A^0)^-1 R^0.  Afterwards
 * mx_precond_apply and mx_gmres with P apply the two-level form `combine` (MX_COARSE_*).  A is
 * borrowed: it must have a device copy and outlive P (the hybrid and deflated forms multiply by
 * it), and it must be the matrix P was built from (same k and bc, xi = the xi of the local
 * problems).  Synchronous on `stream`, which must outlive P.
 * Errors: MX_EINVAL (ratio, matrix, a share, already two-level), MX_ENOMEM, MX_EDEVICE,
 * MX_EPIVOT. */
int mx_precond_add_coarse(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *m,
                          int ratio, int combine, void *stream);
/* The same with a coarse box mesh of cnx x cny x cnz cubes that need not be nested in the fine one
 * (Sec. 6.1 uses non-nested coarse meshes of a chosen coarse size H_cs): each entry of R^0 is
 * the line integral of the coarse Whitney function along the fine edge by an nq-point
 * Gauss-Legendre rule (1 <= nq <= 64; the paper's runs use a fixed number of points per edge,
 * e.g. 12).  On a nested mesh the integrand is affine along every fine edge and any nq gives the
 * exact values up to rounding.  The coarse point of a quadrature node is located in the coarse
 * Kuhn split (cube by floor, tetrahedron by sorting the local coordinates).  Lowest-order
 * matrices only (an order-2 A needs the nested mesh of mx_precond_add_coarse).
 * Errors: as mx_precond_add_coarse. */
int mx_precond_add_coarse_box(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *m,
                              int cnx, int cny, int cnz, int nq, int combine, void *stream);
/* Optional host half of mx_precond_add_coarse (coarse mesh, R^0, A^0 and the plan of its
 * factorisation; no device work, A needs no device copy), so that it can run on another host
 * thread, also on a planned, not yet materialised P.  mx_precond_add_coarse with the same A, m,
 * ratio and combine then only builds the device half; until then P is refused by
 * mx_precond_apply and mx_gmres.  Errors: as mx_precond_add_coarse. */
int mx_precond_plan_coarse(mx_precond *P, const mx_matrix *A, const mx_mesh *m, int ratio,
                           int combine);
/* Host half of mx_precond_add_coarse_box (then completed by mx_precond_add_coarse_box with the
 * same arguments). */
int mx_precond_plan_coarse_box(mx_precond *P, const mx_matrix *A, const mx_mesh *m, int cnx,
                               int cny, int cnz, int nq, int combine);
/* Host copies of the coarse level, for inspection and tests: R^0 as CSR r_rowptr[n_coarse+1],
 * r_col[nnz_r] (fine edge ids), r_val[nnz_r] (real), and A^0 as a_rowptr[n_coarse+1],
 * a_col[nnz_a], a_val[2*nnz_a] (complex128).  Rows are all coarse edges: with PEC the boundary
 * edges carry no basis function, so their R^0 rows are empty and their A^0 rows are unit rows.
 * Any pointer may be NULL (call first with the arrays NULL for the sizes).  Errors: MX_EINVAL
 * (no coarse level). */
int mx_precond_coarse_export(const mx_precond *P, int64_t *n_coarse, int64_t *nnz_r,
                             int64_t *nnz_a, int64_t *r_rowptr, int32_t *r_col, double *r_val,
                             int64_t *a_rowptr, int32_t *a_col, double *a_val);
/* Host-only: the coarse operators mx_precond_add_coarse builds for a matrix A on mesh m (same
 * layout as mx_precond_coarse_export), without a preconditioner or a device.  Call with the six
 * arrays NULL to get the sizes; then *n_coarse, *nnz_r and *nnz_a must hold those sizes.
 * Errors: MX_EINVAL. */
int mx_coarse_operators(const mx_mesh *m, const mx_matrix *A, int ratio, int64_t *n_coarse,
                        int64_t *nnz_r, int64_t *nnz_a, int64_t *r_rowptr, int32_t *r_col,
                        double *r_val, int64_t *a_rowptr, int32_t *a_col, double *a_val);
/* Host-only coarse operators of mx_precond_add_coarse_box (same layout and calling convention as
 * mx_coarse_operators).  Errors: MX_EINVAL. */
int mx_coarse_operators_box(const mx_mesh *m, const mx_matrix *A, int cnx, int cny, int cnz, int nq,
                            int64_t *n_coarse, int64_t *nnz_r, int64_t *nnz_a, int64_t *r_rowptr,
                            int32_t *r_col, double *r_val, int64_t *a_rowptr, int32_t *a_col,
                            double *a_val);
/* Factorisation tuner: sets up the preconditioner that mx_precond_setup would build from these
 * arguments once for each factorisation launch shape -- one stream, and look-ahead with 1, 2, 3
 * and 4 block columns per trailing-update pass (factor_width) -- times each factorisation, frees
 * it, and returns the fastest (best_schedule, best_width for mx_precond_opts; best_ms) and all
 * five times in ms_each[5] (either may be NULL).  opts->factor_schedule and factor_width are
 * ignored.  Every candidate computes the same factors up to rounding.  Costs five setups.
 * Errors: as mx_precond_setup. */
int mx_precond_tune_factor(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                           const mx_precond_opts *opts, void *stream, int32_t *best_schedule,
                           int32_t *best_width, double *best_ms, double *ms_each);
/* Checks the device error word of P (set by a failed pivot or an expired wait).  Once such an
 * error has been reported (by this call, mx_gmres or mx_precond_autotune), P is unusable: its
 * device flags stay set, and every later mx_precond_apply, mx_precond_autotune, mx_gmres and
 * mx_precond_check with P returns the same code without enqueuing work.  Applications enqueued
 * before the report write NaN into z.  Destroy P and set it up again. */
int mx_precond_check(mx_precond *P);
void mx_precond_destroy(mx_precond *P);

/* ---- right-preconditioned restarted (F)GMRES (Sec. 5.2 definition, Sec. 6.1 stopping) ---- */
typedef struct {
  int restart;      /* m, Krylov vectors per cycle                                            */
  int max_iters;    /* cap on total iterations (one iteration = one B^-1 and one A product)   */
  int flexible;     /* 1: keep z_j = B^-1 v_j and update x += Z y (FGMRES)                    */
  int fixed_iters;  /* > 0: run exactly this many iterations, ignoring rtol                   */
  int spmv_c64;     /* 1: Arnoldi products with the complex64 copy of A (FP64 accumulate)     */
  double rtol;      /* stop when ||b - A x|| <= rtol ||b - A x0||                             */
  int graph;        /* 1: each Arnoldi step (preconditioner application, products with A, the */
                    /* Gram-Schmidt passes, the Givens update, the status copy) is captured    */
                    /* once into a HIP graph and replayed, in later cycles and in later solves */
                    /* on the same context with the same matrix, preconditioner and restart;   */
                    /* results are bitwise those of the launched steps.  Ignored while the     */
                    /* preconditioner's sweeps are timed or its applications are batched.      */
} mx_gmres_opts;

typedef struct {
  int iters, cycles, converged;
  double relres_true, relres_est;
  double t_solve;  /* seconds */
} mx_gmres_stats;

/* Orthogonalisation: classical Gram-Schmidt twice; least squares: complex Givens rotations
 * (c = |a|/r, s = (a/|a|) conj(b)/r), all in FP64 on the device.  x_dev holds x0 on entry and
 * the solution on exit.  res_hist (host, may be NULL) receives |g_{j+1}|/||r0|| per iteration
 * (max_iters + 1 entries, entry 0 = 1).  Non-convergence is not an error (converged = 0).
 * Synchronous.  Errors: MX_EINVAL, MX_ENOMEM, MX_EDEVICE, MX_ENAN, MX_ESTALL. */
int mx_gmres(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev, void *x_dev,
             const mx_gmres_opts *opts, mx_gmres_stats *stats, double *res_hist, void *stream);

/* Weighted GMRES (Sec. 5.2, eq:ip): as mx_gmres, but the iterate minimises ||b - A x||_D over
 * the Krylov space, with <v, w>_D = w^H D v for a Hermitian positive definite D (e.g. D_k from
 * mx_weight_assemble).  The Arnoldi process orthonormalises in <.,.>_D (classical Gram-Schmidt
 * twice, D w formed before each pass and for the norm: three products with D per iteration),
 * so the Givens least squares is unchanged, and every residual norm (the estimate, rtol, the
 * true-residual test, res_hist) is the D-norm.  D = NULL is mx_gmres.  Errors: as mx_gmres. */
int mx_gmres_weighted(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const mx_matrix *D,
                      const void *b_dev, void *x_dev, const mx_gmres_opts *opts,
                      mx_gmres_stats *stats, double *res_hist, void *stream);

/* The same solve as mx_gmres for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the Krylov workspace
 * (basis, Hessenberg matrix, rotations, reduction partials, status) lives in a fixed array of
 * 64 MiB per GPU that the library holds from the first mx_ctx_create on that GPU until the
 * process ends, instead of the context's workspace, and the call makes no device allocation.
 * Workspace bytes are about 16 E (restart + 5) (+ 16 E restart when flexible); a call needing
 * more than the array returns MX_EINVAL without enqueuing work.  The preconditioner, matrix and
 * vectors are the caller's as for mx_gmres; results are identical to mx_gmres's.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on the same GPU (from several
 * host threads or on several streams) race and must not be made.  Errors: as mx_gmres. */
int mx_gmres_noalloc(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev,
                     void *x_dev, const mx_gmres_opts *opts, mx_gmres_stats *stats,
                     double *res_hist, void *stream);

/* ---- solve server: continuous batching of independent solves -------------------------------- */
/* Requests are unit-cube problems solved by the path above (Sec. 6.1 workloads).  `slots` worker
 * threads, each with its own HIP stream, pull requests in submission order; a slot first does the
 * request's host work (mesh, assembly, partition, local problems, orderings), which fixes its exact
 * device footprint, then waits until the footprint fits in what is left of `hbm_budget`, runs the
 * device work (upload, factorisation, GMRES) on its stream concurrently with the other admitted
 * requests and returns its memory.  With batch_applies, the preconditioner applications of the
 * requests that are in their GMRES phase are batched: a batcher thread collects one application
 * from each of them (or whatever arrived within batch_window_us) and runs their restrictions,
 * one forward and one backward block-sweep launch over all their subdomains, and their
 * prolongations, on its own stream; each request's stream waits for that batch.  A lone
 * application runs on its request's own stream.  Results do not
 * depend on what else is running (deterministic kernels; a batched application computes exactly
 * what a single one does).  A server is driven from any number of host threads. */
typedef struct {
  uint64_t hbm_budget;  /* device bytes the server may hold; 0 = 85% of the free memory          */
  int slots;            /* requests in flight (worker threads / streams), at most 16               */
  int kind, precision;  /* preconditioner (MX_AS/MX_RAS/MX_ORAS) and factor precision             */
  int layers;           /* overlap sweeps                                                          */
  int restart, max_iters, flexible, spmv_c64;
  double rtol;
  int batch_applies;    /* 1: batch the applications of co-resident requests; 0: each on its own  */
  int batch_window_us;  /* longest wait for the other requests' applications (0 = 50 us)           */
} mx_server_opts;

typedef struct {
  int n;                                     /* cubes per side of the unit cube                  */
  int p;                                     /* subdomains per side (p^3 boxes)                   */
  double k, xi;                              /* wavenumber and absorption                        */
  double center[3], pol[3], sigma;           /* Gaussian source, as mx_rhs_gaussian              */
} mx_request;

typedef struct {
  int status;                  /* MX_OK or the request's error code (message: mx_last_error)    */
  int iters, converged;
  double relres_true;
  int64_t n_dof;
  uint64_t footprint_bytes;    /* device bytes reserved for the request                          */
  double t_queue, t_host, t_device, t_total; /* s: submit->admitted, submit->host work done,
                                                admitted->done, submit->done                     */
} mx_result;

/* Errors: MX_EINVAL, MX_EDEVICE. */
int mx_server_create(int device, const mx_server_opts *opts, mx_server **out);
/* Non-blocking; *ticket identifies the request.  Errors: MX_EINVAL. */
int mx_server_submit(mx_server *s, const mx_request *req, uint64_t *ticket);
/* Blocks until the request is done (timeout_s < 0: no limit) and copies its result; a request
 * whose footprint exceeds the budget finishes with status MX_EHBM.  Errors: MX_EINVAL,
 * MX_ETIMEOUT. */
int mx_server_wait(mx_server *s, uint64_t ticket, double timeout_s, mx_result *res);
/* Copies the solution (complex128[n], host) of a finished, successful request. */
int mx_server_solution(mx_server *s, uint64_t ticket, double *x_host, int64_t n);
/* Forgets a finished request (its stored solution). */
int mx_server_release(mx_server *s, uint64_t ticket);
/* Budget, peak reserved bytes and the largest number of simultaneously admitted requests. */
int mx_server_stats(mx_server *s, uint64_t *budget, uint64_t *peak_used, int *max_admitted);
/* Batched applications so far: launches of the batcher and the applications they carried
 * (equal when nothing was batched; both 0 without batch_applies).  Errors: MX_EINVAL. */
int mx_server_batch_stats(mx_server *s, uint64_t *batches, uint64_t *applications);
/* Test hook of the server's recovery path: the next n device phases fail with MX_ENOMEM right
 * after their preconditioner has been materialised, as a late device allocation failure would.
 * The server then releases the request's device memory, waits for another request to finish (or
 * an idle device) and runs the device phase again from the same host plan; an injected failure
 * is retried even when the request is alone.  For callers that test that path, not for
 * production use.  Errors: MX_EINVAL. */
int mx_server_inject_enomem(mx_server *s, int n);
/* Finishes every submitted request, then stops the workers. */
void mx_server_destroy(mx_server *s);

/* ---- device self-check -------------------------------------------------------------------- */
/* Runs the matrix-core tile product used by the factorisation on random 64x64 complex tiles in
 * both precisions and compares with a plain device loop; *err64, *err32 receive the max
 * relative errors.  Synchronous. */
int mx_selftest(mx_ctx *ctx, double *err64, double *err32);
/* Host-only check of the error path of the library's host thread pool (which runs the per-
 * subdomain host work of setups and plans): n_items items run on up to 16 threads, twice (a
 * work-queue pass and a range-split pass); item fail_item (none if outside [0, n_items)) throws
 * the library's internal error (fail_code = MX_EINVAL) or an allocation failure (MX_ENOMEM).
 * Returns that code, as any entry point would, after every thread has been joined, with
 * *items_run = items completed before the failure stopped the pass; MX_OK when nothing failed
 * and every item ran exactly once per pass. */
int mx_selftest_host(int64_t n_items, int64_t fail_item, int fail_code, int64_t *items_run);

#ifdef __cplusplus
}
#endif
#endif /* MX_H */
