/*
 * hm.h -- C ABI of the hierarchical (H-matrix) view-factor radiosity library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library implements the hot path of "Hierarchical Block Low-rank
 * Approximation of Cavity Radiation" (arXiv 2305.06891):
 *   - facet geometry and the centroid-rule view factor of eq. (10)
 *     (Sec. 3.2): F_ij = max(0,cos_i) max(0,cos_j) A_j / (pi r^2), F_ii = 0,
 *     in the per-area convention (the paper's area-weighted F is diag(A) F);
 *   - the geometric cluster tree of Algorithm 1 and the block tree of
 *     Algorithm 2 with the admissibility condition of Sec. 4.2;
 *   - adaptive cross approximation (Sec. 4.3, eq. (30)) of the admissible
 *     blocks under the block-wise tolerance of eq. (31);
 *   - the block-wise product x -> F x of Sec. 5.2 inside a Krylov solve of the
 *     radiosity system C J = sigma eps T^4 with the reflection matrix of
 *     eq. (11), C = I - diag(1 - eps) F, and the facet flux of eq. (12).
 *
 * Conventions (every function):
 *   - Facet order at the ABI is the caller's ORIGINAL order.  The cluster
 *     permutation never leaks out (except through hm_tree_stats/perm_out).
 *   - Pointers are borrowed for the duration of the call unless stated.
 *     "HOST" pointers are ordinary CPU memory; "DEVICE" pointers must be
 *     device memory on the context's GPU (for example torch tensors) and are
 *     used in stream order on the context's stream.
 *   - Matrices of right-hand sides are column-major with a leading dimension
 *     (ld >= n); column r of X starts at X + r*ld.
 *   - Every call returns an hm_status; nothing throws across the ABI.  On
 *     failure hm_last_error(ctx) describes the cause (NULL ctx: the message
 *     is kept per thread and returned by hm_last_error(NULL)).
 *   - Opaque handles are created by the library and released by the
 *     matching *_destroy; destroying NULL is a no-op.
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HM_OK = 0,
  HM_EINVAL = 1,     /* invalid argument (sizes, ranges, NaN, zero area ...) */
  HM_ENOMEM = 2,     /* device/host allocation failed or budget exceeded     */
  HM_ENOTCONV = 3,   /* iteration did not reach the tolerance; best iterate  */
  HM_EDEVICE = 4,    /* HIP runtime error                                    */
  HM_EBUSY = 5,      /* result not ready yet (hm_poll)                       */
  HM_ENOTFOUND = 6   /* unknown ticket or cavity id                          */
} hm_status;

typedef enum { HM_F64 = 0, HM_F32 = 1, HM_BF16 = 2 } hm_dtype;

typedef struct hm_ctx hm_ctx;
typedef struct hm_tree hm_tree;
typedef struct hm_matrix hm_matrix;
typedef struct hm_server hm_server;

/* ------------------------------------------------------------------ context */

/* Create a context bound to GPU `device` and HIP stream `hip_stream`
 * (hipStream_t passed as void*; NULL = the device's null stream, which is
 * also torch's default stream).  All work of the context is ordered on that
 * stream.  One context per host thread / stream. */
hm_status hm_ctx_create(int device, void* hip_stream, hm_ctx** out);
void hm_ctx_destroy(hm_ctx* ctx);
/* Block until all work the library queued on ctx's stream has finished. */
hm_status hm_ctx_synchronize(hm_ctx* ctx);
const char* hm_status_string(hm_status s);
const char* hm_last_error(const hm_ctx* ctx);
/* Library version string, e.g. "hmrad 1.0 gfx950". */
const char* hm_version(void);

/* ----------------------------------------------------------- facet geometry */

/* Facet centroid, unit normal and area of every triangle (Sec. 3.1-3.2: the
 * radiation surface is a set of flat facets with areas, centroids and plane
 * normals).  HOST, FP64.  v: nv x 3 row-major vertices; tri: nt x 3
 * row-major vertex indices.  The normal is (b-a) x (c-a) normalised, then
 * oriented by `orient`: +1 keep, -1 flip, 0 flip if it points away from the
 * vertex centroid of the mesh (valid for star-shaped cavities).  Outputs
 * (caller-allocated HOST): centroid nt x 3, normal nt x 3, area nt.
 * HM_EINVAL on an index out of range, a degenerate (zero-area) triangle or a
 * non-finite coordinate. */
hm_status hm_facets_from_triangles(int64_t nv, const double* v, int64_t nt, const int32_t* tri,
                                   int orient, double* centroid, double* normal, double* area);

/* ----------------------------------------------------- cluster / block tree */

typedef struct {
  int32_t leaf_size; /* n_min of Algorithm 1: a cluster with #tau <= leaf_size is a leaf (>= 1) */
  double eta;        /* admissibility constant c of Sec. 4.2 (> 0) */
} hm_tree_params;

/* Build the index tree (Algorithm 1: split the centroid bounding box along
 * its longest axis at the median, ties x<y<z, order by (coordinate, original
 * index), left child gets floor(#tau/2)) and the block tree (Algorithm 2:
 * a block is admissible iff min(diam s, diam t) <= eta * dist(s, t) with
 * bounding-box diam/dist and dist > 0; an inadmissible block whose row or
 * column cluster is a leaf becomes a dense leaf).  HOST inputs (copied):
 * centroid n x 3, normal_into_cavity n x 3 (unit), area n (> 0).  ctx may be
 * NULL (the tree is host data).  Destroy with hm_tree_destroy. */
hm_status hm_build_cluster_tree(hm_ctx* ctx, int64_t n, const double* centroid,
                                const double* normal_into_cavity, const double* area,
                                const hm_tree_params* params, hm_tree** out);

/* Counts of the tree; any output pointer may be NULL.  perm_out (HOST, n):
 * perm_out[k] = original index of the facet at permuted position k. */
hm_status hm_tree_stats(const hm_tree* tree, int64_t* n_nodes, int64_t* n_dense, int64_t* n_lowrank,
                        int32_t* perm_out);

/* Leaf blocks of the block tree in permuted positions, sorted by (row begin,
 * column begin): dense_out (HOST, n_dense x 4) and lowrank_out (HOST,
 * n_lowrank x 4), each row (row_begin, row_end, col_begin, col_end).  Either
 * pointer may be NULL. */
hm_status hm_tree_blocks(const hm_tree* tree, int32_t* dense_out, int32_t* lowrank_out);
void hm_tree_destroy(hm_tree* tree);

/* ------------------------------------------------------------- H-matrix */

typedef struct {
  double aca_tol;          /* eps_rel of eq. (31), in (0, 1) */
  int32_t k_max;           /* rank cap of ACA; a block reaching it is stored dense (>= 1) */
  hm_dtype lowrank_dtype;  /* storage of U, V: HM_F64, HM_F32 or HM_BF16 */
  hm_dtype dense_dtype;    /* storage of near-field blocks: HM_F64, HM_F32 or HM_BF16; HM_BF16
                              needs HM_BF16 factors and keep_f32_copy, and no closed_row_scale
                              (HM_EINVAL otherwise) */
  int32_t keep_f32_copy;   /* with HM_BF16 factors: also keep FP32 factors (and an FP32 copy of a
                              BF16 near field); products with FP64 vectors use the copies
                              (refinement residual), products with FP32 vectors the BF16 arrays */
  int32_t closed_row_scale;/* 1: closed-cavity row scaling of eqs. (32)-(34) (clamp the row sum
                              to [0,1], divide rows with non-zero clamped sum by it); default 0 */
  int32_t autotune;        /* k >= 1: time the candidate work splits of the product's first
                              kernel (rows per item, bytes per wave task) on this matrix with
                              products of k columns (1..16: the width it will mostly be applied
                              to; with many columns longer items are candidates too, their
                              partial sums costing k times more) and keep the fastest; 0: fixed
                              defaults (128 rows, 16 KB).  Results are the same bit for bit
                              either way except for the order of partial sums.  HM_EINVAL
                              outside 0..16. */
  int32_t recompress;      /* 1: truncate every block stored low-rank to its smallest rank r whose
                              discarded singular values satisfy sqrt(sum_{i>r} s_i^2) <= aca_tol *
                              |s|_2 (Sec. 4.3 post-processing into U V^T; Sec. 5.1 truncation at
                              eps_rel): FP64 QR-free SVD of the crosses on the GPU, V' with
                              orthonormal columns.  The dense/low-rank decision is taken on the
                              ACA rank; blocks of ACA rank above 256 keep their crosses.  0: the
                              ACA crosses are stored as they are (default).  HM_EINVAL outside
                              0..1. */
  int32_t aca_pivot;       /* 0: partial (row/column) pivoting: each cross evaluates one row and
                              one column, stop when |u_k||v_k| <= aca_tol |sum u_l v_l^T|_F
                              (default); 1: full pivoting (the paper's choice): the block is
                              evaluated whole, each pivot is the largest entry of the residual
                              (first in row-major order on ties) and the stop test is eq. (31)
                              itself, |X - U V^T|_F <= aca_tol |X|_F, so no block can miss it;
                              needs m n doubles of scratch per block being compressed and
                              O(m n k) work.  HM_EINVAL outside 0..1. */
  int32_t lowrank_rounding; /* rounding of FP32 factor entries to HM_BF16 storage: 0 nearest even
                              (default); 1 dithered: up or down to the two BF16 neighbours with
                              the probabilities that make the error's mean zero, drawn by a
                              counter-based generator (SplitMix64 output function) keyed by the
                              entry's factor side, permuted row or column, block and rank index,
                              so the result is deterministic and the same alone or batched.
                              Errors of near-equal entries then do not add up coherently, which
                              lets iterative refinement converge in fewer outer steps.  1 needs
                              HM_BF16 factors and closed_row_scale 0.  HM_EINVAL otherwise. */
} hm_assembly_params;

/* Evaluate the near field (every inadmissible leaf block, FP64 evaluation
 * of eq. (10) rounded to dense_dtype) and compress every admissible block by
 * partial-pivoting ACA in FP64 (eq. (30); stop when |u_k||v_k| <= aca_tol *
 * |sum u_l v_l^T|_F).  An admissible block whose ACA reaches the cap
 * min(k_max, ceil(mn/(m+n))) without meeting the stop test, or whose rank k
 * gives k(m+n) >= mn, is stored dense.  The matrix keeps what it needs; the
 * tree may be destroyed afterwards.  Runs on ctx's stream and synchronises it. */
hm_status hm_assemble_hmatrix(hm_ctx* ctx, const hm_tree* tree, const hm_assembly_params* params,
                              hm_matrix** out);

/* Assembles count cavities as hm_assemble_hmatrix would one by one
 * (trees[i] with params[i], matrix written to out[i]), with the admissible
 * blocks of all cavities compressed in shared ACA launches, largest blocks
 * first: the batching of Sec. 4.3's block-wise compression across cavities.
 * Every matrix equals the one hm_assemble_hmatrix builds from the same tree
 * and parameters (same ranks and factors), except that the cavities whose
 * autotune flag is set share one work split of the product's first kernel,
 * timed on their batched product (as hm_solve_radiosity_batched and
 * hm_hmatvec_profile apply them together).  count >= 1; trees, params and out hold
 * count entries.  On error no matrix is returned.  Runs on ctx's stream and
 * synchronises it. */
hm_status hm_assemble_hmatrix_batched(hm_ctx* ctx, int32_t count, const hm_tree* const* trees,
                                      const hm_assembly_params* params, hm_matrix** out);

/* bytes_device: device bytes held by the matrix; entries_dense: sum of m*n
 * over dense blocks; entries_lowrank: sum of k*(m+n) over low-rank blocks;
 * max_rank; any pointer may be NULL. */
hm_status hm_matrix_stats(const hm_matrix* M, int64_t* bytes_device, int64_t* entries_dense,
                          int64_t* entries_lowrank, int32_t* max_rank);
/* Extended statistics: n, number of dense / low-rank blocks, admissible
 * blocks stored dense (fallbacks), sum of ranks.  Any pointer may be NULL. */
hm_status hm_matrix_info(const hm_matrix* M, int64_t* n, int64_t* n_dense_blocks,
                         int64_t* n_lowrank_blocks, int64_t* n_fallback, int64_t* rank_sum);
/* Work split of the product's first kernel chosen at assembly (fixed or
 * autotuned): rows per item and minimum bytes per wave task; timing_us (may
 * be NULL) receives the measured microseconds of the chosen split, or 0 when
 * nothing was timed.  Any pointer may be NULL. */
hm_status hm_matrix_tuning(const hm_matrix* M, int32_t* p1_rows, int32_t* p1_task_bytes, double* timing_us);
/* Sets the work split of the product's first kernel (the two values
 * hm_matrix_tuning reports), e.g. a split found by timing a batch of
 * matrices that are multiplied together.  p1_rows: rows per item, a positive
 * multiple of 64; p1_task_bytes: minimum bytes per wave task, counted at 4
 * bytes per stored entry, >= 0.  The product's result changes only by the
 * order of partial sums.  Synchronises ctx's stream; must not overlap a
 * product with M on another stream.  HM_EINVAL on bad values. */
hm_status hm_matrix_set_tuning(hm_ctx* ctx, hm_matrix* M, int32_t p1_rows, int32_t p1_task_bytes);
/* Launch shape of the product's second kernel for products of one or two
 * columns, chosen at assembly: waves per workgroup, 2, 4 or 8, timed by the
 * autotuner after the first kernel's split, or 0 when it is chosen by the
 * tile count (4 from 4,096 row tiles on, else 8); timing_us receives the measured
 * microseconds of that kernel with the chosen shape, or 0 when nothing was
 * timed.  Any pointer may be NULL; HM_EINVAL for a NULL matrix. */
hm_status hm_matrix_tuning_phase2(const hm_matrix* M, int32_t* p2_waves, double* timing_us);
/* Sets that shape (0, 2, 4 or 8).  The result does not change: the waves of a
 * workgroup add their sums in a fixed order whatever their number.  A batch
 * of matrices uses a shape only when all its members hold the same one.
 * Synchronises ctx's stream; must not overlap a product with M on another
 * stream.  HM_EINVAL on bad values. */
hm_status hm_matrix_set_tuning_phase2(hm_ctx* ctx, hm_matrix* M, int32_t p2_waves);
void hm_matrix_destroy(hm_matrix* M);

/* Y = alpha * F_H * X + beta * Y (Sec. 5.2: the block-wise product adds no
 * approximation beyond the stored blocks).  X, Y: DEVICE, n x nrhs
 * column-major, leading dims ldx, ldy, of type vec_dtype (HM_F64 or HM_F32).
 * 1 <= nrhs <= 16 (widths 3, 5-7 and 9-15 run in the kernels of the next
 * width of 2, 4, 8 or 16, whose extra columns are neither read from X nor
 * written to Y; 9-16 columns of FP32/BF16 entries run on the matrix cores).  use_f32_copy = 1 reads the FP32 copies of BF16 factors (and of a
 * BF16 near field).  Accumulation is in vec_dtype.  X and Y must not
 * overlap. */
hm_status hm_hmatvec(hm_ctx* ctx, const hm_matrix* M, int32_t nrhs, hm_dtype vec_dtype, const void* X,
                     int64_t ldx, void* Y, int64_t ldy, double alpha, double beta);
hm_status hm_hmatvec_ex(hm_ctx* ctx, const hm_matrix* M, int32_t nrhs, hm_dtype vec_dtype,
                        int32_t use_f32_copy, const void* X, int64_t ldx, void* Y, int64_t ldy,
                        double alpha, double beta);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as hm_hmatvec (same kernels, same result bit for bit, factors as
 * stored), with every workspace in a fixed device array of
 * HM_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends.  It calls no hipMalloc or hipFree, no
 * allocating library routine, and does not synchronise.  The caller still
 * passes X and Y (DEVICE, as for hm_hmatvec).  The array is shared by every
 * call on a device and keeps the last call's contents (nothing in it needs
 * to start at zero): calls that overlap on one device race, so a caller
 * using several streams must order these calls itself.
 * Workspace needed (bytes, each part rounded up to 256): two slot
 * descriptors; 4 per product work item (tasks, reductions and tiles of the
 * matrix's plan, + 1); 2 * n * w * 8 for the permuted vectors (w = nrhs
 * rounded up to 1, 2, 4, 8 or 16); 8 * w * (sum of ranks) for the rank
 * intermediates; 8 * w * 64 per row-split partial of the first kernel; and
 * n * 16 * 8 more when w = 16.  HM_ENOMEM (the product is not run) when this
 * exceeds HM_NOALLOC_SCRATCH_BYTES; hm_hmatvec has no such limit.  Other
 * errors as hm_hmatvec. */
#define HM_NOALLOC_SCRATCH_BYTES (64u << 20)
hm_status hm_hmatvec_noalloc(hm_ctx* ctx, const hm_matrix* M, int32_t nrhs, hm_dtype vec_dtype, const void* X,
                             int64_t ldx, void* Y, int64_t ldy, double alpha, double beta);

/* Timing of the product's two kernels for `count` matrices applied as one
 * block-diagonal operator (one launch per phase, as in the batched solve),
 * measured with HIP events recorded on ctx's stream around each kernel of
 * `reps` products y = F_H x on internal permuted vectors (x = 1).  Before
 * each product `flush_bytes` (>= 0) of device memory are streamed through the
 * caches (read only) so that the 256 MB last-level cache holds none of the
 * matrix.  M: HOST array of count matrices on ctx's device.  Outputs (HOST,
 * any may be NULL): average ms of phase 1 (t = V^T x, with the reduction of
 * row-split partial sums), of phase 2 (y = D x + U t) and of the whole
 * product, and the algorithmic bytes of each phase per product summed over
 * the matrices: phase 1 reads every V factor once plus x and writes t;
 * phase 2 reads every dense block and U factor once plus x and t and writes y. */
hm_status hm_hmatvec_profile(hm_ctx* ctx, int32_t count, const hm_matrix* const* M, int32_t nrhs,
                             hm_dtype vec_dtype, int32_t use_f32_copy, int32_t reps, int64_t flush_bytes,
                             double* ms_phase1, double* ms_phase2, double* ms_total, int64_t* bytes_phase1,
                             int64_t* bytes_phase2);

/* ----------------------------------------------------------- radiosity solve */

typedef struct {
  double rtol;             /* stop when |b - C J|_2 <= rtol |b|_2 per right-hand side */
  int32_t restart;         /* GMRES restart length m (1..64) */
  int32_t max_iter;        /* total Arnoldi steps per solve */
  int32_t mixed_precision; /* 1: iterative refinement: FP64 residual with FP32 (or FP64)
                              factors, inner GMRES with the stored (e.g. BF16) factors */
  double ir_inner_rtol;    /* inner relative tolerance of each refinement step */
  int32_t want_q;          /* compute the facet flux of eq. (12) */
  int32_t vec_dtype;       /* Krylov vectors when not refining: HM_F64 or HM_F32 */
  int32_t use_graphs;      /* 1: the Arnoldi steps run as HIP graphs captured once per workspace
                              (fewer launches; same kernels and results); 0: direct launches */
  int32_t open_cavity;     /* 1: open cavity (eq. (35)): the flux gains the exchange with an
                              ambient at ambient_temperature, -sigma (1 - c_i)(T_i^4 - T_amb^4) into
                              facet i, c_i = clamp(sum_j F_ij, 0, 1) (eqs. (32)-(33), the row sum of
                              the stored H-matrix); the transient's Newton update takes its
                              derivative 4 sigma (1 - c_i) T_i^3.  The server takes closed cavities
                              only: hm_server_create returns HM_EINVAL for 1.  0: closed
                              cavity (default) */
  double ambient_temperature; /* T_amb in K (> 0) when open_cavity = 1; ignored otherwise */
} hm_solve_params;

typedef struct {
  int32_t iters;           /* Arnoldi steps (max over right-hand sides) */
  int32_t outer_iters;     /* refinement steps (0 without refinement) */
  int32_t matvecs;         /* H-matrix products issued (all precisions) */
  double rel_residual;     /* max over right-hand sides of |b - C J| / |b| (FP64) */
  double seconds;          /* wall time of the call */
  int64_t bytes_moved;     /* algorithmic bytes of all products */
} hm_solve_info;

/* Solve (I - diag(1 - eps) F) J = sigma eps T^4 (eq. (11) with the per-area F;
 * the radiosity balance J_i = eps_i sigma T_i^4 + (1 - eps_i) sum_j F_ij J_j)
 * for nrhs temperature fields by restarted GMRES (classical Gram-Schmidt
 * with re-orthogonalisation, x0 = b), and optionally the facet flux of
 * eq. (12), evaluated as q = eps (F J - sigma T^4 g) with g = F C^-1 eps
 * (g is computed once per matrix and emissivity field and cached).
 * eps: DEVICE FP64 n, 0 < eps <= 1.  T: DEVICE FP64 n x nrhs (> 0).
 * J, q: DEVICE FP64 n x nrhs (q may be NULL).  1 <= nrhs <= 16.
 * Returns HM_ENOTCONV with the best iterate in J (and q) when rtol is not
 * met within max_iter; info (may be NULL) is filled either way. */
hm_status hm_solve_radiosity(hm_ctx* ctx, const hm_matrix* M, const double* eps, int32_t nrhs,
                             const double* T, int64_t ldT, double sigma, const hm_solve_params* p,
                             double* J, int64_t ldJ, double* q, int64_t ldq, hm_solve_info* info);

/* Batched form: `count` independent cavities solved together; every
 * H-matrix product and every Krylov kernel covers all of them in one launch
 * (block-diagonal operator).  Arrays of length count; eps[i], T[i], J[i],
 * q[i] are DEVICE pointers for cavity i (n_i rows, one right-hand side;
 * q may be NULL or hold NULL entries).  info_out (HOST, count, may be NULL). */
hm_status hm_solve_radiosity_batched(hm_ctx* ctx, int32_t count, const hm_matrix* const* M,
                                     const double* const* eps, const double* const* T, double sigma,
                                     const hm_solve_params* p, double* const* J, double* const* q,
                                     hm_solve_info* info_out);

/* ------------------------------------------------------------ transient */

typedef struct {
  double mc;          /* heat capacity per area rho*c*thickness, J/(m^2 K) */
  double dt;          /* time step, s */
  int32_t steps;      /* backward-Euler steps */
  double newton_rtol; /* stop when |R|_2 <= newton_rtol |mc T^n / dt|_2 per scenario */
  int32_t max_newton; /* Newton updates per step */
} hm_transient_params;

typedef struct {
  int32_t steps_done;
  int32_t newton_total;   /* Newton iterations summed over steps */
  int32_t newton_max;     /* most Newton iterations in one step */
  int32_t matvecs;
  double seconds;
  double max_rel_residual;/* largest final |R| / |mc T^n/dt| over steps and scenarios */
} hm_transient_info;

/* Lumped implicit-Euler radiative exchange on one cavity (analogue of the
 * time discretisation of Sec. 3.3): mc (T - T^n)/dt = q(T) + s per facet,
 * with q of eq. (12).  Each step runs Newton's method with the local
 * Jacobian D = mc/dt + 4 sigma eps g T^3, T <- T - R/D; each Newton
 * iteration solves the radiosity system for all nrhs scenarios at once.
 * T: DEVICE FP64 n x nrhs, in: T^0, out: T^steps.  src: DEVICE FP64
 * n x nrhs (W/m^2).  eps: DEVICE FP64 n.  history (DEVICE FP64,
 * (steps+1) x ld x nrhs blocks, may be NULL) receives T^0..T^steps. */
hm_status hm_transient_run(hm_ctx* ctx, const hm_matrix* M, const double* eps, int32_t nrhs, double* T,
                           int64_t ldT, const double* src, int64_t ldS, double sigma,
                           const hm_transient_params* tp, const hm_solve_params* sp, double* history,
                           hm_transient_info* info);

/* --------------------------------------------------- hierarchical block LU */

/* Sec. 5.1: the reflection matrix C = I - diag(1 - eps) F (eq. (11)) in the
 * block structure of the tree (Algorithm 2), its admissible blocks
 * compressed by ACA (params->aca_pivot) and truncated at params->aca_tol,
 * factorised C ~ L U by the paper's four recursive steps (dense LU without
 * row exchanges in the leaf blocks; forward substitution for the blocks
 * right of the diagonal, backward substitution for those below it, the
 * Schur complement update) with every addition into a low-rank block
 * truncated at the relative accuracy aca_tol from its singular values.  All
 * in FP64: params->lowrank_dtype and dense_dtype must be HM_F64
 * (HM_EINVAL otherwise); keep_f32_copy, closed_row_scale, autotune and
 * recompress are not used.  eps: DEVICE FP64 n, caller order, in (0, 1].
 * Runs on ctx's stream and synchronises it; the tree may be destroyed
 * afterwards. */
typedef struct hm_hlu hm_hlu;
hm_status hm_hlu_factor(hm_ctx* ctx, const hm_tree* tree, const double* eps, const hm_assembly_params* params,
                        hm_hlu** out);
/* Sec. 5.2: X = U^-1 (L^-1 B) ~ C^-1 B for nrhs right-hand sides (DEVICE
 * FP64 n x nrhs, caller order, leading dimensions ldb, ldx >= n; X may be
 * B).  No further approximation beyond the factors.  The first solve with
 * a given nrhs records the substitutions as a graph kept with the factors
 * (with its own device work buffers; the four most recently used counts
 * are kept); solves on the same factors from several threads are
 * serialised.  Synchronises ctx's stream. */
hm_status hm_hlu_solve(hm_ctx* ctx, const hm_hlu* lu, int32_t nrhs, const double* B, int64_t ldb, double* X,
                       int64_t ldx);
/* Device bytes and stored entries of the factors, their largest rank and the
 * factorisation's wall time in seconds (any pointer may be NULL). */
hm_status hm_hlu_stats(const hm_hlu* lu, int64_t* bytes_device, int64_t* entries, int32_t* max_rank,
                       double* factor_seconds);
void hm_hlu_destroy(hm_hlu* lu);

/* ------------------------------------------------------------- finite-element coupling */

/* Sec. 3.1-3.4: nodal temperatures of a conducting shell whose P1 triangles
 * are the cavity's facets, coupled to the radiation through
 *   eta_M = T_M^4, eta_i = sum_M P_iM eta_M (P_iM = 1/3 for the vertices of
 *   facet i: the facet average of the linear basis function),
 *   R = sigma diag(eps A) F C^-1 diag(eps)  (eq. (Rdef) with this library's
 *   normalised F), R_bar = R - diag(R 1)  (eq. (Rbardef)),
 *   S = P^T R_bar P  (eq. (S_def_matrix)),  Q = S eta;
 * implicit Euler on the Galerkin equations (eq. (SVF_Galerkin_time)):
 *   Res(T) = M (T - T^n)/dt + K T - Q(T) - f,
 * M the consistent mass (rho c_p h A/12 [[2,1,1],[1,2,1],[1,1,2]] per
 * element), K the stiffness (k h (e_a . e_b)/(4A) per element, e_a the edge
 * opposite vertex a), f_N = sum over the facets around N of f_i A_i / 3.
 * Each Newton correction solves (M/dt + K - 4 S diag(T^3)) d = -Res by
 * GMRES on the system preconditioned from the left with (M/dt + K)^-1
 * (eq. (Jprec)), that inverse applied by conjugate gradients; every action
 * of S costs one cavity solve (C^-1 by the H-matrix's Krylov solve). */
typedef struct hm_fe hm_fe;
typedef struct {
  double conductance;      /* k h: conductivity times shell thickness (W/K), >= 0 */
  double capacity;         /* rho c_p h: heat capacity per unit area (J/(m^2 K)), > 0 */
  double dt;               /* implicit Euler step (s), > 0 */
  double newton_rtol;      /* stop when |Res|_2 <= newton_rtol |M T^n / dt|_2 */
  int32_t max_newton;      /* Newton corrections per step (>= 1) */
  int32_t krylov_restart;  /* GMRES restart length (1..64) */
  double krylov_rtol;      /* relative tolerance of each correction's preconditioned solve */
  int32_t max_krylov;      /* Krylov iterations per correction (>= 1) */
  double pc_rtol;          /* conjugate gradients for (M/dt + K)^-1 to this relative residual */
  hm_solve_params solve;   /* the cavity solves (want_q and open_cavity ignored: closed cavity); those
                              inside Jacobian products stop at max(solve.rtol, krylov_rtol / 100) */
  double sigma;            /* Stefan-Boltzmann constant */
} hm_fe_params;

typedef struct {
  int32_t newton;          /* Newton corrections taken */
  int32_t krylov;          /* GMRES iterations over all corrections */
  int32_t cavity_solves;   /* actions of S (each one solve with C) */
  int32_t pc_iterations;   /* conjugate-gradient iterations over all preconditioner applications */
  double residual;         /* final |Res|_2 / |M T^n / dt|_2 */
  int32_t status;          /* HM_OK, or HM_ENOTCONV when max_newton was reached first */
} hm_fe_info;

/* F: the assembled H-matrix of the same facets (triangles in the same
 * order; not copied: it must outlive the object).  vertices: HOST n_nodes x
 * 3 (row-major); triangles: HOST n_facets x 3 vertex indices, oriented as
 * for hm_facets_from_triangles; eps: DEVICE n_facets.  The mesh and
 * eps are copied; the mass, stiffness and projection are built here.
 * HM_EINVAL for sizes that do not match F, bad indices, degenerate
 * triangles or parameters out of range. */
hm_status hm_fe_create(hm_ctx* ctx, const hm_matrix* F, int64_t n_nodes, const double* vertices,
                       int64_t n_facets, const int32_t* triangles, const double* eps, const hm_fe_params* p,
                       hm_fe** out);
/* Q = S T^4 for nodal temperatures T (DEVICE n_nodes in, DEVICE n_nodes
 * out): the radiation load of eq. (flux_residual_3).  One cavity solve on
 * ctx's stream (ctx on the object's device), which it synchronises. */
hm_status hm_fe_cavity_load(hm_ctx* ctx, hm_fe* fe, const double* T, double* Q);
/* One implicit Euler step: T_out (DEVICE n_nodes) from T_n (DEVICE
 * n_nodes) with facet sources f_facet (DEVICE n_facets, W/m^2, or NULL for
 * none); T_out may be T_n.  info may be NULL.  Returns HM_ENOTCONV (with the
 * last iterate in T_out) when Newton did not reach newton_rtol.  Runs on
 * ctx's stream and synchronises it.  Calls on one object must not overlap. */
hm_status hm_fe_step(hm_ctx* ctx, hm_fe* fe, const double* T_n, const double* f_facet, double* T_out,
                     hm_fe_info* info);
void hm_fe_destroy(hm_fe* fe);

/* ------------------------------------------------------------- serving */

typedef struct {
  int64_t hbm_budget_bytes;  /* device bytes allowed for resident H-matrices + solve buffers */
  int32_t max_active;        /* most requests advanced together */
  int32_t max_rhs_per_slot;  /* right-hand sides of one cavity batched in one slot (<= 16) */
  hm_solve_params solve;
  double sigma;
} hm_server_params;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t assemblies, evictions, cache_hits;
  int64_t rounds;            /* batched solve rounds run */
  double busy_seconds;
  int64_t resident_bytes;
} hm_server_stats;

/* A serving loop owned by two background host threads: requests (radiosity
 * solves of registered cavities) are admitted while the resident H-matrices
 * and the solve buffers fit hbm_budget_bytes, advanced together in shared
 * products, and retired as they converge; new requests join at the next
 * round.  H-matrices stay resident across requests (least-recently-used
 * eviction of cavities with no running or waiting request).  A cavity that
 * is not resident is assembled by the second thread on its own stream while
 * the admitted requests keep running; the requests that need it wait for it
 * (its budget share reserved) and then go first.  cache_hits counts
 * requests whose cavity was resident when they were admitted.  Thread-safe. */
hm_status hm_server_create(hm_ctx* ctx, const hm_server_params* p, hm_server** out);
/* Register a cavity: the tree is copied; eps_host (HOST, n) is copied;
 * assembly happens lazily on first use. */
hm_status hm_server_register_cavity(hm_server* s, uint64_t cavity_id, const hm_tree* tree,
                                    const double* eps_host, const hm_assembly_params* ap);
/* Queue a request of nrhs temperature fields (HOST n x nrhs column-major,
 * copied).  HM_ENOTFOUND for an unknown cavity, HM_EINVAL for bad sizes. */
hm_status hm_submit(hm_server* s, uint64_t cavity_id, int32_t nrhs, const double* T_host, uint64_t* ticket);
/* done = 1 when the request finished: J_host / q_host (HOST n x nrhs, may
 * be NULL) and info receive the result and the ticket is released.  Returns
 * HM_EBUSY with done = 0 while running, HM_ENOTFOUND for unknown tickets,
 * or the request's own status when it failed. */
hm_status hm_poll(hm_server* s, uint64_t ticket, int32_t* done, double* J_host, double* q_host,
                  hm_solve_info* info, double* latency_seconds);
hm_status hm_server_stats_get(hm_server* s, hm_server_stats* out);
/* Stop the loop after in-flight work finished; pending tickets stay pollable
 * until destroy. */
void hm_server_destroy(hm_server* s);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
