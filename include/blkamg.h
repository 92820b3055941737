/*
 * blkamg.h - C ABI of the natively blocked smoothed-aggregation AMG solve phase
 * for AMD Instinct MI355X (gfx950).
 *
 * The library implements the recurring ("hot") work of a blocked SA-AMG solve for
 * vector PDEs (paper §3.1): the numeric Galerkin recompute A_c = P^T A P on fixed
 * block patterns, the V-cycle inside preconditioned CG, rectangular-block SpMV and
 * SpMV-transpose, and blocked COO value assembly.  Blocks are dense bs_r x bs_c and
 * may be rectangular (3x3 fine operator, 3x6 prolongator, 6x6 coarse operators;
 * paper §2.3).  A one-time host setup (aggregation, tentative prolongator) is
 * included so that the hierarchy can be built without any other software.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: 0 (BLKAMG_OK) on success, BLKAMG_ENOCONV (1) when an iteration
 *   limit is reached (results are still written), a negative code on failure.
 *   blkamg_last_error() returns a thread-local message describing the last failure.
 *   No C++ exception crosses the ABI.
 * - Pointers named d_* are device pointers (HIP device memory of the current
 *   device); h_* are host pointers.  Indices are int32.  Block values are stored
 *   block after block, each block row-major (bs_r rows of bs_c values).
 * - Vectors are row-major [n][nrhs]: the nrhs right-hand sides of one scalar dof
 *   are contiguous.  A block vector of a matrix with nb block rows of size bs has
 *   n = nb * bs entries per right-hand side.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Calls marked "async" only enqueue work on that stream; calls marked "sync"
 *   wait for the stream before returning.  Asynchronous kernel faults surface at
 *   the next synchronising call.
 * - Borrowed device arrays must stay valid, and their pattern (rowptr/colidx)
 *   unchanged, for the lifetime of every handle that refers to them.
 * - The library allocates its own device memory (plans, caches, library-owned
 *   matrices, hierarchy work vectors) with hipMalloc at create/setup time; the
 *   hot calls (spmv, ptap_numeric, coo_assemble_blocked, vcycle_apply, pcg_solve
 *   after its first call on a hierarchy) allocate nothing.
 */
#ifndef BLKAMG_H
#define BLKAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define BLKAMG_OK 0
#define BLKAMG_ENOCONV 1     /* maximum iterations reached, not converged */
#define BLKAMG_EINVAL (-1)   /* invalid argument, shape or state */
#define BLKAMG_ENOMEM (-2)   /* device or host allocation failed */
#define BLKAMG_EHIP (-3)     /* a HIP runtime call failed */
#define BLKAMG_ESTATE (-4)   /* handle used out of order / pattern changed */
#define BLKAMG_EBREAKDOWN (-5) /* CG breakdown: p^T A p <= 0 (matrix or M not SPD) */
#define BLKAMG_ENOTSPD (-6)  /* coarsest Cholesky found a non-positive pivot */

/* ---- value types --------------------------------------------------------- */
#define BLKAMG_F64 0
#define BLKAMG_F32 1
#define BLKAMG_BF16 2        /* bfloat16 (round to nearest even); matrix values only */

/* COO assembly modes */
#define BLKAMG_INSERT 0
#define BLKAMG_ADD 1

/* source of lambda_hat in the smoother refresh (blkamg_opts.eig_mode) */
#define BLKAMG_EIG_LANCZOS 0 /* k-step Lanczos per level (paper's method) */
#define BLKAMG_EIG_MLP 1     /* learned eigenbound with growth test and Lanczos fallback */

/* guard of the learned eigenbound in the hot refresh (blkamg_opts.mlp_guard) */
#define BLKAMG_GUARD_SMOOTHER 0 /* smoother growth test on every level at every refresh */
#define BLKAMG_GUARD_PCG 1      /* no test at refresh: pcg_solve checks its own residual */

/* eigenbound network 12 -> 64 -> 64 -> 2: parameter count and deployable model size */
#define BLKAMG_MLP_PARAMS 5122
#define BLKAMG_MLP_MODEL 5150

typedef struct bsr_s* bsr_t;
typedef struct coo_plan_s* coo_plan_t;
typedef struct amg_s* amg_t;
typedef struct sa_result_s* sa_result_t;
typedef struct fe_plan_s* fe_plan_t;

/* Thread-local text of the last error ("" if none).  Never NULL. */
const char* blkamg_last_error(void);
/* Library version as an integer (major*10000 + minor*100 + patch). */
int blkamg_version(void);

/* Device memory.  Every device buffer the library allocates (owned patterns and
 * values, plans, hierarchy data, work vectors) comes from alloc_fn(bytes, ctx),
 * which must return memory of the current device aligned to 256 bytes, or NULL
 * (the calling entry point then fails with ENOMEM; a misaligned pointer is handed
 * back to free_fn and the call fails with EINVAL).  free_fn(ptr, bytes, ctx) gets
 * each buffer back with the size it was allocated with, after the library has
 * synchronised the device (as hipFree would), so stream-ordered pools such as
 * PyTorch's caching allocator may reuse it at once.  Both NULL: hipMalloc/hipFree
 * (the default).  Exactly one NULL: EINVAL.  A buffer is returned to the routine
 * that allocated it, so the allocator may be changed while handles are alive;
 * ctx must stay valid until every buffer allocated with it has been freed.
 * Pinned host staging (hipHostMalloc) is not routed.  Not to be called while
 * another thread is inside the library. */
typedef void* (*blkamg_alloc_fn)(size_t bytes, void* ctx);
typedef void (*blkamg_free_fn)(void* ptr, size_t bytes, void* ctx);
int blkamg_set_allocator(blkamg_alloc_fn alloc_fn, blkamg_free_fn free_fn, void* ctx);

/* ==========================================================================
 * Rectangular-block sparse matrix (paper §2.3, §2.4: independent row and column
 * block sizes; one int32 column index per block).
 * ========================================================================== */

/* Wrap caller-owned device arrays as a block matrix (the blocked storage of paper
 * §2.3, §4.2).
 *   nbr, nbc     : block rows / block columns (>= 0)
 *   bs_r, bs_c   : block shape, each in 1..8
 *   nnzb         : stored blocks; d_rowptr[nbr] must equal nnzb
 *   d_rowptr     : int32[nbr+1], d_colidx: int32[nnzb] (ascending within a row)
 *   d_val        : nnzb * bs_r * bs_c values of type `dtype`
 *   stream       : orders the optional validation after the caller's work that
 *                  writes the arrays (NULL = the null stream)
 * Borrowed: the handle stores the pointers only.  Validation of the pattern
 * (monotone rowptr, column range, sorted rows) is done when the environment
 * variable BLKAMG_VALIDATE=1 is set (copies the pattern to the host after the
 * stream's work, sync).  Errors: EINVAL for bad sizes/pointers.  Host-only; no
 * device work otherwise. */
int bsr_create(int32_t nbr, int32_t nbc, int32_t bs_r, int32_t bs_c, int64_t nnzb,
               const int32_t* d_rowptr, const int32_t* d_colidx, void* d_val,
               int dtype, void* stream, bsr_t* out);
/* Free the handle and everything it owns (caches; for library-created matrices
 * also the arrays).  NULL is accepted. */
int bsr_destroy(bsr_t A);
/* Declare that the values changed: bumps the value-state stamp that gates the
 * cached transpose and the prolongator-side data of the Galerkin product
 * (the object-state gating of paper §3.5). */
int bsr_mark_modified(bsr_t A);
/* Shape, size, value type and current value-state stamp. */
int bsr_info(bsr_t A, int32_t* nbr, int32_t* nbc, int32_t* bs_r, int32_t* bs_c,
             int64_t* nnzb, int* dtype, uint64_t* stamp);
/* Device arrays of the matrix (borrowed or library-owned). */
int bsr_arrays(bsr_t A, const int32_t** d_rowptr, const int32_t** d_colidx, void** d_val);

/* y = alpha * A x + beta * y   (the blocked MatMult of paper §4.2).
 *   x: [nbc*bs_c][nrhs], y: [nbr*bs_r][nrhs], both of `vec_dtype`
 *   (F64 with F64 matrices; F32 with F32 or BF16 matrices), nrhs in 1..8.
 * beta == 0 overwrites y (NaNs in y are not propagated).  Async. */
int bsr_spmv(bsr_t A, double alpha, const void* d_x, double beta, void* d_y,
             int vec_dtype, int32_t nrhs, void* stream);
/* y = alpha * S x + beta * y for a square-blocked matrix with a structurally
 * symmetric pattern, S the symmetric completion of A's upper triangle: S_ij = A_ij
 * for j >= i and A_ji^T for j < i (S = A when A is symmetric, as the SPD operators
 * of CG are; paper §2.1, §4.1).  Only the diagonal and upper blocks are streamed from
 * memory; a strictly lower block is read as the transpose of its mirror, which the
 * mirror's own row read shortly before, so the second read is mostly served from the
 * caches.  For symmetric A the result is that of bsr_spmv up to the grouping of the
 * row sums (its own lane shape).  Arguments as bsr_spmv (nrhs > 1 reads every block).  The mirror index (int32 per block) is built
 * on the first call (device, sync, allocates).  EINVAL if A is not square-blocked or
 * its pattern is not symmetric.  Async afterwards. */
int bsr_spmv_sym(bsr_t A, double alpha, const void* d_x, double beta, void* d_y,
                 int vec_dtype, int32_t nrhs, void* stream);
/* y = alpha * A^T x + beta * y through a cached explicit transpose R = A^T
 * (the cached restriction of paper §3.5).  x: [nbr*bs_r][nrhs],
 * y: [nbc*bs_c][nrhs].  The transpose pattern is built on the first call (sync,
 * allocates); its values are refreshed on the stream whenever the value stamp
 * changed since they were last copied.  Async afterwards. */
int bsr_spmv_t(bsr_t A, double alpha, const void* d_x, double beta, void* d_y,
               int vec_dtype, int32_t nrhs, void* stream);
/* Autotuner of the blocked SpMV (paper §4.2 kernel, shapes for gfx950): times every
 * compiled lane shape (G lanes per block row in {8,16,32,64} x U in {1,2} blocks per
 * lane per step) of y = A x with zero vectors of `vec_dtype` and `nrhs` (1 or 8)
 * columns on the stream with device events, and stores the fastest in the handle;
 * later SpMVs of A with that many columns (bsr_spmv, and the fused hierarchy
 * kernels) use it.  *code = G * 8 + U (may be NULL).  Sync; allocates two
 * temporary vectors. */
int bsr_autotune(bsr_t A, int vec_dtype, int32_t nrhs, void* stream, int32_t* code);

/* ==========================================================================
 * Galerkin coarse operator A_c = P^T A P (paper §2.1, §3.1, §3.5)
 * ========================================================================== */

/* Symbolic phase: builds the structural pattern of A_c (no numerical dropping)
 * and the numeric plan (pattern of A P, explicit transpose of P), records P's
 * value stamp, and creates C (library-owned, nbr = nbc = P.nbc, block
 * P.bs_c x P.bs_c, value type of A).  Requirements: A square-blocked
 * (bs_r == bs_c == P.bs_r), A.nbr == A.nbc == P.nbr; A F64 with P F64, or A F32
 * with P F32 or BF16.  Sync (host pattern work).  *C must be destroyed with
 * bsr_destroy. */
int ptap_symbolic(bsr_t A, bsr_t P, bsr_t* C, void* stream);
/* As ptap_symbolic, with flags:
 *   BLKAMG_PTAP_SYMMETRIC - the caller guarantees that A is symmetric (A_ij = A_ji^T),
 *     as for the SPD operators of an AMG hierarchy; then A_c is symmetric, and
 *     ptap_numeric computes only its blocks with column >= row and stores each
 *     off-diagonal one a second time, transposed.  Results on a non-symmetric A are
 *     undefined (the lower triangle mirrors the upper one).
 *   BLKAMG_PTAP_HOST_SYMBOLIC - build the plan on the host.  By default the patterns
 *     of A P and A_c and the contribution lists are built on the device (paper §6:
 *     the device-resident setup): each output row's contributions are sorted in LDS by
 *     one workgroup, or, beyond 4096 of them, in device memory by a segmented radix
 *     sort.  Both builds
 *     produce the same plan, so ptap_numeric gives the same bits either way.
 * Unknown flags are EINVAL. */
#define BLKAMG_PTAP_SYMMETRIC 1
#define BLKAMG_PTAP_HOST_SYMBOLIC 2
int ptap_symbolic_ex(bsr_t A, bsr_t P, int flags, bsr_t* C, void* stream);
/* Numeric phase: C.values = P^T A P on the fixed pattern.  If P's value stamp
 * differs from the one cached, the prolongator-side cache (transpose values) is
 * refreshed first on the stream; if P's or A's block count changed, returns
 * ESTATE.  C must come from ptap_symbolic(A, P).  No allocation, no host
 * synchronisation.  Async. */
int ptap_numeric(bsr_t A, bsr_t P, bsr_t C, void* stream);
/* Sizes of the numeric plan that ptap_symbolic attached to C (paper §3.5), for the
 * flop count of a recompute: *ap_nnzb blocks of A P, *ap_pairs (A block, P block)
 * products of the A P pass and *c_pairs (P^T block, A P block) products of the
 * R (A P) pass (the upper blocks' only when *symmetric).  The pair counts are -1 when
 * the plan holds no contribution lists.  Any output may be NULL.  EINVAL if C carries
 * no plan.  Sync (reads two counts from the device). */
int ptap_plan_info(bsr_t C, int64_t* ap_nnzb, int64_t* ap_pairs, int64_t* c_pairs, int32_t* symmetric);

/* ==========================================================================
 * Blocked COO assembly (paper §3.4 and §5)
 * ========================================================================== */

/* Preallocation: from n block coordinates (i[k], j[k]) (a negative i or j marks an
 * entry that is ignored) build the sorted unique block pattern and the
 * duplicate-summation plan, and create the matrix *A_out (library-owned, values
 * zero, type `val_dtype`).  Coordinates >= nbr / nbc are EINVAL.  The index map is
 * the stable order of the valid entries by (row, column, position), the same bits
 * whichever side builds it.
 *   where = BLKAMG_HOST  : i, j are host arrays; the plan is built on the host
 *                          (stream unused);
 *   where = BLKAMG_DEVICE: i, j are device arrays; the plan is built on the device
 *                          on `stream` (stable radix sort of 64-bit keys
 *                          row * nbc + col), and no host copy of the pattern is made.
 * Sync.  Free with coo_plan_destroy and bsr_destroy. */
#define BLKAMG_HOST 0
#define BLKAMG_DEVICE 1
int coo_plan_create(int32_t nbr, int32_t nbc, int32_t bs_r, int32_t bs_c, int64_t n,
                    const int32_t* i, const int32_t* j, int where, int val_dtype,
                    coo_plan_t* plan, bsr_t* A_out, void* stream);
int coo_plan_destroy(coo_plan_t plan);
/* The plan's index map: d_perm int32[n_valid] (positions of valid entries in
 * sorted order) and d_seg int32[nnzb+1] (block t sums perm[seg[t]..seg[t+1])).
 * Device pointers owned by the plan. */
int coo_plan_map(coo_plan_t plan, const int32_t** d_perm, const int32_t** d_seg,
                 int64_t* n_valid, int64_t* nnzb);
/* Numeric assembly: for each stored block t of A,
 *   INSERT: A_t  = sum_{k in run(t)} V_k        ADD: A_t += sum V_k
 * summed in stream order (deterministic, no atomics).  d_vals holds n blocks of
 * bs_r*bs_c values (same order as the coordinates) of type val_dtype == A's type.
 * A must be the matrix created with the plan (or have its exact pattern).  Async. */
int coo_assemble_blocked(coo_plan_t plan, const void* d_vals, int val_dtype, int mode,
                         bsr_t A, void* stream);

/* ==========================================================================
 * Finite-element assembly of trilinear hexahedral elasticity on the device
 * (paper §5: finite-element assembly is the blocked COO primitive's immediate use
 * beyond the Galerkin product; this pairs it with element-by-element assembly).
 * Element e has 8 nodes d_elem_nodes[8e .. 8e+7] (int32 rows of d_coords, local
 * order (0,0,0), (1,0,0), (0,1,0), (1,1,0), (0,0,1), (1,0,1), (0,1,1), (1,1,1) of
 * the reference cube, x fastest) and Lame parameters d_lam[e], d_mu[e]; d_coords is
 * double [n_nodes][3].  The element stiffness of  int lambda div u div v +
 * 2 mu eps(u):eps(v)  uses the isoparametric map and 2x2x2 Gauss-Legendre points;
 * block K_ab (3x3, row-major) couples local nodes a (rows) and b (columns).  Node
 * indices are not checked on the device: they must index d_coords.
 * ========================================================================== */
#define BLKAMG_AGG_GREEDY 0
#define BLKAMG_AGG_LUBY 1
#define BLKAMG_FE_ATOMIC 0   /* element-by-element, FP64 atomic adds */
#define BLKAMG_FE_COLORED 1  /* element-by-element in colour passes, fixed order */

/* Element blocks as a blocked COO value stream: d_out double [n_elem*64 + n_identity]
 * [3][3], element-major with block 64e + 8a + b = K_ab of element e, followed by
 * n_identity identity blocks (e.g. the Dirichlet diagonal of a clamped mesh).  Feed it
 * to coo_assemble_blocked with the matching coordinates.  d_out must be 16-byte aligned
 * when n_elem > 0 (EINVAL otherwise).  Async, no allocation. */
int fe_q1_stream(int64_t n_elem, const int32_t* d_elem_nodes, const double* d_coords,
                 const double* d_lam, const double* d_mu, int64_t n_identity,
                 double* d_out, void* stream);
/* Plan for element-by-element assembly into A (square, 3x3 F64 blocks, one block row
 * per node): the block of A that receives each (e, a, b) (none when either node is
 * flagged in h_dirichlet, which may be NULL), the diagonal blocks of the flagged
 * nodes, and a greedy colouring in which elements of one colour share no node (at
 * most 64 colours; 8 on structured hexahedral meshes).  h_elem_nodes is the host copy
 * of the element list later passed on the device.  EINVAL if the pattern of A lacks a
 * needed block or a node is out of range.  Sync; allocates (plan owned by the caller,
 * fe_ebe_plan_destroy). */
int fe_ebe_plan_create(bsr_t A, int64_t n_elem, const int32_t* h_elem_nodes,
                       const uint8_t* h_dirichlet, fe_plan_t* out);
/* Number of colours and the plan's device bytes (slots, Dirichlet slots, order). */
int fe_ebe_plan_info(fe_plan_t P, int32_t* n_colors, int64_t* slot_bytes);
int fe_ebe_plan_destroy(fe_plan_t P);
/* A's values := sum of the element blocks (identity on the flagged diagonal blocks,
 * couplings of flagged nodes dropped), computed and added element by element without
 * a value stream.  mode BLKAMG_FE_ATOMIC: one launch, FP64 atomic adds (the summation
 * order varies from run to run); BLKAMG_FE_COLORED: one launch per colour with plain
 * read-modify-writes (deterministic).  Bumps A's value stamp.  Async, no allocation. */
int fe_q1_assemble_ebe(fe_plan_t P, bsr_t A, const int32_t* d_elem_nodes,
                       const double* d_coords, const double* d_lam, const double* d_mu,
                       int mode, void* stream);

/* ==========================================================================
 * Smoothed-aggregation hierarchy and solve (paper §2.1, §2.2, §3.1, §4.1)
 * ========================================================================== */

typedef struct {
  int32_t max_levels;       /* maximum number of levels (>= 1), default 10 */
  int32_t coarse_eq_limit;  /* stop coarsening at <= this many dofs, default 1000 */
  double strength_eps;      /* strength threshold epsilon (paper §2.2), default 0 */
  int32_t cheb_degree;      /* Chebyshev polynomial degree (>= 1), default 2 */
  double cheb_lo, cheb_hi;  /* Chebyshev interval as fractions of lambda_hat, 0.1 / 1.1 */
  int32_t lanczos_steps;    /* Lanczos steps for lambda_hat (2..64), default 10 */
  uint64_t lanczos_seed;    /* start-vector seed, level l uses seed + l, default 0x5EED */
  double omega_scale;       /* prolongator-smoothing weight omega = omega_scale / lambda_hat, 4/3 */
  int32_t hier_dtype;       /* F64 or F32: type of the level operators, smoother and V-cycle */
  int32_t p_dtype;          /* type of the stored prolongators: F64 (with F64), F32 or BF16 (with F32) */
  int32_t pcg_graph_iters;  /* batched CG (several instances or nrhs = 8): iterations per
                               replay of a captured HIP graph; 0 = launch eagerly.
                               Default 4 (0..64) */
  int32_t autotune_nrhs;    /* 0: heuristic SpMV lane shapes; 1 or 8: at setup, time every
                               compiled shape of each hierarchy SpMV (and of A0) for that
                               many right-hand sides and keep the fastest.  Default 0 */
  int32_t eig_mode;         /* BLKAMG_EIG_LANCZOS (default) or BLKAMG_EIG_MLP: refreshes
                               take lambda_hat from the model (eig_model below, or the
                               one set by amg_set_eig_model); with eig_model set, the cold
                               setup also takes each level's lambda_hat and its
                               prolongator-smoothing weight omega from the network
                               (P = (I - omega D^-1 A) P~, paper §2.2) */
  int32_t agg_mode;         /* BLKAMG_AGG_GREEDY (default): host aggregation in natural
                               order; BLKAMG_AGG_LUBY: sa_aggregate_device with agg_seed
                               on every level (one instance, strength_eps = 0) */
  uint64_t agg_seed;        /* priority seed of BLKAMG_AGG_LUBY, default 0x4D495332 */
  int32_t growth_steps;     /* guard of the learned eigenbound: power steps of the
                               smoother's error propagation from a fixed vector; a level
                               whose last step grows the A-norm (or whose prediction is
                               not positive and finite) falls back to Lanczos.  1..16,
                               default 3 */
  const float* eig_model;   /* host copy of a model (BLKAMG_MLP_MODEL floats) used from
                               the cold setup on when eig_mode is BLKAMG_EIG_MLP (copied;
                               NULL = none until amg_set_eig_model).  Default NULL */
  int32_t mlp_guard;        /* BLKAMG_GUARD_SMOOTHER (default): every MLP refresh runs the
                               smoother growth test (growth_steps) and falls back per level.
                               BLKAMG_GUARD_PCG: an MLP refresh of a one-instance hierarchy
                               runs no test; the next pcg_solve with one right-hand side
                               checks its residual recurrence instead (the preconditioned
                               r.z must stay positive and ||r|| must not grow above 1e3
                               times its smallest value so far); when the check fails,
                               every smoothed level is refreshed by Lanczos (all flagged as
                               fallback) and the solve restarts from x = 0.  vcycle_apply
                               and the other solves first run the deferred smoother test.
                               With one instance the cold setup then also takes the
                               network's lambda_hat and omega without the smoother test
                               (omega only shapes the coarse space; the first solve checks
                               the smoother); with several it runs the test. */
  int32_t sym_spmv;         /* 1 (default): the hierarchy's SpMVs on FP64 level operators
                               (smoother, residual, Lanczos, growth test) and pcg_solve's
                               A p read only the diagonal and upper blocks of a
                               structurally symmetric operator from memory and use each
                               strictly lower block as the transpose of its mirror, i.e.
                               they apply the symmetric completion of the upper triangle
                               (A itself when A is symmetric, as CG requires; the results
                               then differ from full reads only in the grouping of the row
                               sums).  0: read every block */
  int32_t ap_residual;      /* 1 (default): with one right-hand side, the post-smoothing's
                               first residual on a level whose Galerkin product A P costs
                               fewer bytes to read than A (the FP32 fine level) is updated
                               from the restricted residual, r - (A P) e_c, with the A P
                               that the last recompute formed (paper §2.1: the same residual
                               as f - A (x + P e_c) up to rounding).  Used only while A and
                               P still hold the values that A P was formed from; otherwise,
                               and with 0, the residual is f - A x */
} blkamg_opts;

/* Fill *o with the defaults listed above. */
void blkamg_opts_default(blkamg_opts* o);

/* Host-only greedy aggregation (paper §2.2 "greedy disjoint covering", paper §3.2
 * graph over blocks), the structural case epsilon = 0: vertices are the block rows
 * with h_dirichlet[i] == 0; neighbours are the other stored columns of the row
 * that are not Dirichlet.  Phase 1 visits rows in natural order and makes a row
 * whose neighbours are all unaggregated the root of {row} + neighbours; phase 2
 * puts each leftover row into the phase-1 aggregate holding most of its
 * neighbours (ties: smallest id).  h_agg[i] = aggregate id or -1 (Dirichlet).
 * h_rowptr/h_colidx: host pattern.  h_dirichlet may be NULL.  Pure host code. */
int sa_aggregate(int32_t nbr, const int32_t* h_rowptr, const int32_t* h_colidx,
                 const uint8_t* h_dirichlet, int32_t* h_agg, int32_t* n_agg);

/* Distance-2 aggregation on the device by Luby rounds (paper §6: the device MIS
 * coarsener with deterministic hash priorities).  The graph is the block pattern of
 * A (square, any block size and dtype; values unused) without the diagonal and
 * without the vertices flagged in d_dirichlet (device uint8[nbr], may be NULL).
 * Vertex i has priority ((splitmix64(seed ^ i) >> 32) << 32) | (i + 1).  Each round,
 * an undecided vertex whose priority is the largest among undecided vertices within
 * distance 2 becomes a root, then undecided vertices within distance 2 of a new root
 * are decided; rounds repeat until none is undecided.  Roots are numbered in vertex
 * order; a root's neighbours join it; the remaining vertices join the neighbouring
 * aggregate that holds most of their neighbours (ties: smallest id).  d_agg: device
 * int32[nbr] output (-1 for flagged vertices); *n_agg aggregates; *n_rounds (may be
 * NULL) rounds taken.  The pattern's rows must be symmetric (an undirected graph).
 * Sync (one 4-byte read per round); allocates scratch. */
int sa_aggregate_device(bsr_t A, const uint8_t* d_dirichlet, uint64_t seed, int32_t* d_agg,
                        int32_t* n_agg, int32_t* n_rounds, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sa_aggregate_device with the same
 * arguments and results, on a static 64 MiB scratch array per GPU (held by the library
 * from the first call on a device until the process ends) instead of an allocation;
 * no hipMalloc, hipFree or allocating library routine is called.  Graphs whose scratch
 * exceeds 64 MiB (30 bytes per vertex plus a scan temporary: about 2.2 million
 * vertices) are refused with EINVAL before any launch.  Every call on one GPU shares
 * that GPU's scratch, so calls that overlap on one GPU (other threads, other streams)
 * race; each call initialises every scratch value it reads.  Sync, as
 * sa_aggregate_device. */
int sa_aggregate_device_noalloc(bsr_t A, const uint8_t* d_dirichlet, uint64_t seed, int32_t* d_agg,
                                int32_t* n_agg, int32_t* n_rounds, void* stream);
/* Tentative prolongator on the device (paper §2.2; the device-resident setup of §6):
 * per aggregate, the near-null-space rows of its members in ascending node order,
 * B_g = Q_g R_g by a thin Householder QR with diag(R_g) > 0; the members' rows of P~
 * are the rows of Q_g and R_g is the coarse near-null space.
 *   d_agg : device int32[nbr], aggregate id 0..n_agg-1 or -1 (row of P~ left zero);
 *           every id must be used
 *   d_B   : device double [nbr][bs][6], the near-null space (bs in 1..8)
 *   d_Pt  : device double [nbr][bs][6] output (values of P~ row by row; its pattern
 *           is one block per aggregated row, in column d_agg[i])
 *   d_Bc  : device double [n_agg][6][6] output (R_g row-major)
 * EINVAL for an aggregate with fewer than 6 rows, a rank-deficient one (|R_kk| <=
 * 1e-10 max(1, max|B_g|)), or one with more than 682 rows.  Sync; allocates scratch. */
int sa_tentative_device(int32_t nbr, int32_t bs, const int32_t* d_agg, int32_t n_agg, const double* d_B,
                        double* d_Pt, double* d_Bc, void* stream);
/* One smoothed-aggregation level on the host from the fine block pattern (paper §2.2,
 * §3.2): the greedy aggregation of sa_aggregate, the tentative prolongator P~ of the
 * six rigid-body modes built from h_coords ([n_nodes][3], bs = 3: per aggregate a thin
 * Householder QR of its members' rows in ascending order, signs with diag(R) > 0), the
 * coarse near-null space R ([n_agg][6][6]) and the pattern of the smoothed prolongator
 * (the structural product of the pattern of A with that of P~; the values follow from
 * D^-1 A on the device).  h_rowptr / h_colidx: the pattern of A with strictly ascending
 * columns per row; h_dirichlet ([n_nodes] flags, may be NULL) excludes rows from the
 * aggregation.  opts may be NULL; its strength_eps must be 0 (no values are given).
 * The arrays belong to the result: read them with sa_result_info / sa_result_arrays,
 * release them with sa_result_free.  EINVAL on a malformed pattern or a rank-deficient
 * aggregate.  Pure host code. */
int sa_setup_host(int32_t n_nodes, const int32_t* h_rowptr, const int32_t* h_colidx,
                  const uint8_t* h_dirichlet, const double* h_coords, const blkamg_opts* opts,
                  sa_result_t* out);
/* Sizes of a result: aggregates, blocks of P~ (one per aggregated row), blocks of the
 * smoothed-prolongator pattern (any pointer may be NULL). */
int sa_result_info(sa_result_t r, int32_t* n_agg, int64_t* pt_nnzb, int64_t* sp_nnzb);
/* Host arrays of a result, valid until sa_result_free (any pointer may be NULL):
 * agg [n_nodes] (aggregate id, -1 for unaggregated rows); P~ as BSR with 3x6 blocks:
 * pt_rowptr [n_nodes + 1], pt_colidx [pt_nnzb], pt_val [pt_nnzb][3][6] row-major;
 * bc [n_agg][6][6]; smoothed pattern sp_rowptr [n_nodes + 1], sp_colidx [sp_nnzb]. */
int sa_result_arrays(sa_result_t r, const int32_t** agg, const int32_t** pt_rowptr,
                     const int32_t** pt_colidx, const double** pt_val, const double** bc,
                     const int32_t** sp_rowptr, const int32_t** sp_colidx);
int sa_result_free(sa_result_t r);

/* Build the hierarchy from the fine operator A0 (square blocks bs = A0.bs_r, F64):
 * per level aggregate, tentative prolongator from the near-null space (thin QR per
 * aggregate, positive diagonal of R), lambda_hat by Lanczos, P = (I - omega D^-1 A) P~
 * with D the block diagonal, A_c = P^T A P; coarsest level factored by dense
 * Cholesky.  h_coords: [nbr][3] node coordinates (bs must be 3: the six rigid-body
 * modes are generated) ; h_dirichlet: [nbr] flags (may be NULL).  A0 is borrowed
 * and must outlive the hierarchy.  Sync; allocates. */
int amg_setup(bsr_t A0, const double* h_coords, const uint8_t* h_dirichlet,
              const blkamg_opts* opts, void* stream, amg_t* out);
/* Hierarchy of a batch of independent problems given as one block-diagonal A0:
 * instance t owns block rows (and columns) [h_inst_row0[t], h_inst_row0[t+1]),
 * h_inst_row0 has n_inst + 1 entries from 0 to A0.nbr, and no stored block may
 * couple two instances (EINVAL otherwise).  Each instance is coarsened exactly as
 * amg_setup would coarsen it alone (own aggregates, own lambda_hat per level, own
 * coarsest level and Cholesky factor); one kernel launch serves all instances of
 * a level.  Instances with at most coarse_eq_limit dofs must come last.  On every
 * level the rows of the instances still smoothed there come first, then those of
 * the instances whose coarsest level it is (amg_instance_rows tells where each
 * instance lives).  Sync; allocates. */
int amg_setup_batched(bsr_t A0, int32_t n_inst, const int32_t* h_inst_row0,
                      const double* h_coords, const uint8_t* h_dirichlet,
                      const blkamg_opts* opts, void* stream, amg_t* out);
int amg_destroy(amg_t M);
int amg_num_levels(amg_t M, int32_t* n_levels);
/* Number of instances (1 for amg_setup). */
int amg_num_instances(amg_t M, int32_t* n_inst);
/* Where each instance lives on `level` (host arrays of n_inst entries, any may be
 * NULL): first block row, number of block rows, and state 0 = the instance has no
 * such level, 1 = smoothed there, 2 = this is its coarsest level (dense solve). */
int amg_instance_rows(amg_t M, int32_t level, int32_t* h_row0, int32_t* h_nrows,
                      int32_t* h_state);
/* Level operators (library-owned; level 0 is A0 itself for F64 hierarchies and a
 * library-owned F32 copy for F32 hierarchies) and prolongators (NULL on the
 * coarsest level).  Handles remain owned by the hierarchy. */
int amg_level(amg_t M, int32_t level, bsr_t* A, bsr_t* P);
/* Host copy of the aggregates of `level`: one id (row of level + 1) per smoothed
 * row, int32[number of smoothed rows of that level] (all rows for one instance);
 * -1 for Dirichlet rows. */
int amg_aggregates(amg_t M, int32_t level, int32_t* h_agg);
/* Host copy of lambda_hat, double[n_levels - 1][n_inst] (level-major); 0 where the
 * instance is not smoothed on that level.  Sync. */
int amg_lambdas(amg_t M, double* h_lam);
/* Hot Galerkin recompute with reused interpolation (paper §3.1, §3.5): after A0's
 * values changed, recompute every coarse operator with ptap_numeric on the fixed
 * patterns (F32 hierarchies first cast A0 to their F32 copy).  Async, no allocation. */
int amg_galerkin_recompute(amg_t M, void* stream);
/* Refresh the smoother data after a recompute: block-diagonal inverses,
 * lambda_hat (Lanczos, or taken from h_lambda[level * n_inst + instance] when
 * h_lambda != NULL; entries of instances not smoothed on a level are ignored),
 * Chebyshev coefficients and the coarsest Cholesky factor.  Returns ENOTSPD if the
 * factorisation meets a non-positive pivot (sync check at the end).  Sync. */
int amg_smoother_refresh(amg_t M, const double* h_lambda, void* stream);

/* Hierarchy from operators the caller already has (paper §2.1: the V-cycle needs
 * the level operators, the prolongators and the smoother data; §3.1: the coarse
 * operators may come from elsewhere, e.g. ptap_numeric).  A: n_levels handles,
 * A[0] F64 with 3x3 blocks, A[l >= 1] F64 with 6x6 blocks, all square; P:
 * n_levels - 1 handles (may be NULL when n_levels = 1), P[l] F64 with
 * A[l].nbr x A[l+1].nbr block rows x columns and A[l].bs x 6 blocks.  The A
 * handles are borrowed and must outlive the hierarchy; the P values and patterns
 * are copied.  Computes the smoother data as amg_smoother_refresh does (block-
 * diagonal inverses, lambda_hat by Lanczos or the learned model as opts.eig_mode
 * says, Chebyshev coefficients, Cholesky factor of A[n_levels - 1]).  One instance;
 * opts.hier_dtype must be F64 (EINVAL otherwise), opts may be NULL.  Such a
 * hierarchy has no aggregates (amg_aggregates returns EINVAL) and
 * amg_galerkin_recompute refuses it: the caller recomputes A[l >= 1] and then calls
 * amg_hierarchy_update.  ENOTSPD if the coarsest factorisation fails.  Sync;
 * allocates. */
int amg_hierarchy_create(int32_t n_levels, const bsr_t* A, const bsr_t* P,
                         const blkamg_opts* opts, void* stream, amg_t* out);
/* Refresh the smoother data from the current level operators (paper §3.1; any
 * hierarchy): as amg_smoother_refresh, with lambda_hat given in single precision,
 * h_lambda float[n_levels - 1][n_inst] (level-major; entries of instances not
 * smoothed on a level are ignored, the others must be positive, EINVAL otherwise),
 * or computed by the configured estimator when h_lambda is NULL.  Sync. */
int amg_hierarchy_update(amg_t M, const float* h_lambda, void* stream);

/* One V-cycle from a zero guess, z = M^-1 r (paper §2.1): Chebyshev/point-block-
 * Jacobi pre-smoothing, residual, restriction with P^T, recursion, prolongation,
 * post-smoothing, coarsest solve with the Cholesky factor.  d_r, d_z: F64
 * [n_dof(A0)][nrhs], nrhs 1 or 8 (F32 hierarchies convert at entry and exit).
 * Async (the first call with nrhs = 8 allocates the wider work vectors). */
int vcycle_apply(amg_t M, const double* d_r, double* d_z, int32_t nrhs, void* stream);
/* vcycle_apply with the vectors' type: vec_dtype BLKAMG_F64 (as vcycle_apply, any
 * hierarchy) or BLKAMG_F32 (F32 hierarchies only: the V-cycle reads d_r and writes
 * d_z, FP32 [n_dof][nrhs], directly, with no conversion; EINVAL on an F64 hierarchy).
 * Async. */
int vcycle_apply_ex(amg_t M, const void* d_r, void* d_z, int vec_dtype, int32_t nrhs, void* stream);

/* Preconditioned CG on A x = b (the CG accelerator of paper §4.1) from x0 = 0 with
 * M = one V-cycle; stops when the recurrence residual satisfies
 * ||r||_2 <= rtol ||b||_2 (unpreconditioned norm, paper §4.1) or after maxit
 * iterations.  A: F64, n_dof = A0's; d_b, d_x: F64 [n_dof][nrhs], nrhs 1 or 8.
 * Every (instance, column) pair is its own system with its own CG scalars and
 * stopping test; a system that stopped is frozen while the others go on.
 * iters, relres (may be NULL): [n_inst][nrhs] number of solution updates and
 * ||r||/||b|| (0 for b = 0).  Returns ENOCONV if any system reached maxit,
 * EBREAKDOWN if p^T A p <= 0 in any (results of the others are still written).
 * One instance with one column: one 8-byte read per iteration.  Otherwise the
 * stopping tests stay on the device and the host reads an 8-byte status every
 * pcg_graph_iters iterations, each block of iterations replayed from a captured
 * HIP graph (captured on a library stream on first use, recaptured when x, A,
 * nrhs, rtol or maxit change).  Sync. */
int pcg_solve(bsr_t A, amg_t M, const double* d_b, double* d_x, double rtol,
              int32_t maxit, int32_t nrhs, int32_t* iters, double* relres, void* stream);

/* ==========================================================================
 * Learned eigenbound (replaces the per-level Lanczos estimate of lambda_max(D^-1 A)
 * that sets the Chebyshev interval, paper §4.1, and the prolongator-smoothing
 * weight, paper §2.2; Lanczos stays as fallback and as reference)
 * ========================================================================== */

/* C[m][n] = op(A) op(B) on the matrix cores (v_mfma_f32_16x16x4_f32), FP32.
 * op(A) is m x k: A row-major [m][lda] (trans_a = 0) or [k][lda] read transposed
 * (trans_a = 1); likewise op(B) k x n from [k][ldb] or [n][ldb].  C row-major
 * [m][ldc] is overwritten.  Async. */
int mlp_gemm_f32(int32_t trans_a, int32_t trans_b, int32_t m, int32_t n, int32_t k,
                 const float* d_a, int32_t lda, const float* d_b, int32_t ldb,
                 float* d_c, int32_t ldc, void* stream);
/* Network forward on n standardised feature rows d_x [n][12]:
 * H1 = relu(X W1 + b1) [n][64], H2 = relu(H1 W2 + b2) [n][64], Y = H2 W3 + b3 [n][2].
 * d_theta: BLKAMG_MLP_PARAMS floats, W1 [12][64], b1 [64], W2 [64][64], b2 [64],
 * W3 [64][2], b3 [2] (row-major, in x out).  Async. */
int mlp_forward(const float* d_theta, const float* d_x, int32_t n, float* d_h1,
                float* d_h2, float* d_y, void* stream);
/* Gradient of L = 1/(2n) sum (Y - T)^2 with respect to theta, from the forward
 * results; d_t [n][2]; d_work: 130 n floats of scratch; d_grad: BLKAMG_MLP_PARAMS
 * floats (overwritten); *d_loss (device double, may be NULL) = L.  Async. */
int mlp_loss_grad(const float* d_theta, const float* d_x, const float* d_h1,
                  const float* d_h2, const float* d_y, const float* d_t, int32_t n,
                  float* d_work, float* d_grad, double* d_loss, void* stream);
/* One Adam step (Kingma & Ba, Algorithm 1) on n_params FP32 master weights with
 * moments d_m, d_v (start at zero); step counts from 1.  Async. */
int mlp_adam(float* d_theta, const float* d_grad, float* d_m, float* d_v, int32_t n_params,
             int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Network inputs of every smoothed (level, instance) pair, computed by one
 * block-row reduction kernel per level from the current operators (block-diagonal
 * inverses are refreshed first): d_feat [n_samples][12] FP32 (may be NULL to only
 * count), samples level-major, instances in level order; h_level, h_inst
 * (n_samples entries each, may be NULL) name each sample.  The twelve features are
 * logs of the max, mean and RMS of the Gershgorin row bounds of D^-1 A, of
 * 1 + max and 1 + mean of the off-diagonal block norms of D^-1 A, of the
 * diagonal-block norm contrast, the mean and max blocks per row, log scalar rows,
 * level index, block size / 6, and feature 4 minus feature 1.  Sync. */
int amg_features(amg_t M, float* d_feat, int32_t* n_samples, int32_t* h_level,
                 int32_t* h_inst, void* stream);
/* Reference lambda_max(D^-1 A) per (level, instance), double[n_levels-1][n_inst]
 * (0 where not smoothed): k steps (2..64) of Lanczos in the D inner product with
 * full reorthogonalisation, FP64 vectors, started like the level's estimate.
 * Uses the current block-diagonal inverses (amg_smoother_refresh or setup).  Sync. */
int amg_judge_lambdas(amg_t M, int32_t k, double* h_lam, void* stream);
/* Install a trained model: h_model = BLKAMG_MLP_MODEL floats, the parameters then
 * feature mean[12], feature std[12], target mean[2], target std[2]; targets are
 * (log lambda_max, omega).  With eig_mode BLKAMG_EIG_MLP, amg_smoother_refresh
 * then takes lambda_hat = exp(prediction) per (level, instance), runs the smoother
 * growth test on every level (A-norm of the last of opts.growth_steps smoother
 * applications to a fixed splitmix64 vector, from f = 0, must not grow) and falls back
 * to Lanczos on each level where some instance fails it.  Sync (copies the model). */
int amg_set_eig_model(amg_t M, const float* h_model, int32_t n_floats);
/* Outcome of the last MLP refresh: h_fallback[n_levels-1] (1 = level fell back to
 * Lanczos), h_growth and h_omega [n_levels-1][n_inst] (growth factor of the test
 * and predicted prolongator weight; 0 where not smoothed).  Any may be NULL. */
int amg_eig_status(amg_t M, int32_t* h_fallback, double* h_growth, double* h_omega);
/* State of the deferred guard (opts.mlp_guard = BLKAMG_GUARD_PCG): *armed = 1 while
 * the smoother scalars come from the network and no check has rejected them;
 * *restarts = solves restarted so far because CG's residual check failed.  Either
 * may be NULL. */
int amg_guard_status(amg_t M, int32_t* armed, int32_t* restarts);
/* What the cold setup used on each smoothed level (paper §2.2: P = (I - omega D^-1 A) P~):
 * h_lambda and h_omega [n_levels-1][n_inst] (the lambda_hat the setup's smoother
 * and the weight its prolongator smoothing used; 0 where not smoothed) and
 * h_learned[n_levels-1] (1 = from the network, which passed the growth test; 0 =
 * Lanczos with omega = omega_scale / lambda_hat).  Any may be NULL.  Hierarchies
 * from caller operators report zeros. */
int amg_setup_weights(amg_t M, double* h_lambda, double* h_omega, int32_t* h_learned);

#ifdef __cplusplus
}
#endif
#endif /* BLKAMG_H */
