/*
 * h2lr -- H^2-matrix local low-rank updates, H^2 Cholesky factorisation and
 * preconditioned CG on one AMD Instinct MI355X (gfx950).
 *
 * Method: S. Boerm, K. Reimer, "Efficient arithmetic operations for
 * rank-structured matrices based on hierarchical low-rank updates".
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status codes only; no C++ exception crosses this interface.  After an
 *   error h2_last_error() returns a message for the calling thread.
 * - Index order: a cluster tree permutes the n indices so that every cluster
 *   is a contiguous range ("cluster order").  Vectors passed to h2_matvec,
 *   h2_precond, h2_pcg and h2_spmv are in the caller's ORIGINAL order.  The
 *   factors X, Y of h2_lowrank_update use cluster order restricted to the
 *   block's row / column cluster (row i of X belongs to index
 *   perm[offset(t0) + i]).
 * - Matrices passed by pointer are column-major with the given leading
 *   dimension.  Pointers documented as "device" must be HIP device memory
 *   owned by the caller and stay valid until the context stream is
 *   synchronised; "host" pointers are read before the call returns.
 * - All device work is issued on the stream given to h2_ctx_create.  Calls
 *   that return host values (info/stats/export, h2_pcg counters) synchronise
 *   that stream; every other call may return before the device work ends.
 * - Device memory of matrices, sparse matrices and tree tables is allocated
 *   and released in the order of that stream (hipMallocAsync/hipFreeAsync),
 *   so destroying an object does not wait for other streams; the stream
 *   must therefore outlive every object created on the context, and a tree
 *   must outlive the matrices built on it.
 * - Objects are not thread safe; use one context per host thread.
 */
#ifndef H2LR_H
#define H2LR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_OK = 0,
  H2_ERR_ARG = -1,              /* invalid argument (null, size, range)        */
  H2_ERR_NOMEM = -2,            /* device or host allocation failed            */
  H2_ERR_HIP = -3,              /* a HIP runtime call failed                   */
  H2_ERR_NOT_SPD = -4,          /* non-positive pivot in a leaf factorisation  */
  H2_ERR_RANK_CAP = -5,         /* a recompressed rank exceeded the rank cap   */
  H2_ERR_NONZERO_FARFIELD = -6, /* sparse input has a non-zero in an admissible block */
  H2_ERR_NOT_CONVERGED = -7,    /* PCG reached maxit before the tolerance      */
  H2_ERR_STATE = -8,            /* object poisoned by an earlier failed update */
  H2_ERR_ZERO_PIVOT = -9        /* zero pivot in a leaf of the LR factorisation */
} h2_status;

typedef struct h2_ctx_s *h2_ctx;
typedef struct h2_ctree_s *h2_ctree;
typedef struct h2_btree_s *h2_btree;
typedef struct h2_mat_s *h2_mat;
typedef struct h2_csr_s *h2_csr;
typedef struct h2_job_s *h2_job;

/* Recompression accuracy (Section 4, last paragraph; Section 7 "block-relative
 * accuracy").  mode 0 = block-relative: every block entering a weight stack is
 * scaled by 1/||block||_F and singular values <= eps are dropped; mode 1 =
 * constant relative: drop sigma <= eps*sigma_1; mode 2 = no truncation (keep
 * all numerically non-zero singular values).  In every mode a basis
 * recompression of an m x n matrix also drops sigma <= max(m,n) eps_mach
 * sigma_1 (rounding noise).  rank_cap: 1..H2_MAX_RANK, exceeding it fails
 * with H2_ERR_RANK_CAP.  precision: H2_PREC_FP64, or H2_PREC_MIXED: the
 * coupling projections S_b <- R_t S_b R_s^* and the transfer / basis-change
 * products (R_t' E_t', R_t = Q_t^* V_t, R_t0 E_t0) of every local update take
 * float operands and accumulate in float on the matrix cores; QR, SVD,
 * weights, nearfield and all vector solves stay FP64 (results stored FP64).
 * H2_PREC_MIXED_BF16 (a trial): as H2_PREC_MIXED, and every new leaf basis
 * is stored rounded to bfloat16 precision.  accumulate (products, hence
 * Cholesky, LR and the triangular inverse): 0 = every temporary low-rank
 * matrix of an admissible product target (one per pair of sons, Section 6)
 * is added by its own local update; 1 = accumulated updates: the
 * temporaries of one target are concatenated, in order, into as few local
 * updates as the update rank H2_MAX_UPDATE_RANK allows (greedy), so fewer
 * recompressions run (a truncation strategy of the kind named at the end of
 * Section 4; it changes the truncation sequence).  level_factor q in (0, 1]
 * (0 means 1): variable-order weighting of the cluster-basis recompression,
 * the threshold of a cluster at level l of a tree of depth p multiplied by
 * q^(p - l) (formed by repeated products), so larger clusters are kept more
 * accurately, as in a variable-order scheme (the weighting the end of
 * Section 4 names; q = 1 changes nothing).  Temporaries are not affected. */
typedef struct {
  double eps;
  int32_t mode;
  int32_t rank_cap;
  int32_t precision;
  int32_t accumulate;
  double level_factor;
} h2_trunc;
#define H2_PREC_FP64 0
#define H2_PREC_MIXED 1
#define H2_PREC_MIXED_BF16 2

#define H2_MAX_RANK 32       /* rank capacity of every basis slot            */
#define H2_MAX_LEAF 32       /* largest leaf cluster                          */
#define H2_MAX_COLS 64       /* right-hand sides of one matvec / solve        */
#define H2_MAX_UPDATE_RANK 32 /* columns of a low-rank update factor          */
#define H2_MAX_BATCH_UPDATES 4 /* updates per matrix in one batched call      */

/* ---------------------------------------------------------------- context */
/* device: HIP device ordinal, or -1 for a host-only context that can build
 * and export trees but holds no device data; stream: hipStream_t to issue
 * work on (NULL = the default stream).  The context owns no matrix data. */
h2_status h2_ctx_create(int device, void *stream, h2_ctx *out);
h2_status h2_ctx_destroy(h2_ctx ctx);
h2_status h2_ctx_synchronize(h2_ctx ctx);
const char *h2_last_error(void);

/* ------------------------------------------------------------ cluster tree */
/* Cluster tree (Def. "Cluster tree", Section 2; binary as in Section 3) by
 * geometric bisection of integer points: a cluster with more than leaf_size
 * points is split at the midpoint of the longest side of its bounding box
 * (lowest axis on ties), son 0 keeping the points with 2c <= lo+hi in their
 * current order.  Clusters are numbered breadth first.
 * coords: host, n x dim int32 row-major (point i at coords[i*dim ..]).
 * leaf_size: 1..H2_MAX_LEAF; dim 1..3.  Result owned by the caller. */
h2_status h2_ctree_build(h2_ctx ctx, int32_t dim, int64_t n, const int32_t *coords,
                         int32_t leaf_size, h2_ctree *out);
/* Cluster tree by domain decomposition (Section 7 uses a domain decomposition
 * cluster strategy; the paper gives no details).  Binary, like every tree
 * here: a domain cluster with more than leaf_size points is cut by the grid
 * hyperplane x_d = floor((lo_d + hi_d)/2) of its longest side d (lowest axis
 * on ties) into D1 (x_d below), D2 (x_d above) and the interface I (on the
 * plane); its sons are the union D1+D2 and I, ordered D1, D2, I (each in its
 * current order), and the union, if larger than leaf_size, has the domain
 * sons D1 and D2.  Interfaces and their descendants are bisected as in
 * h2_ctree_build; a domain whose cut leaves D1, D2 or I empty is bisected and
 * its sons stay domains.  A block tree built on this tree makes the pairs
 * (D1, D2), (D2, D1) of every cut admissible leaves: on a stencil that
 * couples only points at most one grid step apart in each axis they vanish,
 * and, the order being a nested dissection, so does the Cholesky factor, so
 * they keep rank 0.  Arguments, result and errors as for h2_ctree_build. */
h2_status h2_ctree_build_dd(h2_ctx ctx, int32_t dim, int64_t n, const int32_t *coords,
                            int32_t leaf_size, h2_ctree *out);
h2_status h2_ctree_info(h2_ctree ct, int64_t *n, int64_t *nclusters, int32_t *depth);
/* Host copies of the tree tables (each array nclusters long, perm n long);
 * any pointer may be NULL. */
h2_status h2_ctree_export(h2_ctree ct, int64_t *perm, int32_t *offset, int32_t *size,
                          int32_t *level, int32_t *son0, int32_t *son1, int32_t *parent);
h2_status h2_ctree_destroy(h2_ctree ct);

/* -------------------------------------------------------------- block tree */
/* Block tree (Def. "Block tree", Section 2) of ct x ct: (t,s) is an
 * admissible leaf iff max(diam^2) <= eta^2 dist^2 for the integer bounding
 * boxes and the boxes are at least two grid steps apart along some axis (no
 * stencil of reach one couples them), or (t,s) is a zero pair of a
 * domain-decomposition tree (h2_ctree_build_dd); a pair of leaf clusters is an inadmissible leaf;
 * other pairs are split into sons+(t) x sons+(s), t' outer.  Breadth-first
 * block numbering.  The block tree keeps a reference to ct. */
h2_status h2_btree_build(h2_ctx ctx, h2_ctree ct, double eta, h2_btree *out);
/* csp: largest number of admissible leaves in one block row. */
h2_status h2_btree_info(h2_btree bt, int64_t *nblocks, int64_t *nadm, int64_t *nnear,
                        int32_t *csp);
/* kind: 0 subdivided, 1 admissible leaf, 2 inadmissible leaf.  Arrays are
 * nblocks long; any pointer may be NULL. */
h2_status h2_btree_export(h2_btree bt, int32_t *row, int32_t *col, int32_t *kind,
                          int32_t *parent);
/* block id of the pair (t, s), or -1 if it is not a block of the tree. */
h2_status h2_btree_find(h2_btree bt, int64_t t, int64_t s, int64_t *block);
h2_status h2_btree_destroy(h2_btree bt);

/* ---------------------------------------------------------------- matrices */
/* H^2 representation (Def. "H^2-matrix", eq. (vsw)) of a sparse matrix whose
 * admissible blocks vanish: all ranks 0, inadmissible leaves dense.
 * rowptr (n+1), col (nnz), val (nnz): host CSR in original order.
 * lower != 0 stores only the blocks on or below the diagonal (the storage
 * of a Cholesky factor).  rank_cap as in h2_trunc.
 * Fails with H2_ERR_NONZERO_FARFIELD if a non-zero lies in an admissible
 * block. */
h2_status h2_mat_from_csr(h2_ctx ctx, h2_btree bt, int64_t n, const int64_t *rowptr,
                          const int32_t *col, const double *val, int32_t lower,
                          h2_mat *out);
h2_status h2_mat_copy(h2_mat src, h2_mat *out);
/* Overwrite dst with the contents of src (same block tree and storage);
 * device-to-device copies only, no allocation.  Clears a poisoned dst. */
h2_status h2_mat_assign(h2_mat dst, h2_mat src);
h2_status h2_mat_destroy(h2_mat m);
/* Device bytes h2_mat_from_csr allocates for a matrix on bt (lower: as its
 * argument): storage, work areas and block lists; task lists (made by the
 * first factorisation / solve), PCG vectors and the tree tables (shared by
 * the matrices of one tree) come on top.  Host-only; for admission by an HBM
 * budget. */
h2_status h2_estimate_bytes(h2_btree bt, int32_t lower, int64_t *bytes);
/* Device bytes the matrix holds now, task lists and PCG vectors included
 * (tree tables excluded). */
h2_status h2_mat_bytes(h2_mat m, int64_t *bytes);
/* stored_values: floating point values held by bases, transfers, couplings
 * and nearfield blocks at the current ranks; max ranks of both bases. */
h2_status h2_mat_stats(h2_mat m, int64_t *stored_values, int32_t *max_rank_row,
                       int32_t *max_rank_col);
/* Host copies of the current ranks k_t of the row basis (rank_row) and of
 * the column basis (rank_col), nclusters entries each, cluster ids as in
 * h2_ctree_export; either pointer may be NULL.  Synchronises the stream. */
h2_status h2_mat_ranks(h2_mat m, int32_t *rank_row, int32_t *rank_col);
/* Algorithmic floating point operations performed on m since the last reset
 * (products 2mnk, Householder R-factors 2mn^2-2n^3/3, SVDs 4ab^2+8b^3 with
 * a = max, b = min of the dimensions; vector substitutions n^2 per column);
 * reset != 0 zeroes the counter afterwards.  Synchronises the stream. */
h2_status h2_mat_flops(h2_mat m, double *flops, int32_t reset);
/* Tracing: if counters != NULL, copy the first n (<= 204) profile counters
 * of m (task counts per kind [0,32), device ticks of a 100 MHz clock per kind
 * [32,64), ticks per stage of the low-rank update [64,80), ticks and counts
 * of sub-block products by size class [80,96), per-wave ticks of update
 * sub-steps [96,112) and event counts [112,128), ticks and counts of
 * low-rank updates by tree level of t0 [128,144) and [144,160), ticks per
 * stage of updates of leaf blocks [160,168), ticks and counts of the
 * recompression SVDs by column count (<= 8, 16, 32, more) [168,176), ticks
 * and counts of truncated additions by row count (<= 32, 128, 512, 2048,
 * more) [176,184) and [184,192), algorithmic flops [192,198) and bytes of
 * H^2 data read and written [198,204) of the update steps: R-factors,
 * weights, recompression (with the E_t0 update), couplings, R-factor path
 * refresh, nearfield); then enable (enable != 0, counters reset to zero) or
 * disable collection. */
h2_status h2_profile(h2_mat m, int32_t enable, int64_t *counters, int32_t n);

/* Local low-rank update Z|_{t0 x s0} += X Y^* of the block tree node
 * `block` = (t0, s0) (Section 4 for the recompression, Section 5 for the
 * local update).  X: device, #t0 x k, leading dimension ldx >= #t0;
 * Y: device, #s0 x k, ldy >= #s0; 0 <= k <= H2_MAX_UPDATE_RANK.  Truncation per tr.
 * A zero X or Y (or k = 0) leaves Z unchanged.  On H2_ERR_RANK_CAP the matrix
 * is poisoned (H2_ERR_STATE on later calls). */
h2_status h2_lowrank_update(h2_mat z, int64_t block, int32_t k, const double *X, int64_t ldx,
                            const double *Y, int64_t ldy, const h2_trunc *tr);

/* Accumulated local update: the count updates (blocks[i], X_i, Y_i), with
 * arguments as for h2_lowrank_update, are merged into ONE local update of
 * the smallest block b* = (t*, s*) of the block tree that contains every
 * target, with factors X* = [P_1 X_1 ... P_m X_m], Y* = [Q_1 Y_1 ... Q_m Y_m]
 * (P_i, Q_i place the rows of t_i, s_i inside t*, s*; zeros elsewhere), so
 * X* Y*^* = sum_i P_i X_i Y_i^* Q_i^* and one recompression replaces m
 * (the accumulation variant of the truncation strategies at the end of
 * Section 4).  sum_i k_i <= H2_MAX_UPDATE_RANK.  merged_block (may be NULL)
 * receives b*.  H2_ERR_ARG for bad arguments; H2_ERR_RANK_CAP poisons. */
h2_status h2_lowrank_update_accumulated(h2_mat z, int32_t count, const int64_t *blocks, const int32_t *ks,
                                        const double *const *Xs, const int64_t *ldxs, const double *const *Ys,
                                        const int64_t *ldys, const h2_trunc *tr, int64_t *merged_block);

/* Local low-rank updates of count distinct matrices in one launch (one
 * workgroup per matrix; each matrix's updates run in order with the
 * arithmetic of h2_lowrank_update, so the results equal the single calls).
 * Matrix i receives nupd[i] (0..H2_MAX_BATCH_UPDATES) updates, taken in order
 * from the flat host arrays blocks, ks, Xs, ldxs, Ys, ldys (argument meaning
 * as for h2_lowrank_update); the matrices share one device and stream.
 * Arguments are checked before any device work.  status: optional, count
 * entries; a matrix whose update fails (H2_ERR_RANK_CAP) is poisoned, the
 * others are updated, the first failure is returned.  Blocks until done. */
h2_status h2_lowrank_update_batched(h2_mat *mats, int32_t count, const int32_t *nupd, const int64_t *blocks,
                                   const int32_t *ks, const double *const *Xs, const int64_t *ldxs,
                                   const double *const *Ys, const int64_t *ldys, const h2_trunc *tr,
                                   h2_status *status);

/* y = alpha op(Z) x + beta y, op = identity (trans = 0) or transpose.
 * x, y: device, n x nrhs column-major (leading dimension n), original order,
 * 1 <= nrhs <= H2_MAX_COLS.  Evaluated by forward transformation, coupling,
 * backward transformation and nearfield products (linear complexity, as
 * stated in the abstract and for the k matrix-vector products of Section 6,
 * Case 2). */
h2_status h2_matvec(h2_mat z, int32_t trans, double alpha, const double *x, double beta,
                    double *y, int32_t nrhs);

/* In-place approximate Cholesky factorisation A = L L^* of a matrix created
 * with lower != 0 (Section 3 recursion with R = L^*, block substitution and
 * products expressed by local low-rank updates; Section 7 uses it as the
 * preconditioner).  Fails with H2_ERR_NOT_SPD (message names the leaf) or
 * H2_ERR_RANK_CAP; the matrix is then poisoned. */
h2_status h2_cholesky(h2_mat a, const h2_trunc *tr);

/* In-place approximate LR factorisation A = L R of a matrix created with
 * lower = 0 (Section 3: LR recursion with L unit lower and R upper
 * triangular, leaves by Gaussian elimination without pivoting, the block
 * forward substitutions L_11 R_12 = A_12 and L_21 R_11 = A_21, the Schur
 * product A_22 - L_21 R_12 by the product recursion, all expressed by local
 * low-rank updates).  Afterwards the matrix holds L - I below the diagonal
 * and R on and above it in the same H^2 structure (h2_matvec applies that
 * packed operator).  Fails with H2_ERR_ZERO_PIVOT (message names the leaf)
 * or H2_ERR_RANK_CAP; the matrix is then poisoned. */
h2_status h2_lr(h2_mat a, const h2_trunc *tr);

/* z = R^{-1} L^{-1} r with the factors made by h2_lr (block forward
 * substitution with L, then block backward substitution with R, Section 3,
 * vector right-hand sides).  r, z: device, n x nrhs, original order (may
 * alias), 1 <= nrhs <= H2_MAX_COLS.  H2_ERR_ARG if a holds no LR factors. */
h2_status h2_lr_solve(h2_mat f, const double *r, double *z, int32_t nrhs);

/* Z += alpha X Y for three distinct full-storage (lower = 0) matrices on one
 * block tree and device (Section 3, product of H^2-matrices: Case 1
 * recursion over the sons, with temporary low-rank matrices for admissible
 * leaf targets added by local updates; Case 2 emissions of low-rank
 * products when a factor is a leaf; Section 6 for the cost).  X and Y are
 * only read; pending work on their streams is waited for.  Truncation per
 * tr.  Fails with H2_ERR_RANK_CAP (Z then poisoned). */
h2_status h2_product(h2_mat z, double alpha, h2_mat x, h2_mat y, const h2_trunc *tr);

/* h2_cholesky of count independent matrices in one launch (one workgroup
 * per matrix; the same Section 3 recursion and arithmetic as h2_cholesky,
 * so each factor equals the one h2_cholesky makes alone).  mats: host array
 * of distinct lower-stored matrices on one device and stream, any sizes.
 * status: optional host array of count entries receiving each matrix's
 * result.  Every matrix is factorised; a failed one is poisoned and the
 * call returns the status of the first failure (message names its index),
 * the others keep valid factors.  Blocks until the launch has finished. */
h2_status h2_cholesky_batched(h2_mat *mats, int32_t count, const h2_trunc *tr, h2_status *status);

/* The launch half of h2_cholesky_batched: plans (first call per matrix),
 * starts the factorisations on the matrices' stream and returns at once.
 * Until h2_job_finish, the matrices are busy: every other call on them fails
 * with H2_ERR_ARG (h2_mat_destroy with H2_ERR_STATE).  Launches on different
 * streams run concurrently on the device. */
h2_status h2_cholesky_launch(h2_mat *mats, int32_t count, const h2_trunc *tr, h2_job *job);
/* Local low-rank updates and Cholesky factorisations of distinct matrices
 * in ONE launch (one workgroup per matrix): matrices umats[0..ucount)
 * receive their updates as in h2_lowrank_update_batched (same argument
 * arrays and checks, the same arithmetic, so each result equals the single
 * calls), matrices cmats[0..ccount) (lower-stored) are factorised as in
 * h2_cholesky_launch (Section 3 recursion).  ucount or ccount may be 0, not
 * both; no matrix may appear twice; all share one device and stream.
 * Returns at once with a job (h2_job_query, h2_job_finish); the factors X, Y
 * are read on that stream before the launch, so they must stay valid until
 * the stream reaches it (h2_job_finish waits for it).  h2_job_finish's status
 * array has ucount + ccount entries, updated matrices first. */
h2_status h2_update_cholesky_launch(h2_mat *umats, int32_t ucount, const int32_t *nupd, const int64_t *blocks,
                                    const int32_t *ks, const double *const *Xs, const int64_t *ldxs,
                                    const double *const *Ys, const int64_t *ldys, h2_mat *cmats,
                                    int32_t ccount, const h2_trunc *tr, h2_job *job);
/* *done = 1 once the launched work has finished (does not block). */
h2_status h2_job_query(h2_job job, int32_t *done);
/* Waits for the job, checks every matrix as h2_cholesky_batched does (status
 * optional, count entries), releases the matrices and frees the job (also
 * when it returns an error). */
h2_status h2_job_finish(h2_job job, h2_status *status);

/* In-place approximate inverse G ~ L^{-1} of a Cholesky factor made by
 * h2_cholesky (the inversion remark at the end of Section 6, with the upper
 * off-diagonal block zero: C_11 = L_11^{-1}, C_22 = L_22^{-1},
 * C_21 = -C_22 L_21 C_11, the products by the Section 3 recursion with local
 * low-rank updates).  G keeps the block structure of L; its diagonal leaves
 * hold dense lower triangular inverses (zero above the diagonal).  After
 * the call h2_precond and h2_pcg apply G^* G, and h2_matvec applies G.
 * Fails with H2_ERR_RANK_CAP (matrix then poisoned), H2_ERR_ARG if the
 * matrix is not lower-stored or already inverted. */
h2_status h2_tri_invert(h2_mat l, const h2_trunc *tr);
/* *inverse = 1 if h2_tri_invert has turned the matrix into G ~ L^{-1}. */
h2_status h2_mat_is_inverse(h2_mat m, int32_t *inverse);

/* z = (L L^*)^{-1} r by forward and backward substitution with the factor
 * (Section 3, block forward substitution with vector right-hand sides), or
 * z = G^* G r by two H^2 matrix-vector products after h2_tri_invert.
 * r, z: device, n x nrhs, original order; r and z may alias. */
h2_status h2_precond(h2_mat l, const double *r, double *z, int32_t nrhs);

/* One triangular solve with a Cholesky factor (Section 3, block forward
 * substitution with vector right-hand sides): z = L^{-1} r (trans = 0) or
 * z = L^{-*} r (trans = 1); h2_precond is the two in sequence.  r, z:
 * device, n x nrhs, original order (may alias), 1 <= nrhs <= H2_MAX_COLS.
 * H2_ERR_ARG for a matrix that is not a (non-inverted) lower factor. */
h2_status h2_trsv(h2_mat l, int32_t trans, const double *r, double *z, int32_t nrhs);

/* Launch shape of the substitutions with a Cholesky factor (h2_precond,
 * h2_trsv, the preconditioner of h2_pcg and h2_pcg_batched) for nrhs
 * columns: threads per workgroup, 128, 256 or 512 (0 restores the default,
 * 256).  The substitutions compute every column, cluster and block group in
 * one wave in a fixed order, so the shape changes the time, never the
 * result.  h2_pcg_batched launches all systems with the largest shape of
 * its members.  H2_ERR_ARG for another value or a non-factor. */
h2_status h2_precond_config(h2_mat l, int32_t nrhs, int32_t threads);

/* Autotuner of that launch shape: times reps applications of the
 * substitution pair (z = (L L^*)^{-1} r on a work vector it allocates) for
 * each shape with events on the matrix's stream, keeps the fastest for
 * this matrix and nrhs, and reports it (threads, ms_per_apply).  With a
 * cache_path (may be NULL), a result recorded there for the same key (the
 * device architecture, n, cluster and block counts, stored values and nrhs)
 * is applied without timing (*from_cache = 1); a new result is appended as
 * one text line "key threads ms".  ms_by_shape: 3 entries, the time per
 * application at 128, 256 and 512 threads (zeros when taken from the
 * cache).  Output pointers may be NULL. */
h2_status h2_autotune_precond(h2_mat l, int32_t nrhs, int32_t reps, const char *cache_path, int32_t *threads,
                              double *ms_per_apply, int32_t *from_cache, double *ms_by_shape);

/* ------------------------------------------------------- sparse A and PCG */
/* Device copy of a CSR matrix (host arrays, original order). */
h2_status h2_csr_create(h2_ctx ctx, int64_t n, const int64_t *rowptr, const int32_t *col,
                        const double *val, h2_csr *out);
h2_status h2_csr_destroy(h2_csr a);
/* y = A x, device vectors of length n. */
h2_status h2_spmv(h2_csr a, const double *x, double *y);

/* Preconditioned conjugate gradients (Section 1; stopping rule of Section 7)
 * for A x = b with preconditioner (L L^*)^{-1} (G^* G after h2_tri_invert): x0 = 0, stop when the
 * recursive residual satisfies ||r||_2 <= rtol ||b||_2.  b, x: device,
 * length n, original order.  iters: products with A performed; relres: final
 * ||r||/||b||.  Returns H2_ERR_NOT_CONVERGED if maxit is reached. */
h2_status h2_pcg(h2_csr a, h2_mat l, const double *b, double *x, double rtol, int32_t maxit,
                 int32_t *iters, double *relres);

/* h2_pcg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * arguments, arithmetic and results as h2_pcg, but the PCG vectors, dot
 * product partial sums and scalars live in a fixed device area owned by the
 * library (one per device, 8 MiB, held until the process ends) instead of
 * memory the factor allocates, and x is cleared by a fill kernel.  No
 * device memory is allocated or freed.  Requirements, each an H2_ERR_ARG
 * otherwise: n <= H2_NOALLOC_MAX_N; the factor's preconditioner task list
 * already exists (made by the first h2_precond or h2_pcg call on l).
 * Every call on one device uses the same area and overwrites what the last
 * call left there; calls that overlap on one device (other host threads,
 * other streams) race and must be serialised by the caller. */
#define H2_NOALLOC_MAX_N 262144
h2_status h2_pcg_noalloc(h2_csr a, h2_mat l, const double *b, double *x, double rtol, int32_t maxit,
                         int32_t *iters, double *relres);

/* h2_pcg for count independent systems A_i X_i = B_i in lockstep on one
 * stream, each with nrhs[i] right-hand sides (one CG iteration per column):
 * the products and vector updates of each column are launched one after
 * another, the preconditioner applications of all systems with an
 * unconverged column run in one launch (one workgroup per system, all its
 * columns at once); a converged column stops.  as, ls, bs, xs, nrhs: host
 * arrays of count entries; bs[i], xs[i]: device, n_i x nrhs[i] column-major
 * (leading dimension n_i), original order; nrhs NULL means one column each,
 * 1 <= nrhs[i] <= H2_MAX_COLS; ls distinct Cholesky factors (not inverted)
 * on one stream.  iters, relres, status: optional host arrays with one entry
 * per column (systems in order, columns in order).  Returns the first
 * failure (H2_ERR_NOT_CONVERGED if a column reached maxit). */
h2_status h2_pcg_batched(h2_csr *as, h2_mat *ls, const double *const *bs, double *const *xs,
                         const int32_t *nrhs, int32_t count, double rtol, int32_t maxit, int32_t *iters,
                         double *relres, h2_status *status);

/* h2_pcg_batched with the iterations replayed from a HIP graph: one CG
 * iteration of every column (product, dot products, updates, convergence
 * test, the preconditioner launch, the next direction) is captured once,
 * with all columns in each launch and the convergence test on the device
 * switching columns and systems off; the host replays it and reads one
 * counter per iteration.  Same arguments, arithmetic and results (bit for
 * bit) as h2_pcg_batched; at most 65535 columns in all. */
h2_status h2_pcg_batched_graph(h2_csr *as, h2_mat *ls, const double *const *bs, double *const *xs,
                               const int32_t *nrhs, int32_t count, double rtol, int32_t maxit, int32_t *iters,
                               double *relres, h2_status *status);

#ifdef __cplusplus
}
#endif
#endif /* H2LR_H */
