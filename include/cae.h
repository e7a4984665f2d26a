/*
 * cae.h -- C ABI of the compress-and-eliminate (CE) preconditioner for
 * sparse symmetric positive definite matrices on one MI355X (gfx950).
 *
 * The method (Sushnikova & Oseledets, "Compress and eliminate" solver for
 * symmetric positive definite sparse matrices):
 *   A0 = P A P^T is split into blocks by the permutation P and the block
 *   partition (Section 2, eq. (init_perm)).  Level by level, every block row
 *   i is compressed -- the far blocks F_i of the row are approximated by a
 *   low-rank factor, U_i^T F_i = [F^_i; E_i] with ||E_i|| below the tolerance
 *   (eq. (rreav), Remark 2.1) -- and the trailing b_i - r_i rotated unknowns
 *   are eliminated by block Cholesky (eq. (sm_L)).  The remaining (basis)
 *   unknowns of 2^d Morton siblings form the blocks of the next level
 *   (Section 2.5, eq. (bsp)); the last remainder is factored densely.  The
 *   result is A ~ Q^T L L^T Q (Proposition 2.1); the solve is
 *   x = Q^T L^{-T} L^{-1} Q b (Proposition 2.2).
 *
 * Conventions for every entry point:
 *   - Return value: 0 (CAE_OK) or a negative cae_status_t.  On error no
 *     output handle is created and nothing leaks; cae_last_error(NULL)
 *     returns a description (thread-local), cae_last_error(h) the last one of
 *     a call on handle h.
 *   - "host" pointers are read during the call only and never retained.
 *   - "device" pointers are HIP device memory owned by the caller.  They
 *     must stay valid until the call returns; work is issued on the stream
 *     given in cae_options_t (0 = the null stream) and every entry point
 *     synchronises that stream before it returns.
 *   - Vectors are FP64, column-major n x nrhs with leading dimension >= n,
 *     in the ORIGINAL (unpermuted) ordering.
 *   - A handle may be used by one host thread / stream at a time.
 */
#ifndef CAE_H_
#define CAE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CAE_OK = 0,
  CAE_EINVAL = -1,    /* invalid argument (shape, range, pattern) */
  CAE_ENOMEM = -2,    /* device or host allocation failed */
  CAE_ENOTSPD = -3,   /* a pivot block is not positive definite */
  CAE_ENOCONV = -4,   /* PCG did not reach the tolerance in maxit */
  CAE_EDEVICE = -5    /* a HIP call failed */
} cae_status_t;

typedef enum { CAE_RANK_EPS = 0, CAE_RANK_FIXED = 1, CAE_RANK_LEARNED = 2, CAE_RANK_LEARNED_CAP = 3 } cae_rank_mode_t;
/* FP32_BF16: FP32 factor whose Schur-complement products take BF16 inputs
 * with FP32 accumulation on the matrix cores */
typedef enum { CAE_FP64 = 0, CAE_FP32 = 1, CAE_FP32_BF16 = 2 } cae_precision_t;
typedef enum { CAE_ORDER_PAPER = 0, CAE_ORDER_MULTICOLOUR = 1 } cae_order_t;

typedef struct {
  int32_t struct_size;     /* sizeof(cae_options_t) */
  int32_t rank_mode;       /* CE(eps) (Remark 2.1, first strategy), CE(r) (second), or
                              LEARNED: CE(eps) with the cheaper rank-revealing step the
                              paper's conclusion proposes -- an MLP predicts the rank, a
                              Gaussian sketch of that width (plus 8) gives the range, an
                              a-posteriori check guarantees ||E_i||_2 <= eps * tau and
                              steps that fail it take the exact SVD (blocks <= 64);
                              LEARNED_CAP: CE(eps) where the MLP's width (plus 8) caps the
                              pivoted Cholesky of the far row's Gram matrix in the exact
                              compression (any block size); a capped step is kept only if
                              the energy left out cannot change the rank (sigma_{r+1}^2 +
                              bound <= (eps tau)^2, so its rank is the exact one and
                              ||E_i||_2 <= eps * tau), else it is redone without the cap */
  int32_t fixed_rank;      /* r for CE(r) */
  int32_t precision;       /* arithmetic of the block factorization; the coarse
                              remainder, the apply vectors and PCG are FP64 */
  int32_t order;           /* elimination order of every level: PAPER = block order
                              (Algorithm 2, i = 1..M_j); MULTICOLOUR = greedy colouring
                              of the block graph at distance 2, blocks ordered by
                              (colour, index) */
  int32_t max_levels;      /* K of Algorithm 1; 0 = until one block is left or the
                              remainder dimension is <= coarse_max_dim */
  int32_t timing;          /* 1 = time the compression launches with HIP events
                              (reported by cae_get_stats) */
  int32_t compensate;      /* 1: for every dropped far block E_il add its Frobenius norm to the
                              diagonal of i's eliminated rows and of l's live columns
                              (robustness option, not in the paper): M - A0 is then
                              positive semidefinite and no pivot can fail */
  int64_t coarse_max_dim;  /* remainder size factored densely (default 2048) */
  void* stream;            /* hipStream_t; NULL = null stream */
  const float* mlp_params; /* LEARNED: DEVICE, cae_mlp_param_count() floats (see cae_mlp_train) */
  uint64_t seed;           /* LEARNED: key of the counter-based (Philox4x32-10) sketches */
  float* record;           /* DEVICE or NULL: training records, CAE_RECORD_WIDTH floats per block
                              of every factored level (level after level): 16 features of
                              the far row, then the rank fraction r_i / b_i of the step
                              (-1 where the step compressed nothing); CE(eps) or LEARNED */
  int64_t record_cap;      /* rows available in record */
  int32_t coarsen;         /* cae_analyze with coordinates: 0 = the 2^d Morton siblings form a
                              block of the next level; 1 = pairs of blocks along the Morton
                              curve (axis x, y, z in turn: J = 2, keeping J r ~ B, Section
                              2.5, when ranks are about half the block) */
  int32_t graphs;          /* 1 (default): the iterative solvers (cae_pcg_solve,
                              cae_minres_solve) capture the preconditioner apply of a
                              handle into a HIP graph after its first three applies with
                              the same vectors and replay it from then on (the same
                              kernels, launched as one graph); 0 = launch the kernels one
                              by one */
  int32_t apply_split_steps; /* elimination waves with fewer steps than this (default 1024)
                              update the close blocks in the apply one workgroup per
                              (step, close block), larger waves one workgroup per step;
                              0 = always one workgroup per step.  Only the order of the
                              FP64 sums in the backward pass differs */
  void* workspace;         /* DEVICE or NULL: caller-owned arena (256-byte aligned) that
                              holds every device buffer of the numeric factorization (level
                              blocks, bases, factors, dense remainder, scratch), so that
                              cae_factor_numeric allocates no device memory; it must outlive
                              the handle.  Size it with cae_workspace_query.  The analysis'
                              own device arrays and the solvers' work vectors are not in it */
  size_t workspace_bytes;  /* size of workspace */
  int32_t big_pivot_cap;   /* blocks of 129..512 unknowns: most rows of the pivoted Cholesky
                              of the far row's Gram matrix (1..128; 0 = 128).  A step that
                              needs more is certified by a spectral bound on its dropped
                              part, or redone with an uncapped pivoted Cholesky (counted in
                              cae_stats_t.big_*); a smaller cap sends more steps there */
} cae_options_t;

#define CAE_RECORD_WIDTH 17

/* Fill *opt with the defaults (CE(eps), FP64, MULTICOLOUR, coarse 2048, graphs on,
   apply split below 1024 steps). */
void cae_default_options(cae_options_t* opt);

typedef struct cae_analysis_s* cae_analysis_t;
typedef struct cae_factor_s* cae_handle_t;

/*
 * Initial permutation for a tensor grid (Section 2, eq. (init_perm); Section
 * 2.8 on the choice of P): patches of patch[k] points per axis, visited in
 * Z (Morton) order of their coordinates; x fastest inside a patch.  The grid
 * is numbered naturally with axis 0 fastest.  Partial patches at the high end
 * of an axis keep their smaller size.
 *   ndim in {1,2,3}; dims, patch: host, ndim entries, all > 0.
 *   Query mode: perm == NULL writes only *nblocks.
 *   Outputs (host, caller-allocated): perm[new] = old (n entries),
 *   block_ptr (nblocks+1), coords (nblocks*ndim patch coordinates).
 */
int cae_grid_order(int32_t ndim, const int32_t* dims, const int32_t* patch,
                   int32_t* perm, int32_t* block_ptr, int32_t* coords, int32_t* nblocks);

/*
 * Ordering for a general sparse SPD matrix with no grid (robustness and
 * generality option, not in the paper, which orders grids geometrically,
 * Section 2.8): nested bisection of the graph of A -- each part split into
 * halves along the breadth-first order from a pseudo-peripheral vertex --
 * to a uniform depth so that every block has at most B unknowns.  The halves
 * of a part are consecutive, so cae_analyze with coords = NULL and ndim = 1
 * (groups of J = 2 blocks) coarsens along the bisection tree.
 *   n, row_ptr, col_idx: host CSR structure (both triangles).
 *   Query mode: perm == NULL writes only *nblocks.
 *   Outputs (host, caller-allocated): perm[new] = old (n), block_ptr (nblocks+1).
 */
int cae_graph_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t B,
                    int32_t* perm, int32_t* block_ptr, int32_t* nblocks);

/*
 * Symbolic analysis (host only, no GPU call): level-1 block pattern of A0
 * (close blocks, Section 2), elimination order and dependency waves of every
 * level, the far blocks created by the eliminations (eq. (A_st); remark after
 * eq. (sm_L)), blocks eliminated whole (empty far row: the first-row
 * elimination of Section 2.1), and the Morton coarsening (Section 2.5, eq. (bsp)).
 *   n, row_ptr (n+1), col_idx (row_ptr[n]): host CSR structure of the full
 *   symmetric matrix A (both triangles, sorted columns, diagonal present).
 *   perm: host, n entries, A0[i][j] = A[perm[i]][perm[j]].
 *   block_ptr: host, nblocks+1 bounds of the blocks of A0; NULL = uniform
 *   blocks of B (the last one may be smaller).
 *   coords: host, nblocks*ndim block coordinates used for coarsening (parent =
 *   coordinate >> 1, Morton siblings); NULL = consecutive groups of 2^ndim.
 *   opt: order and level options (the numeric fields are ignored here).
 *   The analysis may be shared by several factorizations and outlives them
 *   only if the caller destroys it last.
 */
int cae_analyze(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                const int32_t* perm, const int32_t* block_ptr, int32_t nblocks,
                int32_t B, const int32_t* coords, int32_t ndim,
                const cae_options_t* opt, cae_analysis_t* out);

typedef struct {
  int32_t M;            /* blocks of the level */
  int32_t nclose;       /* close pairs p < q at the start of the level */
  int32_t nfar;         /* far pairs created during the level */
  int32_t nremoved;     /* blocks eliminated whole */
  int32_t nwaves;       /* dependency waves of the order */
  int32_t Mnext;        /* blocks of the next level */
} cae_level_info_t;

/* Number of structural levels (until one block is left). */
int cae_analysis_levels(cae_analysis_t a, int32_t* nlevels);
int cae_analysis_level_info(cae_analysis_t a, int32_t level, cae_level_info_t* info);
/* Host arrays, sized from cae_level_info_t; any may be NULL.
 *   order[M] (elimination order), wave[M] (wave of every block),
 *   close_pairs[2*nclose], far_pairs[2*nfar] (p<q, sorted),
 *   removed[M] (1 = eliminated whole), parent[M] (block of the next level). */
int cae_analysis_level_arrays(cae_analysis_t a, int32_t level, int32_t* order, int32_t* wave,
                              int32_t* close_pairs, int32_t* far_pairs, uint8_t* removed,
                              int32_t* parent);
/* Permutation and level-1 blocks the analysis uses (host, n and nblocks+1). */
int cae_analysis_perm(cae_analysis_t a, int32_t* perm, int32_t* block_ptr);
void cae_analysis_destroy(cae_analysis_t a);

/*
 * Numeric CE factorization on the GPU (Algorithm 1 with Algorithm 2 per
 * level), A ~ Q^T L L^T Q.
 *   vals: DEVICE pointer, row_ptr[n] FP64 values of A in the CSR order given
 *   to cae_analyze.  eps: tolerance of CE(eps); the kept rank of a far row is
 *   the number of its singular values > eps * max_i A_ii (spectral-norm
 *   reading of ||E_i|| < eps).  The handle keeps a reference to the analysis
 *   (destroy the handle first) and a device copy of A for PCG.
 *   Errors: CAE_ENOTSPD (message names level and block), CAE_EDEVICE.
 */
int cae_factor_numeric(cae_analysis_t a, const double* vals, double eps,
                       const cae_options_t* opt, cae_handle_t* out);

/*
 * Bytes of device workspace a cae_factor_numeric of these values and options
 * carves when given cae_options_t.workspace (the options' own workspace fields
 * are ignored here).  The level sizes after the first depend on the ranks, so
 * the figure is exact for these values: the call runs the factorization with
 * the library's own memory, counts, and releases it.  It also uploads the
 * analysis' device arrays, which a factorization into a workspace requires.
 *   vals: DEVICE, as for cae_factor_numeric.  bytes: host, one size_t.
 *   Errors: as cae_factor_numeric.  A factorization whose workspace is too
 *   small returns CAE_ENOMEM and names the bytes it had reached.
 */
int cae_workspace_query(cae_analysis_t a, const double* vals, double eps, const cae_options_t* opt,
                        size_t* bytes);

/*
 * One call from the statement of the problem (Section 2: A x = b with A sparse
 * SPD, the permutation P of eq. (init_perm), the block size, the tolerance; the
 * result A ~ Q^T L L^T Q of Proposition 2.1): cae_analyze followed by
 * cae_factor_numeric.  Arguments as for cae_analyze, plus vals: HOST, row_ptr[n]
 * FP64 values in the CSR order (copied to the device), and eps.  The handle
 * owns the analysis (cae_destroy releases both); with cae_options_t.workspace
 * the numeric factorization is carved from it as in cae_factor_numeric.
 */
int cae_factor(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
               const int32_t* perm, const int32_t* block_ptr, int32_t nblocks, int32_t B,
               const int32_t* coords, int32_t ndim, double eps, const cae_options_t* opt,
               cae_handle_t* out);

/* z = M^{-1} r, M = Q^T L L^T Q (Proposition 2.2).  r, z: device, n x nrhs. */
int cae_apply_precond(cae_handle_t h, int32_t nrhs, const double* r, int64_t ldr,
                      double* z, int64_t ldz);

/*
 * z = M^{-1} r exactly as cae_apply_precond computes it (the same kernels in
 * the same order, bitwise the same result), for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The level vectors, the coarse product and the
 * partial products live in a 64 MiB array of static device memory that every
 * GPU loading the library holds until the process ends; this entry point
 * calls no hipMalloc, hipFree or other allocating routine.
 *   r, z: device, n x nrhs (ldr, ldz >= n).  stream: hipStream_t to enqueue
 *   on, NULL = the handle's stream.  The work is enqueued and the call
 *   returns without waiting for it.
 *   Errors: CAE_EINVAL when the work vectors of this factor and nrhs exceed
 *   the 64 MiB (the message states the bytes needed) or the factor has more
 *   than 63 levels; nothing is enqueued then.
 *   Every call on one GPU shares that GPU's array, which keeps the last
 *   call's contents (nothing in it needs to start at zero): calls that
 *   overlap on one GPU (other streams, other threads) race; calls enqueued on
 *   one stream are ordered by it.
 */
int cae_apply_precond_noalloc(cae_handle_t h, int32_t nrhs, const double* r, int64_t ldr,
                              double* z, int64_t ldz, void* stream);

/* y = M x with the stored factor (the approximation of A itself). */
int cae_apply_factor(cae_handle_t h, int32_t nrhs, const double* x, int64_t ldx,
                     double* y, int64_t ldy);

/*
 * FP64 preconditioned conjugate gradients with M^{-1} as preconditioner,
 * x0 = 0, every column stops when ||r_k||_2 <= rtol ||b||_2 (recurrence
 * residual), at most maxit iterations.
 *   b, x: device n x nrhs.  iters, relres: host, nrhs entries (iterations and
 *   true residual ||b - A x|| / ||b|| at exit).  Returns CAE_ENOCONV when a
 *   column did not converge (x still holds the last iterate).
 */
int cae_pcg_solve(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb,
                  double* x, int64_t ldx, double rtol, int32_t maxit,
                  int32_t* iters, double* relres);

/*
 * A batch of independent problems in one factorization (Algorithms 1 and 2
 * applied to each problem; the problems share every level's launches).  A
 * problem is a sparse SPD matrix on a tensor grid whose unknowns are numbered
 * lexicographically with the first axis fastest; its level-1 blocks are
 * patches of the given shape in Morton order (Section 2.5, eq. (bsp)).
 */
typedef struct {
  int64_t n;                /* unknowns: the product of dims */
  const int64_t* row_ptr;   /* HOST, n+1 (row_ptr[0] may be nonzero) */
  const int32_t* col_idx;   /* HOST, both triangles, sorted, diagonal present */
  const double* vals;       /* DEVICE, FP64 values in that CSR order */
  int32_t ndim;             /* 2 or 3 */
  int32_t dims[3];          /* grid sizes (dims[2] ignored for ndim 2) */
  int32_t patch[3];         /* patch shape; all zero = 8 x 8 (2D) or 4 x 4 x 4 (3D) */
} cae_problem_t;

/*
 * Symbolic analysis (host only) of nprob problems joined into one block-
 * diagonal matrix: problem t's rows follow those of problems 0..t-1 in the
 * joint ordering.  Problem t's block coordinates are offset by t's binary
 * digits dealt to the three axes in turn above 8 bits, so the Morton order of
 * the joint blocks runs problem by problem and the coarsening never joins
 * blocks of two problems before each is one block; a problem may have at
 * most 256 patches along an axis.  vals may be NULL here.  A numeric
 * factorization of the analysis (values: the problems' values stacked in the
 * joint CSR order) supports cae_pcg_solve_batched.
 *   Errors: CAE_EINVAL (the message names the problem), CAE_ENOMEM.
 */
int cae_analyze_batched(int32_t nprob, const cae_problem_t* probs, const cae_options_t* opt,
                        cae_analysis_t* out);

/* Problems of an analysis and their first rows (row_off: host, nprob+1
 * entries, or NULL); an analysis of one matrix reports one problem. */
int cae_analysis_batch_rows(cae_analysis_t a, int32_t* nprob, int64_t* row_off);

/*
 * cae_analyze_batched followed by the numeric factorization of the stacked
 * values (copied from the problems' device arrays), in one handle that owns
 * the joint analysis.  The threshold is eps * the largest diagonal entry of
 * the whole batch.  Every other call on handles works on the joint vectors
 * (problems stacked).  The host arrays may be freed after the call.
 *   Errors: as cae_analyze_batched and cae_factor_numeric.
 */
int cae_factor_batched(int32_t nprob, const cae_problem_t* probs, double eps,
                       const cae_options_t* opt, cae_handle_t* out);

/*
 * PCG as cae_pcg_solve, run independently on every problem of a batched
 * handle: each (problem, column) pair has its own step lengths and stops when
 * its residual over the problem's rows satisfies ||r|| <= rtol ||b|| there.
 * The sums over a problem's rows are formed in tiles of 4096 rows added in a
 * fixed order (the result does not depend on the launch).
 *   b, x: device, joint n x nrhs.  iters, relres: host, nprob * nrhs entries,
 *   entry t * nrhs + k for problem t and column k.  CAE_ENOCONV when a pair
 *   did not converge; CAE_EINVAL for a handle not made from a batch.
 */
int cae_pcg_solve_batched(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb,
                          double* x, int64_t ldx, double rtol, int32_t maxit,
                          int32_t* iters, double* relres);

/*
 * FP64 preconditioned MINRES (the Krylov method of the paper's Section 3),
 * with M^{-1} as the symmetric positive definite preconditioner, x0 = 0.  The
 * iterate minimises ||b - A x||_{M^{-1}} over the preconditioned Krylov space
 * (Paige-Saunders recurrences: three-term Lanczos with M^{-1}, Givens QR of
 * the tridiagonal matrix, three-term update of the search directions).
 * Every column stops when the preconditioned residual norm satisfies
 * ||r_k||_{M^{-1}} <= rtol ||b||_{M^{-1}}, or at maxit.  Arguments, outputs
 * (true residual ||b - A x|| / ||b|| in relres) and errors as for
 * cae_pcg_solve.
 */
int cae_minres_solve(cae_handle_t h, int32_t nrhs, const double* b, int64_t ldb,
                     double* x, int64_t ldx, double rtol, int32_t maxit,
                     int32_t* iters, double* relres);

typedef struct {
  int32_t nlevels;          /* levels factored (K) */
  int64_t coarse_dim;       /* dimension of the dense remainder */
  double tau;               /* max diagonal of A0; threshold = eps * tau */
  double dropped_sq;        /* sum over all steps of ||E_i||_F^2 */
  double min_pivot;         /* smallest diagonal entry of L */
  int64_t factor_bytes;     /* device bytes of the stored factor */
  double factor_ms;         /* wall time of the last numeric factorization */
  /* with cae_options_t.timing: the compression kernels (far row -> U_i, r_i) */
  int32_t compress_launches;
  double compress_ms;       /* summed device time of those launches */
  double compress_flops;    /* (always counted) algorithmic flops: per far row b x w,
                               2 w b^2 - 2 b^3 / 3 (QR, w >= b; else 2 b w^2 - 2 w^3 / 3)
                               + 12 b^3 (SVD of the triangular factor) */
  int32_t compressions;     /* far rows compressed (steps with a non-empty far row) */
  int32_t sketch_accepted;  /* LEARNED: steps the sketch settled */
  int32_t sketch_rejected;  /* LEARNED: steps that failed the check and took the exact SVD */
  int64_t record_rows;      /* rows written to cae_options_t.record */
  /* algorithmic flops of the other block operations of the factorization, from
     the recorded sizes and ranks (b = b_i, r = r_i, n = b - r, s_c live widths
     of the close blocks, w far width; see compress_flops for the compression):
     rotation 4 b^3 + 2 b^2 sum_c b_c + 2 r b w (steps with a far row),
     elimination n^3 / 3 + n^2 (r + sum_c s_c), Schur sum_{a <= c} 2 n s_a s_c
     over the panel widths {r, s_c}, dense remainder dim^3 / 3 */
  double rotate_flops;
  double elim_flops;
  double schur_flops;
  double coarse_flops;
  /* compressions of blocks of 129..512 unknowns, by how their rank was settled:
     the pivoted Cholesky ran to the rounding level; it was truncated and the
     energy left out (Frobenius norm) cannot change the rank; the spectral norm
     of the dropped part was bounded by repeated squaring of its Gram matrix;
     the bound failed and the step was redone with an uncapped pivoted
     Cholesky and a Jacobi on its rows */
  int32_t big_untruncated;
  int32_t big_frobenius;
  int32_t big_certified;
  int32_t big_uncapped;
  /* with cae_options_t.timing: the Schur updates of every wave (after the
     triangular solves; their flops are schur_flops) */
  int32_t schur_launches;
  double schur_ms;          /* summed device time of those launches */
} cae_stats_t;

int cae_get_stats(cae_handle_t h, cae_stats_t* s);
/* Host wall time of one level of the last factorization (level < K: from the
 * end of the previous level until its ranks were read back; level = K: the
 * dense remainder and the final read-backs).  The levels sum to factor_ms. */
int cae_get_level_ms(cae_handle_t h, int32_t level, double* ms);
/* Ranks r_i of a factored level (host, M entries, block index order). */
int cae_get_ranks(cae_handle_t h, int32_t level, int32_t* ranks);
/* Block sizes b_i of a factored level (host, M entries). */
int cae_get_sizes(cae_handle_t h, int32_t level, int32_t* sizes);
/* Dropped energy ||E_i||_F^2 of every step of a factored level (host, M
 * doubles, block index order; 0 where nothing was compressed): the terms of
 * cae_stats_t.dropped_sq, for which ||A0 - M||_F^2 = 2 sum_i ||E_i||_F^2
 * (every step is an orthogonal change of basis followed by an exact
 * elimination, Proposition 2.1). */
int cae_get_drops(cae_handle_t h, int32_t level, double* e);
/*
 * Write the factor to a file for parity checks and offline inspection
 * (little-endian binary; T = float or double as the factor's precision, int32
 * unless noted): "CAEFACT1"; esize (4 | 8), K; int64 n, int64 coarse_dim;
 * double tau; perm[n]; then per factored level l < K: M, nslots; sizes[M],
 * ranks[M]; slot_p[nslots], slot_q[nslots]; int64 slot_off[nslots + 1]; T
 * arena[slot_off[nslots]] (the in-place factor: slot (p, q), p <= q, is a
 * row-major b_p x b_q block; after step i the rows n_i = b_i - r_i (trailing)
 * of block i's close views hold L(c, n_i)^T and the trailing n_i x n_i part of
 * the diagonal slot L_nn, lower triangle); int64 u_off[M + 1]; T U[u_off[M]]
 * (U_i row-major b_i x b_i, columns by decreasing singular value); T
 * Li[u_off[M]] (L_nn^{-1}, n_i x n_i, row-major); parent[M],
 * off_in_parent[M] (where block i's r_i basis unknowns sit in the next level);
 * order[M] (elimination order); finally the dense remainder A_K and -A_K^{-1}
 * (double, coarse_dim^2 each, row-major).  Errors: CAE_EINVAL when the file
 * cannot be written.
 */
int cae_export_factor(cae_handle_t h, const char* path);
void cae_destroy(cae_handle_t h);

/*
 * Rank-predicting MLP of the LEARNED mode: 16 features -> 64 -> 64 -> 1,
 * ReLU, output z ~ r_i / b_i; the predicted rank is ceil(b_i z) clamped to
 * [0, b_i].  Parameters (FP32, DEVICE, cae_mlp_param_count() floats): feature
 * mean[16], std[16], W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Records (DEVICE, n rows of CAE_RECORD_WIDTH floats) come from a
 * factorization with cae_options_t.record; rows with a negative label are
 * skipped.
 */
int32_t cae_mlp_param_count(void);
/* Sets the feature mean/std from the records, then runs `epochs` full-batch
 * Adam steps (learning rate lr) on 0.5 mean (z - label)^2 from the given
 * weights.  *loss (host) receives the loss of the last step. */
int cae_mlp_train(const float* records, int64_t n, float* params, int32_t epochs, float lr,
                  float* loss, void* stream);
/* Loss and gradient (DEVICE grad, cae_mlp_param_count() floats, zero for the
 * normalisation entries) at the given parameters, FP32. */
int cae_mlp_loss_grad(const float* params, const float* records, int64_t n, float* grad,
                      float* loss, void* stream);
/* z for every record (DEVICE, n floats), FP64 arithmetic as in the factorization. */
int cae_mlp_predict(const float* params, const float* records, int64_t n, float* z, void* stream);

/* Message of the last failing call: h = NULL gives the calling thread's last
 * failure (any entry point, valid until the thread's next failing call);
 * otherwise the last failure of a call on that handle (empty if none), valid
 * until the handle's next failing call or its destruction. */
const char* cae_last_error(cae_handle_t h);

#ifdef __cplusplus
}
#endif
#endif /* CAE_H_ */
