// Launch interfaces of the HIP kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cae_internal.h"

namespace cae {

// Largest dynamic LDS allocation of one workgroup (set from the device).
size_t max_lds_bytes();
void set_max_lds_bytes(size_t b);

template <typename T>
struct LevelArgs {
  T* arena;                 // slots of the level
  const int64_t* slot_off;  // element offset of every slot
  const int32_t* bsz;       // block sizes b_i
  T* U;                     // U_i, b_i x b_i row-major
  const int64_t* u_off;
  T* Li;                    // L_nn^{-1} of every step, n_i x n_i row-major at u_off
  int32_t* rank;            // r_i (written by the compression of step i)
  double* edrop;            // ||E_i||_F^2
  double* minpiv;           // smallest diagonal entry of the Cholesky factor of S_ii
  const Step* steps;
  const View* views;
  const Item* items;        // set per kernel (rotation or triangular-solve items)
  const Item* rot;
  const Item* trsm;
  const Pair* pairs;
  int32_t* err;             // [0] non-SPD flag, [1] block
  const double* theta;      // eps * max diag(A0)
  int32_t rank_mode;        // 0 CE(eps), 1 CE(r)
  int32_t fixed_rank;
  int64_t* dbg;             // optional per-block compression counters (8 per block) or null
  int32_t small_by_wave;    // blocks of at most this size are compressed by the wavefront kernel
  // learned-rank compression (sketch + MLP) and training-data recording
  const float* mlp;         // MLP parameters (MLP_NPARAM floats) or null
  uint64_t seed;            // Philox key of the sketches
  int32_t level;            // level index (0-based), part of the sketch counter
  int32_t feat_only;        // 1: the sketch kernel only records features and defers every step
  float* rec;               // REC_W floats per block: 16 features, label r/b (or -1), or null
  int64_t rec_off;          // first record row of this level
  int32_t* need_exact;      // per block: 1 = the exact compression must take the step, or null
  int32_t* lcount;          // [0] sketches accepted, [1] sketches rejected
  int32_t bf16_schur;       // FP32 factor: Schur products with BF16 inputs on the matrix cores
  int32_t compensate;       // add |E_i| to the diagonals (k_compensate) instead of plain dropping
  // big-block compression (blocks above 128 unknowns): per-step scratch of
  // the wave (Gram matrix, pivoted Cholesky rows, U_i in FP64, work),
  // bg_stride(bmax) doubles per step of the wave, or null
  double* big;
  int64_t big_stride;
  int32_t* big_fail;        // per block: 1 = left to k_bg_full (then the generic kernel), 2 = to k_bg_cert
  int32_t bg_cap;           // most pivoted Cholesky rows (<= BG_MA)
  int32_t* bg_count;        // [0] untruncated, [1] Frobenius-accepted, [2] certified, [3] generic
  int32_t big_retry;        // generic compression: only the blocks flagged in big_fail
  // learned ranks by a capped rank-revealing factorization (LEARNED_CAP)
  int32_t* lwidth;          // per block: the MLP's width, caps the pivoted Cholesky; or null
};

// doubles of big-block compression scratch per step of a wave
int64_t bg_stride(int bmax);

// learned rank: feature count, record width, MLP parameter layout (floats):
// mean[16], std[16], W1[64x16], b1[64], W2[64x64], b2[64], w3[64], b3
constexpr int NFEAT = 16;
constexpr int REC_W = NFEAT + 1;
constexpr int MLP_H = 64;
constexpr int MLP_OFF_MEAN = 0, MLP_OFF_STD = 16, MLP_OFF_W1 = 32, MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * NFEAT,
              MLP_OFF_W2 = MLP_OFF_B1 + MLP_H, MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H,
              MLP_OFF_W3 = MLP_OFF_B2 + MLP_H, MLP_OFF_B3 = MLP_OFF_W3 + MLP_H, MLP_NPARAM = MLP_OFF_B3 + 1;
constexpr int SKETCH_OVERSAMPLE = 8;

// Workgroup b of nb (dispatched round-robin over the eight XCDs, each with
// its own L2) mapped to a contiguous range of logical workgroups per XCD, so
// that work items adjacent in index (grid neighbours, the items of one
// elimination step) share an L2.  A bijection of [0, nb).
__device__ inline int64_t xcd_swizzle(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, rem = nb % 8, x = b % 8, k = b / 8;
  return x < rem ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

struct WaveRange {
  int32_t s0, s1;   // steps
  int32_t r0, r1;   // rotation items
  int32_t t0, t1;   // triangular-solve items
  int32_t p0, p1;   // Schur targets
  int32_t maxclose; // most close views of one step
};

template <typename T>
size_t factor_scratch_elems(int bmax);
template <typename T>
bool factor_needs_global(int bmax);
// workgroups sharing the global scratch at once (generic kernels run in chunks)
template <typename T>
int32_t scratch_group(int bmax);
// the compression of a wave, then rotation, elimination and Schur update
template <typename T>
void launch_wave_compress(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gscratch, hipStream_t stream);
// A second stream for the diagonal blocks of big steps (their rotation and
// Cholesky run while the main stream rotates the views), with the events that
// fork it from and join it to the main stream.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
// Returns the first error of the side stream's event calls (kernel launch
// errors are left to hipGetLastError).
template <typename T>
hipError_t launch_wave_rest(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gscratch, hipStream_t stream,
                            const SideStream* side = nullptr);
// The Schur updates of a wave, after launch_wave_rest.
template <typename T>
void launch_wave_schur(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gscratch, hipStream_t stream);
template <typename T>
void launch_scatter_a0(T* arena, const double* vals, const int64_t* dst, int64_t nnz, hipStream_t stream);
void launch_theta(const double* vals, const int64_t* diag_pos, int64_t n, double eps, double* out,
                  hipStream_t stream);
template <typename T>
void launch_gather_next(const Trans* items, int32_t nitems, const T* src, const int64_t* src_off,
                        const int32_t* bsz, const int32_t* rank, const int32_t* parent,
                        const int32_t* off_in_parent, T* dst, const int64_t* dst_off, const int32_t* bsz_next,
                        hipStream_t stream);
template <typename T>
void launch_coarse_assemble(const int32_t* slot_p, const int32_t* slot_q, int32_t nslots, const T* arena,
                            const int64_t* slot_off, const int32_t* bsz, const int64_t* dof_off, double* Ad,
                            int64_t dim, hipStream_t stream);
// In place: Ad (dim x dim, symmetric positive definite) -> -Ad^{-1}.
// Pinv: 64*64, W and R0: 64*dim scratch.  err[0] set on a non-positive pivot.
void launch_gj_inverse(double* Ad, int64_t dim, double* Pinv, double* W, double* R0, int32_t* err,
                       hipStream_t stream);

// ------------------------------------------------------------------ apply ---
template <typename T>
struct ApplyArgs {
  const T* arena;
  const int64_t* slot_off;
  const int32_t* bsz;
  const int32_t* rank;
  const T* U;
  const int64_t* u_off;
  const T* Li;              // L_nn^{-1} of every step (n_i x n_i at u_off)
  const int64_t* dof_off;   // first unknown of every block in the level vector
  const Step* steps;
  const View* views;
  int32_t nrhs;
};

// y_i <- U_i^T y_i (dir 0) or U_i y_i (dir 1) for every block with a far row.
template <typename T>
void launch_ap_rotate(const ApplyArgs<T>& A, int32_t nsteps, double* y, int dir, int bmax, hipStream_t stream);
// forward / backward block solves of one wave
// (waves of fewer than split_steps steps update their close blocks one
// workgroup per (step, view); the backward pass then needs `part`,
// ap_part_elems doubles, else nullptr selects the one-workgroup-per-step form)
template <typename T>
void launch_ap_fwd(const ApplyArgs<T>& A, const WaveRange& w, double* y, int bmax, int32_t split_steps,
                   hipStream_t stream);
template <typename T>
void launch_ap_bwd(const ApplyArgs<T>& A, const WaveRange& w, double* y, int bmax, double* part,
                   int32_t split_steps, hipStream_t stream);
template <typename T>
bool ap_split(const WaveRange& w, int bmax, int32_t split_steps);
size_t ap_part_elems(const WaveRange& w, int bmax, int nrhs);
// multiply: w = Lcheck^T z (all steps), out += Lcheck w (one wave)
template <typename T>
void launch_mul_w(const ApplyArgs<T>& A, int32_t nsteps, const double* z, double* w, int bmax,
                  hipStream_t stream);
template <typename T>
void launch_mul_lw(const ApplyArgs<T>& A, int32_t s0, int32_t s1, const double* w, double* out, int bmax,
                   hipStream_t stream);
// basis parts between a level vector and the next level vector
void launch_to_next(int32_t M, const int64_t* dof_off, const int32_t* rank, const int32_t* parent,
                    const int32_t* off_in_parent, const int64_t* dof_off_next, int32_t nrhs, const double* y,
                    double* ynext, int dir, hipStream_t stream);
// out = -Ainv_store * y  (Ainv_store holds -A_K^{-1})
void launch_coarse_apply(const double* Aneg_inv, int64_t dim, int32_t nrhs, const double* y, double* out,
                         hipStream_t stream);
void launch_coarse_mul(const double* Ad, int64_t dim, int32_t nrhs, const double* y, double* out,
                       hipStream_t stream);
// permutations between column-major user vectors and the level-1 layout
void launch_perm_in(int64_t n, int32_t nrhs, const int32_t* perm, const double* x, int64_t ldx, double* y,
                    hipStream_t stream);
void launch_perm_out(int64_t n, int32_t nrhs, const int32_t* perm, const double* y, double* x, int64_t ldx,
                     hipStream_t stream);

// -------------------------------------------------------------------- PCG ---
void launch_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals, int32_t nrhs,
                 const double* x, int64_t ldx, double* y, int64_t ldy, hipStream_t stream);
// out[k] = sum_i a[i + k*lda] * b[i + k*ldb]; partial: scratch of nrhs * 1024
void launch_dots(int64_t n, int32_t nrhs, const double* a, int64_t lda, const double* b, int64_t ldb,
                 double* partial, double* out, hipStream_t stream);
// x += alpha p, r -= alpha q with alpha[k] = active[k] ? rz[k] / pq[k] : 0
void launch_pcg_xr(int64_t n, int32_t nrhs, const double* rz, const double* pq, const int32_t* active,
                   double* x, int64_t ldx, const double* p, double* r, const double* q, hipStream_t stream);
// p = z + beta p with beta[k] = rz_new[k] / rz[k] (active columns), then rz = rz_new
void launch_pcg_p(int64_t n, int32_t nrhs, double* rz, const double* rz_new, const int32_t* active,
                  const double* z, double* p, double* beta, hipStream_t stream);
// Independent PCG runs of the problems of a batch: the rows of the joint
// vectors split into tiles that never straddle two problems (segments), and
// every (segment, column) lane has its own scalars, lane = k * nseg + segment.
struct SegTiles {
  const int64_t* tb;       // first row of every tile
  const int64_t* te;       // one past its last row
  const int32_t* ts;       // segment of every tile
  const int32_t* sfirst;   // first tile of every segment (nseg + 1)
  int32_t ntiles = 0, nseg = 0;
};
constexpr int SEG_TILE_ROWS = 4096;
// out[k * nseg + s] = sum over the rows of segment s of a .* b (column k), the
// tiles' partial sums added in tile order; partial: nrhs * ntiles doubles
void launch_seg_dots(const SegTiles& sg, int32_t nrhs, const double* a, int64_t lda, const double* b, int64_t ldb,
                     double* partial, double* out, hipStream_t stream);
// launch_pcg_xr / launch_pcg_p with the scalars of each row's lane
void launch_seg_pcg_xr(const SegTiles& sg, int64_t n, int32_t nrhs, const double* rz, const double* pq,
                       const int32_t* active, double* x, int64_t ldx, const double* p, double* r, const double* q,
                       hipStream_t stream);
void launch_seg_pcg_p(const SegTiles& sg, int64_t n, int32_t nrhs, double* rz, const double* rz_new,
                      const int32_t* active, const double* z, double* p, double* beta, hipStream_t stream);
// ----------------------------------------------------------------- MINRES ---
// fields of the per-column MINRES state st[f * nrhs + k]
enum {
  MR_BETA = 0, MR_OLDB, MR_DBAR, MR_EPSLN, MR_PHIBAR, MR_CS, MR_SN, MR_ALPHA, MR_BSQ, MR_OLDEPS, MR_DELTA,
  MR_GAMMA, MR_PHI, MR_NFIELDS
};
void launch_mr_v(int64_t n, int32_t nrhs, const int32_t* active, const double* st, const double* y, double* v,
                 hipStream_t stream);
void launch_mr_y(int64_t n, int32_t nrhs, const int32_t* active, const double* st, const double* r, double* y,
                 int which, hipStream_t stream);
void launch_mr_scalars(int32_t nrhs, const int32_t* active, double* st, hipStream_t stream);
// w_new = (v - oldeps w_prev2 - delta w_prev) / gamma into wout, x += phi w_new
void launch_mr_wx(int64_t n, int32_t nrhs, const int32_t* active, const double* st, const double* v,
                  const double* wprev2, const double* wprev, double* wout, double* x, int64_t ldx,
                  hipStream_t stream);
void launch_copy_cols(int64_t n, int32_t nrhs, const double* a, int64_t lda, double* b, int64_t ldb,
                      hipStream_t stream);
void launch_fill(double* a, int64_t count, double v, hipStream_t stream);
// r = b - r (true residual after r = A x)
void launch_residual(int64_t n, int32_t nrhs, const double* b, int64_t ldb, double* r, hipStream_t stream);

// ------------------------------------------------------- rank MLP training ---
void launch_mlp_stats(const float* rec, int64_t n, float* P, int* nvalid, hipStream_t s);
void launch_mlp_predict(const float* P, const float* rec, int64_t n, float* z, hipStream_t s);
void launch_mlp_grad(const float* P, const float* rec, int64_t n, float inv_n, float* grad, float* loss,
                     hipStream_t s);
void launch_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, int step, hipStream_t s);
void launch_mlp_zero(float* a, int n, hipStream_t s);

}  // namespace cae
