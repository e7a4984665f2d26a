// HIP kernels (gfx950) of the numeric CE factorization.
//
// One level of Algorithm 2 runs as a sequence of dependency waves; inside a
// wave every step (block row) is independent, and each step is split into
// five batched kernels:
//   k_compress : far row F_i -> U_i, r_i                    (eq. (rreav))
//   k_rotate   : row/column i and stored factor rows by U_i (eq. (q), (big_L))
//   k_potrf    : Cholesky of S_ii and L(basis_i, n_i)       (eq. (sm_L))
//   k_trsm     : factor panels L(c, n_i) of close blocks c  (eq. (sm_L))
//   k_schur    : Schur complement into close and far blocks (eq. (A_st))
// Every workgroup keeps its operands in LDS when they fit (the `work`
// pointer), otherwise in a global scratch slice of its own.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "cae_internal.h"
#include "kernels.h"

namespace cae {

constexpr int NT = 256;

template <typename T>
struct Eps;
template <>
struct Eps<double> {
  static __device__ double v() { return DBL_EPSILON; }
  // squared column norms below this are treated as zero by the reflectors:
  // 2 / tiny stays finite, and such columns are far below any threshold
  static __device__ double tiny() { return 1e-290; }
};
template <>
struct Eps<float> {
  static __device__ float v() { return FLT_EPSILON; }
  static __device__ float tiny() { return 1e-30f; }
};

// Element (a, c) of the view (i, x) of a step: b_i x b_x.
template <typename T>
__device__ inline T* view_ptr(T* base, int trans, int bi, int bx, int a, int c) {
  return trans ? base + (int64_t)c * bi + a : base + (int64_t)a * bx + c;
}

template <typename T>
__device__ inline T* dyn_work(T* gscratch, int64_t per_wg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (gscratch) return gscratch + per_wg * blockIdx.x;
  return reinterpret_cast<T*>(smem_raw);
}

// ---------------------------------------------------------------------------
// Compression: Householder QR of F_i^T, streamed over the far blocks in chunks
// of 64 rows ([R; C] -> R), then one-sided (Hestenes) Jacobi on the columns of
// R: R V = X S, so V holds the right singular vectors of R, which are the left
// singular vectors of F_i.  U_i = V with columns sorted by decreasing sigma.
// ---------------------------------------------------------------------------
constexpr int QR_CH = 64;
// blocks of BG_MIN..BG_MAXB unknowns: big-block compression of the FP32
// factor (k_bg_gram / k_bg_eig), at most BG_MA pivoted Cholesky rows
constexpr int BG_MIN = 129, BG_MAXB = 512, BG_MA = 128;

template <typename T>
__global__ __launch_bounds__(NT) void k_compress(LevelArgs<T> A, int32_t s0, T* gscratch, int64_t per_wg) {
  // FP64 arithmetic for either storage type (an FP32 far row is read into
  // FP64); the rounding levels below are those of the stored entries
  using W = double;
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int tid = threadIdx.x;
  if (A.small_by_wave && b <= A.small_by_wave) return;   // done by the wavefront kernel
  if (A.big_retry && b >= BG_MIN && b <= BG_MAXB && !A.big_fail[i]) return;   // settled by the big-block kernels
  T* Ug = A.U + A.u_off[i];
  if (st.nfar == 0 || b == 0) {
    for (int e = tid; e < b * b; e += NT) Ug[e] = (e / b == e % b) ? T(1) : T(0);
    if (tid == 0) {
      A.rank[i] = 0;
      A.edrop[i] = 0.0;
    }
    return;
  }
  W* work = reinterpret_cast<W*>(dyn_work<T>(gscratch, per_wg));
  const int ld = b + 1;
  W* R = work;                       // b x ld
  W* C = R + (int64_t)b * ld;        // max(QR_CH, b) x ld  (chunk, then V)
  W* part = C + (int64_t)max(QR_CH, b) * ld;   // 4 x b partial dots, then sigma
  W* cf = part + 4 * b;                        // b reflector coefficients
  for (int e = tid; e < b * ld; e += NT) R[e] = W(0);
  __syncthreads();

  const int jl = tid & 63, g = tid >> 6;   // column lane, row group (4 groups)
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    T* base = A.arena + A.slot_off[v.slot];
    for (int c0 = 0; c0 < w; c0 += QR_CH) {
      const int m = min(QR_CH, w - c0);
      // chunk row t = column c0 + t of F_i (row j of the chunk = unknown j of block i)
      for (int e = tid; e < m * b; e += NT) {
        int t = e % m, j = e / m;
        C[t * ld + j] = (W)*view_ptr(base, v.trans, b, bx, j, c0 + t);
      }
      __syncthreads();
      for (int k = 0; k < b; ++k) {
        // (a) partial dots of column k with columns j >= k over rows t = g mod 4
        for (int j = k + jl; j < b; j += 64) {
          W s = 0;
          for (int t = g; t < m; t += 4) s += C[t * ld + k] * C[t * ld + j];
          part[g * b + j] = s;
        }
        __syncthreads();
        // (b) reflector H = I - tau v v^T with v = [R_kk - alpha; C(:,k)]
        const W xn2 = part[k] + part[b + k] + part[2 * b + k] + part[3 * b + k];
        const bool reflect = xn2 > Eps<W>::tiny();
        if (reflect) {
          const W rkk = R[k * ld + k];
          const W nrm = sqrt(rkk * rkk + xn2);
          const W alpha = rkk >= W(0) ? -nrm : nrm;
          const W v0 = rkk - alpha;
          const W tau = W(2) / (v0 * v0 + xn2);
          for (int j = k + 1 + jl; j < b; j += 64) {
            const W s = v0 * R[k * ld + j] + part[j] + part[b + j] + part[2 * b + j] + part[3 * b + j];
            const W coef = tau * s;
            if (g == 0) cf[j] = coef;
            for (int t = g; t < m; t += 4) C[t * ld + j] -= coef * C[t * ld + k];
          }
        }
        __syncthreads();
        // (c) row k of R: every thread has read it; wave 0 updates it while
        // the other waves start the next column (they touch C and part only)
        if (g == 0 && reflect) {
          const W rkk = R[k * ld + k];
          const W nrm = sqrt(rkk * rkk + xn2);
          const W alpha = rkk >= W(0) ? -nrm : nrm;
          const W v0 = rkk - alpha;
          for (int j = k + 1 + jl; j < b; j += 64) R[k * ld + j] -= cf[j] * v0;
          if (jl == 0) R[k * ld + k] = alpha;
        }
      }
      __syncthreads();
    }
  }

  // one-sided Jacobi on the columns of R; V accumulates the rotations
  W* V = C;
  for (int e = tid; e < b * ld; e += NT) V[e] = (e / ld == e % ld) ? W(1) : W(0);
  // ||R||_F^2: columns below eps * ||R||_F are rounding noise of the QR; a
  // pair of two such columns is left alone (their mixing only touches
  // directions far below any resolvable singular value)
  {
    W s = 0;
    for (int e = tid; e < b * b; e += NT) {
      const W x = R[(e / b) * ld + e % b];
      s += x * x;
    }
    part[tid] = s;     // the part/cf area holds at least NT entries
  }
  __syncthreads();
  __shared__ W sh_norm2;
  if (tid == 0) {
    W s = 0;
    for (int k = 0; k < NT; ++k) s += part[k];
    sh_norm2 = s;
  }
  __syncthreads();
  const W noise = (W)Eps<T>::v() * sqrt(sh_norm2);
  // two rows that both stay below theta/64 end in the dropped set whatever
  // their mutual rotation; they are left alone
  const W negl = A.rank_mode == 0 ? max(noise, (W)(*A.theta / 64.0)) : noise;
  const int nb = b + (b & 1);
  const int npair = nb / 2;
  // rotation threshold: the computed a_p^T a_q of exactly orthogonal columns
  // carries a rounding error of a few b*eps, so the threshold must be above it
  const W tol = W(max(b, 16)) * Eps<W>::v();
  // a rotation moves the smaller row of a pair by about |d| / max(na, nc);
  // below the absolute rounding level of the stored entries and of the FP64
  // QR it is skipped (then the singular values near theta, and so the rank,
  // are those of the stored far row to that level)
  const W aerr = max(noise, W(max(b, 16)) * Eps<W>::v() * sqrt(sh_norm2));
  const int lane8 = tid & 7;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int round = 0; round < nb - 1; ++round) {
      for (int pp = tid >> 3; pp < npair; pp += NT / 8) {
        int p, q;
        if (pp == 0) {
          p = nb - 1;
          q = round;
        } else {
          p = (round + pp) % (nb - 1);
          q = (round - pp + (nb - 1)) % (nb - 1);
        }
        if (p >= b || q >= b) continue;
        W a = 0, c = 0, d = 0;
        for (int l = lane8; l < b; l += 8) {
          const W x = R[l * ld + p], y = R[l * ld + q];
          a += x * x;
          c += y * y;
          d += x * y;
        }
        for (int o = 1; o < 8; o <<= 1) {
          a += __shfl_xor(a, o, 8);
          c += __shfl_xor(c, o, 8);
          d += __shfl_xor(d, o, 8);
        }
        const W na = sqrt(a), nc = sqrt(c);
        if (d != W(0) && fabs(d) > tol * na * nc && (na > negl || nc > negl) &&
            fabs(d) > aerr * max(na, nc)) {
          const W zeta = (c - a) / (W(2) * d);
          W t;
          if (fabs(zeta) > W(1e15))
            t = W(0.5) / zeta;
          else
            t = (zeta >= W(0) ? W(1) : W(-1)) / (fabs(zeta) + sqrt(W(1) + zeta * zeta));
          const W cs = W(1) / sqrt(W(1) + t * t), sn = cs * t;
          for (int l = lane8; l < b; l += 8) {
            const W x = R[l * ld + p], y = R[l * ld + q];
            R[l * ld + p] = cs * x - sn * y;
            R[l * ld + q] = sn * x + cs * y;
            const W u = V[l * ld + p], z = V[l * ld + q];
            V[l * ld + p] = cs * u - sn * z;
            V[l * ld + q] = sn * u + cs * z;
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  // singular values = column norms; sort decreasing (ties by index)
  W* sig = part;
  for (int j = tid; j < b; j += NT) {
    W s = 0;
    for (int l = 0; l < b; ++l) s += R[l * ld + j] * R[l * ld + j];
    sig[j] = sqrt(s);
  }
  __syncthreads();
  const double theta = *A.theta;
  int r;
  if (A.rank_mode == 0) {
    int cnt = 0;
    for (int j = 0; j < b; ++j) cnt += (double)sig[j] > theta ? 1 : 0;
    r = cnt;
  } else {
    r = min(A.fixed_rank, b);
  }
  for (int j = tid; j < b; j += NT) {
    const W sj = sig[j];
    int pos = 0;
    for (int k = 0; k < b; ++k) pos += (sig[k] > sj || (sig[k] == sj && k < j)) ? 1 : 0;
    for (int l = 0; l < b; ++l) Ug[(int64_t)l * b + pos] = (T)V[l * ld + j];
    part[b + j] = (W)pos;
  }
  __syncthreads();
  if (tid == 0) {
    double e = 0.0;
    for (int j = 0; j < b; ++j)
      if ((int)part[b + j] >= r) e += (double)sig[j] * (double)sig[j];
    A.rank[i] = r;
    A.edrop[i] = e;
  }
}

// ---------------------------------------------------------------------------
// Compression, one wavefront per step (b <= 64 * NCOL).  Same mathematics as
// k_compress, organised for one 64-lane wavefront without workgroup
// barriers:
//   1. TSQR of F_i^T: lane j owns column j of a chunk of rows (registers);
//      column k is broadcast with readlane; R stays in LDS;
//   2. rows of R below eps * ||R||_F are rounding noise of the QR and are set
//      aside (their directions carry no resolvable singular value);
//   3. one-sided Jacobi on the remaining rows of R (the columns of R^T): the
//      rows converge to sigma_k v_k^T, v_k the right singular vectors of R =
//      the left singular vectors of F_i; no rotation has to be accumulated;
//   4. the r_i leading directions are completed to an orthonormal U_i by
//      Householder reflections (U_i is unique only up to rotations inside the
//      kept and the dropped subspaces, which leave the factorization intact).
// ---------------------------------------------------------------------------
constexpr int WV = 64;

__device__ inline float rdl(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double rdl(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WV);
  return v;
}

template <typename T>
struct WaveCh;
template <>
struct WaveCh<float> {
  static constexpr int CH = 64;
};
template <>
struct WaveCh<double> {
  static constexpr int CH = 32;
};

// Sum of products with four independent accumulators.
template <typename T, int N>
__device__ inline T dot_u(const T (&x)[N], const T (&y)[N]) {
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
  for (int t = 0; t < N; t += 4) {
    s0 += x[t] * y[t];
    if (t + 1 < N) s1 += x[t + 1] * y[t + 1];
    if (t + 2 < N) s2 += x[t + 2] * y[t + 2];
    if (t + 3 < N) s3 += x[t + 3] * y[t + 3];
  }
  return (s0 + s1) + (s2 + s3);
}

template <int WB>
struct WaveLd {
  static constexpr int LD = WB + 4;   // LDS row stride (16-byte aligned rows)
};

template <typename T, int WB>
size_t work_compress_wave() {
  return (size_t)2 * WB * WaveLd<WB>::LD + 4 * (size_t)WB + 16;
}

// Partial dot products over the entries t = sub, sub + LP, ... of two LDS rows.
template <typename T, int LP>
__device__ inline void pair_dots(const T* x, const T* y, int b, int sub, T& a, T& c, T& d) {
  T a0 = 0, c0 = 0, d0 = 0, a1 = 0, c1 = 0, d1 = 0;
  int t = sub;
  for (; t + LP < b; t += 2 * LP) {
    const T x0 = x[t], y0 = y[t], x1 = x[t + LP], y1 = y[t + LP];
    a0 += x0 * x0;
    c0 += y0 * y0;
    d0 += x0 * y0;
    a1 += x1 * x1;
    c1 += y1 * y1;
    d1 += x1 * y1;
  }
  if (t < b) {
    const T x0 = x[t], y0 = y[t];
    a0 += x0 * x0;
    c0 += y0 * y0;
    d0 += x0 * y0;
  }
  a = a0 + a1;
  c = c0 + c1;
  d = d0 + d1;
}

template <typename T, int WB>
__global__ __launch_bounds__(WV) void k_compress_wave(LevelArgs<T> A, int32_t s0) {
  constexpr int NCOL = WB / WV;                    // columns of F_i^T per lane in the TSQR
  constexpr int CH = WaveCh<T>::CH / NCOL;         // rows of F_i^T per TSQR chunk
  constexpr int LD = WaveLd<WB>::LD;
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b > WB || (WB > WV && b <= WB / 2)) return;   // another size class handles it
  const int lane = threadIdx.x;
  T* Ug = A.U + A.u_off[i];
  if (st.nfar == 0 || b == 0) {
    for (int e = lane; e < b * b; e += WV) Ug[e] = (e / b == e % b) ? T(1) : T(0);
    if (lane == 0) {
      A.rank[i] = 0;
      A.edrop[i] = 0.0;
    }
    return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* R = reinterpret_cast<T*>(smem_raw);  // WB x LD: R, the active rows X, then Q
  T* Bv = R + WB * LD;                    // WB x LD: broadcast row, then kept directions / reflectors
  T* sg = Bv + WB * LD;                   // singular values
  T* tau = sg + WB;
  int* posv = reinterpret_cast<int*>(tau + WB);
  for (int e = lane; e < WB * LD; e += WV) R[e] = T(0);
  __syncthreads();
  const int64_t t_start = clock64();
  int wtot = 0;

  // ---- 1. TSQR: lane j keeps columns j, j+64, ... of the chunk in registers --
  T* bc = Bv;
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    wtot += w;
    for (int c0 = 0; c0 < w; c0 += CH) {
      const int m = min(CH, w - c0);
      T c[NCOL][CH];
#pragma unroll
      for (int ci = 0; ci < NCOL; ++ci) {
        const int j = lane + WV * ci;
#pragma unroll
        for (int t = 0; t < CH; ++t) c[ci][t] = (j < b && t < m) ? *view_ptr(base, v.trans, b, bx, j, c0 + t) : T(0);
      }
      for (int k = 0; k < b; ++k) {
        const int kl = k % WV, kc = k / WV;
        if (lane == kl) {
#pragma unroll
          for (int t = 0; t < CH; ++t) bc[t] = (kc == 0) ? c[0][t] : c[NCOL - 1][t];
        }
        __syncthreads();
        T ck[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) ck[t] = bc[t];
        T sdot[NCOL];
#pragma unroll
        for (int ci = 0; ci < NCOL; ++ci) sdot[ci] = dot_u(ck, c[ci]);
        const T xn2 = rdl(kc == 0 ? sdot[0] : sdot[NCOL - 1], kl);
        if (xn2 > Eps<T>::tiny()) {
          const T rkk = R[k * LD + k];
          const T nrm = sqrt(rkk * rkk + xn2);
          const T alpha = rkk >= T(0) ? -nrm : nrm;
          const T v0 = rkk - alpha;
          const T tk = T(2) / (v0 * v0 + xn2);
#pragma unroll
          for (int ci = 0; ci < NCOL; ++ci) {
            const int j = lane + WV * ci;
            T coef = T(0);
            if (j > k && j < b) {
              coef = tk * (v0 * R[k * LD + j] + sdot[ci]);
              R[k * LD + j] -= coef * v0;
            }
#pragma unroll
            for (int t = 0; t < CH; ++t) c[ci][t] -= coef * ck[t];
          }
          __syncthreads();
          if (lane == kl) R[k * LD + k] = alpha;
        }
        __syncthreads();
      }
    }
  }
  const int64_t t_qr = clock64();

  // ---- 2. active rows ---------------------------------------------------------
  T rn[NCOL];
  T fro = 0;
#pragma unroll
  for (int ci = 0; ci < NCOL; ++ci) {
    const int k = lane + WV * ci;
    T s2 = 0;
    for (int j = k; j < b; ++j) s2 += R[k * LD + j] * R[k * LD + j];   // rows >= b are zero
    rn[ci] = k < b ? s2 : T(0);
    fro += rn[ci];
  }
  fro = wave_sum(fro);
  const T noise = Eps<T>::v() * sqrt(fro);
  const T negl = A.rank_mode == 0 ? max(noise, (T)(*A.theta / 64.0)) : noise;
  uint64_t mask[NCOL];
  int before[NCOL];
  int ma = 0;
  double inactive = 0.0;
#pragma unroll
  for (int ci = 0; ci < NCOL; ++ci) {
    const int k = lane + WV * ci;
    const bool act = k < b && sqrt(rn[ci]) > noise;
    mask[ci] = __ballot(act);
    before[ci] = ma + __popcll(mask[ci] & ((1ull << lane) - 1ull));
    ma += __popcll(mask[ci]);
    if (k < b && !act) inactive += (double)rn[ci];
  }
  inactive = wave_sum(inactive);
  T* X = R;
  // compact in place, 16 columns at a time: every lane loads before any stores
#pragma unroll
  for (int ci = 0; ci < NCOL; ++ci) {
    const int k = lane + WV * ci;
    const bool act = (mask[ci] >> lane) & 1ull;
    for (int j0 = 0; j0 < b; j0 += 16) {
      T tmp[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) tmp[t] = (j0 + t < LD) ? R[k * LD + j0 + t] : T(0);
      __syncthreads();
      if (act) {
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (j0 + t < LD) X[before[ci] * LD + j0 + t] = tmp[t];
      }
      __syncthreads();
    }
  }
  const int64_t t_cmp = clock64();

  // ---- 3. one-sided Jacobi: LP lanes rotate the pair (p, q) of round rho ------
  const int mm = ma + (ma & 1);
  const T tol = T(max(b, 16)) * Eps<T>::v();
  // a rotation moves the smaller row of a pair by about |d| / max(na, nc);
  // below the QR's own absolute rounding level (tol * ||R||) it is skipped
  const T aerr = A.rank_mode == 0 ? max(noise, min(T(max(b, 16)) * noise, (T)(*A.theta / 32.0)))
                                  : T(max(b, 16)) * noise;
  const int LPs = (mm / 2 <= 16) ? 4 : ((mm / 2 <= 32) ? 2 : 1);
  const int pp = lane / LPs, sub = lane % LPs;
  int nsweep = 0;
  for (int sweep = 0; sweep < 40 && ma > 1; ++sweep) {
    ++nsweep;
    int rotated = 0;
    for (int rho = 0; rho < mm - 1; ++rho) {
      for (int pbase = 0; pbase < mm / 2; pbase += WV / LPs) {
        const int mypair = pbase + pp;
        int p = -1, q = -1;
        if (mypair < mm / 2) {
          if (mypair == 0) {
            p = mm - 1;
            q = rho;
          } else {
            p = (rho + mypair) % (mm - 1);
            q = (rho - mypair + (mm - 1)) % (mm - 1);
          }
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          if (q >= ma) p = -1;
        }
        T a = 0, cc = 0, d = 0;
        if (p >= 0) {
          if (LPs == 4)
            pair_dots<T, 4>(X + p * LD, X + q * LD, b, sub, a, cc, d);
          else if (LPs == 2)
            pair_dots<T, 2>(X + p * LD, X + q * LD, b, sub, a, cc, d);
          else
            pair_dots<T, 1>(X + p * LD, X + q * LD, b, sub, a, cc, d);
        }
        for (int o = 1; o < LPs; o <<= 1) {
          a += __shfl_xor(a, o, WV);
          cc += __shfl_xor(cc, o, WV);
          d += __shfl_xor(d, o, WV);
        }
        if (p >= 0) {
          const T na = sqrt(a), nc = sqrt(cc);
          if (d != T(0) && fabs(d) > tol * na * nc && (na > negl || nc > negl) &&
            fabs(d) > aerr * max(na, nc)) {
            const T zeta = (cc - a) / (T(2) * d);
            T tt;
            if (fabs(zeta) > T(1e15))
              tt = T(0.5) / zeta;
            else
              tt = (zeta >= T(0) ? T(1) : T(-1)) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
            const T cs = T(1) / sqrt(T(1) + tt * tt), sn = cs * tt;
            T* xp = X + p * LD;
            T* xq = X + q * LD;
            for (int t = sub; t < b; t += LPs) {
              const T x = xp[t], y = xq[t];
              xp[t] = cs * x - sn * y;
              xq[t] = sn * x + cs * y;
            }
            rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  const int64_t t_jac = clock64();

  // ---- singular values, order, rank -----------------------------------------
  for (int p = lane; p < ma; p += WV) {
    T s2 = 0;
    for (int t = 0; t < b; ++t) s2 += X[p * LD + t] * X[p * LD + t];
    sg[p] = sqrt(s2);
  }
  __syncthreads();
  for (int p = lane; p < ma; p += WV) {
    const T sp = sg[p];
    int pos = 0;
    for (int q = 0; q < ma; ++q) pos += (sg[q] > sp || (sg[q] == sp && q < p)) ? 1 : 0;
    posv[p] = pos;
  }
  __syncthreads();
  const double theta = *A.theta;
  int r;
  double edrop = 0.0;
  {
    int cnt = 0;
    for (int p = lane; p < ma; p += WV) cnt += (double)sg[p] > theta ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, WV);
    r = A.rank_mode == 0 ? cnt : min(A.fixed_rank, b);
    for (int p = lane; p < ma; p += WV)
      if (posv[p] >= r) edrop += (double)sg[p] * (double)sg[p];
    edrop = wave_sum(edrop) + inactive;
  }

  // ---- 4. orthonormal completion of the kb leading directions ----------------
  const int kb = min(r, ma);
  for (int p = 0; p < ma; ++p) {
    const int c2 = posv[p];
    if (c2 < kb) {
      const T inv = sg[p] > T(0) ? T(1) / sg[p] : T(0);
      for (int t = lane; t < LD; t += WV) Bv[c2 * LD + t] = t < b ? X[p * LD + t] * inv : T(0);
    }
  }
  __syncthreads();
  for (int cv = 0; cv < kb; ++cv) {
    T loc = 0;
    for (int t = cv + lane; t < b; t += WV) loc += Bv[cv * LD + t] * Bv[cv * LD + t];
    const T nrm2 = wave_sum(loc);
    const T x0 = Bv[cv * LD + cv];
    const T nrm = sqrt(nrm2);
    const T alpha = x0 >= T(0) ? -nrm : nrm;
    const T v0 = x0 - alpha;
    const T vv = v0 * v0 + (nrm2 - x0 * x0);
    const T tc = vv > T(0) ? T(2) / vv : T(0);
    __syncthreads();
    if (lane == 0) {
      Bv[cv * LD + cv] = v0;
      tau[cv] = tc;
    }
    for (int t = lane; t < cv; t += WV) Bv[cv * LD + t] = T(0);
    __syncthreads();
    for (int c2 = cv + 1 + lane; c2 < kb; c2 += WV) {
      T dd = 0;
      for (int t = cv; t < b; ++t) dd += Bv[cv * LD + t] * Bv[c2 * LD + t];
      dd *= tc;
      for (int t = cv; t < b; ++t) Bv[c2 * LD + t] -= dd * Bv[cv * LD + t];
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{kb-1}: lane col updates column col (in X's space)
  T* Q = X;
  for (int e = lane; e < WB * LD; e += WV) Q[e] = (e / LD == e % LD) ? T(1) : T(0);
  __syncthreads();
  for (int cv = kb - 1; cv >= 0; --cv) {
    const T tc = tau[cv];
    for (int col = lane; col < b; col += WV) {
      T dd = 0;
      for (int t = cv; t < b; ++t) dd += Bv[cv * LD + t] * Q[t * LD + col];
      dd *= tc;
      for (int t = cv; t < b; ++t) Q[t * LD + col] -= dd * Bv[cv * LD + t];
    }
    __syncthreads();
  }
  for (int e = lane; e < b * b; e += WV) Ug[e] = Q[(e / b) * LD + e % b];
  if (lane == 0) {
    A.rank[i] = r;
    A.edrop[i] = edrop;
    if (A.dbg) {
      int64_t* dd = A.dbg + 72 * (int64_t)i;
      dd[0] = ma;
      dd[1] = nsweep;
      dd[2] = wtot;
      dd[3] = b;
      dd[4] = t_qr - t_start;
      dd[5] = t_cmp - t_qr;
      dd[6] = t_jac - t_cmp;
      dd[7] = clock64() - t_jac;
    }
  }
}

// Phases shared by the cooperative compression kernels: one-sided Jacobi on
// the ma rows of X (their Gram matrix is F_i F_i^T, up to the coordinate
// permutation piv, or none), singular values, rank, ||E_i||_F^2, and the
// orthonormal completion of the kept directions into U_i (Householder), all
// in the compute type CT; U_i is written in the factor type T.
template <typename CT, typename T>
__device__ void jacobi_basis_wg(const LevelArgs<T>& A, int i, int b, int ma, CT* X, CT* R, int LD, const int* piv,
                                double inactive, CT negl, CT aerr, CT* sg, CT* tau, int* posv, int* shi, double* shd,
                                T* Ug, int wtot, int64_t t_start, int64_t t_qr, int64_t t_cmp, int ncoord = -1,
                                const CT* Qm = nullptr, double out2 = -1.0) {
  if (ncoord < 0) ncoord = b;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // ---- 3. one-sided Jacobi on the ma rows of X ------------------------------
  const int mm = ma + (ma & 1);
  const CT tol = CT(max(b, 16)) * Eps<CT>::v();
  const int LP = (mm / 2 <= 16) ? 16 : 8;   // lanes per pair (power of two, divides 64)
  const int pp = tid / LP, sub = tid % LP;
  int nsweep = 0;
  for (int sweep = 0; sweep < 40 && ma > 1; ++sweep) {
    ++nsweep;
    int rotated = 0;
    for (int rho = 0; rho < mm - 1; ++rho) {
      int p = -1, q = -1;
      if (pp < mm / 2) {
        if (pp == 0) {
          p = mm - 1;
          q = rho;
        } else {
          p = (rho + pp) % (mm - 1);
          q = (rho - pp + (mm - 1)) % (mm - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q >= ma) p = -1;
      }
      CT a = 0, cc = 0, d = 0;
      if (p >= 0) {
        for (int t = sub; t < ncoord; t += LP) {
          const CT x = X[p * LD + t], y = X[q * LD + t];
          a += x * x;
          cc += y * y;
          d += x * y;
        }
      }
      for (int o = 1; o < LP; o <<= 1) {
        a += __shfl_xor(a, o, WV);
        cc += __shfl_xor(cc, o, WV);
        d += __shfl_xor(d, o, WV);
      }
      if (p >= 0) {
        const CT na = sqrt(a), nc = sqrt(cc);
        if (d != CT(0) && fabs(d) > tol * na * nc && (na > negl || nc > negl) &&
            fabs(d) > aerr * max(na, nc)) {
          const CT zeta = (cc - a) / (CT(2) * d);
          CT tt;
          if (fabs(zeta) > CT(1e15))
            tt = CT(0.5) / zeta;
          else
            tt = (zeta >= CT(0) ? CT(1) : CT(-1)) / (fabs(zeta) + sqrt(CT(1) + zeta * zeta));
          const CT cs = CT(1) / sqrt(CT(1) + tt * tt), sn = cs * tt;
          for (int t = sub; t < ncoord; t += LP) {
            const CT x = X[p * LD + t], y = X[q * LD + t];
            X[p * LD + t] = cs * x - sn * y;
            X[q * LD + t] = sn * x + cs * y;
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  const int64_t t_jac = clock64();

  // ---- singular values, order, rank -----------------------------------------
  if (wv == 0) {
    CT s2 = 0;
    if (lane < ma)
      for (int t = 0; t < ncoord; ++t) s2 += X[lane * LD + t] * X[lane * LD + t];
    if (lane < ma) sg[lane] = sqrt(s2);
  }
  __syncthreads();
  if (wv == 0) {
    int pos = 0;
    if (lane < ma) {
      const CT sp = sg[lane];
      for (int q = 0; q < ma; ++q) pos += (sg[q] > sp || (sg[q] == sp && q < lane)) ? 1 : 0;
      posv[lane] = pos;
    }
    const double theta = *A.theta;
    const int cnt = __popcll(__ballot(lane < ma && (double)sg[lane] > theta));
    const int r = A.rank_mode == 0 ? cnt : min(A.fixed_rank, b);
    const double ed = wave_sum((lane < ma && pos >= r) ? (double)sg[lane] * (double)sg[lane] : 0.0);
    // largest dropped singular value (the sketch's a-posteriori check)
    double nx = (lane < ma && pos == r) ? (double)sg[lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) nx = fmax(nx, __shfl_xor(nx, o, WV));
    if (lane == 0) {
      shi[1] = r;
      shd[2] = ed + inactive + (out2 > 0.0 ? out2 : 0.0);
      shi[2] = (out2 >= 0.0 && out2 + nx * nx > theta * theta) ? 1 : 0;
    }
  }
  __syncthreads();
  if (shi[2]) {   // sketch rejected: the exact compression takes the step
    if (threadIdx.x == 0) {
      A.need_exact[i] = 1;
      atomicAdd(A.lcount + 1, 1);
    }
    return;
  }
  if (out2 >= 0.0 && threadIdx.x == 0) atomicAdd(A.lcount, 1);
  const int r = shi[1];
  const int kb = min(r, ma);
  if (A.rec) {
    // training label: the smallest sketch width k >= r that an ideal sketch
    // would need to pass the check, tail(k) + (k > r ? sigma_r^2 : 0) <= theta^2,
    // tail(k) = sum of sigma_j^2 over positions j >= k plus the inactive energy
    if (wv == 0) {
      if (lane < ma) tau[posv[lane]] = sg[lane] * sg[lane];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane == 0) {
        const double th2 = (*A.theta) * (*A.theta);
        const double sr2 = r < ma ? (double)tau[r] : 0.0;
        double tail = inactive;
        int kf = ma;
        for (int k = ma; k >= r; --k) {   // tail = sum over positions >= k
          if (k < ma) tail += (double)tau[k];
          if (tail + (k > r ? sr2 : 0.0) <= th2) kf = k;
        }
        shi[3] = max(kf, r);
      }
    }
    __syncthreads();
  }

  // ---- 4. orthonormal completion ----------------------------------------------
  CT* Bv = R;   // R is free: the kept directions, then the reflectors
  for (int e = tid; e < ma * 64; e += NT) {
    const int p = e >> 6, t = e & 63;
    const int c2 = posv[p];
    if (c2 < kb) {
      const CT inv = sg[p] > CT(0) ? CT(1) / sg[p] : CT(0);
      if (Qm) {          // sketch coordinates -> block coordinates
        CT s = 0;
        if (t < b)
          for (int u = 0; u < ncoord; ++u) s += Qm[t * LD + u] * X[p * LD + u];
        Bv[c2 * LD + t] = s * inv;
      } else if (t < b) {
        Bv[c2 * LD + (piv ? piv[t] : t)] = X[p * LD + t] * inv;
      } else {
        Bv[c2 * LD + t] = CT(0);
      }
    }
  }
  __syncthreads();
  for (int cv = 0; cv < kb; ++cv) {
    if (wv == 0) {
      const CT x = (lane >= cv && lane < b) ? Bv[cv * LD + lane] : CT(0);
      const CT nrm2 = wave_sum(x * x);
      const CT x0 = Bv[cv * LD + cv];
      const CT nrm = sqrt(nrm2);
      const CT alpha = x0 >= CT(0) ? -nrm : nrm;
      const CT v0 = x0 - alpha;
      const CT vv = v0 * v0 + (nrm2 - x0 * x0);
      if (lane < cv) Bv[cv * LD + lane] = CT(0);
      if (lane == cv) {
        Bv[cv * LD + cv] = v0;
        tau[cv] = vv > CT(0) ? CT(2) / vv : CT(0);
      }
    }
    __syncthreads();
    // apply H_cv to the later vectors: 16 lanes per vector
    {
      const CT tc = tau[cv];
      for (int c2 = cv + 1 + tid / 16; c2 - tid / 16 < kb; c2 += NT / 16) {
        const int sb = tid % 16;
        CT dd = 0;
        if (c2 < kb)
          for (int t = cv + sb; t < b; t += 16) dd += Bv[cv * LD + t] * Bv[c2 * LD + t];
        for (int o = 1; o < 16; o <<= 1) dd += __shfl_xor(dd, o, WV);
        if (c2 < kb)
          for (int t = cv + sb; t < b; t += 16) Bv[c2 * LD + t] -= tc * dd * Bv[cv * LD + t];
      }
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{kb-1}: 4 lanes per column
  CT* Q = X;
  for (int e = tid; e < 64 * LD; e += NT) Q[e] = (e / LD == e % LD) ? CT(1) : CT(0);
  __syncthreads();
  for (int cv = kb - 1; cv >= 0; --cv) {
    const CT tc = tau[cv];
    const int col = tid >> 2, sb = tid & 3;
    CT dd = 0;
    for (int t = cv + sb; t < b; t += 4) dd += Bv[cv * LD + t] * Q[t * LD + col];
    dd += __shfl_xor(dd, 1, WV);
    dd += __shfl_xor(dd, 2, WV);
    for (int t = cv + sb; t < b; t += 4) Q[t * LD + col] -= tc * dd * Bv[cv * LD + t];
    __syncthreads();
  }
  for (int e = tid; e < b * b; e += NT) Ug[e] = (T)Q[(e / b) * LD + e % b];
  if (A.dbg && tid < ma && tid < 64) {
    double* sv = reinterpret_cast<double*>(A.dbg + 72 * (int64_t)i + 8);
    sv[tid] = (double)sg[tid];
  }
  if (tid == 0) {
    A.rank[i] = r;
    A.edrop[i] = shd[2];
    if (A.rec) A.rec[(A.rec_off + i) * REC_W + NFEAT] = (float)shi[3] / (float)b;
    if (A.dbg) {
      int64_t* dd = A.dbg + 72 * (int64_t)i;
      dd[0] = ma;
      dd[1] = nsweep;
      dd[2] = wtot;
      dd[3] = b;
      dd[4] = t_qr - t_start;
      dd[5] = t_cmp - t_qr;
      dd[6] = t_jac - t_cmp;
      dd[7] = clock64() - t_jac;
    }
  }
}

// ---------------------------------------------------------------------------
// Compression by one 256-thread workgroup per step (b <= 64): the same four
// phases as k_compress_wave, with the four wavefronts cooperating so that a
// single step finishes sooner (a wave's compression time is set by its
// slowest step):
//   TSQR  : wavefront w owns rows w*RW .. w*RW+RW-1 of each chunk, lane j
//           column j; one barrier per column (partial dots double-buffered);
//   Jacobi: LP = 8 or 16 lanes per row pair, shuffle-reduced dots;
//   basis : reflectors and Q built by all threads.
// ---------------------------------------------------------------------------
template <typename T>
size_t work_compress_wg() {
  constexpr int LD = WaveLd<64>::LD;
  return (size_t)2 * 64 * LD + 2 * 4 * 64 + 4 * WaveCh<T>::CH + 4 * 64 + 16;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_compress_wg(LevelArgs<T> A, int32_t s0) {
  constexpr int CH = WaveCh<T>::CH;   // chunk rows (FP32 64, FP64 32)
  constexpr int RW = CH / 4;          // rows per wavefront
  constexpr int LD = WaveLd<64>::LD;
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  if (A.need_exact && !A.need_exact[i]) return;   // taken by the sketch kernel
  const int b = A.bsz[i];
  if (b > 64) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T* Ug = A.U + A.u_off[i];
  if (st.nfar == 0 || b == 0) {
    for (int e = tid; e < b * b; e += NT) Ug[e] = (e / b == e % b) ? T(1) : T(0);
    if (tid == 0) {
      A.rank[i] = 0;
      A.edrop[i] = 0.0;
    }
    return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* R = reinterpret_cast<T*>(smem_raw);   // 64 x LD: R, then kept directions / reflectors
  T* X = R + 64 * LD;                      // 64 x LD: active rows, then Q
  T* part = X + 64 * LD;                   // 2 x 4 x 64 partial dots
  T* bc = part + 2 * 4 * 64;               // 4 x RW broadcast strips
  T* sg = bc + 4 * CH;                     // 64 singular values
  T* tau = sg + 64;                        // 64 reflector coefficients
  int* posv = reinterpret_cast<int*>(tau + 64);
  __shared__ double shd[4];
  __shared__ int shi[4];
  for (int e = tid; e < 64 * LD; e += NT) R[e] = T(0);
  __syncthreads();
  const int64_t t_start = clock64();
  int wtot = 0;

  // ---- 1. TSQR --------------------------------------------------------------
  T* bcw = bc + wv * RW;
  int buf = 0;
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    wtot += w;
    for (int c0 = 0; c0 < w; c0 += CH) {
      const int m = min(CH, w - c0);
      T c[RW];
#pragma unroll
      for (int t = 0; t < RW; ++t) {
        const int row = wv * RW + t;
        c[t] = (lane < b && row < m) ? *view_ptr(base, v.trans, b, bx, lane, c0 + row) : T(0);
      }
      for (int k = 0; k < b; ++k) {
        if (lane == k) {
#pragma unroll
          for (int t = 0; t < RW; ++t) bcw[t] = c[t];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        T ck[RW];
#pragma unroll
        for (int t = 0; t < RW; ++t) ck[t] = bcw[t];
        part[buf * 256 + wv * 64 + lane] = dot_u(ck, c);
        const T rkk = R[k * LD + k];
        const T rkj = R[k * LD + lane];
        __syncthreads();
        const T* pb = part + buf * 256;
        const T sdot = pb[lane] + pb[64 + lane] + pb[128 + lane] + pb[192 + lane];
        const T xn2 = pb[k] + pb[64 + k] + pb[128 + k] + pb[192 + k];
        buf ^= 1;
        if (xn2 > Eps<T>::tiny()) {
          const T nrm = sqrt(rkk * rkk + xn2);
          const T alpha = rkk >= T(0) ? -nrm : nrm;
          const T v0 = rkk - alpha;
          const T tk = T(2) / (v0 * v0 + xn2);
          const T coef = (lane > k && lane < b) ? tk * (v0 * rkj + sdot) : T(0);
#pragma unroll
          for (int t = 0; t < RW; ++t) c[t] -= coef * ck[t];
          if (wv == 0) {
            if (lane > k && lane < b) R[k * LD + lane] = rkj - coef * v0;
            if (lane == k) R[k * LD + k] = alpha;
          }
        }
        // the next column's partials go to the other buffer; row k of R is
        // read again only after further barriers
      }
      __syncthreads();
    }
  }
  const int64_t t_qr = clock64();

  // ---- 2. active rows (wave 0 measures, all copy) ----------------------------
  if (wv == 0) {
    T s2 = 0;
    if (lane < b)
      for (int j = lane; j < b; ++j) s2 += R[lane * LD + j] * R[lane * LD + j];
    const T fro = wave_sum(s2);
    const T noise = Eps<T>::v() * sqrt(fro);
    const bool act = lane < b && sqrt(s2) > noise;
    const uint64_t mask = __ballot(act);
    const double inactive = wave_sum((lane < b && !act) ? (double)s2 : 0.0);
    posv[lane] = act ? __popcll(mask & ((1ull << lane) - 1ull)) : -1;
    if (lane == 0) {
      shi[0] = __popcll(mask);
      shd[0] = inactive;
      shd[1] = (double)noise;
    }
  }
  __syncthreads();
  int ma = shi[0];
  double inactive = shd[0];
  const T noise = (T)shd[1];
  const T negl = A.rank_mode == 0 ? max(noise, (T)(*A.theta / 64.0)) : noise;
  // a Jacobi rotation moves the smaller row of a pair by about |d| / max(na, nc);
  // below the QR's absolute rounding level (b * eps * ||R||) it is skipped; in
  // CE(eps) that level is capped at theta / 32 so that it cannot add to a rank
  const T aerr = A.rank_mode == 0 ? max(noise, min(T(max(b, 16)) * noise, (T)(*A.theta / 32.0)))
                                  : T(max(b, 16)) * noise;
  for (int e = tid; e < 64 * 64; e += NT) {
    const int k = e >> 6, j = e & 63;
    const int dst = posv[k];
    if (dst >= 0) X[dst * LD + j] = R[k * LD + j];
  }

  // ---- 2b. column-pivoted QR of the active rows (a left orthogonal transform,
  // so the Gram matrix R^T R and hence the left singular vectors of the far row
  // are unchanged).  Its rows come out graded, which lets the one-sided Jacobi
  // converge in a few sweeps (Jacobi preconditioned by a pivoted QR, after
  // Drmac and Veselic).  It stops once the trailing block is below the
  // rounding level aerr; that block joins the dropped part.  Columns are
  // permuted: piv[t] is the coordinate held in column t.
  T* cn = part;                             // squared trailing column norms
  T* vh = part + 64;                        // reflector of the current column
  int* piv = reinterpret_cast<int*>(part + 192);
  __shared__ T qtau;
  {
    const int col = tid >> 2, sb = tid & 3;
    __syncthreads();
    T s2 = 0;
    if (col < b)
      for (int p = sb; p < ma; p += 4) s2 += X[p * LD + col] * X[p * LD + col];
    s2 += __shfl_xor(s2, 1, WV);
    s2 += __shfl_xor(s2, 2, WV);
    if (sb == 0 && col < 64) {
      cn[col] = col < b ? s2 : T(0);
      piv[col] = col;
    }
    __syncthreads();
    const T stop2 = aerr * aerr;
    const int kmax = min(ma, b);
    int k = 0;
    for (; k < kmax; ++k) {
      if (wv == 0) {
        const bool in = lane >= k && lane < b;
        T cv = in ? cn[lane] : T(-1);
        int ci = lane;
        const T rs = wave_sum(in ? cn[lane] : T(0));
        for (int o = 32; o > 0; o >>= 1) {
          const T ov = __shfl_xor(cv, o, WV);
          const int oi = __shfl_xor(ci, o, WV);
          if (ov > cv || (ov == cv && oi < ci)) {
            cv = ov;
            ci = oi;
          }
        }
        const bool stop = rs <= stop2;
        if (!stop) {
          const int jm = ci;
          T xk = lane < ma ? X[lane * LD + k] : T(0);
          if (jm != k) {
            const T xm = lane < ma ? X[lane * LD + jm] : T(0);
            if (lane < ma) {
              X[lane * LD + k] = xm;
              X[lane * LD + jm] = xk;
            }
            xk = xm;
            if (lane == 0) {
              const T c0 = cn[k];
              cn[k] = cn[jm];
              cn[jm] = c0;
              const int p0 = piv[k];
              piv[k] = piv[jm];
              piv[jm] = p0;
            }
          }
          const T x = (lane >= k && lane < ma) ? xk : T(0);
          const T nrm2 = wave_sum(x * x);
          const T x0 = __shfl(xk, k, WV);
          T tq = 0;
          if (nrm2 > Eps<T>::tiny()) {
            const T nrm = sqrt(nrm2);
            const T alpha = x0 >= T(0) ? -nrm : nrm;
            const T v0 = x0 - alpha;
            const T vv = v0 * v0 + (nrm2 - x0 * x0);
            tq = vv > T(0) ? T(2) / vv : T(0);
            vh[lane] = lane == k ? v0 : x;
            if (lane == k) X[k * LD + k] = alpha;
            if (lane > k && lane < ma) X[lane * LD + k] = T(0);
          } else {
            vh[lane] = T(0);
          }
          if (lane == 0) qtau = tq;
        }
        if (lane == 0) {
          shi[2] = stop ? 1 : 0;
          shd[3] = (double)rs;
        }
      }
      __syncthreads();
      if (shi[2]) break;
      // apply the reflector to the later columns, then refresh their trailing
      // norms (4 threads per column)
      const int j = k + 1 + col;
      if (j < b) {
        const T tq = qtau;
        T dd = 0;
        for (int p = k + sb; p < ma; p += 4) dd += vh[p] * X[p * LD + j];
        dd += __shfl_xor(dd, 1, WV);
        dd += __shfl_xor(dd, 2, WV);
        T t2 = 0;
        for (int p = k + sb; p < ma; p += 4) {
          const T y = X[p * LD + j] - tq * dd * vh[p];
          X[p * LD + j] = y;
          if (p > k) t2 += y * y;
        }
        t2 += __shfl_xor(t2, 1, WV);
        t2 += __shfl_xor(t2, 2, WV);
        if (sb == 0) cn[j] = t2;
      }
      __syncthreads();
    }
    if (k < kmax) inactive += shd[3];
    ma = k;
  }
  __syncthreads();
  const int64_t t_cmp = clock64();

  jacobi_basis_wg<T, T>(A, i, b, ma, X, R, LD, piv, inactive, negl, aerr, sg, tau, posv, shi, shd, Ug, wtot, t_start,
                        t_qr, t_cmp);
}

// ---------------------------------------------------------------------------
// Rotation: V_ix <- U_i^T V_ix for close and far views (far views then lose
// their rows r_i..b_i-1), D <- U_i^T D U_i for the diagonal block.
// ---------------------------------------------------------------------------
constexpr int ROT_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT) void k_rotate(LevelArgs<T> A, int32_t it0, T* gscratch, int64_t per_wg) {
  const Item item = A.items[it0 + blockIdx.x];
  const Step st = A.steps[item.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (A.small_by_wave && b <= A.small_by_wave) return;
  const int tid = threadIdx.x;
  if (b == 0) return;
  const T* Ug = A.U + A.u_off[i];
  T* work = dyn_work<T>(gscratch, per_wg);
  const int ld = b + 1;
  T* Us = work;                         // U, b x ld
  T* X = Us + (int64_t)b * ld;          // b x (ROT_TC+1)  or  b x ld for the diagonal
  for (int e = tid; e < b * b; e += NT) Us[(e / b) * ld + e % b] = Ug[e];
  if (item.view < 0) {
    T* D = A.arena + A.slot_off[i];
    T* Y = X;
    __syncthreads();
    // Y = U^T D  (D read from memory)
    for (int e = tid; e < b * b; e += NT) {
      const int a = e / b, c = e % b;
      T s = 0;
      for (int k = 0; k < b; ++k) s += Us[k * ld + a] * D[(int64_t)k * b + c];
      Y[a * ld + c] = s;
    }
    __syncthreads();
    // D = Y U, stored exactly symmetric (lower triangle mirrored)
    for (int e = tid; e < b * b; e += NT) {
      const int a = e / b, c = e % b;
      if (c > a) continue;
      T s = 0;
      for (int k = 0; k < b; ++k) s += Y[a * ld + k] * Us[k * ld + c];
      D[e] = s;
      D[(int64_t)c * b + a] = s;
    }
    return;
  }
  const View v = A.views[item.view];
  const int bx = A.bsz[v.x];
  const bool far = (item.view - st.view0) >= st.nclose;
  const int r = A.rank[i];
  T* base = A.arena + A.slot_off[v.slot];
  const int ldx = ROT_TC + 1;
  for (int c0 = 0; c0 < bx; c0 += ROT_TC) {
    const int tc = min(ROT_TC, bx - c0);
    __syncthreads();
    for (int e = tid; e < b * tc; e += NT) {
      const int a = e / tc, c = e % tc;
      X[a * ldx + c] = *view_ptr(base, v.trans, b, bx, a, c0 + c);
    }
    __syncthreads();
    for (int e = tid; e < b * tc; e += NT) {
      const int a = e / tc, c = e % tc;
      T s = 0;
      if (!(far && a >= r && !A.compensate))
        for (int k = 0; k < b; ++k) s += Us[k * ld + a] * X[k * ldx + c];
      *view_ptr(base, v.trans, b, bx, a, c0 + c) = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Elimination of S_i: Cholesky of the trailing n x n block of the rotated
// diagonal block and L(basis_i, n_i)^T = L^{-1} D[n, basis].
// ---------------------------------------------------------------------------
template <typename T>
__device__ void chol_inplace(T* S, int n, int ld, int* bad) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      T p = S[k * ld + k];
      if (!(p > T(0))) {
        *bad = 1;
        p = T(1);
      }
      S[k * ld + k] = sqrt(p);
    }
    __syncthreads();
    const T d = S[k * ld + k];
    for (int j = k + 1 + tid; j < n; j += NT) S[j * ld + k] /= d;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += NT) {
      const int j = k + 1 + e / m, l = k + 1 + e % m;
      if (l <= j) S[j * ld + l] -= S[j * ld + k] * S[l * ld + k];
    }
    __syncthreads();
  }
}

// X (n x w, ld ldx) <- L^{-1} X with L lower (n x n, ld ldl).
template <typename T>
__device__ void trsm_lower(const T* L, int ldl, T* X, int n, int w, int ldx) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    const T d = L[k * ldl + k];
    for (int c = tid; c < w; c += NT) X[k * ldx + c] /= d;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = tid; e < m * w; e += NT) {
      const int j = k + 1 + e / w, c = e % w;
      X[j * ldx + c] -= L[j * ldl + k] * X[k * ldx + c];
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_potrf(LevelArgs<T> A, int32_t s0, T* gscratch, int64_t per_wg) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (A.small_by_wave && b <= A.small_by_wave) return;
  const int r = A.rank[i];
  const int n = b - r;
  const int tid = threadIdx.x;
  if (n <= 0) return;
  T* D = A.arena + A.slot_off[i];
  T* work = dyn_work<T>(gscratch, per_wg);
  const int ld = b + 1;
  T* S = work;                      // n x ld
  T* X = S + (int64_t)n * ld;       // n x ld (basis columns)
  __shared__ int bad;
  if (tid == 0) bad = 0;
  for (int e = tid; e < n * b; e += NT) {
    const int j = e / b, c = e % b;
    const T val = D[(int64_t)(r + j) * b + c];
    if (c >= r)
      S[j * ld + (c - r)] = val;
    else
      X[j * ld + c] = val;
  }
  __syncthreads();
  chol_inplace(S, n, ld, &bad);
  if (r > 0) trsm_lower(S, ld, X, n, r, ld);
  __syncthreads();
  for (int e = tid; e < n * b; e += NT) {
    const int j = e / b, c = e % b;
    T val;
    if (c >= r)
      val = (c - r) <= j ? S[j * ld + (c - r)] : T(0);
    else
      val = X[j * ld + c];
    D[(int64_t)(r + j) * b + c] = val;
  }
  // L^{-1} for the preconditioner apply (X is free now)
  __syncthreads();
  for (int e = tid; e < n * n; e += NT) X[(e / n) * ld + e % n] = (e / n == e % n) ? T(1) : T(0);
  __syncthreads();
  trsm_lower(S, ld, X, n, n, ld);
  T* Lig = A.Li + A.u_off[i];
  for (int e = tid; e < n * n; e += NT) Lig[e] = X[(e / n) * ld + e % n];
  for (int e = tid; e < r * n; e += NT) D[(int64_t)(e / n) * b + r + e % n] = T(0);
  if (tid == 0) {
    double mp = 1e300;
    for (int k = 0; k < n; ++k) mp = fmin(mp, (double)S[k * ld + k]);
    A.minpiv[i] = mp;
    if (bad) {
      if (atomicCAS(A.err, 0, 1) == 0) A.err[1] = i;
    }
  }
}

// L(c, n_i)^T = L^{-1} V_ic[n_i, live_c] for a close block c.
constexpr int TRSM_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT) void k_trsm(LevelArgs<T> A, int32_t it0, T* gscratch, int64_t per_wg) {
  const Item item = A.items[it0 + blockIdx.x];
  const Step st = A.steps[item.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (A.small_by_wave && b <= A.small_by_wave) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const View v = A.views[item.view];
  const int bx = A.bsz[v.x];
  const int lc = v.proc ? A.rank[v.x] : bx;
  if (lc == 0) return;
  const int tid = threadIdx.x;
  const T* D = A.arena + A.slot_off[i];
  T* base = A.arena + A.slot_off[v.slot];
  T* work = dyn_work<T>(gscratch, per_wg);
  const int ld = n + 1, ldx = TRSM_TC + 1;
  T* Ls = work;                       // n x ld
  T* X = Ls + (int64_t)n * ld;        // n x ldx
  for (int e = tid; e < n * n; e += NT) {
    const int j = e / n, c = e % n;
    Ls[j * ld + c] = D[(int64_t)(r + j) * b + r + c];
  }
  for (int c0 = 0; c0 < lc; c0 += TRSM_TC) {
    const int tc = min(TRSM_TC, lc - c0);
    __syncthreads();
    for (int e = tid; e < n * tc; e += NT) {
      const int j = e / tc, c = e % tc;
      X[j * ldx + c] = *view_ptr(base, v.trans, b, bx, r + j, c0 + c);
    }
    __syncthreads();
    trsm_lower(Ls, ld, X, n, tc, ldx);
    for (int e = tid; e < n * tc; e += NT) {
      const int j = e / tc, c = e % tc;
      *view_ptr(base, v.trans, b, bx, r + j, c0 + c) = X[j * ldx + c];
    }
  }
}

// ---------------------------------------------------------------------------
// Schur complement: T(a, c) -= P_a^T P_c with P_a = rows n_i of view a
// (a = 0: basis columns of the diagonal block).
// ---------------------------------------------------------------------------
constexpr int SCH_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT) void k_schur(LevelArgs<T> A, int32_t p0, T* gscratch, int64_t per_wg) {
  const Pair pr = A.pairs[p0 + blockIdx.x];
  const Step st = A.steps[pr.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (A.small_by_wave && b <= A.small_by_wave) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int tid = threadIdx.x;
  T* D = A.arena + A.slot_off[i];
  // panel a
  int la, lc, ba = b, bc = b, ta = 0, tc_ = 0;
  T* pa;
  T* pc;
  if (pr.a == 0) {
    la = r;
    pa = D;
  } else {
    const View va = A.views[st.view0 + pr.a - 1];
    ba = A.bsz[va.x];
    la = va.proc ? A.rank[va.x] : ba;
    pa = A.arena + A.slot_off[va.slot];
    ta = va.trans;
  }
  if (pr.c == 0) {
    lc = r;
    pc = D;
  } else {
    const View vc = A.views[st.view0 + pr.c - 1];
    bc = A.bsz[vc.x];
    lc = vc.proc ? A.rank[vc.x] : bc;
    pc = A.arena + A.slot_off[vc.slot];
    tc_ = vc.trans;
  }
  if (la == 0 || lc == 0) return;
  // target accessor
  T* tbase;
  int64_t ts_a, ts_c;       // strides for (alpha, gamma)
  if (pr.a == 0) {
    if (pr.c == 0) {
      tbase = D;
      ts_a = b;
      ts_c = 1;
    } else {
      tbase = pc;           // rows 0..r-1 of view c
      ts_a = tc_ ? 1 : bc;
      ts_c = tc_ ? b : 1;
    }
  } else {
    tbase = A.arena + A.slot_off[pr.slot];
    if (pr.trans) {         // stored with the rows of x_c: (gamma, alpha)
      ts_a = 1;
      ts_c = ba;
    } else {
      ts_a = bc;
      ts_c = 1;
    }
  }
  T* work = dyn_work<T>(gscratch, per_wg);
  const int lda = la + 1, ldc = SCH_TC + 1;
  T* Pa = work;                         // n x lda
  T* Pc = Pa + (int64_t)n * lda;        // n x ldc
  for (int e = tid; e < n * la; e += NT) {
    const int t = e / la, al = e % la;
    Pa[t * lda + al] = *view_ptr(pa, ta, b, ba, r + t, al);
  }
  for (int c0 = 0; c0 < lc; c0 += SCH_TC) {
    const int tcn = min(SCH_TC, lc - c0);
    __syncthreads();
    for (int e = tid; e < n * tcn; e += NT) {
      const int t = e / tcn, gm = e % tcn;
      Pc[t * ldc + gm] = *view_ptr(pc, tc_, b, bc, r + t, c0 + gm);
    }
    __syncthreads();
    for (int e = tid; e < la * tcn; e += NT) {
      const int al = e / tcn, gm = e % tcn;
      T s = 0;
      for (int t = 0; t < n; ++t) s += Pa[t * lda + al] * Pc[t * ldc + gm];
      tbase[al * ts_a + (int64_t)(c0 + gm) * ts_c] -= s;
    }
  }
}

// ---------------------------------------------------------------------------
// Tiled variants of rotation, triangular solve and Schur update for steps
// with b_i <= 64.  Every product is C = A^T B with A (K x 64) and B (K x 64)
// staged in LDS (row stride TLD).  The Schur update, the view rotation and
// the coarse Gauss-Jordan products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64, one 16-row strip of C per wavefront, accumulators
// in dbl4); the others use register tiles: thread (ty, tx) = (tid / 16,
// tid % 16) accumulates the 4 x 4 tile rows 4ty.., columns 4tx.., so one k
// step costs 8 LDS reads for 16 FMAs.  Global tiles are moved with the thread
// mapping that makes consecutive threads touch consecutive addresses for
// either storage orientation of a view.
// ---------------------------------------------------------------------------
constexpr int TLD = 68;
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <typename TI, typename TA>
__device__ inline void gemm_tn_4x4(const TI* A, const TI* B, int K, TA acc[4][4]) {
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const TI* a = A + 4 * ty;
  const TI* bb = B + 4 * tx;
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
    TA av[4], bv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      av[q] = (TA)a[k * TLD + q];
      bv[q] = (TA)bb[k * TLD + q];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] += av[p] * bv[q];
  }
}

// accumulator type of the tiled products: FP64 for every factor precision
// (products of FP32 entries are exact in FP64, so an FP32 factor takes one
// rounding per stored entry instead of one per term)
template <typename T>
struct AccT {
  using type = double;
};

// C = A^T B with A (K x 64, type TA) and B (K x 64, type TB) in LDS, FP64 or
// FP32 accumulation in TC (the same thread tiling as gemm_tn_4x4)
template <typename TA, typename TB, typename TC>
__device__ inline void gemm_tn_4x4m(const TA* A, const TB* B, int K, TC acc[4][4]) {
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const TA* a = A + 4 * ty;
  const TB* bb = B + 4 * tx;
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
    TC av[4], bv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      av[q] = (TC)a[k * TLD + q];
      bv[q] = (TC)bb[k * TLD + q];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] += av[p] * bv[q];
  }
}

template <typename T>
__device__ inline void zero_acc(T acc[4][4]) {
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = T(0);
}

// S[a][c] = view(rows row0 + a, columns c0 + c) for a < na, c < nc (both
// <= 64): 16 slots per thread of the 64 x 64 window, the unit-stride index on
// consecutive threads, loads issued in two groups of eight before their stores.
template <typename T>
__device__ inline void load_view_tile(T* S, const T* base, int trans, int bi, int bx, int row0, int na, int c0,
                                      int nc) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + NT * (8 * h + u);
      const int a = trans ? (e & 63) : (e >> 6), c = trans ? (e >> 6) : (e & 63);
      v[u] = (a < na && c < nc)
                 ? (trans ? base[(int64_t)(c0 + c) * bi + row0 + a] : base[(int64_t)(row0 + a) * bx + c0 + c])
                 : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + NT * (8 * h + u);
      const int a = trans ? (e & 63) : (e >> 6), c = trans ? (e >> 6) : (e & 63);
      if (a < na && c < nc) S[a * TLD + c] = v[u];
    }
  }
}

// The same tile with one element per thread and iteration (fewer live
// registers: the Schur kernels keep their occupancy).
template <typename T>
__device__ inline void load_view_tile_lean(T* S, const T* base, int trans, int bi, int bx, int row0, int na, int c0,
                                           int nc) {
  if (trans) {
    for (int e = threadIdx.x; e < na * nc; e += NT) {
      const int c = e / na, a = e % na;
      S[a * TLD + c] = base[(int64_t)(c0 + c) * bi + row0 + a];
    }
  } else {
    for (int e = threadIdx.x; e < na * nc; e += NT) {
      const int a = e / nc, c = e % nc;
      S[a * TLD + c] = base[(int64_t)(row0 + a) * bx + c0 + c];
    }
  }
}

// Two view tiles (as load_view_tile_lean, operand Q into S + 64 TLD only when
// nq > 0) with their elements enumerated densely and, per round of 16 per
// thread, every load issued before the first LDS store, with 32-bit offsets
// into the views: many loads in flight for few registers.
struct TileSrc {
  int trans, bi, bx, c0, nc;
};
template <typename T>
__device__ inline void load_tile_pair(T* S, const T* pb, TileSrc P, const T* qb, TileSrc Q, int row0, int na) {
  // (predicated loads here: unconditional ones with clamped addresses
  // measured slower, holding more registers for the sixteen in flight)
  const int tp = P.nc > 0 ? na * P.nc : 0;
  const int tot = tp + (Q.nc > 0 ? na * Q.nc : 0);
  for (int e0 = 0; e0 < tot; e0 += 16 * NT) {
    T v[16];
    int so[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      int e = e0 + threadIdx.x + NT * u;
      so[u] = -1;
      if (e < tot) {
        const bool q = e >= tp;
        if (q) e -= tp;
        const TileSrc& V = q ? Q : P;
        const T* base = q ? qb : pb;
        const int ld = V.trans ? na : V.nc;
        const int x = e / ld, m = e - x * ld;
        const int a = V.trans ? m : x, c = V.trans ? x : m;
        v[u] = V.trans ? base[(V.c0 + c) * V.bi + row0 + a] : base[(row0 + a) * V.bx + V.c0 + c];
        so[u] = (q ? 64 * TLD : 0) + a * TLD + c;
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (so[u] >= 0) S[so[u]] = v[u];
  }
}

template <typename T>
__device__ inline void store_view_tile(const T* S, T* base, int trans, int bi, int bx, int row0, int na, int c0,
                                       int nc) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + NT * u;
    const int a = trans ? (e & 63) : (e >> 6), c = trans ? (e >> 6) : (e & 63);
    if (a < na && c < nc) {
      if (trans) base[(int64_t)(c0 + c) * bi + row0 + a] = S[a * TLD + c];
      else base[(int64_t)(row0 + a) * bx + c0 + c] = S[a * TLD + c];
    }
  }
}

template <typename TA, typename T>
__device__ inline void acc_to_lds(const TA acc[4][4], T* S) {
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) S[(4 * ty + p) * TLD + 4 * tx + q] = (T)acc[p][q];
}

template <typename T>
size_t work_tiled() {
  return (size_t)2 * 64 * TLD;
}

// In-place Cholesky S = L L^T of the n x n block (n <= 64, row stride TLD)
// and X <- L^{-1} (X holds the identity on entry), 256 threads, one barrier
// per column for each: the scaling of column k and the final write of row k
// of the inverse are deferred to the next column, which no longer reads them.
// A non-positive pivot sets *bad.
template <typename CT>
__device__ void chol_inv_lds(CT* S, CT* X, int n, int* bad) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  // right-looking Cholesky on the unscaled column k: S_jl -= S_jk S_lk / S_kk
  for (int k = 0; k < n; ++k) {
    const CT p = S[k * TLD + k];
    if (k > 0) {
      const CT dprev = sqrt(S[(k - 1) * TLD + (k - 1)]);
      for (int j = k + tid; j < n; j += NT) S[j * TLD + (k - 1)] /= dprev;
    }
    if (p > CT(0)) {
      const CT ip = CT(1) / p;
      for (int j = k + 1 + ty; j < n; j += 16) {
        const CT f = S[j * TLD + k] * ip;
        for (int l = k + 1 + tx; l <= j; l += 16) S[j * TLD + l] -= f * S[l * TLD + k];
      }
    } else if (tid == 0) {
      *bad = 1;
    }
    __syncthreads();
  }
  // columns 0..n-2 are scaled (column n-1 has nothing below the diagonal);
  // the diagonal still holds the pivots p_k, and L_kk = sqrt(p_k)
  for (int k = tid; k < n; k += NT) S[k * TLD + k] = sqrt(fmax(S[k * TLD + k], CT(0)));
  __syncthreads();
  // X <- L^{-1}: forward substitution, row k final in the next step
  for (int k = 0; k < n; ++k) {
    const CT lkk = S[k * TLD + k];
    if (k > 0) {
      const CT lp = S[(k - 1) * TLD + (k - 1)];
      for (int c = tid; c < k; c += NT) X[(k - 1) * TLD + c] /= lp;
    }
    for (int j = k + 1 + ty; j < n; j += 16) {
      const CT f = S[j * TLD + k] / lkk;
      for (int c = tx; c <= k; c += 16) X[j * TLD + c] -= f * X[k * TLD + c];
    }
    __syncthreads();
  }
  {
    const CT lp = S[(n - 1) * TLD + (n - 1)];
    for (int c = tid; c < n; c += NT) X[(n - 1) * TLD + c] /= lp;
  }
  __syncthreads();
}

// Diagonal compensation of the dropped E_i (rows r_i.. of the rotated far
// views): for every far block the Frobenius norm e of its dropped part is
// added to the diagonal of i's eliminated rows and of the neighbour's live
// columns, then E_i is zeroed.  M - A0 gains [[e I, -E], [-E^T, e I]] per far
// block, positive semidefinite since ||E||_2 <= e, so no pivot can fail; e
// and the identities do not depend on the bases chosen inside the kept and
// dropped subspaces.  One workgroup per step; the neighbour's diagonal may be
// shared by other steps of the wave (atomics), D_i is not.
template <typename T>
__global__ __launch_bounds__(NT) void k_compensate(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  if (st.nfar == 0 || b - r <= 0) return;
  __shared__ double red[NT / WV];
  T* D = A.arena + A.slot_off[i];
  double dsum = 0.0;   // compensation of i's eliminated rows (uniform over the workgroup)
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    T* base = A.arena + A.slot_off[v.slot];
    double s2 = 0.0;
    for (int e = threadIdx.x; e < (b - r) * w; e += NT) {
      const double x = (double)*view_ptr(base, v.trans, b, bx, r + e / w, e % w);
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    if ((threadIdx.x & (WV - 1)) == 0) red[threadIdx.x / WV] = s2;
    __syncthreads();
    const double eF = sqrt(red[0] + red[1] + red[2] + red[3]);
    __syncthreads();
    dsum += eF;
    T* Dx = A.arena + A.slot_off[v.x];
    if (eF > 0.0)
      for (int c = threadIdx.x; c < w; c += NT) atomicAdd(Dx + (int64_t)c * bx + c, (T)eF);
    for (int e = threadIdx.x; e < (b - r) * bx; e += NT) *view_ptr(base, v.trans, b, bx, r + e / bx, e % bx) = T(0);
  }
  for (int a = r + threadIdx.x; a < b; a += NT) {
    T* dp = D + (int64_t)a * b + a;
    *dp = (T)((double)*dp + dsum);
  }
}

// ---------------------------------------------------------------------------
// Compression of a reduced-precision factor (b <= 128) through the Gram matrix
// G = F_i F_i^T accumulated in FP64: products of FP32 entries are exact in
// FP64, so G carries the far row to FP64 accuracy, and its eigenvalues sigma^2
// resolve singular values down to about 1e-7 sigma_1, well below the FP32
// rounding level of F_i itself.  A pivoted Cholesky G = R^T R (pivot = largest
// remaining diagonal, the Gram form of a column-pivoted QR of F_i^T) gives
// graded rows R, stopped once the trailing diagonal sum is below the rounding
// level; the one-sided Jacobi and the completion then run in FP64 on R.
//
// The kernel is organised for the latency of one step, which bounds every
// dependency wave with fewer steps than the chip holds at once:
//   * the far row is gathered through a column map (one descriptor per far
//     view, staged in parallel), so a chunk of 64 columns of F_i mixes views
//     and its 16 loads per thread are all in flight together; the next chunk
//     is loaded while the current one is multiplied (one barrier per chunk);
//   * the pivoted Cholesky is left-looking and runs in one wavefront (no
//     workgroup barriers): row k of R is written over row p_k of G, which no
//     later pivot reads;
//   * the Jacobi rounds run in one wavefront with the pair reductions done by
//     DPP lane exchanges inside rows of 16 lanes;
//   * the reflectors of the completion are built by one wavefront, and the
//     four wavefronts then form 16 columns of U_i each with no barrier.
// Two instances: b <= 64 (LDS 48 KB, three workgroups per compute unit) and
// 64 < b <= 128 (LDS 139 KB, each lane owning two coordinates).
// ---------------------------------------------------------------------------
constexpr int GCW = 64;     // columns of F_i per staged chunk
constexpr int GVB = 256;    // far-view descriptors staged at once
constexpr int GCOLS = 512;  // columns of F_i mapped at once

constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int DPP_MIRROR8 = 0x141;      // row_half_mirror: lane i <-> 7 - i within 8
constexpr int DPP_MIRROR16 = 0x140;     // row_mirror: lane i <-> 15 - i within 16

template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)bits, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of G lanes (G = 2, 4, 8, 16), all lanes active:
// every lane of a group ends with the same bits (each stage adds two equal
// partial sums in either order).
template <int G>
__device__ inline double group_sum(double v) {
  v += dpp_f64<DPP_XOR1>(v);
  if (G >= 4) v += dpp_f64<DPP_XOR2>(v);
  if (G >= 8) v += dpp_f64<DPP_MIRROR8>(v);
  if (G >= 16) v += dpp_f64<DPP_MIRROR16>(v);
  return v;
}

// Sum over the wavefront, the same value in every lane.
__device__ inline double wave_sum_u(double v) {
  v = group_sum<16>(v);
  return (rdl(v, 0) + rdl(v, 16)) + (rdl(v, 32) + rdl(v, 48));
}

__device__ inline void amax_step(double& v, int& ix, double ov, int oi) {
  if (ov > v || (ov == v && oi < ix)) {
    v = ov;
    ix = oi;
  }
}
template <int CTRL>
__device__ inline void amax_dpp(double& v, int& ix) {
  amax_step(v, ix, dpp_f64<CTRL>(v), __builtin_amdgcn_mov_dpp(ix, CTRL, 0xF, 0xF, false));
}
// Largest value over the wavefront and its lane (ties: the lower index), the
// same in every lane.
__device__ inline void wave_argmax_u(double& v, int& ix) {
  amax_dpp<DPP_XOR1>(v, ix);
  amax_dpp<DPP_XOR2>(v, ix);
  amax_dpp<DPP_MIRROR8>(v, ix);
  amax_dpp<DPP_MIRROR16>(v, ix);
  double bv = rdl(v, 0);
  int bi = __builtin_amdgcn_readlane(ix, 0);
  amax_step(bv, bi, rdl(v, 16), __builtin_amdgcn_readlane(ix, 16));
  amax_step(bv, bi, rdl(v, 32), __builtin_amdgcn_readlane(ix, 32));
  amax_step(bv, bi, rdl(v, 48), __builtin_amdgcn_readlane(ix, 48));
  v = bv;
  ix = bi;
}

// LDS writes of one lane visible to the other lanes of its wavefront.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Elimination of the trailing n_i unknowns of a step (eq. (sm_L)), FP64
// arithmetic: the left-looking Cholesky S_ii = L L^T and the forward
// substitution L [X | P] = [I | D(n, basis)] in one pass over k, so that
// X = L^{-1} and the panel P = L(basis_i, n_i)^T come out together.  Lane j
// owns row j of L and column j of [X | P] (n + r = b <= 64 columns).  LDS:
// one 64 x 64 array W of (L column m, [X | P] row m) pairs, read as one
// 16-byte load per lane per term.
// ---------------------------------------------------------------------------
constexpr int PW_LDS = 64 * 64 * 2 * 8;

// Four wavefronts of one workgroup share W (its LDS allows two blocks per
// compute unit, so a single wavefront per block would leave half of the
// SIMDs idle): for column k, wavefront w sums the
// terms m = w, w + 4, ... < k of both quantities, the four partial sums meet
// in LDS (two alternating buffers, one barrier per column) and are combined
// in wavefront order by every wavefront; row k of W is then written by
// wavefront k mod 4, the only one that reads it again.
constexpr int PW4_LDS = PW_LDS + 2 * 4 * 64 * 16;

template <typename T>
__global__ __launch_bounds__(NT) void k_potrf_w(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b > 64) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* W = reinterpret_cast<double2*>(smem_raw);   // W[m * 64 + l] = (L(l, m), [X | P](m, l))
  double2* Pp = W + 64 * 64;                            // [2][4][64] partial sums
  T* D = A.arena + A.slot_off[i];
  T* Lig = A.Li + A.u_off[i];
  // row k of S_ii (lanes < n, from its lower triangle: column k) and of
  // D(n, basis) (lanes n .. b-1), sixteen loads in flight per thread
  for (int e0 = 0; e0 < n * 64; e0 += 16 * NT) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + tid + NT * u, k = e >> 6, l = e & 63;
      v[u] = (k < n) ? (l < n ? D[(int64_t)(r + l) * b + r + k] : (l < b ? D[(int64_t)(r + k) * b + l - n] : T(0)))
                     : T(0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + tid + NT * u, k = e >> 6, l = e & 63;
      if (k < n) {
        const double sv = (double)v[u];
        W[e] = make_double2(l < n ? sv : 0.0, l < n ? (l == k ? 1.0 : 0.0) : sv);
      }
    }
  }
  __syncthreads();
  bool ok = true;
  double mp = 1e300;
  for (int k = 0; k < n; ++k) {
    const double2 sx = W[k * 64 + lane];   // read by all before any wavefront rewrites row k
    double s0 = 0.0, x0 = 0.0, s1 = 0.0, x1 = 0.0;
    int m = wv;
    for (; m + 28 < k; m += 32) {
      double2 w[8];
      double bk[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        w[u] = W[(m + 4 * u) * 64 + lane];
        bk[u] = W[(m + 4 * u) * 64 + k].x;
      }
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        s0 += w[u].x * bk[u];
        x0 += bk[u] * w[u].y;
        s1 += w[u + 1].x * bk[u + 1];
        x1 += bk[u + 1] * w[u + 1].y;
      }
    }
    for (; m < k; m += 4) {
      const double2 w0 = W[m * 64 + lane];
      const double b0 = W[m * 64 + k].x;
      s0 += w0.x * b0;
      x0 += b0 * w0.y;
    }
    double2* pb = Pp + (k & 1) * 256;
    pb[wv * 64 + lane] = make_double2(s0 + s1, x0 + x1);
    __syncthreads();
    const double2 p0 = pb[lane], p1 = pb[64 + lane], p2 = pb[128 + lane], p3 = pb[192 + lane];
    const double s = sx.x - ((p0.x + p1.x) + (p2.x + p3.x));
    const double x = sx.y - ((p0.y + p1.y) + (p2.y + p3.y));
    const double d = rdl(s, k);
    double inv = 0.0, lkk = 0.0;
    if (d > 0.0) {
      inv = 1.0 / sqrt(d);
      lkk = d * inv;
    } else {
      ok = false;
    }
    mp = fmin(mp, lkk);
    if (wv == (k & 3)) {
      const double lv = (lane > k && lane < n) ? s * inv : (lane == k ? lkk : 0.0);
      W[k * 64 + lane] = make_double2(lv, x * inv);
    }
  }
  // results leave through W after the last column: a global store inside the
  // loop would make every barrier wait for its completion
  __syncthreads();
  for (int e = tid; e < n * 64; e += NT) {
    const int k = e >> 6, l = e & 63;
    const double2 w = W[e];
    if (l < n) {
      D[(int64_t)(r + l) * b + r + k] = (T)w.x;
      Lig[k * n + l] = (T)w.y;
    } else if (l < b) {
      D[(int64_t)(r + k) * b + (l - n)] = (T)w.y;
    }
  }
  // the basis rows of the eliminated columns are zero after the elimination
  for (int e = tid; e < r * n; e += NT) D[(int64_t)(e / n) * b + r + e % n] = T(0);
  if (tid == 0) {
    A.minpiv[i] = mp;
    if (!ok && atomicCAS(A.err, 0, 1) == 0) A.err[1] = i;
  }
}

// 1/sqrt(x) for x >= 1: the hardware estimate refined by two Newton steps
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
}

// One-sided Jacobi on the ma rows R[row[k]] (BM coordinates, zero beyond b,
// row stride ld) by one wavefront: LP lanes per row pair, 64 / LP pairs per
// pass, the round-robin pairing of the rows, the rotation tests of
// jacobi_basis_wg.
template <int LP, int BM>
__device__ int jacobi_rows_wave(double* R, int ld, const int* row, int ma, double negl, double aerr, double tol) {
  constexpr int NC = BM / LP, PPASS = 64 / LP;
  const int lane = threadIdx.x & 63, sub = lane % LP;
  const int mm = ma + (ma & 1), np = mm / 2, m1 = mm - 1;
  const double negl2 = negl * negl, aerr2 = aerr * aerr, tol2 = tol * tol;
  int nsweep = 0;
  for (int sweep = 0; sweep < 40 && ma > 1; ++sweep) {
    ++nsweep;
    bool rotated = false;
    for (int rho = 0; rho < m1; ++rho) {
      for (int pb = 0; pb < np; pb += PPASS) {
        const int pp = pb + lane / LP;
        int p = -1, q = -1;
        if (pp < np) {
          if (pp == 0) {
            p = m1;
            q = rho;
          } else {
            p = rho + pp;
            if (p >= m1) p -= m1;
            q = rho - pp;
            if (q < 0) q += m1;
          }
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          if (q >= ma) p = -1;
        }
        double x[NC], y[NC];
        double a = 0.0, c = 0.0, d = 0.0;
        double* xr = R;
        double* yr = R;
        if (p >= 0) {
          xr = R + row[p] * ld;
          yr = R + row[q] * ld;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            x[u] = xr[sub + LP * u];
            y[u] = yr[sub + LP * u];
            a += x[u] * x[u];
            c += y[u] * y[u];
            d += x[u] * y[u];
          }
        }
        a = group_sum<LP>(a);
        c = group_sum<LP>(c);
        d = group_sum<LP>(d);
        // the tests of jacobi_basis_wg on squares: |d| > tol |x||y|, one of
        // the rows above negl, |d| > aerr max(|x|, |y|)
        const double d2 = d * d;
        if (p >= 0 && d != 0.0 && d2 > tol2 * a * c && (a > negl2 || c > negl2) && d2 > aerr2 * fmax(a, c)) {
          // t = tan of the rotation angle, the smaller root of
          // t^2 + 2 zeta t - 1 = 0 with zeta = (c - a) / 2d
          const double e = c - a, f = 2.0 * d;
          const double h = sqrt(e * e + f * f);
          const double tt = (e >= 0.0 ? f : -f) / (fabs(e) + h);
          const double cs = rsqrt_nr(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            xr[sub + LP * u] = cs * x[u] - sn * y[u];
            yr[sub + LP * u] = sn * x[u] + cs * y[u];
          }
          rotated = true;
        }
        wave_sync();
      }
    }
    if (__ballot(rotated) == 0) break;
  }
  return nsweep;
}

// The same rotations by the four wavefronts of a workgroup: the pairs of a
// round are split over the wavefronts, one workgroup barrier per round (every
// thread of the workgroup must call it).  Returns the number of sweeps.
template <int LP, int BM>
__device__ int jacobi_rows_wg(double* R, int ld, const int* row, int ma, double negl, double aerr, double tol) {
  constexpr int NC = BM / LP, PPASS = 64 / LP;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, sub = lane % LP;
  const int mm = ma + (ma & 1), np = mm / 2, m1 = mm - 1;
  const double negl2 = negl * negl, aerr2 = aerr * aerr, tol2 = tol * tol;
  int nsweep = 0;
  for (int sweep = 0; sweep < 40 && ma > 1; ++sweep) {
    ++nsweep;
    int rotated = 0;
    for (int rho = 0; rho < m1; ++rho) {
      for (int pb = wv * PPASS; pb < np; pb += 4 * PPASS) {
        const int pp = pb + lane / LP;
        int p = -1, q = -1;
        if (pp < np) {
          if (pp == 0) {
            p = m1;
            q = rho;
          } else {
            p = rho + pp;
            if (p >= m1) p -= m1;
            q = rho - pp;
            if (q < 0) q += m1;
          }
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          if (q >= ma) p = -1;
        }
        double x[NC], y[NC];
        double a = 0.0, c = 0.0, d = 0.0;
        double* xr = R;
        double* yr = R;
        if (p >= 0) {
          xr = R + row[p] * ld;
          yr = R + row[q] * ld;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            x[u] = xr[sub + LP * u];
            y[u] = yr[sub + LP * u];
            a += x[u] * x[u];
            c += y[u] * y[u];
            d += x[u] * y[u];
          }
        }
        a = group_sum<LP>(a);
        c = group_sum<LP>(c);
        d = group_sum<LP>(d);
        const double d2 = d * d;
        if (p >= 0 && d != 0.0 && d2 > tol2 * a * c && (a > negl2 || c > negl2) && d2 > aerr2 * fmax(a, c)) {
          const double e = c - a, f = 2.0 * d;
          const double h = sqrt(e * e + f * f);
          const double tt = (e >= 0.0 ? f : -f) / (fabs(e) + h);
          const double cs = rsqrt_nr(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            xr[sub + LP * u] = cs * x[u] - sn * y[u];
            yr[sub + LP * u] = sn * x[u] + cs * y[u];
          }
          rotated = 1;
        }
      }
      __syncthreads();   // the rows of this round rotated before the next pairing
    }
    if (!__syncthreads_or(rotated)) break;
  }
  return nsweep;
}

// C[TM x TM tile of thread (ty, tx)] += A^T A over K rows of the staged chunk
// S (row stride ld, BM = 16 TM columns), FP64 accumulation.
template <int TM, typename T>
__device__ inline void gram_tile(const T* S, int ld, int K, double acc[TM][TM]) {
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const T* a = S + TM * ty;
  const T* bb = S + TM * tx;
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
    double av[TM], bv[TM];
#pragma unroll
    for (int q = 0; q < TM; ++q) {
      av[q] = (double)a[k * ld + q];
      bv[q] = (double)bb[k * ld + q];
    }
#pragma unroll
    for (int p = 0; p < TM; ++p)
#pragma unroll
      for (int q = 0; q < TM; ++q) acc[p][q] += av[p] * bv[q];
  }
}

// LDS layout of the Gram compression for blocks of at most BM unknowns.
template <typename T, int BM>
struct GramLds {
  static constexpr int GL = BM + 1;                // row stride of G (doubles)
  static constexpr int SL = BM + 4;                // row stride of a staged chunk
  static constexpr size_t gram_phase =
      (size_t)2 * GCW * SL * sizeof(T) + (size_t)GCOLS * 12 + (size_t)GVB * 16 + (size_t)(GVB + 1) * 4;
  static constexpr size_t factor_phase = (size_t)BM * GL * sizeof(double);
  static constexpr size_t big =
      ((gram_phase > factor_phase ? gram_phase : factor_phase) + 15) & ~(size_t)15;
  static constexpr size_t total = big + 3 * BM * sizeof(double) + 3 * BM * sizeof(int);
};

template <typename T, int BM>
size_t work_compress_gram() {
  return GramLds<T, BM>::total;
}

// Blocks with BM - 64 < b <= BM (all b <= 64 for BM = 64).
template <typename T, int BM>
__global__ __launch_bounds__(NT) void k_compress_gram(LevelArgs<T> A, int32_t s0) {
  if constexpr (sizeof(T) != sizeof(float)) {
    return;   // FP64 factors take k_compress_wg
  } else {
    using L = GramLds<T, BM>;
    constexpr int GL = L::GL, SL = L::SL, NL = BM / 64, TM = BM / 16;
    const Step st = A.steps[s0 + blockIdx.x];
    const int i = st.blk;
    if (A.need_exact && !A.need_exact[i]) return;   // taken by the sketch kernel
    const int b = A.bsz[i];
    // size class (BM - 64, BM]; the first class also takes empty blocks
    if (b > BM || (b <= BM - 64 && !(BM == 64 && b == 0))) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, ty = tid >> 4, tx = tid & 15;
    T* Ug = A.U + A.u_off[i];
    if (st.nfar == 0 || b == 0) {
      for (int e = tid; e < b * b; e += NT) Ug[e] = (e / b == e % b) ? T(1) : T(0);
      if (tid == 0) {
        A.rank[i] = 0;
        A.edrop[i] = 0.0;
      }
      return;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // Gram phase: two staged chunks, the column map, the view descriptors
    T* stg0 = reinterpret_cast<T*>(smem_raw);
    T* stg1 = stg0 + GCW * SL;
    int64_t* coff = reinterpret_cast<int64_t*>(stg1 + GCW * SL);
    int64_t* voff = coff + GCOLS;
    int* cstr = reinterpret_cast<int*>(voff + GVB);
    int* vbx = cstr + GCOLS;
    int* vtr = vbx + GVB;
    int* vst = vtr + GVB;   // GVB + 1 column starts
    // factor phases: G (BM x GL); rows of R overwrite the pivot rows of G
    double* G = reinterpret_cast<double*>(smem_raw);
    double* sg = reinterpret_cast<double*>(smem_raw + L::big);
    double* tau = sg + BM;
    double* isg = tau + BM;
    int* prow = reinterpret_cast<int*>(isg + BM);   // G row holding row k of R
    int* posv = prow + BM;                          // rank order of row k
    int* brow = posv + BM;                          // G row holding kept direction c
    __shared__ int wsum[4];
    __shared__ double shd[4];
    __shared__ int shi[4];
    __shared__ int64_t shj;
    const int64_t t_start = clock64();

    // ---- 1. G = F_i F_i^T ----------------------------------------------------
    double acc[TM][TM];
#pragma unroll
    for (int p = 0; p < TM; ++p)
#pragma unroll
      for (int q = 0; q < TM; ++q) acc[p][q] = 0.0;
    int wtot = 0;
    for (int f0 = 0; f0 < st.nfar;) {
      const int nv = min(GVB, st.nfar - f0);
      __syncthreads();
      int wme = 0;
      if (tid < nv) {
        const View v = A.views[st.view0 + st.nclose + f0 + tid];
        const int bx = A.bsz[v.x];
        wme = v.proc ? A.rank[v.x] : bx;
        voff[tid] = A.slot_off[v.slot];
        vbx[tid] = bx;
        vtr[tid] = v.trans;
      }
      int incl = wme;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, WV);
        if (lane >= o) incl += y;
      }
      if (lane == 63) wsum[wv] = incl;
      __syncthreads();
      int base = 0;
      for (int k = 0; k < wv; ++k) base += wsum[k];
      if (tid < nv) vst[tid + 1] = base + incl;
      if (tid == 0) vst[0] = 0;
      __syncthreads();
      // the views whose columns end within the map (at least one: w <= BM)
      const int nb = __syncthreads_count(tid < nv && vst[tid + 1] <= GCOLS);
      const int Wb = vst[nb];
      for (int c = tid; c < Wb; c += NT) {
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (vst[mid] <= c) lo = mid;
          else hi = mid - 1;
        }
        const int m = c - vst[lo];
        coff[c] = voff[lo] + (vtr[lo] ? (int64_t)m * b : (int64_t)m);
        cstr[c] = vtr[lo] ? 1 : vbx[lo];
      }
      __syncthreads();
      const int nch = (Wb + GCW - 1) / GCW;
      T rg[NL][GCW / 4];
      auto load = [&](int c0) {
#pragma unroll
        for (int h = 0; h < NL; ++h)
#pragma unroll
          for (int k = 0; k < GCW / 4; ++k) {
            const int c = c0 + wv + 4 * k, a = lane + 64 * h;
            rg[h][k] = (a < b && c < Wb) ? A.arena[coff[c] + (int64_t)a * cstr[c]] : T(0);
          }
      };
      auto store = [&](T* S) {
#pragma unroll
        for (int h = 0; h < NL; ++h)
#pragma unroll
          for (int k = 0; k < GCW / 4; ++k) S[(wv + 4 * k) * SL + lane + 64 * h] = rg[h][k];
      };
      load(0);
      store(stg0);
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        if (ch + 1 < nch) load((ch + 1) * GCW);
        T* S = (ch & 1) ? stg1 : stg0;
        gram_tile<TM, T>(S, SL, min(GCW, Wb - ch * GCW), acc);
        if (ch + 1 < nch) store((ch & 1) ? stg0 : stg1);
        __syncthreads();
      }
      wtot += Wb;
      f0 += nb;
    }
#pragma unroll
    for (int p = 0; p < TM; ++p)
#pragma unroll
      for (int q = 0; q < TM; ++q) G[(TM * ty + p) * GL + TM * tx + q] = acc[p][q];
    __syncthreads();
    const int64_t t_qr = clock64();

    // ---- 2-4. one wavefront: pivoted Cholesky, Jacobi, rank, reflectors -------
    // lane owns the coordinates t = lane + 64 h, h < NL
    if (wv == 0) {
      const double theta = *A.theta;
      double dgl[NL];
      double tr0 = 0.0;
#pragma unroll
      for (int h = 0; h < NL; ++h) {
        const int t = lane + 64 * h;
        dgl[h] = t < b ? G[t * GL + t] : 0.0;
        tr0 += dgl[h];
      }
      const double fro2 = wave_sum_u(tr0);
      // rounding level of the factor's own entries (its precision T), as in
      // the other compression kernels
      const double noise = (double)Eps<T>::v() * sqrt(fro2);
      const double negl = A.rank_mode == 0 ? fmax(noise, theta / 64.0) : noise;
      const double aerr = A.rank_mode == 0 ? fmax(noise, fmin((double)max(b, 16) * noise, theta / 32.0))
                                           : (double)max(b, 16) * noise;
      const double stop2 = aerr * aerr;
      bool chosen[NL];
#pragma unroll
      for (int h = 0; h < NL; ++h) chosen[h] = false;
      double inactive = 0.0;
      // learned cap (LEARNED_CAP): at most the predicted width of pivots
      const int cap = A.lwidth ? A.lwidth[i] : b;
      bool capped = false;
      int k = 0;
      for (; k < b; ++k) {
        double rsl = 0.0, cv = -1.0;
        int ci = lane;
#pragma unroll
        for (int h = 0; h < NL; ++h) {
          const int t = lane + 64 * h;
          const bool in = t < b && !chosen[h];
          if (in) rsl += dgl[h];
          if (in && dgl[h] > cv) {
            cv = dgl[h];
            ci = t;
          }
        }
        const double rs = wave_sum_u(rsl);
        wave_argmax_u(cv, ci);
        if (rs <= stop2 || !(cv > 0.0)) {
          inactive = rs;
          break;
        }
        if (k >= cap) {
          inactive = rs;
          capped = true;
          break;
        }
        const int p = ci;
        const double ilpp = 1.0 / sqrt(cv), lpp = cv * ilpp;
        // column p of the trailing matrix: G(:, p) - sum_j R(j, :)^T R(j, p)
        double s[NL];
#pragma unroll
        for (int h = 0; h < NL; ++h) s[h] = G[p * GL + lane + 64 * h];
        int j = 0;
        for (; j + 4 <= k; j += 4) {
          const double* r0 = G + prow[j] * GL;
          const double* r1 = G + prow[j + 1] * GL;
          const double* r2 = G + prow[j + 2] * GL;
          const double* r3 = G + prow[j + 3] * GL;
          const double b0 = r0[p], b1 = r1[p], b2 = r2[p], b3 = r3[p];
#pragma unroll
          for (int h = 0; h < NL; ++h) {
            const int t = lane + 64 * h;
            s[h] -= (r0[t] * b0 + r1[t] * b1) + (r2[t] * b2 + r3[t] * b3);
          }
        }
        for (; j < k; ++j) {
          const double* rj = G + prow[j] * GL;
          const double bj = rj[p];
#pragma unroll
          for (int h = 0; h < NL; ++h) s[h] -= rj[lane + 64 * h] * bj;
        }
#pragma unroll
        for (int h = 0; h < NL; ++h) {
          const int t = lane + 64 * h;
          const bool in = t < b && !chosen[h];
          const double lv = (t >= b || chosen[h]) ? 0.0 : (t == p ? lpp : s[h] * ilpp);
          G[p * GL + t] = lv;   // row k of R replaces row p of G
          if (t == p) chosen[h] = true;
          else if (in) dgl[h] -= lv * lv;
        }
        if (lane == 0) prow[k] = p;
        wave_sync();
      }
      const int ma = k;
      const int64_t t_cmp = clock64();
      // ---- Jacobi on the ma rows of R
      const double tol = (double)max(b, 16) * DBL_EPSILON;
      const int np = (ma + 1) / 2;
      int nsweep;
      if (np <= 4) nsweep = jacobi_rows_wave<16, BM>(G, GL, prow, ma, negl, aerr, tol);
      else if (np <= 8) nsweep = jacobi_rows_wave<8, BM>(G, GL, prow, ma, negl, aerr, tol);
      else nsweep = jacobi_rows_wave<4, BM>(G, GL, prow, ma, negl, aerr, tol);
      const int64_t t_jac = clock64();
      // ---- singular values, order, rank (lane owns rows lane + 64 h)
      double sgl[NL];
#pragma unroll
      for (int h = 0; h < NL; ++h) {
        const int q = lane + 64 * h;
        sgl[h] = 0.0;
        if (q < ma) {
          const double* rr = G + prow[q] * GL;
          double s0 = 0.0, s1 = 0.0;
          for (int t = 0; t < BM; t += 2) {
            s0 += rr[t] * rr[t];
            s1 += rr[t + 1] * rr[t + 1];
          }
          sgl[h] = sqrt(s0 + s1);
          sg[q] = sgl[h];
        }
      }
      wave_sync();
      int pos[NL];
      int cnt = 0;
      double edl = 0.0;
#pragma unroll
      for (int h = 0; h < NL; ++h) {
        const int q0 = lane + 64 * h;
        pos[h] = 0;
        if (q0 < ma) {
          for (int q = 0; q < ma; ++q) pos[h] += (sg[q] > sgl[h] || (sg[q] == sgl[h] && q < q0)) ? 1 : 0;
          posv[q0] = pos[h];
        }
        cnt += __popcll(__ballot(q0 < ma && sgl[h] > theta));
      }
      const int r = A.rank_mode == 0 ? cnt : min(A.fixed_rank, b);
      // a capped step is kept only if the energy the cap left out (the
      // trailing trace, G - R^T R being positive semidefinite) cannot change
      // the rank: sigma_{r+1}^2 + inactive <= theta^2 gives sigma_{r+1}(F) <=
      // theta (Weyl), so r is the rank of F_i and ||E_i||_2 <= theta
      if (capped && A.rank_mode == 0) {
        double s1 = 0.0;
#pragma unroll
        for (int h = 0; h < NL; ++h)
          if (lane + 64 * h < ma && pos[h] == r) s1 = sgl[h] * sgl[h];
        s1 = wave_sum_u(s1);
        if (lane == 0) shi[3] = s1 + inactive > theta * theta ? 1 : 0;
      } else if (lane == 0) {
        shi[3] = 0;
      }
#pragma unroll
      for (int h = 0; h < NL; ++h)
        if (lane + 64 * h < ma && pos[h] >= r) edl += sgl[h] * sgl[h];
      const double ed = wave_sum_u(edl);
      const int kb = min(r, ma);
      int label = 0;
      if (A.rec) {
        // training label: the smallest sketch width k >= r that an ideal
        // sketch would need to pass the a-posteriori check,
        // tail(k) + (k > r ? sigma_r^2 : 0) <= theta^2, tail(k) = sum of
        // sigma_j^2 over positions j >= k plus the inactive energy
#pragma unroll
        for (int h = 0; h < NL; ++h)
          if (lane + 64 * h < ma) tau[pos[h]] = sgl[h] * sgl[h];
        wave_sync();
        const double th2 = theta * theta;
        const double sr2 = r < ma ? tau[r] : 0.0;
        double tail = inactive;
        int kf = ma;
        for (int kk = ma; kk >= r; --kk) {
          if (kk < ma) tail += tau[kk];
          if (tail + (kk > r ? sr2 : 0.0) <= th2) kf = kk;
        }
        label = max(kf, r);
        wave_sync();
      }
      // kept directions, normalised, in rank order
#pragma unroll
      for (int h = 0; h < NL; ++h) {
        const int q = lane + 64 * h;
        if (q < ma && pos[h] < kb) {
          brow[pos[h]] = prow[q];
          isg[pos[h]] = sgl[h] > 0.0 ? 1.0 / sgl[h] : 0.0;
        }
      }
      wave_sync();
      for (int c2 = 0; c2 < kb; ++c2) {
        const double f = isg[c2];
#pragma unroll
        for (int h = 0; h < NL; ++h) G[brow[c2] * GL + lane + 64 * h] *= f;
      }
      wave_sync();
      // ---- Householder reflectors of the kept directions
      for (int cv = 0; cv < kb; ++cv) {
        double* vr = G + brow[cv] * GL;
        double xs = 0.0;
#pragma unroll
        for (int h = 0; h < NL; ++h) {
          const int t = lane + 64 * h;
          const double x = (t >= cv && t < b) ? vr[t] : 0.0;
          xs += x * x;
        }
        const double nrm2 = wave_sum_u(xs);
        const double x0 = vr[cv];
        const double nrm = sqrt(nrm2);
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double vv = v0 * v0 + (nrm2 - x0 * x0);
        const double tc = vv > 0.0 ? 2.0 / vv : 0.0;
        wave_sync();
#pragma unroll
        for (int h = 0; h < NL; ++h) {
          const int t = lane + 64 * h;
          if (t < cv) vr[t] = 0.0;
          if (t == cv) vr[cv] = v0;
        }
        if (lane == 0) tau[cv] = tc;
        wave_sync();
        // H_cv on the later directions: 4 lanes per direction, BM / 4
        // coordinates per lane
        for (int cb = cv + 1; cb < kb; cb += 16) {
          const int c2 = cb + (lane >> 2), sb = lane & 3;
          double vreg[BM / 4], breg[BM / 4];
          double dd = 0.0;
          double* br = G + brow[min(c2, kb - 1)] * GL;
#pragma unroll
          for (int u = 0; u < BM / 4; ++u) {
            vreg[u] = vr[sb + 4 * u];
            breg[u] = br[sb + 4 * u];
            dd += vreg[u] * breg[u];
          }
          dd = group_sum<4>(dd);
          if (c2 < kb) {
#pragma unroll
            for (int u = 0; u < BM / 4; ++u) br[sb + 4 * u] = breg[u] - tc * dd * vreg[u];
          }
          wave_sync();
        }
      }
      if (lane == 0) {
        shi[0] = kb;
        shi[1] = r;
        shi[2] = label;
        shd[0] = ed + inactive;
        shj = t_jac;
        if (A.dbg) {
          int64_t* dd = A.dbg + 72 * (int64_t)i;
          dd[0] = ma;
          dd[1] = nsweep;
          dd[2] = wtot;
          dd[3] = b;
          dd[4] = t_qr - t_start;
          dd[5] = t_cmp - t_qr;
          dd[6] = t_jac - t_cmp;
        }
      }
      if (A.dbg && lane < ma && lane < 64) {
        double* sv = reinterpret_cast<double*>(A.dbg + 72 * (int64_t)i + 8);
        sv[lane] = sg[lane];
      }
    }
    __syncthreads();

    if (A.lwidth) {
      // learned cap: a rejected step is redone without the cap
      if (tid == 0) {
        if (shi[3]) A.big_fail[i] = 1;
        atomicAdd(A.lcount + (shi[3] ? 1 : 0), 1);
      }
      if (shi[3]) return;
    }
    // ---- 5. U_i = H_0 ... H_{kb-1}: 4 lanes per column, BM / 4 coordinates
    // per lane, 16 columns per wavefront and pass --------------------------------
    const int kb = shi[0];
    for (int col0 = 16 * wv; col0 < BM; col0 += 64) {
      const int col = col0 + (lane >> 2), sb = lane & 3;
      double qv[BM / 4];
#pragma unroll
      for (int u = 0; u < BM / 4; ++u) qv[u] = (sb + 4 * u == col) ? 1.0 : 0.0;
      for (int cv = kb - 1; cv >= 0; --cv) {
        const double* vr = G + brow[cv] * GL;
        const double tc = tau[cv];
        double vreg[BM / 4];
        double dd = 0.0;
#pragma unroll
        for (int u = 0; u < BM / 4; ++u) {
          vreg[u] = vr[sb + 4 * u];
          dd += vreg[u] * qv[u];
        }
        dd = group_sum<4>(dd);
#pragma unroll
        for (int u = 0; u < BM / 4; ++u) qv[u] -= tc * dd * vreg[u];
      }
      if (col < b) {
#pragma unroll
        for (int u = 0; u < BM / 4; ++u) {
          const int t = sb + 4 * u;
          if (t < b) Ug[t * b + col] = (T)qv[u];
        }
      }
    }
    if (tid == 0) {
      A.rank[i] = shi[1];
      A.edrop[i] = shd[0];
      if (A.rec) A.rec[(A.rec_off + i) * REC_W + NFEAT] = (float)shi[2] / (float)b;
      if (A.dbg) A.dbg[72 * (int64_t)i + 7] = clock64() - shj;
    }
  }
}

// ---------------------------------------------------------------------------
// Learned-rank compression (b <= 64): the cheaper rank-revealing variant of
// eq. (rreav).  One 256-thread workgroup per step, FP64 arithmetic:
//   1. features of the far row (Frobenius norms of the row and of its far
//      blocks against theta, widths, neighbour ranks: all invariant under the
//      rotations inside kept bases that leave the method unchanged);
//   2. MLP 16 -> 64 -> 64 -> 1 (ReLU) predicts z ~ r/b, k = ceil(b z);
//   3. sketch Y = F Omega with l = min(k + p, b, w) columns, Omega drawn by
//      Philox4x32-10 (counter (column of F, j/2, block, level), key seed),
//      Box-Muller in FP64;
//   4. Q = orth(Y) (Householder), B = Q^T F, H = B B^T (l x l);
//   5. pivoted Cholesky + one-sided Jacobi on H give sigma(B) and its left
//      singular vectors; r = #{sigma > theta}; accept when
//      ||F||_F^2 - ||B||_F^2 + sigma_{r+1}^2 <= theta^2 (then ||E_i||_2 <=
//      theta), else flag the step for the exact kernel.
// With feat_only the kernel records the features and flags every step.
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// the two normals of sketch entries (m, 2 jp) and (m, 2 jp + 1)
__device__ inline void sketch_pair(uint64_t seed, int level, int block, int m, int jp, double& n0, double& n1) {
  uint32_t c[4] = {(uint32_t)m, (uint32_t)jp, (uint32_t)block, (uint32_t)level};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double ua = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) / 9007199254740992.0;
  const double ub = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) / 9007199254740992.0;
  const double rad = sqrt(-2.0 * log(ua));
  n0 = rad * cos(6.283185307179586 * ub);
  n1 = rad * sin(6.283185307179586 * ub);
}

__device__ inline double clog10(double v, double theta) {
  return fmin(fmax(log10(fmax(v, 1e-300) / theta), -30.0), 30.0);
}

template <typename T>
size_t work_compress_rand() {
  return (size_t)4 * 64 * TLD * sizeof(double) + (size_t)(4 * 64 + 3 * 64 + 64 + 16) * sizeof(double) +
         64 * sizeof(int);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_compress_rand(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, ty = tid >> 4, tx = tid & 15;
  T* Ug = A.U + A.u_off[i];
  if (tid == 0) A.need_exact[i] = 0;
  if (A.rec && tid < REC_W) A.rec[(A.rec_off + i) * REC_W + tid] = tid < NFEAT ? 0.0f : -1.0f;
  if (b > 64 || A.feat_only && (st.nfar == 0 || b == 0)) {
    if (tid == 0) A.need_exact[i] = 1;
    return;
  }
  if (st.nfar == 0 || b == 0) {
    for (int e = tid; e < b * b; e += NT) Ug[e] = (e / b == e % b) ? T(1) : T(0);
    if (tid == 0) {
      A.rank[i] = 0;
      A.edrop[i] = 0.0;
    }
    return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* R1 = reinterpret_cast<double*>(smem_raw);   // F tiles (type T)
  double* R2 = R1 + 64 * TLD;                          // Omega tiles (T), then B^T tiles, then Jacobi rows
  double* YQ = R2 + 64 * TLD;                          // Y, Householder vectors, then H, then kept vectors
  double* Qx = YQ + 64 * TLD;                          // explicit Q (b x l)
  double* red = Qx + 64 * TLD;                         // 4 x 64 partial sums
  double* sg = red + 4 * 64;
  double* tau = sg + 64;
  double* lc = tau + 64;
  double* hbuf = lc + 64;                              // hidden layer
  double* xf = hbuf + 64;                              // 16 features
  int* posv = reinterpret_cast<int*>(xf + 16);
  __shared__ double shd[8];
  __shared__ int shi[8];
  T* Fs = reinterpret_cast<T*>(R1);
  T* Os = reinterpret_cast<T*>(R2);
  const double theta = *A.theta;
  const int64_t t_start = clock64();

  // ---- 1. features ------------------------------------------------------------
  double racc = 0.0, cmax2 = 0.0, bsum4 = 0.0;   // squared block norms: max, sum of squares, count above theta
  int ccnt = 0, wtot = 0, nproc = 0;
  double prs = 0.0, pss = 0.0;
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    wtot += w;
    if (v.proc) {
      ++nproc;
      prs += A.rank[v.x];
      pss += bx;
    }
    double blk = 0.0;   // this thread's part of the block's squared norm
    for (int c0 = 0; c0 < w; c0 += 64) {
      const int mc = min(64, w - c0);
      __syncthreads();
      load_view_tile(Fs, base, v.trans, b, bx, 0, b, c0, mc);
      __syncthreads();
      if (lane < b)
        for (int m = wv; m < mc; m += 4) {
          const double x = (double)Fs[lane * TLD + m];
          racc += x * x;
          blk += x * x;
        }
    }
    // block norm: reduce blk over the workgroup (uniform control flow)
    __syncthreads();
    blk = wave_sum(blk);
    if (lane == 0) red[wv] = blk;
    __syncthreads();
    const double bn2 = red[0] + red[1] + red[2] + red[3];
    cmax2 = fmax(cmax2, bn2);
    ccnt += bn2 > theta * theta ? 1 : 0;
    bsum4 += bn2 * bn2;
    __syncthreads();
  }
  red[wv * 64 + lane] = racc;
  __syncthreads();
  {
    // column statistics: block reductions through red (after the row sums are read)
    double rn2 = 0.0;
    if (wv == 0) rn2 = red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
    __syncthreads();
    // cmax2 and ccnt are uniform over the workgroup (block norms)
    if (wv == 0) {
      const double fro2 = wave_sum(lane < b ? rn2 : 0.0);
      const double cmx2 = cmax2;
      const double ccn = (double)ccnt;
      if (lane == 0) {
        const double cmax = sqrt(cmx2), fro = sqrt(fro2);
        xf[0] = log2((double)b + 1.0);
        xf[1] = log2((double)wtot + 1.0);
        xf[2] = (double)A.level;
        xf[3] = (double)st.nfar;
        xf[4] = (double)st.nclose;
        xf[5] = clog10(fro, theta);
        xf[6] = clog10(sqrt(fro2 / max(b, 1)), theta);
        xf[7] = clog10(cmax, theta);
        xf[8] = clog10(sqrt(fro2 / max(wtot, 1)), theta);
        xf[9] = ccn / (double)max(st.nfar, 1);
        xf[10] = fro2 > 0.0 ? bsum4 / (fro2 * fro2) : 0.0;
        xf[11] = cmx2 > 0.0 ? fro2 / (cmx2 * st.nfar) : 0.0;
        xf[12] = (double)nproc / (double)max(st.nfar, 1);
        xf[13] = pss > 0.0 ? prs / pss : 0.0;
        xf[14] = b / 64.0;
        xf[15] = 1.0;
        shd[0] = fro2;
      }
    }
  }
  __syncthreads();
  if (A.rec && tid < NFEAT) A.rec[(A.rec_off + i) * REC_W + tid] = (float)xf[tid];
  if (A.feat_only) {
    if (tid == 0) A.need_exact[i] = 1;
    return;
  }
  const double fro2 = shd[0];

  // ---- 2. rank prediction ----------------------------------------------------
  if (wv == 0) {
    const float* P = A.mlp;
    double h = P[MLP_OFF_B1 + lane];
    for (int k = 0; k < NFEAT; ++k)
      h += (double)P[MLP_OFF_W1 + lane * NFEAT + k] * ((xf[k] - (double)P[MLP_OFF_MEAN + k]) / (double)P[MLP_OFF_STD + k]);
    hbuf[lane] = fmax(h, 0.0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double h2 = P[MLP_OFF_B2 + lane];
    for (int k = 0; k < MLP_H; ++k) h2 += (double)P[MLP_OFF_W2 + lane * MLP_H + k] * hbuf[k];
    h2 = fmax(h2, 0.0);
    const double z = wave_sum((double)P[MLP_OFF_W3 + lane] * h2) + (double)P[MLP_OFF_B3];
    if (lane == 0) {
      const double bz = z * b;
      int k = (bz == bz) ? (int)fmin(fmax(ceil(bz), 0.0), (double)b) : b;
      shi[0] = min(min(k + SKETCH_OVERSAMPLE, b), min(wtot, 64));
    }
  }
  __syncthreads();
  const int l = shi[0];

  // ---- 3. sketch Y = F Omega ----------------------------------------------------
  double acc[4][4];
  zero_acc(acc);
  int mbase = 0;
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    for (int c0 = 0; c0 < w; c0 += 64) {
      const int mc = min(64, w - c0);
      __syncthreads();
      if (v.trans) {
        for (int e = tid; e < mc * b; e += NT) {
          const int m = e / b, a = e % b;
          Fs[m * TLD + a] = base[(int64_t)(c0 + m) * b + a];
        }
      } else {
        for (int e = tid; e < mc * b; e += NT) {
          const int a = e / mc, m = e % mc;
          Fs[m * TLD + a] = base[(int64_t)a * bx + c0 + m];
        }
      }
      const int np = (l + 1) >> 1;
      for (int e = tid; e < mc * np; e += NT) {
        const int m = e / np, jp = e % np;
        double n0, n1;
        sketch_pair(A.seed, A.level, i, mbase + c0 + m, jp, n0, n1);
        Os[m * TLD + 2 * jp] = (T)n0;
        if (2 * jp + 1 < l) Os[m * TLD + 2 * jp + 1] = (T)n1;
      }
      __syncthreads();
      gemm_tn_4x4m(Fs, Os, mc, acc);
    }
    mbase += w;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) YQ[(4 * ty + p) * TLD + 4 * tx + q] = acc[p][q];
  __syncthreads();
  const int64_t t_qr = clock64();

  // ---- 4a. Householder QR of Y (b x l), explicit Q ----------------------------
  const int nref = min(l, b);
  for (int k = 0; k < nref; ++k) {
    if (wv == 0) {
      const double x = (lane >= k && lane < b) ? YQ[lane * TLD + k] : 0.0;
      const double nrm2 = wave_sum(x * x);
      const double x0 = __shfl(x, k, WV);
      double tq = 0.0;
      if (nrm2 > 1e-290) {
        const double nrm = sqrt(nrm2);
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double vv = v0 * v0 + (nrm2 - x0 * x0);
        tq = vv > 0.0 ? 2.0 / vv : 0.0;
        if (lane == k) YQ[k * TLD + k] = v0;
      }
      if (lane == 0) tau[k] = tq;
    }
    __syncthreads();
    {
      const int j = k + 1 + (tid >> 2), pt = tid & 3;
      const double tq = tau[k];
      double dd = 0.0;
      if (j < l)
        for (int a = k + pt; a < b; a += 4) dd += YQ[a * TLD + k] * YQ[a * TLD + j];
      dd += __shfl_xor(dd, 1, WV);
      dd += __shfl_xor(dd, 2, WV);
      if (j < l && tq != 0.0)
        for (int a = k + pt; a < b; a += 4) YQ[a * TLD + j] -= tq * dd * YQ[a * TLD + k];
    }
    __syncthreads();
  }
  for (int e = tid; e < 64 * 64; e += NT) Qx[(e >> 6) * TLD + (e & 63)] = ((e >> 6) == (e & 63)) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = nref - 1; k >= 0; --k) {
    const int j = tid >> 2, pt = tid & 3;
    const double tq = tau[k];
    double dd = 0.0;
    if (j < l && tq != 0.0)
      for (int a = k + pt; a < b; a += 4) dd += YQ[a * TLD + k] * Qx[a * TLD + j];
    dd += __shfl_xor(dd, 1, WV);
    dd += __shfl_xor(dd, 2, WV);
    if (j < l && tq != 0.0)
      for (int a = k + pt; a < b; a += 4) Qx[a * TLD + j] -= tq * dd * YQ[a * TLD + k];
    __syncthreads();
  }

  // ---- 4b. B = Q^T F, H = B B^T ------------------------------------------------
  double accH[4][4];
  zero_acc(accH);
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    for (int c0 = 0; c0 < w; c0 += 64) {
      const int mc = min(64, w - c0);
      __syncthreads();
      load_view_tile(Fs, base, v.trans, b, bx, 0, b, c0, mc);
      __syncthreads();
      zero_acc(acc);
      gemm_tn_4x4m(Qx, Fs, b, acc);   // acc[p][q] = B[4ty+p][4tx+q]
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) R2[(4 * tx + q) * TLD + 4 * ty + p] = (4 * tx + q < mc) ? acc[p][q] : 0.0;
      __syncthreads();
      gemm_tn_4x4m(R2, R2, mc, accH);
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) YQ[(4 * ty + p) * TLD + 4 * tx + q] = accH[p][q];
  __syncthreads();

  // ---- 5. pivoted Cholesky of H, rows into R2 ------------------------------------
  double* G = YQ;
  double* X = R2;
  if (wv == 0) {
    const double gd = lane < l ? G[lane * TLD + lane] : 0.0;
    const double tr = wave_sum(gd);
    lc[lane] = gd;   // trailing diagonal
    posv[lane] = 0;  // chosen flags
    if (lane == 0) shd[1] = tr;
  }
  __syncthreads();
  const double out2 = fmax(fro2 - shd[1], 0.0);
  const double noise = (double)Eps<T>::v() * sqrt(fro2);
  const double negl = A.rank_mode == 0 ? fmax(noise, theta / 64.0) : noise;
  const double aerr = A.rank_mode == 0 ? fmax(noise, fmin((double)max(b, 16) * noise, theta / 32.0))
                                       : (double)max(b, 16) * noise;
  const double stop2 = aerr * aerr;
  int k = 0;
  for (; k < l; ++k) {
    if (wv == 0) {
      const bool in = lane < l && !posv[lane];
      const double dv = in ? lc[lane] : 0.0;
      const double rs = wave_sum(dv);
      double cv = in ? dv : -1.0;
      int ci = lane;
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(cv, o, WV);
        const int oi = __shfl_xor(ci, o, WV);
        if (ov > cv || (ov == cv && oi < ci)) {
          cv = ov;
          ci = oi;
        }
      }
      const bool stop = rs <= stop2 || !(cv > 0.0);
      if (lane == 0) {
        shi[3] = stop ? 1 : 0;
        shd[2] = rs;
        if (!stop) {
          shi[2] = ci;
          shd[3] = sqrt(cv);
          posv[ci] = 1;
        }
      }
    }
    __syncthreads();
    if (shi[3]) break;
    const int p = shi[2];
    const double lpp = shd[3];
    if (tid < 64) {
      const int t = tid;
      const double lv = t >= l ? 0.0 : (t == p ? lpp : (posv[t] ? 0.0 : G[t * TLD + p] / lpp));
      tau[t] = lv;
      X[k * TLD + t] = lv;
    }
    __syncthreads();
    for (int t = ty; t < l; t += 16) {
      const double lt = tau[t];
      for (int u = tx; u < l; u += 16) {
        const double g = G[t * TLD + u] - lt * tau[u];
        G[t * TLD + u] = g;
        if (u == t) lc[t] = g;
      }
    }
    __syncthreads();
  }
  const int ma = k;
  const double inactive = k < l ? shd[2] : 0.0;
  const int64_t t_cmp = clock64();
  __syncthreads();
  jacobi_basis_wg<double, T>(A, i, b, ma, X, YQ, TLD, nullptr, inactive, negl, aerr, sg, tau, posv, shi, shd, Ug,
                             wtot, t_start, t_qr, t_cmp, l, Qx, out2);
}

// V_ix <- U_i^T V_ix (far views keep rows 0..r_i-1), D_i <- U_i^T D_i U_i.
template <typename T>
__global__ __launch_bounds__(NT) void k_rotate_t(LevelArgs<T> A, int32_t it0) {
  // the items of one step (consecutive) on one XCD: U_i is fetched into one L2
  const Item item = A.items[it0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[item.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b == 0 || b > 64) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Us = reinterpret_cast<T*>(smem_raw);
  T* X = Us + 64 * TLD;
  const T* Ug = A.U + A.u_off[i];
  load_view_tile(Us, Ug, 0, b, b, 0, b, 0, b);
  typename AccT<T>::type acc[4][4];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  if (item.view < 0) {
    T* D = A.arena + A.slot_off[i];
    load_view_tile(X, D, 0, b, b, 0, b, 0, b);
    __syncthreads();
    zero_acc(acc);
    gemm_tn_4x4(X, Us, b, acc);       // Z = D U (D symmetric)
    __syncthreads();
    acc_to_lds(acc, X);
    __syncthreads();
    zero_acc(acc);
    gemm_tn_4x4(Us, X, b, acc);       // U^T Z
    // the rotated block is stored exactly symmetric: the lower triangle is
    // mirrored (the two triangles of U^T Z differ by the rounding of Z)
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int a = 4 * ty + p;
      if (a < b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = 4 * tx + q;
          if (c <= a) {
            const T v = (T)acc[p][q];
            D[a * b + c] = v;
            D[c * b + a] = v;
          }
        }
    }
    return;
  }
  const View v = A.views[item.view];
  const int bx = A.bsz[v.x];
  const bool far = (item.view - st.view0) >= st.nclose;
  const int r = A.rank[i];
  T* base = A.arena + A.slot_off[v.slot];
  // U^T X on the FP64 matrix cores: wavefront w owns rows 16 w .. 16 w + 15
  // of the product as four 16 x 16 tiles (v_mfma_f64_16x16x4f64 lanes:
  // A (row l % 16, k l / 16), B (k l / 16, column l % 16); result register j
  // of lane l: (row 4 j + l / 16, column l % 16)); rows b .. b4 - 1 of both
  // operands are zero so the k loop runs in whole steps of four
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int b4 = (b + 3) & ~3;
  for (int e = threadIdx.x; e < (b4 - b) * 64; e += NT) Us[(b + (e >> 6)) * TLD + (e & 63)] = T(0);
  // a far view keeps only its rows < r_i (E_i is dropped): wavefronts whose
  // rows all lie beyond r_i skip the product (with compensation k_compensate
  // reads E_i and zeroes it afterwards)
  const bool drop = far && !A.compensate;
  for (int c0 = 0; c0 < bx; c0 += 64) {
    const int tc = min(64, bx - c0);
    __syncthreads();
    load_view_tile(X, base, v.trans, b, bx, 0, b, c0, tc);
    for (int e = threadIdx.x; e < (b4 - b) * 64; e += NT) X[(b + (e >> 6)) * TLD + (e & 63)] = T(0);
    __syncthreads();
    dbl4 dacc[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) dacc[tj] = dbl4{0.0, 0.0, 0.0, 0.0};
    if (!drop || 16 * wv < r) {
      const T* fa = Us + fk * TLD + 16 * wv + fr;
      const T* fb = X + fk * TLD + fr;
#pragma unroll 2
      for (int k0 = 0; k0 < b4; k0 += 4) {
        const double av = (double)fa[k0 * TLD];
        double bv[4];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) bv[tj] = (double)fb[k0 * TLD + 16 * tj];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          dacc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tj], dacc[tj], 0, 0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * wv + 4 * j + fk;
        X[row * TLD + 16 * tj + fr] = (drop && row >= r) ? T(0) : (T)dacc[tj][j];
      }
    __syncthreads();
    store_view_tile(X, base, v.trans, b, bx, 0, b, c0, tc);
  }
}

// L(c, n_i)^T = L_nn^{-1} V_ic[n_i, live_c] as a product with the stored inverse.
template <typename T>
__global__ __launch_bounds__(NT) void k_trsm_t(LevelArgs<T> A, int32_t it0) {
  // the items of one step (consecutive) on one XCD: L_nn^{-1} is fetched into one L2
  const Item item = A.items[it0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[item.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b > 64) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const View v = A.views[item.view];
  const int bx = A.bsz[v.x];
  const int lc = v.proc ? A.rank[v.x] : bx;
  if (lc == 0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Lt = reinterpret_cast<T*>(smem_raw);   // Lt[k][j] = Li[j][k]
  T* X = Lt + 64 * TLD;
  const T* Lig = A.Li + A.u_off[i];
  load_view_tile(Lt, Lig, 1, n, n, 0, n, 0, n);   // Lt[k][j] = Li(j, k)
  T* base = A.arena + A.slot_off[v.slot];
  typename AccT<T>::type acc[4][4];
  for (int c0 = 0; c0 < lc; c0 += 64) {
    const int tc = min(64, lc - c0);
    __syncthreads();
    load_view_tile(X, base, v.trans, b, bx, r, n, c0, tc);
    __syncthreads();
    zero_acc(acc);
    gemm_tn_4x4(Lt, X, n, acc);
    __syncthreads();
    acc_to_lds(acc, X);
    __syncthreads();
    store_view_tile(X, base, v.trans, b, bx, r, n, c0, tc);
  }
}

// T(a, c) -= P_a^T P_c, P_a = rows n_i of panel a (0 = basis columns of D_i).
template <typename T>
__global__ __launch_bounds__(NT) void k_schur_t(LevelArgs<T> A, int32_t p0) {
  // the pairs of one step (consecutive) on one XCD: their panels are fetched
  // into one L2 and reused there
  const Pair pr = A.pairs[p0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[pr.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b > 64) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  T* D = A.arena + A.slot_off[i];
  int la, lc, ba = b, bc = b, ta = 0, tcv = 0;
  T* pa;
  T* pc;
  if (pr.a == 0) {
    la = r;
    pa = D;
  } else {
    const View va = A.views[st.view0 + pr.a - 1];
    ba = A.bsz[va.x];
    la = va.proc ? A.rank[va.x] : ba;
    pa = A.arena + A.slot_off[va.slot];
    ta = va.trans;
  }
  if (pr.c == 0) {
    lc = r;
    pc = D;
  } else {
    const View vc = A.views[st.view0 + pr.c - 1];
    bc = A.bsz[vc.x];
    lc = vc.proc ? A.rank[vc.x] : bc;
    pc = A.arena + A.slot_off[vc.slot];
    tcv = vc.trans;
  }
  if (la == 0 || lc == 0) return;
  T* tbase;
  int ts_a, ts_c;   // target strides (a slot of at most 64 x bmax entries)
  if (pr.a == 0) {
    if (pr.c == 0) {
      tbase = D;
      ts_a = b;
      ts_c = 1;
    } else {
      tbase = pc;
      ts_a = tcv ? 1 : bc;
      ts_c = tcv ? b : 1;
    }
  } else {
    tbase = A.arena + A.slot_off[pr.slot];
    if (pr.trans) {
      ts_a = 1;
      ts_c = ba;
    } else {
      ts_a = bc;
      ts_c = 1;
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Pa = reinterpret_cast<T*>(smem_raw);
  T* Pc = Pa + 64 * TLD;
  // FP64 matrix cores: wavefront w owns rows 16w .. 16w + 15 of the 64 x 64
  // target tile, as four 16 x 16 tiles; v_mfma_f64_16x16x4f64 operand
  // lanes: A (row l % 16, k l / 16), B (k l / 16, column l % 16); result
  // register j of lane l holds (row 4 j + l / 16, column l % 16)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  // rows n .. n4 - 1 of both tiles stay zero: the k loop runs in whole steps
  // of four without predicates (the loads only write rows below n)
  const int n4 = (n + 3) & ~3;
  for (int e = threadIdx.x; e < (n4 - n) * 64; e += NT) {
    Pa[(n + (e >> 6)) * TLD + (e & 63)] = T(0);
    Pc[(n + (e >> 6)) * TLD + (e & 63)] = T(0);
  }
  const T* fa = Pa + fk * TLD + 16 * wv + fr;
  const T* fc = Pc + fk * TLD + fr;
  for (int a0 = 0; a0 < la; a0 += 64) {
    const int tan = min(64, la - a0);
    for (int c0 = 0; c0 < lc; c0 += 64) {
      const int tcn = min(64, lc - c0);
      __syncthreads();
      // both operand tiles in one round of loads, then the target entries
      // this lane updates, in flight while the products run
      // the Pa tile is loaded with the first Pc tile of its row of targets
      load_tile_pair(Pa, pa, TileSrc{ta, b, ba, a0, c0 == 0 ? tan : 0}, pc, TileSrc{tcv, b, bc, c0, tcn}, r, n);
      T tv[4][4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int al = 16 * wv + 4 * j + fk, gm = 16 * tj + fr;
          tv[tj][j] = (al < tan && gm < tcn) ? tbase[(a0 + al) * ts_a + (c0 + gm) * ts_c] : T(0);
        }
      __syncthreads();
      dbl4 dacc[4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) dacc[tj] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
      for (int k0 = 0; k0 < n4; k0 += 4) {
        const double av = (double)fa[k0 * TLD];
        double bv[4];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) bv[tj] = (double)fc[k0 * TLD + 16 * tj];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) dacc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tj], dacc[tj], 0, 0, 0);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int al = 16 * wv + 4 * j + fk, gm = 16 * tj + fr;
          if (al < tan && gm < tcn)
            tbase[(a0 + al) * ts_a + (c0 + gm) * ts_c] = (T)((double)tv[tj][j] - dacc[tj][j]);
        }
    }
  }
}

// Schur update with BF16 inputs and FP32 accumulation on the matrix cores
// (FP32 factor, reduced-precision mode): the 64 x 64 target tile is four
// 32 x 32 MFMA tiles, one per wavefront, v_mfma_f32_32x32x8bf16_1k over the
// n_i rows of the panels (zero-padded to a multiple of 8).  Operand lanes: A
// row i = lane % 32, k = 4 (lane / 32) + 0..3; B column j = lane % 32, same k;
// result register v holds row 8 (v / 4) + 4 (lane / 32) + v % 4, column
// lane % 32.  Panels are staged in LDS in FP32 and rounded to BF16 (nearest
// even) when loaded into the operands.
// ---------------------------------------------------------------------------
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ inline short to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_schur_bf16(LevelArgs<T> A, int32_t p0) {
  const Pair pr = A.pairs[p0 + blockIdx.x];
  const Step st = A.steps[pr.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b > 64) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  T* D = A.arena + A.slot_off[i];
  int la, lc, ba = b, bc = b, ta = 0, tcv = 0;
  T* pa;
  T* pc;
  if (pr.a == 0) {
    la = r;
    pa = D;
  } else {
    const View va = A.views[st.view0 + pr.a - 1];
    ba = A.bsz[va.x];
    la = va.proc ? A.rank[va.x] : ba;
    pa = A.arena + A.slot_off[va.slot];
    ta = va.trans;
  }
  if (pr.c == 0) {
    lc = r;
    pc = D;
  } else {
    const View vc = A.views[st.view0 + pr.c - 1];
    bc = A.bsz[vc.x];
    lc = vc.proc ? A.rank[vc.x] : bc;
    pc = A.arena + A.slot_off[vc.slot];
    tcv = vc.trans;
  }
  if (la == 0 || lc == 0) return;
  T* tbase;
  int64_t ts_a, ts_c;
  if (pr.a == 0) {
    if (pr.c == 0) {
      tbase = D;
      ts_a = b;
      ts_c = 1;
    } else {
      tbase = pc;
      ts_a = tcv ? 1 : bc;
      ts_c = tcv ? b : 1;
    }
  } else {
    tbase = A.arena + A.slot_off[pr.slot];
    if (pr.trans) {
      ts_a = 1;
      ts_c = ba;
    } else {
      ts_a = bc;
      ts_c = 1;
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Pa = reinterpret_cast<T*>(smem_raw);
  T* Pc = Pa + 64 * TLD;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int si = wv >> 1, sj = wv & 1;
  const int nk = (n + 7) & ~7;
  for (int a0 = 0; a0 < la; a0 += 64) {
    const int tan = min(64, la - a0);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += NT) Pa[(e >> 6) * TLD + (e & 63)] = T(0);
    __syncthreads();
    load_view_tile_lean(Pa, pa, ta, b, ba, r, n, a0, tan);
    for (int c0 = 0; c0 < lc; c0 += 64) {
      const int tcn = min(64, lc - c0);
      __syncthreads();
      for (int e = threadIdx.x; e < 64 * 64; e += NT) Pc[(e >> 6) * TLD + (e & 63)] = T(0);
      __syncthreads();
      load_view_tile_lean(Pc, pc, tcv, b, bc, r, n, c0, tcn);
      __syncthreads();
      f32x16_t acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
      const int ia = si * 32 + (lane & 31), jb = sj * 32 + (lane & 31);
      for (int k0 = 0; k0 < nk; k0 += 8) {
        bf16x4_t av, bv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int k = k0 + 4 * (lane >> 5) + t;
          av[t] = to_bf16((float)Pa[k * TLD + ia]);
          bv[t] = to_bf16((float)Pc[k * TLD + jb]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int al = si * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int gm = sj * 32 + (lane & 31);
        if (al < tan && gm < tcn) {
          T* tp = tbase + (int64_t)(a0 + al) * ts_a + (int64_t)(c0 + gm) * ts_c;
          *tp = (T)((float)*tp - acc[v]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Level set-up and transition.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_scatter_a0(T* arena, const double* vals, const int64_t* dst, int64_t nnz) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = dst[e];
    if (d >= 0) arena[d] = (T)vals[e];
  }
}

// out[0] = eps * max_i A_ii, out[1] = max_i A_ii.  Diagonal entries of an SPD
// matrix are positive, so their IEEE bit patterns order like the values;
// out[1] is cleared beforehand.
__global__ void k_theta_max(const double* vals, const int64_t* diag_pos, int64_t n, unsigned long long* out_bits) {
  __shared__ double red[NT];
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    m = fmax(m, vals[diag_pos[i]]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.0) atomicMax(out_bits, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_theta_fin(double eps, double* out) { out[0] = eps * out[1]; }

template <typename T>
__global__ void k_gather_next(const Trans* items, const T* src, const int64_t* src_off, const int32_t* bsz,
                              const int32_t* rank, const int32_t* parent, const int32_t* off_in_parent,
                              T* dst, const int64_t* dst_off, const int32_t* bsz_next) {
  const Trans t = items[blockIdx.x];
  const int rp = rank[t.p], rq = rank[t.q];
  if (rp == 0 || rq == 0) return;
  const int bq = bsz[t.q];
  const int ldn = bsz_next[parent[t.q]];
  const int op = off_in_parent[t.p], oq = off_in_parent[t.q];
  const T* s = src + src_off[t.src_slot];
  T* d = dst + dst_off[t.dst_slot];
  const bool mirror = (t.p != t.q) && (parent[t.p] == parent[t.q]);
  for (int e = threadIdx.x; e < rp * rq; e += blockDim.x) {
    const int a = e / rq, c = e % rq;
    const T val = s[(int64_t)a * bq + c];
    d[(int64_t)(op + a) * ldn + oq + c] = val;
    if (mirror) d[(int64_t)(oq + c) * ldn + op + a] = val;
  }
}

// Dense remainder A_K (FP64, row-major dim x dim) from the slots of a level.
template <typename T>
__global__ void k_coarse_assemble(const int32_t* slot_p, const int32_t* slot_q, const T* arena,
                                  const int64_t* slot_off, const int32_t* bsz, const int64_t* dof_off,
                                  double* Ad, int64_t dim) {
  const int s = blockIdx.x;
  const int p = slot_p[s], q = slot_q[s];
  const int bp = bsz[p], bq = bsz[q];
  const T* src = arena + slot_off[s];
  const int64_t op = dof_off[p], oq = dof_off[q];
  for (int e = threadIdx.x; e < bp * bq; e += blockDim.x) {
    const int a = e / bq, c = e % bq;
    const double v = (double)src[e];
    Ad[(op + a) * dim + oq + c] = v;
    if (p != q) Ad[(oq + c) * dim + op + a] = v;
  }
}

// ---------------------------------------------------------------------------
// Dense inverse of the remainder by symmetric block Gauss-Jordan sweeps:
// after sweeping every pivot block the matrix holds -A_K^{-1}.
// ---------------------------------------------------------------------------
constexpr int GJ = 64;

constexpr int GJP = 4;                            // pivot inverse: a GJP x GJP tile per thread
constexpr int GJT = (64 / GJP) * (64 / GJP);      // its threads

static_assert(GJT == NT, "the pivot inverse runs inside the 256-thread update kernel too");

__device__ void gj_pivot_block(const double* Ad, int64_t dim, int64_t k0, int kb, double* Pinv, int32_t* err,
                               double* Sy) {
  // Gauss-Jordan elimination without pivoting of the kb x kb pivot block
  // (read from its lower triangle), in place: after step k the leading k + 1
  // rows and columns hold the inverse of the leading block, the rest its Schur
  // complement.  Each thread keeps a GJP x GJP tile of the 64 x 64 array in
  // registers (identity beyond kb); row k and column k reach the other
  // threads through LDS, two alternating buffers, one barrier per step, and
  // the step itself is straight-line code (the steps unrolled by GJP, so the
  // row and column a thread publishes are fixed registers).  The pivots are
  // the leading entries of the successive Schur complements: all positive
  // exactly when the block is positive definite.
  constexpr int TS = 64 / GJP;
  __shared__ double Rb[2][64], Cb[2][64];
  // Sy: 64 x TLD doubles of LDS, the result before symmetrisation
  const int tid = threadIdx.x, ty = tid / TS, tx = tid % TS;
  double a[GJP][GJP];
#pragma unroll
  for (int p = 0; p < GJP; ++p)
#pragma unroll
    for (int q = 0; q < GJP; ++q) {
      const int i = GJP * ty + p, j = GJP * tx + q;
      a[p][q] = (i < kb && j < kb) ? Ad[(k0 + max(i, j)) * dim + k0 + min(i, j)] : (i == j ? 1.0 : 0.0);
    }
  bool bad = false;
  for (int kg = 0; kg < kb; kg += GJP)
#pragma unroll
    for (int kq = 0; kq < GJP; ++kq) {
      const int k = kg + kq, h = kq & 1;
      if (k >= kb) break;
      if (ty == kg / GJP)
#pragma unroll
        for (int q = 0; q < GJP; ++q) Rb[h][GJP * tx + q] = a[kq][q];
      if (tx == kg / GJP)
#pragma unroll
        for (int p = 0; p < GJP; ++p) Cb[h][GJP * ty + p] = a[p][kq];
      __syncthreads();
      const double piv = Rb[h][k];
      bad = bad || !(piv > 0.0);
      // 1 / piv: the hardware estimate and two Newton steps
      const double pv = piv > 0.0 ? piv : 1.0;
      double ip = __builtin_amdgcn_rcp(pv);
      ip = fma(ip, fma(-pv, ip, 1.0), ip);
      ip = fma(ip, fma(-pv, ip, 1.0), ip);
      double rk[GJP], ck[GJP];
#pragma unroll
      for (int q = 0; q < GJP; ++q) rk[q] = Rb[h][GJP * tx + q] * ip;
#pragma unroll
      for (int p = 0; p < GJP; ++p) ck[p] = Cb[h][GJP * ty + p];
#pragma unroll
      for (int p = 0; p < GJP; ++p) {
        const bool ri = GJP * ty + p == k;
        const double nc = -ck[p] * ip;
#pragma unroll
        for (int q = 0; q < GJP; ++q) {
          const bool cj = GJP * tx + q == k;
          const double g = fma(-ck[p], rk[q], a[p][q]);
          const double rv = cj ? ip : rk[q];
          const double ov = cj ? nc : g;
          a[p][q] = ri ? rv : ov;
        }
      }
    }
  // the inverse is symmetric: store the mean of the two triangles
#pragma unroll
  for (int p = 0; p < GJP; ++p)
#pragma unroll
    for (int q = 0; q < GJP; ++q) Sy[(GJP * ty + p) * TLD + GJP * tx + q] = a[p][q];
  __syncthreads();
#pragma unroll
  for (int p = 0; p < GJP; ++p)
#pragma unroll
    for (int q = 0; q < GJP; ++q) {
      const int i = GJP * ty + p, j = GJP * tx + q;
      if (i < kb && j < kb) Pinv[i * GJ + j] = 0.5 * (a[p][q] + Sy[j * TLD + i]);
    }
  if (tid == 0 && bad) {
    if (atomicCAS(err, 0, 1) == 0) err[1] = -1;
  }
}

// The pivot inverse of the first panel (later ones run inside k_gj_update).
__global__ __launch_bounds__(GJT) void k_gj_pivot(double* Ad, int64_t dim, int64_t k0, int kb, double* Pinv,
                                                  int32_t* err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  gj_pivot_block(Ad, dim, k0, kb, Pinv, err, reinterpret_cast<double*>(smem_raw));
}

// W = Pinv * A[k-block, :] and R0 = A[k-block, :]  (kb x dim each, ld dim);
// the product on the FP64 matrix cores as in k_gj_update (Pinv symmetric).
__device__ inline void stage_panel64(double* S, const double* src, int64_t ld, int64_t c0, int kb, int kb4, int nc);
__global__ __launch_bounds__(NT) void k_gj_rows(const double* Ad, int64_t dim, int64_t k0, int kb,
                                                const double* Pinv, double* W, double* R0) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* P = reinterpret_cast<double*>(smem_raw);
  double* X = P + 64 * TLD;
  const int64_t c0 = (int64_t)blockIdx.x * GJ;
  const int tc = (int)min<int64_t>(GJ, dim - c0);
  const int kb4 = (kb + 3) & ~3;
  stage_panel64(P, Pinv, GJ, 0, kb, kb4, kb);
  stage_panel64(X, Ad + k0 * dim, dim, c0, kb, kb4, tc);
  __syncthreads();
  for (int e = threadIdx.x; e < kb * 64; e += NT) {
    const int t = e >> 6, c = e & 63;
    if (c < tc) R0[t * dim + c0 + c] = X[t * TLD + c];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  dbl4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  const double* fa = P + fk * TLD + 16 * wv + fr;
  const double* fb = X + fk * TLD + fr;
#pragma unroll 2
  for (int t0 = 0; t0 < kb4; t0 += 4) {
    const double av = fa[t0 * TLD];
    double bv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = fb[t0 * TLD + 16 * c];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[c], acc[c], 0, 0, 0);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ra = 16 * wv + 4 * j + fk, cc = 16 * c + fr;
      if (ra < kb && cc < tc) W[ra * dim + c0 + cc] = acc[c][j];
    }
}

// Rows t < kb4 of the 64-column window [c0, c0 + nc) of the kb x ? row panel
// src (leading dimension ld) into S (row stride TLD), zero in rows kb .. kb4 - 1
// and in the columns beyond nc; eight loads in flight per thread.
__device__ inline void stage_panel64(double* S, const double* src, int64_t ld, int64_t c0, int kb, int kb4, int nc) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + NT * (8 * h + u), t = e >> 6, c = e & 63;
      v[u] = (t < kb && c < nc) ? src[t * ld + c0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + NT * (8 * h + u), t = e >> 6;
      if (t < kb4) S[t * TLD + (e & 63)] = v[u];
    }
  }
}

// A <- A - R0^T W on the 64 x 64 tile (i0, j0), the pivot rows and columns
// replaced by the corresponding rows of W and -Pinv (the Gauss-Jordan step).
// The product on the FP64 matrix cores: wavefront w owns tile rows
// 16w .. 16w + 15 as four 16 x 16 tiles of v_mfma_f64_16x16x4f64 (operand
// lanes: A (row l % 16, k l / 16), B (k l / 16, column l % 16); result
// register j of lane l: (row 4 j + l / 16, column l % 16)).
__global__ __launch_bounds__(NT) void k_gj_update(double* Ad, int64_t dim, int64_t k0, int kb,
                                                  const double* Pinv, const double* W, const double* R0,
                                                  double* Pnext, int32_t* err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Ri = reinterpret_cast<double*>(smem_raw);
  double* Wj = Ri + 64 * TLD;
  const int64_t i0 = (int64_t)blockIdx.y * GJ, j0 = (int64_t)blockIdx.x * GJ;
  const int ti = (int)min<int64_t>(GJ, dim - i0), tj = (int)min<int64_t>(GJ, dim - j0);
  const int kb4 = (kb + 3) & ~3;
  stage_panel64(Ri, R0, dim, i0, kb, kb4, ti);
  stage_panel64(Wj, W, dim, j0, kb, kb4, tj);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  // the tile entries this lane rewrites, in flight while the products run
  double old[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int li = 16 * wv + 4 * j + fk, lj = 16 * c + fr;
      old[c][j] = (li < ti && lj < tj) ? Ad[(i0 + li) * dim + j0 + lj] : 0.0;
    }
  __syncthreads();
  dbl4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  const double* fa = Ri + fk * TLD + 16 * wv + fr;
  const double* fb = Wj + fk * TLD + fr;
#pragma unroll 2
  for (int t0 = 0; t0 < kb4; t0 += 4) {
    const double av = fa[t0 * TLD];
    double bv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = fb[t0 * TLD + 16 * c];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[c], acc[c], 0, 0, 0);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int li = 16 * wv + 4 * j + fk, lj = 16 * c + fr;
      if (li >= ti || lj >= tj) continue;
      const int64_t i = i0 + li, jj = j0 + lj;
      const bool ik = i >= k0 && i < k0 + kb, jk = jj >= k0 && jj < k0 + kb;
      double v;
      if (ik && jk)
        v = -Pinv[(i - k0) * GJ + (jj - k0)];
      else if (ik)
        v = W[(i - k0) * dim + jj];
      else if (jk)
        v = W[(jj - k0) * dim + i];
      else
        v = old[c][j] - acc[c][j];
      Ad[i * dim + jj] = v;
    }
  // the workgroup holding the next pivot block inverts it as soon as it is
  // written (into the other pivot buffer): no separate launch per panel
  const int64_t kn = k0 + kb;
  if (Pnext && i0 == kn && j0 == kn) {
    __syncthreads();   // the block's entries, written by all threads, visible to all
    gj_pivot_block(Ad, dim, kn, (int)min<int64_t>(GJ, dim - kn), Pnext, err, Ri);
  }
}

// C (m x n, row stride ldc) = alpha op(A) op(B) + diag I by one workgroup on
// the FP64 matrix cores: 64 x 64 output tiles in turn, 64 columns of the
// inner dimension at a time staged in LDS (Sa, Sb: 64 x TLD doubles each);
// operand and result lanes as in k_bg_gram.  op(A)(p, q) = A[p lda + q], or
// A[q lda + p] with ta; op(B)(q, c) = B[q ldb + c], or B[c ldb + q] with tb.
// With sym the product is known to be symmetric: only the tiles on and above
// the diagonal are formed, and mirrored.  C takes the result in its own type,
// C2 (if not null, same layout) in FP64.  Returns, to every thread, the sum
// of squares of the result and its trace.
template <typename TO>
__device__ double2 wg_gemm_f64(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, TO* C, int ldc,
                               int m, int n, int kd, bool sym, double alpha, double diag, double* C2, double* Sa,
                               double* Sb, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = lane >> 4;
  const int mt = (m + 63) / 64, nt = (n + 63) / 64;
  double f2 = 0.0, trc = 0.0;
  for (int ti = 0; ti < mt; ++ti)
    for (int tj = sym ? ti : 0; tj < nt; ++tj) {
      const int ra = 64 * ti, rb = 64 * tj, na = min(64, m - ra), nb = min(64, n - rb);
      dbl4 acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
      for (int kc = 0; kc < kd; kc += 64) {
        const int mc = min(64, kd - kc), mc4 = (mc + 3) & ~3;
        __syncthreads();   // the previous chunk's operands consumed
        // the unit-stride index of each operand on consecutive threads
        for (int e = tid; e < 64 * 64; e += NT) {
          const int k = ta ? (e >> 6) : (e & 63);
          const int a = ta ? (e & 63) : (e >> 6);
          double x = 0.0;
          if (k < mc && a < na)
            x = ta ? A[(int64_t)(kc + k) * lda + ra + a] : A[(int64_t)(ra + a) * lda + kc + k];
          Sa[k * TLD + a] = x;
          const int kq = tb ? (e & 63) : (e >> 6), c = tb ? (e >> 6) : (e & 63);
          double yv = 0.0;
          if (kq < mc && c < nb) yv = tb ? B[(int64_t)(rb + c) * ldb + kc + kq] : B[(int64_t)(kc + kq) * ldb + rb + c];
          Sb[kq * TLD + c] = yv;
        }
        __syncthreads();
        const double* fa = Sa + fk * TLD + 16 * wv + fr;
        const double* fb = Sb + fk * TLD + fr;
        for (int k0 = 0; k0 < mc4; k0 += 4) {
          const double av = fa[k0 * TLD];
          double bv[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) bv[c] = fb[k0 * TLD + 16 * c];
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[c], acc[c], 0, 0, 0);
        }
      }
      const double wgt = (sym && ti != tj) ? 2.0 : 1.0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 16 * wv + 4 * j + fk, col = 16 * c + fr;
          if (row < na && col < nb) {
            const bool dgl = ra + row == rb + col;
            const double v = alpha * acc[c][j] + (dgl ? diag : 0.0);
            C[(int64_t)(ra + row) * ldc + rb + col] = (TO)v;
            if (C2) C2[(int64_t)(ra + row) * ldc + rb + col] = v;
            if (sym && ti != tj) {
              C[(int64_t)(rb + col) * ldc + ra + row] = (TO)v;
              if (C2) C2[(int64_t)(rb + col) * ldc + ra + row] = v;
            }
            f2 += wgt * v * v;
            if (dgl) trc += v;
          }
        }
    }
  f2 = wave_sum_u(f2);
  trc = wave_sum_u(trc);
  __syncthreads();   // red free
  if (lane == 0) {
    red[wv] = f2;
    red[4 + wv] = trc;
  }
  __syncthreads();
  const double2 out = {(red[0] + red[1]) + (red[2] + red[3]), (red[4] + red[5]) + (red[6] + red[7])};
  // C visible to the whole workgroup before it is read as an operand
  __threadfence();
  __syncthreads();
  return out;
}

// ---------------------------------------------------------------------------
// Compression of blocks of BG_MIN..BG_MAXB unknowns (FP32 factor: the coarse
// levels of 3D problems with sibling coarsening, whose blocks join the kept
// unknowns of eight children).  The far row F_i (b x w) is reduced to its
// Gram matrix G = F F^T in FP64 on the matrix cores by many workgroups
// (k_bg_gram, one 64 x 64 tile of G each: the products of FP32 entries are
// exact in FP64).  One workgroup per step then (k_bg_eig):
//   1. pivoted Cholesky G ~ X^T X, stopped at the rounding level the smaller
//      blocks use (at most BG_MA rows);
//   2. S = X X^T (ma x ma): its eigenvalues are those of G, sigma_k(F)^2, and
//      an eigenvector w_k gives the left singular vector v_k = X^T w_k /
//      sigma_k of F;
//   3. one-sided Jacobi on the rows of S (the rows converge to lambda_k w_k^T);
//   4. r_i = #{sigma_k > theta}, the dropped energy, the kept v_k;
//   5. Householder reflectors of the kept directions and U_i = H_0 ... H_{r-1},
//      one wavefront per column of U_i.
// A step whose Gram matrix needs more than BG_MA pivots is flagged in big_fail
// for the generic kernel.
// ---------------------------------------------------------------------------
constexpr int BG_SLD = BG_MA + 4;   // row stride of S in LDS

// per step: G (b x b), X (BG_MA x b), U in FP64 (b x b), two work areas (b x b)
int64_t bg_stride(int bmax) { return (int64_t)4 * bmax * bmax + (int64_t)BG_MA * bmax; }

template <typename T>
__global__ __launch_bounds__(NT) void k_bg_gram(LevelArgs<T> A, int32_t s0, int32_t ntile) {
  // the ntile tile pairs of one step on one XCD, dispatched together: the
  // strips of F_i they share are fetched from HBM into that XCD's L2 once
  const int64_t lg = xcd_swizzle(blockIdx.x, gridDim.x);
  const int sx = (int)(lg / ntile);
  const Step st = A.steps[s0 + sx];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b < BG_MIN || b > BG_MAXB || st.nfar == 0) return;
  if (A.need_exact && !A.need_exact[i]) return;
  // tile pair (ti <= tj) of this workgroup
  const int nt = (b + 63) / 64;
  int t = (int)(lg % ntile), ti = 0;
  while (ti < nt && t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  if (ti >= nt) return;
  const int tj = ti + t;
  const int ra = 64 * ti, rb = 64 * tj;
  const int na = min(64, b - ra), nb = min(64, b - rb);
  double* G = A.big + (int64_t)sx * A.big_stride;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Sa = reinterpret_cast<T*>(smem_raw);   // Sa[k][a] = F(ra + a, column k of the chunk)
  T* Sb = Sa + 64 * TLD;                     // Sb[k][a] = F(rb + a, column k of the chunk)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, fr = lane & 15, fk = lane >> 4;
  dbl4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    for (int c0 = 0; c0 < w; c0 += 64) {
      const int mc = min(64, w - c0), mc4 = (mc + 3) & ~3;
      __syncthreads();
      // rows of the chunk k < mc4 (zero from mc on; a row-major view stages
      // all 64, so that the indices are shifts, not divisions), 64
      // coordinates (zero beyond na / nb); the unit-stride index on
      // consecutive threads
      for (int e = threadIdx.x; e < (v.trans ? 64 * mc4 : 64 * 64); e += NT) {
        const int k = v.trans ? (e >> 6) : (e & 63);
        const int a = v.trans ? (e & 63) : (e >> 6);
        // unconditional loads (the view's first entry outside the chunk)
        const bool oka = k < mc && a < na, okb = k < mc && a < nb;
        const T xa = base[oka ? (v.trans ? (int64_t)(c0 + k) * b + ra + a : (int64_t)(ra + a) * bx + c0 + k) : 0];
        const T xb = base[okb ? (v.trans ? (int64_t)(c0 + k) * b + rb + a : (int64_t)(rb + a) * bx + c0 + k) : 0];
        Sa[k * TLD + a] = oka ? xa : T(0);
        Sb[k * TLD + a] = okb ? xb : T(0);
      }
      __syncthreads();
      // FP64 matrix cores: wavefront w owns rows 16 w .. 16 w + 15 of the tile
      // as four 16 x 16 tiles (operand and result lanes as in k_schur_t)
      const T* fa = Sa + fk * TLD + 16 * wv + fr;
      const T* fb = Sb + fk * TLD + fr;
      for (int k0 = 0; k0 < mc4; k0 += 4) {
        const double av = (double)fa[k0 * TLD];
        double bv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = (double)fb[k0 * TLD + 16 * c];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[c], acc[c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 16 * wv + 4 * j + fk, col = 16 * c + fr;
      if (row < na && col < nb) {
        G[(int64_t)(ra + row) * b + rb + col] = acc[c][j];
        if (ti != tj) G[(int64_t)(rb + col) * b + ra + row] = acc[c][j];
      }
    }
}

// Left-looking pivoted Cholesky G ~ X^T X of a b x b Gram matrix (row
// stride b): row k of X (stride ldx, columns in G's order) from column p of G,
// p the largest trailing diagonal entry, until the trailing trace is at most
// stop2 or cap rows are written.  dg (b doubles, G's diagonal on entry) and
// chosen (b bytes, zero on entry) in LDS, xp (cap doubles), rd / ri (8
// slots); every thread of the workgroup calls it.  Returns the number of rows;
// *inactive = the trailing trace, *truncated = stopped by the cap.
__device__ int gram_pivoted_chol(const double* G, double* X, int ldx, int b, double stop2, int cap, double* dg,
                                 double* xp, unsigned char* chosen, double* rd, int* ri, double* inactive,
                                 bool* truncated) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int k = 0;
  *truncated = false;
  for (;; ++k) {
    __syncthreads();   // dg and chosen of the previous pivot, rd free
    double rs = 0.0, cv = -1.0;
    int ci = 0x7fffffff;
    for (int t = tid; t < b; t += NT)
      if (!chosen[t]) {
        rs += dg[t];
        if (dg[t] > cv) {
          cv = dg[t];
          ci = t;
        }
      }
    rs = wave_sum_u(rs);
    wave_argmax_u(cv, ci);
    if (lane == 0) {
      rd[wv] = rs;
      rd[4 + wv] = cv;
      ri[wv] = ci;
    }
    __syncthreads();
    rs = (rd[0] + rd[1]) + (rd[2] + rd[3]);
    cv = rd[4];
    ci = ri[0];
    for (int u = 1; u < 4; ++u) amax_step(cv, ci, rd[4 + u], ri[u]);
    if (rs <= stop2 || !(cv > 0.0)) {
      *inactive = rs;
      break;
    }
    if (k == cap) {
      // truncated: the trailing energy rs stays outside X
      *inactive = rs;
      *truncated = true;
      break;
    }
    const int p = ci;
    const double ilpp = 1.0 / sqrt(cv), lpp = cv * ilpp;
    for (int j = tid; j < k; j += NT) xp[j] = X[(int64_t)j * ldx + p];
    __syncthreads();
    for (int t = tid; t < b; t += NT) {
      double s = G[(int64_t)p * b + t];
      int j = 0;
      for (; j + 4 <= k; j += 4)
        s -= (X[(int64_t)j * ldx + t] * xp[j] + X[(int64_t)(j + 1) * ldx + t] * xp[j + 1]) +
             (X[(int64_t)(j + 2) * ldx + t] * xp[j + 2] + X[(int64_t)(j + 3) * ldx + t] * xp[j + 3]);
      for (; j < k; ++j) s -= X[(int64_t)j * ldx + t] * xp[j];
      const double lv = chosen[t] ? 0.0 : (t == p ? lpp : s * ilpp);
      X[(int64_t)k * ldx + t] = lv;
      if (!chosen[t] && t != p) dg[t] -= lv * lv;
    }
    __syncthreads();
    if (tid == 0) chosen[p] = 1;
  }
  return k;
}

template <typename T>
size_t work_bg_eig() {
  return (size_t)BG_MA * BG_SLD * sizeof(double) + (size_t)BG_MAXB * sizeof(double) +
         (size_t)4 * BG_MA * sizeof(double) + (size_t)3 * BG_MA * sizeof(int) + (size_t)BG_MAXB;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_bg_eig(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b < BG_MIN || b > BG_MAXB) return;
  if (A.need_exact && !A.need_exact[i]) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T* Ug = A.U + A.u_off[i];
  if (st.nfar == 0) {
    for (int e = tid; e < b * b; e += NT) Ug[e] = (e / b == e % b) ? T(1) : T(0);
    if (tid == 0) {
      A.rank[i] = 0;
      A.edrop[i] = 0.0;
      if (A.rec) A.rec[(A.rec_off + i) * REC_W + NFEAT] = -1.0f;
    }
    return;
  }
  double* G = A.big + (int64_t)blockIdx.x * A.big_stride;   // b x b, left intact
  double* X = G + (int64_t)b * b;                              // BG_MA x b rows of the Cholesky factor
  double* U64 = X + (int64_t)BG_MA * b;                        // U_i in FP64 (steps left to k_bg_cert)
  double* V = U64 + (int64_t)b * b;                            // kept directions, then reflectors
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = reinterpret_cast<double*>(smem_raw);   // BG_MA x BG_SLD
  double* dg = S + BG_MA * BG_SLD;                   // trailing diagonal
  double* xp = dg + BG_MAXB;                         // X(j, p) of the current pivot
  double* sg = xp + BG_MA;                           // eigenvalues of S
  double* tau = sg + BG_MA;                          // sorted eigenvalues, then reflector coefficients
  double* isg = tau + BG_MA;
  int* posv = reinterpret_cast<int*>(isg + BG_MA);
  int* brow = posv + BG_MA;
  int* rowix = brow + BG_MA;
  unsigned char* chosen = reinterpret_cast<unsigned char*>(rowix + BG_MA);
  __shared__ double rd[8];
  __shared__ int ri[8];
  __shared__ double shd[4];
  __shared__ int shi[4];
  const double theta = *A.theta;
  const int64_t t_start = clock64();

  // ---- 1. pivoted Cholesky (left-looking): row k of X from column p of G ----
  double tr = 0.0;
  for (int t = tid; t < b; t += NT) {
    dg[t] = G[(int64_t)t * b + t];
    chosen[t] = 0;
    tr += dg[t];
  }
  tr = wave_sum_u(tr);
  if (lane == 0) rd[wv] = tr;
  __syncthreads();
  const double fro2 = rd[0] + rd[1] + rd[2] + rd[3];
  const double noise = (double)Eps<T>::v() * sqrt(fro2);
  const double negl = A.rank_mode == 0 ? fmax(noise, theta / 64.0) : noise;
  const double aerr = A.rank_mode == 0 ? fmax(noise, fmin((double)max(b, 16) * noise, theta / 32.0))
                                       : (double)max(b, 16) * noise;
  // CE(eps): pivots stop once the trailing energy is below (theta / 32)^2 at
  // the latest (it shifts a sigma near theta by at most theta / 2048); an FP64
  // factor would otherwise pivot down to its rounding level
  const double stop2 = A.rank_mode == 0 ? fmax(aerr * aerr, theta * theta / 1024.0) : aerr * aerr;
  double inactive = 0.0;
  bool truncated = false;
  // at most bg_cap <= BG_MA pivots (the learned width does not cap big blocks:
  // their far rows carry long tails of singular values just below theta)
  const int k = gram_pivoted_chol(G, X, b, b, stop2, min(max(A.bg_cap, 1), BG_MA), dg, xp, chosen, rd, ri,
                                  &inactive, &truncated);
  const int ma = k;
  __syncthreads();
  const int64_t t_chol = clock64();
  // the products' LDS staging shares the region of S (never live together)
  double* Sa = S;
  double* Sb = S + 64 * TLD;

  // a truncated Cholesky leaves G2 = G - X^T X (positive semidefinite); the
  // step is kept if lambda_{r+1}(X^T X) + ||G2||_F <= theta^2: then
  // lambda_{r+1}(G) <= theta^2 too (Weyl, ||G2||_2 <= ||G2||_F), so r is the
  // rank of F_i and the dropped part has spectral norm <= theta; otherwise
  // k_bg_cert bounds the dropped part's spectral norm itself (big_fail = 2)
  // from the basis this kernel still writes (lambda_r(G) >= lambda_r(X^T X) >
  // theta^2 holds in any case, as G - X^T X is positive semidefinite).
  // ||G2||_F from X^T X formed on the matrix cores (in U64's storage).
  double g2n = 0.0;
  if (truncated && A.rank_mode == 0) {
    wg_gemm_f64<double>(X, b, true, X, b, false, U64, b, b, b, ma, true, 1.0, 0.0, nullptr, Sa, Sb, rd);
    double f2 = 0.0;
    for (int e = tid; e < b * b; e += NT) {
      const double g = G[e] - U64[e];
      f2 += g * g;
    }
    f2 = wave_sum_u(f2);
    if (lane == 0) rd[wv] = f2;
    __syncthreads();
    g2n = sqrt((rd[0] + rd[1]) + (rd[2] + rd[3]));
    __syncthreads();   // rd free
  }

  // ---- 2. S = X X^T (ma x ma) on the matrix cores, through V's storage ------
  wg_gemm_f64<double>(X, b, false, X, b, true, V, ma, ma, ma, b, true, 1.0, 0.0, nullptr, Sa, Sb, rd);
  for (int e = tid; e < BG_MA * BG_MA; e += NT) {
    const int p = e / BG_MA, q = e % BG_MA;
    S[p * BG_SLD + q] = (p < ma && q < ma) ? V[p * ma + q] : 0.0;
  }
  if (tid < BG_MA) rowix[tid] = tid;
  __syncthreads();
  const int64_t t_s = clock64();

  // ---- 3. one-sided Jacobi on the rows of S (the four wavefronts) -----------
  // the row norms are lambda = sigma^2: the thresholds of the sigma-scale
  // tests squared
  int nsweep = 0;
  if (ma > 1) {
    const double tol = (double)max(b, 16) * DBL_EPSILON;
    const int np = (ma + 1) / 2;
    if (np <= 4) nsweep = jacobi_rows_wg<16, BG_MA>(S, BG_SLD, rowix, ma, negl * negl, aerr * aerr, tol);
    else if (np <= 8) nsweep = jacobi_rows_wg<8, BG_MA>(S, BG_SLD, rowix, ma, negl * negl, aerr * aerr, tol);
    // rows of 64, 96 or 128 coordinates (those beyond ma are zero): fewer LDS
    // reads for the steps with fewer pivots, loops of a fixed trip count
    else if (ma <= 64) nsweep = jacobi_rows_wg<4, 64>(S, BG_SLD, rowix, ma, negl * negl, aerr * aerr, tol);
    else if (ma <= 96) nsweep = jacobi_rows_wg<4, 96>(S, BG_SLD, rowix, ma, negl * negl, aerr * aerr, tol);
    else nsweep = jacobi_rows_wg<4, BG_MA>(S, BG_SLD, rowix, ma, negl * negl, aerr * aerr, tol);
  }
  __syncthreads();
  const int64_t t_eig = clock64();

  // ---- 4. eigenvalues, order, rank, dropped energy ---------------------------
  if (tid < ma) {
    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < BG_MA; q += 2) {
      s0 += S[tid * BG_SLD + q] * S[tid * BG_SLD + q];
      s1 += S[tid * BG_SLD + q + 1] * S[tid * BG_SLD + q + 1];
    }
    sg[tid] = sqrt(s0 + s1);   // lambda_k = sigma_k(F)^2
  }
  __syncthreads();
  int cnt = 0;
  if (tid < ma) {
    int pos = 0;
    const double l0 = sg[tid];
    for (int q = 0; q < ma; ++q) pos += (sg[q] > l0 || (sg[q] == l0 && q < tid)) ? 1 : 0;
    posv[tid] = pos;
    tau[pos] = l0;
    cnt = sqrt(l0) > theta ? 1 : 0;
  }
  cnt = __syncthreads_count(cnt);
  const int r = A.rank_mode == 0 ? cnt : min(A.fixed_rank, b);
  const int kb = min(r, ma);
  const bool cert = truncated && A.rank_mode == 0 && (r < ma ? tau[r] : 0.0) + g2n > theta * theta;
  if (tid == 0 && cert) A.big_fail[i] = 2;
  if (tid == 0 && A.bg_count && !cert) atomicAdd(A.bg_count + (truncated ? 1 : 0), 1);
  if (tid == 0) {
    double ed = inactive;
    for (int q = r; q < ma; ++q) ed += tau[q];
    shd[0] = ed;
    int label = 0;
    if (A.rec) {
      // the smallest sketch width that an ideal sketch would need to pass the
      // a-posteriori check (as the other compression kernels record it)
      const double th2 = theta * theta, sr2 = r < ma ? tau[r] : 0.0;
      double tail = inactive;
      int kf = ma;
      for (int kk = ma; kk >= r; --kk) {
        if (kk < ma) tail += tau[kk];
        if (tail + (kk > r ? sr2 : 0.0) <= th2) kf = kk;
      }
      label = max(kf, r);
    }
    shi[0] = label;
  }
  if (tid < ma && posv[tid] < kb) {
    brow[posv[tid]] = tid;
    // v = X^T w / sigma with w = row / lambda: X^T row * lambda^{-3/2}
    const double l0 = sg[tid];
    isg[posv[tid]] = l0 > 0.0 ? 1.0 / (l0 * sqrt(l0)) : 0.0;
  }
  __syncthreads();

  // ---- 5. kept directions v_k (b-vectors) ----------------------------------
  for (int t = tid; t < b; t += NT) {
    for (int c0 = 0; c0 < kb; c0 += 16) {
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.0;
      for (int j = 0; j < ma; ++j) {
        const double x = X[(int64_t)j * b + t];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c0 + u < kb) acc[u] += x * S[brow[c0 + u] * BG_SLD + j];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c0 + u < kb) V[(int64_t)(c0 + u) * b + t] = acc[u] * isg[c0 + u];
    }
  }
  __syncthreads();   // S consumed: its LDS is free from here on
  if (truncated && !cert && A.rank_mode == 0) {
    // a truncated step's dropped energy against G itself (the eigenvalues
    // leave G - X^T X out): ||E_i||_F^2 = ||F_i||_F^2 - sum_k v_k^T G v_k,
    // with V G formed on the matrix cores (in U64's storage)
    wg_gemm_f64<double>(V, b, false, G, b, false, U64, b, kb, b, b, false, 1.0, 0.0, nullptr, Sa, Sb, rd);
    double kept = 0.0;
    for (int e = tid; e < kb * b; e += NT) kept += V[e] * U64[e];
    kept = wave_sum_u(kept);
    if (lane == 0) rd[wv] = kept;
    __syncthreads();
    if (tid == 0) shd[0] = fmax(fro2 - ((rd[0] + rd[1]) + (rd[2] + rd[3])), 0.0);
    __syncthreads();
  }
  const int64_t t_dirs = clock64();

  // ---- 6. Householder reflectors of the kept directions ----------------------
  for (int cv = 0; cv < kb; ++cv) {
    double* vr = V + (int64_t)cv * b;
    if (wv == 0) {
      double xs = 0.0;
      for (int t = cv + lane; t < b; t += 64) xs += vr[t] * vr[t];
      const double nrm2 = wave_sum_u(xs);
      const double x0 = vr[cv];
      const double nrm = sqrt(nrm2);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vv = v0 * v0 + (nrm2 - x0 * x0);
      wave_sync();
      for (int t = lane; t < cv; t += 64) vr[t] = 0.0;
      if (lane == 0) {
        vr[cv] = v0;
        tau[cv] = vv > 0.0 ? 2.0 / vv : 0.0;
      }
    }
    __syncthreads();
    const double tc = tau[cv];
    for (int c2 = cv + 1 + wv; c2 < kb; c2 += 4) {
      double* br = V + (int64_t)c2 * b;
      double dd = 0.0;
      for (int t = cv + lane; t < b; t += 64) dd += vr[t] * br[t];
      dd = wave_sum_u(dd);
      for (int t = cv + lane; t < b; t += 64) br[t] -= tc * dd * vr[t];
    }
    __syncthreads();
  }

  // ---- 7. U_i = H_0 ... H_{kb-1} = I - V T V^T (compact WY form, T upper
  // triangular: T_jj = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) V(:, 0:j)^T v_j),
  // then U_i = I - V (T V^T) on the matrix cores ---------------------------
  double* Tm = S;   // kb x kb in LDS, stride BG_SLD: T above the diagonal, v_l^T v_j below
  for (int pq = wv; pq < kb * kb; pq += 4) {
    const int l = pq / kb, j = pq % kb;
    if (l >= j) continue;
    const double* vl = V + (int64_t)l * b;
    const double* vj = V + (int64_t)j * b;
    double dd = 0.0;
    for (int t = j + lane; t < b; t += 64) dd += vl[t] * vj[t];   // v_j is zero above row j
    dd = wave_sum_u(dd);
    if (lane == 0) Tm[j * BG_SLD + l] = dd;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    // T(l, j) for l < j from the finished columns 0..j-1
    if (tid < j) {
      double s = 0.0;
      for (int q = tid; q < j; ++q) s += Tm[tid * BG_SLD + q] * Tm[j * BG_SLD + q];
      Tm[tid * BG_SLD + j] = -tau[j] * s;
    }
    if (tid == 0) Tm[j * BG_SLD + j] = tau[j];
    __syncthreads();
  }
  // Z = T V^T (kb x b) into X's storage: thread t, 16 rows of Z at a time
  double* Z = X;
  for (int t = tid; t < b; t += NT) {
    for (int j0 = 0; j0 < kb; j0 += 16) {
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.0;
      for (int l = j0; l < kb; ++l) {
        const double x = V[(int64_t)l * b + t];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (j0 + u <= l) acc[u] += Tm[(j0 + u) * BG_SLD + l] * x;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (j0 + u < kb) Z[(int64_t)(j0 + u) * b + t] = acc[u];
    }
  }
  __syncthreads();   // Z complete, T consumed: the LDS holds the staging again
  wg_gemm_f64<T>(V, b, true, Z, b, false, Ug, b, b, b, kb, false, -1.0, 1.0, cert ? U64 : nullptr, Sa, Sb, rd);
  if (tid == 0) {
    A.rank[i] = r;
    A.edrop[i] = shd[0];
    if (A.rec) A.rec[(A.rec_off + i) * REC_W + NFEAT] = (float)shi[0] / (float)b;
    if (A.dbg) {
      // phase cycles: pivoted Cholesky, X X^T and Jacobi, truncation checks
      // and kept directions, reflectors and U_i
      int64_t* dd = A.dbg + 72 * (int64_t)i;
      dd[0] = ma;
      dd[1] = (truncated ? 1 : 0) + (cert ? 2 : 0);
      dd[2] = nsweep;
      dd[3] = b;
      dd[8] = t_s - t_chol;   // of which X X^T
      dd[4] = t_chol - t_start;
      dd[5] = t_eig - t_chol;
      dd[6] = t_dirs - t_eig;
      dd[7] = clock64() - t_dirs;
    }
  }
}

// Certificate for a big-block step whose truncated pivoted Cholesky did not
// settle its rank (big_fail = 2; k_bg_eig has written r_i and U_i, and U_i in
// FP64).  With U_2 the last b - r columns of U_i, the dropped part of the far
// row is U_2^T F_i, and C = U_2^T G U_2 is its Gram matrix.  For any r-column
// orthonormal basis, lambda_{r+1}(G) <= lambda_max(C) (Courant-Fischer), and
// lambda_r(G) > theta^2 already holds; so r_i is the rank of F_i at theta (eq.
// (rreav)) once lambda_max(C) <= theta^2, which also bounds the dropped part's
// spectral norm by theta as the compression requires (Section 2.3).  The
// bound: for symmetric C of order n and q >= 0,
//   ||C^(2^q)||_F^(1/2^q) / n^(1/2^(q+1)) <= lambda_max(C) <= ||C^(2^q)||_F^(1/2^q),
// with C^(2^q) formed by repeated squaring (each square normalized to unit
// Frobenius norm, the logarithm of the scale carried alongside).  Certified:
// big_fail = 0 and the dropped energy is trace(C).  Refuted, or undecided
// after BG_QMAX squarings: big_fail = 1, and the generic kernel redoes the
// step.
constexpr int BG_QMAX = 7;

template <typename T>
__global__ __launch_bounds__(NT) void k_bg_cert(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b < BG_MIN || b > BG_MAXB || st.nfar == 0) return;
  if (A.need_exact && !A.need_exact[i]) return;
  if (A.big_fail[i] != 2) return;
  const int r = A.rank[i], n2 = b - r;
  const double* G = A.big + (int64_t)blockIdx.x * A.big_stride;   // left intact (k_bg_full)
  const double* U64 = G + (int64_t)b * b + (int64_t)BG_MA * b;
  double* Y = const_cast<double*>(U64) + (int64_t)b * b;
  double* W = Y + (int64_t)b * b;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Sa = reinterpret_cast<double*>(smem_raw);
  double* Sb = Sa + 64 * TLD;
  __shared__ double red[8];
  const double theta = *A.theta, th2 = theta * theta;
  if (n2 <= 0) {
    if (threadIdx.x == 0) {
      A.big_fail[i] = 0;
      A.edrop[i] = 0.0;
      if (A.bg_count) atomicAdd(A.bg_count + 2, 1);
    }
    return;
  }
  // Y = G U_2 (b x n2), then C = U_2^T Y (n2 x n2) into W
  wg_gemm_f64<double>(G, b, false, U64 + r, b, false, Y, n2, b, n2, b, false, 1.0, 0.0, nullptr, Sa, Sb, red);
  const double2 ft =
      wg_gemm_f64<double>(U64 + r, b, true, Y, n2, false, W, n2, n2, n2, b, true, 1.0, 0.0, nullptr, Sa, Sb, red);
  const double tol = 1e-6;   // far above the rounding of the products
  int verdict = 0;           // 1 certified, -1 refuted
  if (ft.x > 0.0) {
    double ell = 0.5 * log(ft.x);   // log ||C^(2^q)||_F
    double* M = W;
    double* P = Y;
    double scale = exp(-ell);        // 1 / ||M||_F
    const double ln = log((double)n2);
    for (int q = 0;; ++q) {
      const double ub = exp(ell / (double)(1 << q));
      const double lb = exp(ell / (double)(1 << q) - ln / (double)(2 << q));
      if (ub * (1.0 + tol) <= th2) {
        verdict = 1;
        break;
      }
      if (lb * (1.0 - tol) > th2 || q == BG_QMAX) {
        verdict = -1;
        break;
      }
      // P = (M / ||M||_F)^2: its norm g gives log ||C^(2^(q+1))||_F = 2 ell + log g
      const double2 pg = wg_gemm_f64<double>(M, n2, false, M, n2, false, P, n2, n2, n2, n2, true, scale * scale, 0.0,
                                             nullptr, Sa, Sb, red);
      if (!(pg.x > 0.0)) {
        verdict = -1;   // not possible for a symmetric M of unit norm: left to the generic kernel
        break;
      }
      const double lg = 0.5 * log(pg.x);
      ell = 2.0 * ell + lg;
      scale = exp(-lg);
      double* tmp = M;
      M = P;
      P = tmp;
    }
  } else {
    verdict = 1;   // nothing dropped
  }
  if (threadIdx.x == 0) {
    A.big_fail[i] = verdict > 0 ? 0 : 1;
    if (verdict > 0) A.edrop[i] = fmax(ft.y, 0.0);
    if (A.bg_count && verdict > 0) atomicAdd(A.bg_count + 2, 1);
  }
}

// A big step the certificate refuted (big_fail = 1): the exact rank without a
// pivot cap.  The pivoted Cholesky of its Gram matrix runs to the end (up to b
// rows, the trailing energy of k_bg_eig), then a one-sided Jacobi on the rows
// of X (four wavefronts, rows of BM coordinates in global memory): X^T X ~ G
// is kept by the rotations and the rows converge to sigma_k u_k^T, u_k the
// left singular vectors of F_i, so r_i = #{sigma_k > theta}, the kept
// directions are the normalised leading rows, and reflectors complete them to
// U_i.  Settles the step (big_fail = 0).
template <int BM>
__device__ void bg_full_jacobi(double* Xr, const int* rowix, int ma, double negl, double aerr, double tol) {
  constexpr int LP = BM / 32;   // 32 coordinates per lane
  jacobi_rows_wg<LP, BM>(Xr, BM, rowix, ma, negl, aerr, tol);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_bg_full(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b < BG_MIN || b > BG_MAXB || st.nfar == 0) return;
  if (A.need_exact && !A.need_exact[i]) return;
  if (A.big_fail[i] != 1) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int BMr = b <= 256 ? 256 : 512;   // row length of X in the Jacobi
  const double* G = A.big + (int64_t)blockIdx.x * A.big_stride;
  double* Vk = const_cast<double*>(G) + (int64_t)b * b + (int64_t)BG_MA * b;   // kept directions (U64's area)
  double* Xr = Vk + (int64_t)b * b;                                           // ma x BMr rows (the two work areas)
  T* Ug = A.U + A.u_off[i];
  __shared__ double dg[BG_MAXB], xp[BG_MAXB], sg[BG_MAXB], tau[BG_MAXB];
  __shared__ int rowix[BG_MAXB], posv[BG_MAXB];
  __shared__ unsigned char chosen[BG_MAXB];
  __shared__ double rd[8];
  __shared__ int ri[8];
  const double theta = *A.theta;
  double tr = 0.0;
  for (int t = tid; t < b; t += NT) {
    dg[t] = G[(int64_t)t * b + t];
    chosen[t] = 0;
    tr += dg[t];
  }
  tr = wave_sum_u(tr);
  if (lane == 0) rd[wv] = tr;
  __syncthreads();
  const double fro2 = rd[0] + rd[1] + rd[2] + rd[3];
  const double noise = (double)Eps<T>::v() * sqrt(fro2);
  const double negl = A.rank_mode == 0 ? fmax(noise, theta / 64.0) : noise;
  const double aerr = A.rank_mode == 0 ? fmax(noise, fmin((double)max(b, 16) * noise, theta / 32.0))
                                       : (double)max(b, 16) * noise;
  const double stop2 = A.rank_mode == 0 ? fmax(aerr * aerr, theta * theta / 1024.0) : aerr * aerr;
  double inactive = 0.0;
  bool truncated = false;
  const int ma = gram_pivoted_chol(G, Xr, BMr, b, stop2, b, dg, xp, chosen, rd, ri, &inactive, &truncated);
  // zero coordinates b .. BMr - 1 of every row
  for (int e = tid; e < ma * (BMr - b); e += NT) Xr[(int64_t)(e / (BMr - b)) * BMr + b + e % (BMr - b)] = 0.0;
  for (int t = tid; t < ma; t += NT) rowix[t] = t;
  __syncthreads();
  if (ma > 1) {
    // rotations are skipped only below the rounding level of the stored
    // entries and of FP64 (the rows are on the sigma scale: a coarser level
    // would move a sigma near theta by that much)
    const double tol = (double)max(b, 16) * DBL_EPSILON;
    const double aerr_r = fmax(noise, tol * sqrt(fro2));
    if (BMr == 256) bg_full_jacobi<256>(Xr, rowix, ma, negl, aerr_r, tol);
    else bg_full_jacobi<512>(Xr, rowix, ma, negl, aerr_r, tol);
  }
  __syncthreads();
  // singular values, order, rank, dropped energy
  for (int k = tid; k < ma; k += NT) {
    double s2 = 0.0;
    for (int t = 0; t < b; ++t) s2 += Xr[(int64_t)k * BMr + t] * Xr[(int64_t)k * BMr + t];
    sg[k] = sqrt(s2);
  }
  __syncthreads();
  double cnt = 0.0;
  for (int k = tid; k < ma; k += NT) {
    int pos = 0;
    const double l0 = sg[k];
    for (int q = 0; q < ma; ++q) pos += (sg[q] > l0 || (sg[q] == l0 && q < k)) ? 1 : 0;
    posv[k] = pos;
    cnt += l0 > theta ? 1.0 : 0.0;
  }
  cnt = wave_sum_u(cnt);
  if (lane == 0) rd[4 + wv] = cnt;
  __syncthreads();
  const int r = A.rank_mode == 0 ? (int)((rd[4] + rd[5]) + (rd[6] + rd[7])) : min(A.fixed_rank, ma);
  if (tid == 0) {
    double ed = inactive;
    for (int k = 0; k < ma; ++k)
      if (posv[k] >= r) ed += sg[k] * sg[k];
    rd[0] = ed;
  }
  // kept directions: row k / sigma_k at position posv[k]
  for (int e = tid; e < ma * b; e += NT) {
    const int k = e / b, t = e % b;
    if (posv[k] < r) Vk[(int64_t)posv[k] * b + t] = sg[k] > 0.0 ? Xr[(int64_t)k * BMr + t] / sg[k] : 0.0;
  }
  __syncthreads();
  // reflectors of the kept directions (as in k_bg_eig)
  for (int cv = 0; cv < r; ++cv) {
    double* vr = Vk + (int64_t)cv * b;
    if (wv == 0) {
      double xs = 0.0;
      for (int t = cv + lane; t < b; t += 64) xs += vr[t] * vr[t];
      const double nrm2 = wave_sum_u(xs);
      const double x0 = vr[cv];
      const double nrm = sqrt(nrm2);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vv = v0 * v0 + (nrm2 - x0 * x0);
      wave_sync();
      for (int t = lane; t < cv; t += 64) vr[t] = 0.0;
      if (lane == 0) {
        vr[cv] = v0;
        tau[cv] = vv > 0.0 ? 2.0 / vv : 0.0;
      }
    }
    __syncthreads();
    const double tc = tau[cv];
    for (int c2 = cv + 1 + wv; c2 < r; c2 += 4) {
      double* br = Vk + (int64_t)c2 * b;
      double dd = 0.0;
      for (int t = cv + lane; t < b; t += 64) dd += vr[t] * br[t];
      dd = wave_sum_u(dd);
      for (int t = cv + lane; t < b; t += 64) br[t] -= tc * dd * vr[t];
    }
    __syncthreads();
  }
  // U_i = H_0 ... H_{r-1}: one wavefront per column
  for (int col = wv; col < b; col += 4) {
    double q[BG_MAXB / 64];
#pragma unroll
    for (int u = 0; u < BG_MAXB / 64; ++u) q[u] = (lane + 64 * u == col) ? 1.0 : 0.0;
    for (int cv = r - 1; cv >= 0; --cv) {
      const double* vr = Vk + (int64_t)cv * b;
      double dd = 0.0;
#pragma unroll
      for (int u = 0; u < BG_MAXB / 64; ++u) {
        const int t = lane + 64 * u;
        if (t < b) dd += vr[t] * q[u];
      }
      dd = wave_sum_u(dd) * tau[cv];
#pragma unroll
      for (int u = 0; u < BG_MAXB / 64; ++u) {
        const int t = lane + 64 * u;
        if (t < b) q[u] -= dd * vr[t];
      }
    }
#pragma unroll
    for (int u = 0; u < BG_MAXB / 64; ++u) {
      const int t = lane + 64 * u;
      if (t < b) Ug[(int64_t)t * b + col] = (T)q[u];
    }
  }
  if (tid == 0) {
    A.rank[i] = r;
    A.edrop[i] = rd[0];
    A.big_fail[i] = 0;
    if (A.bg_count) atomicAdd(A.bg_count + 3, 1);
  }
}

// Schur update for steps with 64 < b_i <= BG_MAXB (any n_i): T(a, c) -=
// P_a^T P_c over the 64 x 64 target tiles in turn, the n_i rows of the two
// panels staged in LDS 64 at a time, the products on the FP64 matrix cores
// (operand and result lanes as in k_schur_t).
template <typename T>
__global__ __launch_bounds__(NT) void k_schur_big(LevelArgs<T> A, int32_t p0) {
  const Pair pr = A.pairs[p0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[pr.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  T* D = A.arena + A.slot_off[i];
  int la, lc, ba = b, bc = b, ta = 0, tcv = 0;
  T* pa;
  T* pc;
  if (pr.a == 0) {
    la = r;
    pa = D;
  } else {
    const View va = A.views[st.view0 + pr.a - 1];
    ba = A.bsz[va.x];
    la = va.proc ? A.rank[va.x] : ba;
    pa = A.arena + A.slot_off[va.slot];
    ta = va.trans;
  }
  if (pr.c == 0) {
    lc = r;
    pc = D;
  } else {
    const View vc = A.views[st.view0 + pr.c - 1];
    bc = A.bsz[vc.x];
    lc = vc.proc ? A.rank[vc.x] : bc;
    pc = A.arena + A.slot_off[vc.slot];
    tcv = vc.trans;
  }
  if (la == 0 || lc == 0) return;
  T* tbase;
  int64_t ts_a, ts_c;
  if (pr.a == 0) {
    if (pr.c == 0) {
      tbase = D;
      ts_a = b;
      ts_c = 1;
    } else {
      tbase = pc;
      ts_a = tcv ? 1 : bc;
      ts_c = tcv ? b : 1;
    }
  } else {
    tbase = A.arena + A.slot_off[pr.slot];
    if (pr.trans) {
      ts_a = 1;
      ts_c = ba;
    } else {
      ts_a = bc;
      ts_c = 1;
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Pa = reinterpret_cast<T*>(smem_raw);
  T* Pc = Pa + 64 * TLD;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const T* fa = Pa + fk * TLD + 16 * wv + fr;
  const T* fc = Pc + fk * TLD + fr;
  for (int a0 = 0; a0 < la; a0 += 64) {
    const int tan = min(64, la - a0);
    for (int c0 = 0; c0 < lc; c0 += 64) {
      const int tcn = min(64, lc - c0);
      T tv[4][4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int al = 16 * wv + 4 * j + fk, gm = 16 * tj + fr;
          tv[tj][j] = (al < tan && gm < tcn) ? tbase[(a0 + al) * ts_a + (c0 + gm) * ts_c] : T(0);
        }
      dbl4 dacc[4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) dacc[tj] = dbl4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < n; k0 += 64) {
        const int nk = min(64, n - k0), nk4 = (nk + 3) & ~3;
        __syncthreads();
        load_tile_pair(Pa, pa, TileSrc{ta, b, ba, a0, tan}, pc, TileSrc{tcv, b, bc, c0, tcn}, r + k0, nk);
        // rows nk .. nk4 - 1 of both tiles are zero: the k loop runs in steps of four
        for (int e = threadIdx.x; e < (nk4 - nk) * 64; e += NT) {
          Pa[(nk + (e >> 6)) * TLD + (e & 63)] = T(0);
          Pc[(nk + (e >> 6)) * TLD + (e & 63)] = T(0);
        }
        __syncthreads();
#pragma unroll 2
        for (int k = 0; k < nk4; k += 4) {
          const double av = (double)fa[k * TLD];
          double bv[4];
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) bv[tj] = (double)fc[k * TLD + 16 * tj];
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) dacc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tj], dacc[tj], 0, 0, 0);
        }
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int al = 16 * wv + 4 * j + fk, gm = 16 * tj + fr;
          if (al < tan && gm < tcn)
            tbase[(a0 + al) * ts_a + (c0 + gm) * ts_c] = (T)((double)tv[tj][j] - dacc[tj][j]);
        }
    }
  }
}

// The two panels and the target block of a Schur pair (a, c) of step i: the
// basis rows (index 0, width r_i) or close view a - 1 (live width), and the
// strides of the target T(a, c) within its slot; the panels are exchanged
// where that gives the target unit stride along c.
template <typename T>
struct SchurPair {
  const T* pa;
  const T* pc;
  T* tbase;
  int64_t ts_a, ts_c;
  int la, lc, ba, bc, ta, tcv;
};

template <typename T>
__device__ inline SchurPair<T> schur_pair(const LevelArgs<T>& A, const Pair& pr, const Step& st, int b, int r) {
  SchurPair<T> o;
  T* D = A.arena + A.slot_off[st.blk];
  o.ba = b;
  o.bc = b;
  o.ta = 0;
  o.tcv = 0;
  if (pr.a == 0) {
    o.la = r;
    o.pa = D;
  } else {
    const View va = A.views[st.view0 + pr.a - 1];
    o.ba = A.bsz[va.x];
    o.la = va.proc ? A.rank[va.x] : o.ba;
    o.pa = A.arena + A.slot_off[va.slot];
    o.ta = va.trans;
  }
  T* pcw;
  if (pr.c == 0) {
    o.lc = r;
    pcw = D;
  } else {
    const View vc = A.views[st.view0 + pr.c - 1];
    o.bc = A.bsz[vc.x];
    o.lc = vc.proc ? A.rank[vc.x] : o.bc;
    pcw = A.arena + A.slot_off[vc.slot];
    o.tcv = vc.trans;
  }
  o.pc = pcw;
  if (pr.a == 0) {
    if (pr.c == 0) {
      o.tbase = D;
      o.ts_a = b;
      o.ts_c = 1;
    } else {
      o.tbase = pcw;
      o.ts_a = o.tcv ? 1 : o.bc;
      o.ts_c = o.tcv ? b : 1;
    }
  } else {
    o.tbase = A.arena + A.slot_off[pr.slot];
    if (pr.trans) {
      o.ts_a = 1;
      o.ts_c = o.ba;
    } else {
      o.ts_a = o.bc;
      o.ts_c = 1;
    }
  }
  if (o.ts_c != 1) {
    // T(a, c)^T = P_c^T P_a: with the roles of the panels exchanged the
    // target's unit stride runs along the lanes of an output row
    const T* tp = o.pa;
    o.pa = o.pc;
    o.pc = tp;
    int t = o.la;
    o.la = o.lc;
    o.lc = t;
    t = o.ba;
    o.ba = o.bc;
    o.bc = t;
    t = o.ta;
    o.ta = o.tcv;
    o.tcv = t;
    const int64_t u = o.ts_a;
    o.ts_a = o.ts_c;
    o.ts_c = u;
  }
  return o;
}

// Schur update of the FP32 factor with BF16-input products for steps with
// 64 < b_i <= BG_MAXB: T(a, c) -= P_a^T P_c.  Pairs of two panels wider than
// 64 columns (k_schur_big_bf16w): output blocks of 128 x 128
// (wavefront w the 64 x 64 quarter (w / 2, w % 2), as 2 x 2 tiles of 32 x 32 on
// v_mfma_f32_32x32x8bf16_1k with FP32 accumulation, lanes as in
// k_schur_bf16), the n_i panel rows staged 32 at a time in LDS as FP32; each
// thread holds its share of the next chunk in registers while the current one
// is multiplied.  Other pairs (k_schur_big_bf16): 64 x 64 tiles, 64 panel
// rows at a time.
// (an odd LDS row stride: the transposed views' stores, consecutive rows on
// consecutive lanes, fall on different banks; the products read along rows)
constexpr int SB_W = 128, SB_K = 16, SB_LD = SB_W + 1, SB_U = SB_K * SB_W / NT;
// the wide kernel's chunks in LDS as BF16, [column][k] with k contiguous: one
// 8-byte read gives a lane its four k values of an MFMA operand; the row
// stride of 20 (10 dwords) puts the 32 columns of a half-wavefront on
// distinct banks
constexpr int SB_KS = SB_K + 4;

template <typename T>
size_t work_schur_big_bf16() {
  return (size_t)2 * SB_W * SB_KS * sizeof(short);
}

// This thread's share of a chunk of one panel: SB_U entries (row k, column
// c), k = kt + u kstep, c = ct + u cstep (u < SB_U), the unit-stride index on
// consecutive threads (rows for a transposed view, columns otherwise), so
// that one offset and one stride per panel address all of them.
template <typename T>
struct SbShare {
  const T* p;       // panel base
  int64_t off;      // offset of u = 0 at chunk row 0
  int64_t step;     // offset between u and u + 1
  int64_t rstep;    // offset of one chunk row
  int kt, ct, kstep, cstep, tw;
};

template <typename T>
__device__ inline SbShare<T> sb_share(const T* p, int trans, int b, int bx, int col0, int tw, int row0) {
  SbShare<T> s;
  const int tid = threadIdx.x;
  s.p = p;
  s.tw = tw;
  if (trans) {
    s.kt = tid & (SB_K - 1);
    s.ct = tid / SB_K;
    s.kstep = 0;
    s.cstep = NT / SB_K;
    s.off = (int64_t)(col0 + s.ct) * b + row0 + s.kt;
    s.step = (int64_t)s.cstep * b;
    s.rstep = 1;
  } else {
    s.kt = tid / SB_W;
    s.ct = tid & (SB_W - 1);
    s.kstep = NT / SB_W;
    s.cstep = 0;
    s.off = (int64_t)(row0 + s.kt) * bx + col0 + s.ct;
    s.step = (int64_t)s.kstep * bx;
    s.rstep = bx;
  }
  return s;
}

// the SB_U entries of chunk row k0 (nk rows valid), zero outside the panel
// (the loads are unconditional, entries outside the panel read its first
// entry and are replaced by zero: a predicated load per entry would be a
// branch of its own)
template <typename T>
__device__ inline void sb_fetch(const SbShare<T>& s, int k0, int nk, T (&v)[SB_U]) {
  const int64_t o = s.off + (int64_t)k0 * s.rstep;
#pragma unroll
  for (int u = 0; u < SB_U; ++u) {
    const bool ok = s.kt + u * s.kstep < nk && s.ct + u * s.cstep < s.tw;
    const T x = s.p[ok ? o + u * s.step : 0];
    v[u] = ok ? x : T(0);
  }
}

template <typename T>
__device__ inline void sb_store(const SbShare<T>& s, T* L, const T (&v)[SB_U]) {
#pragma unroll
  for (int u = 0; u < SB_U; ++u) L[(s.kt + u * s.kstep) * SB_LD + s.ct + u * s.cstep] = v[u];
}

// the same entries rounded to BF16 once, into the [column][k] layout
template <typename T>
__device__ inline void sb_store_bf16(const SbShare<T>& s, short* L, const T (&v)[SB_U]) {
#pragma unroll
  for (int u = 0; u < SB_U; ++u) L[(s.ct + u * s.cstep) * SB_KS + s.kt + u * s.kstep] = to_bf16((float)v[u]);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_schur_big_bf16(LevelArgs<T> A, int32_t p0) {
  const Pair pr = A.pairs[p0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[pr.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const SchurPair<T> P = schur_pair(A, pr, st, b, r);
  if (P.la == 0 || P.lc == 0) return;
  if (P.la > 64 && P.lc > 64) return;   // k_schur_big_bf16w
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l32 = lane & 31, kh = 4 * (lane >> 5);
  // a narrow panel: 64 x 64 output tiles, the four wavefronts 2 x 2 tiles of
  // 32 x 32, panel rows staged 64 at a time (stride TLD)
  T* Qa = reinterpret_cast<T*>(smem_raw);
  T* Qc = Qa + 64 * TLD;
  const int si = wv >> 1, sj = wv & 1;
  const int ia = si * 32 + l32, jb = sj * 32 + l32;
  for (int a0 = 0; a0 < P.la; a0 += 64) {
    const int tan = min(64, P.la - a0);
    for (int c0 = 0; c0 < P.lc; c0 += 64) {
      const int tcn = min(64, P.lc - c0);
      f32x16_t acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
      for (int k0 = 0; k0 < n; k0 += 64) {
        const int nk = min(64, n - k0), nk8 = (nk + 7) & ~7;
        __syncthreads();
        load_tile_pair(Qa, P.pa, TileSrc{P.ta, b, P.ba, a0, tan}, P.pc, TileSrc{P.tcv, b, P.bc, c0, tcn}, r + k0,
                       nk);
        // rows nk .. nk8 - 1 of both tiles are zero: the k loop runs in steps of eight
        for (int e = threadIdx.x; e < (nk8 - nk) * 64; e += NT) {
          Qa[(nk + (e >> 6)) * TLD + (e & 63)] = T(0);
          Qc[(nk + (e >> 6)) * TLD + (e & 63)] = T(0);
        }
        __syncthreads();
        for (int k = 0; k < nk8; k += 8) {
          bf16x4_t av, bv;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            av[t] = to_bf16((float)Qa[(k + kh + t) * TLD + ia]);
            bv[t] = to_bf16((float)Qc[(k + kh + t) * TLD + jb]);
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int al = si * 32 + 8 * (v >> 2) + kh + (v & 3);
        const int gm = sj * 32 + l32;
        if (al < tan && gm < tcn) {
          T* tp = P.tbase + (int64_t)(a0 + al) * P.ts_a + (int64_t)(c0 + gm) * P.ts_c;
          *tp = (T)((float)*tp - acc[v]);
        }
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_schur_big_bf16w(LevelArgs<T> A, int32_t p0) {
  const Pair pr = A.pairs[p0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[pr.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const SchurPair<T> P = schur_pair(A, pr, st, b, r);
  if (P.la == 0 || P.lc == 0) return;
  if (P.la <= 64 || P.lc <= 64) return;   // k_schur_big_bf16
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l32 = lane & 31, kh = 4 * (lane >> 5);
  short* Pa = reinterpret_cast<short*>(smem_raw);   // [a][k], SB_W x SB_KS (BF16)
  short* Pc = Pa + SB_W * SB_KS;                     // [c][k]
  const int ra = 64 * (wv >> 1), rc = 64 * (wv & 1);
  for (int a0 = 0; a0 < P.la; a0 += SB_W) {
    const int tan = min(SB_W, P.la - a0);
    for (int c0 = 0; c0 < P.lc; c0 += SB_W) {
      const int tcn = min(SB_W, P.lc - c0);
      f32x16_t acc[2][2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[ti][tj][v] = 0.0f;
      const SbShare<T> sa = sb_share(P.pa, P.ta, b, P.ba, a0, tan, r);
      const SbShare<T> sc = sb_share(P.pc, P.tcv, b, P.bc, c0, tcn, r);
      T na[SB_U], nc[SB_U];
      sb_fetch(sa, 0, min(SB_K, n), na);
      sb_fetch(sc, 0, min(SB_K, n), nc);
      for (int k0 = 0; k0 < n; k0 += SB_K) {
        __syncthreads();   // the previous chunk consumed
        sb_store_bf16(sa, Pa, na);
        sb_store_bf16(sc, Pc, nc);
        __syncthreads();
        if (k0 + SB_K < n) {
          const int nk2 = min(SB_K, n - k0 - SB_K);
          sb_fetch(sa, k0 + SB_K, nk2, na);
          sb_fetch(sc, k0 + SB_K, nk2, nc);
        }
        // rows beyond the chunk's end are zero (loaded as zero), so the k
        // loop always runs over SB_K
#pragma unroll 1
        for (int kk = 0; kk < SB_K; kk += 8) {
          bf16x4_t av[2], bv[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            av[h] = *reinterpret_cast<const bf16x4_t*>(Pa + (ra + 32 * h + l32) * SB_KS + kk + kh);
            bv[h] = *reinterpret_cast<const bf16x4_t*>(Pc + (rc + 32 * h + l32) * SB_KS + kk + kh);
          }
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
              acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
        }
      }
      // the target's unit stride runs along the lanes (ts_c = 1, see schur_pair)
      T* const tb = P.tbase + (int64_t)(a0 + ra + kh) * P.ts_a + c0 + rc + l32;
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int dr = 32 * ti + 8 * (v >> 2) + (v & 3);
            const bool ok = ra + kh + dr < tan && rc + 32 * tj + l32 < tcn;
            T* tp = ok ? tb + (int64_t)dr * P.ts_a + 32 * tj : P.tbase;   // (an entry of the target)
            const T old = *tp;
            if (ok) *tp = (T)((float)old - acc[ti][tj][v]);
          }
    }
  }
}

// Strip products of the steps with 64 < b_i <= BG_MAXB.  A strip of SW
// columns of a view (its rows row0 .. row0 + m; SW = 64 for an FP32 factor,
// 32 for FP64, so that BG_MAXB rows fit in LDS) is staged in LDS and
// multiplied from the left by an m x m matrix read from global memory (L2):
// wavefront w owns the output row blocks 16 w, 16 (w + 4), ..., each as SW / 16
// tiles of 16 x 16 on the FP64 matrix cores (lanes as in k_schur_t).  Rows m ..
// m4 - 1 of the strip stay zero so the k loop runs in steps of four.
template <typename T, int W = (sizeof(T) == sizeof(float) ? 64 : 32)>
struct Strip {
  static constexpr int SW = W;         // columns
  static constexpr int LD = SW + 4;    // LDS row stride
  static constexpr int NTJ = SW / 16;  // 16-column tiles
};
//   op = 0: out = M^T X with M row-major m x m (the rotation by U_i^T);
//   op = 1: out = M X (the triangular solve by the stored L_nn^{-1}).
// Output rows >= mout are not computed (far views keep their rows < r_i).
// NS strips side by side (the second at X + m4 LD, columns c0 + SW ..): each
// entry of M loaded from L2 feeds NS times as many products.
template <typename T, int OP, int NS = 1, int W = Strip<T>::SW>
__device__ void strip_product(const T* M, int m, const T* X, int mout, int tc, T* base, int trans, int bi, int bx,
                              int row0, int c0) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, fr = lane & 15, fk = lane >> 4;
  constexpr int NTJ = Strip<T, W>::NTJ, LD = Strip<T, W>::LD, SW = W;
  const int m4 = (m + 3) & ~3;
  for (int rb = wv; 16 * rb < mout; rb += 4) {
    dbl4 acc[NS][NTJ];
#pragma unroll
    for (int h = 0; h < NS; ++h)
#pragma unroll
      for (int tj = 0; tj < NTJ; ++tj) acc[h][tj] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int row = 16 * rb + fr;
#pragma unroll 8
    for (int k0 = 0; k0 < m4; k0 += 4) {
      const int k = k0 + fk;
      // unconditional load (M[0] outside the matrix), then zero: a
      // predicated load would be a branch per k step
      const bool ok = k < m && row < m;
      const T mv = M[ok ? (OP == 0 ? (int64_t)k * m + row : (int64_t)row * m + k) : 0];
      const double av = ok ? (double)mv : 0.0;
#pragma unroll
      for (int h = 0; h < NS; ++h) {
        double bv[NTJ];
#pragma unroll
        for (int tj = 0; tj < NTJ; ++tj) bv[tj] = (double)X[h * m4 * LD + k * LD + 16 * tj + fr];
#pragma unroll
        for (int tj = 0; tj < NTJ; ++tj)
          acc[h][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tj], acc[h][tj], 0, 0, 0);
      }
    }
#pragma unroll
    for (int h = 0; h < NS; ++h)
#pragma unroll
      for (int tj = 0; tj < NTJ; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 16 * rb + 4 * j + fk, c = h * SW + 16 * tj + fr;
          if (a < mout && c < tc) *view_ptr(base, trans, bi, bx, row0 + a, c0 + c) = (T)acc[h][tj][j];
        }
  }
}

// The strip X[a][c] = view(row0 + a, c0 + c), a < m, c < tc <= SW (rows m ..
// m4 - 1 zero), the unit-stride index on consecutive threads.
template <typename T, int W = Strip<T>::SW>
__device__ inline void load_strip(T* X, const T* base, int trans, int bi, int bx, int row0, int m, int c0, int tc) {
  constexpr int SW = W, LD = Strip<T, W>::LD;
  const int m4 = (m + 3) & ~3;
  if (trans) {
    for (int e = threadIdx.x; e < tc * m4; e += NT) {
      const int c = e / m4, a = e % m4;
      const T x = base[a < m ? (int64_t)(c0 + c) * bi + row0 + a : 0];
      X[a * LD + c] = a < m ? x : T(0);
    }
  } else {
    for (int e = threadIdx.x; e < m4 * SW; e += NT) {
      const int a = e / SW, c = e % SW;
      const bool ok = a < m && c < tc;
      const T x = base[ok ? (int64_t)(row0 + a) * bx + c0 + c : 0];
      X[a * LD + c] = ok ? x : T(0);
    }
  }
}

template <typename T, int W = Strip<T>::SW>
size_t work_strip_big(int bmax) {
  return (size_t)((std::min(bmax, BG_MAXB) + 3) & ~3) * Strip<T, W>::LD * sizeof(T);
}
// the strip width of the rotation of the views: 32 columns, so that a
// compute unit holds twice the workgroups of 64-column strips (10% faster on
// the 3D Laplacian; the triangular solve keeps 64, where 32 was slower)
constexpr int SW_VIEW = 32;

// V_ix <- U_i^T V_ix for the close and far views of big steps (far views keep
// rows < r_i; with compensation k_compensate reads E_i and zeroes it).
template <typename T, int NS, int W>
__global__ __launch_bounds__(NT) void k_rot_big(LevelArgs<T> A, int32_t it0) {
  const Item item = A.items[it0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  if (item.view < 0) return;
  const Step st = A.steps[item.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB) return;
  const View v = A.views[item.view];
  const int bx = A.bsz[v.x];
  const bool drop = (item.view - st.view0) >= st.nclose && !A.compensate;
  const int r = A.rank[i];
  T* base = A.arena + A.slot_off[v.slot];
  const T* Ug = A.U + A.u_off[i];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  constexpr int SW = W, LD = Strip<T, W>::LD;
  const int b4 = (b + 3) & ~3;
  for (int c0 = 0; c0 < bx; c0 += NS * SW) {
    const int tc = min(NS * SW, bx - c0);
    __syncthreads();
    for (int h = 0; h < NS; ++h)
      if (h * SW < tc)
        load_strip<T, W>(X + h * b4 * LD, base, v.trans, b, bx, 0, b, c0 + h * SW, min(SW, tc - h * SW));
    __syncthreads();
    strip_product<T, 0, NS, W>(Ug, b, X, drop ? r : b, tc, base, v.trans, b, bx, 0, c0);
    if (drop)
      for (int e = threadIdx.x; e < (b - r) * tc; e += NT)
        *view_ptr(base, v.trans, b, bx, r + e / tc, c0 + e % tc) = T(0);
  }
}

// D_i <- U_i^T D_i U_i for big steps, stored exactly symmetric, in two
// launches of one workgroup per (step, 32-column strip; the diagonal blocks
// run on a side stream beside the views' rotation, and narrow strips let
// their workgroups find room on the busy compute units), the strips of one
// step on one XCD: PHASE 0 T1 = U^T D (a strip of D's columns) into the step's FP64
// scratch; PHASE 1 D = T1 U (a strip of U's columns), the entries (a, c) with
// a >= c written to both triangles (the strip that holds c writes both, so the
// strips write disjoint entries).
template <typename T, int PHASE>
__global__ __launch_bounds__(NT) void k_rot_big_diag(LevelArgs<T> A, int32_t s0, int32_t nstrip) {
  constexpr int SW = Strip<T, 32>::SW, LD = Strip<T, 32>::LD, NTJ = Strip<T, 32>::NTJ;
  const int64_t lg = xcd_swizzle(blockIdx.x, gridDim.x);
  const int sx = (int)(lg / nstrip), c0 = (int)(lg % nstrip) * SW;
  const Step st = A.steps[s0 + sx];
  if (st.nfar == 0) return;   // U_i = I
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB || c0 >= b) return;
  T* D = A.arena + A.slot_off[i];
  const T* Ug = A.U + A.u_off[i];
  double* T1 = A.big + (int64_t)sx * A.big_stride;   // b x b
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, fr = lane & 15, fk = lane >> 4;
  const int b4 = (b + 3) & ~3;
  const int tc = min(SW, b - c0);
  load_strip<T, 32>(X, PHASE == 0 ? (const T*)D : Ug, 0, b, b, 0, b, c0, tc);
  __syncthreads();
  for (int rb = wv; 16 * rb < b; rb += 4) {
    if (PHASE == 1 && 16 * rb + 15 < c0) continue;   // a block entirely above the diagonal of this strip
    dbl4 acc[NTJ];
#pragma unroll
    for (int tj = 0; tj < NTJ; ++tj) acc[tj] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int row = 16 * rb + fr;
#pragma unroll 4
    for (int k0 = 0; k0 < b4; k0 += 4) {
      const int k = k0 + fk;
      double av;
      if (PHASE == 0)
        av = (k < b && row < b) ? (double)Ug[(int64_t)k * b + row] : 0.0;   // U^T
      else
        av = (k < b && row < b) ? T1[(int64_t)row * b + k] : 0.0;
      double bv[NTJ];
#pragma unroll
      for (int tj = 0; tj < NTJ; ++tj) bv[tj] = (double)X[k * LD + 16 * tj + fr];
#pragma unroll
      for (int tj = 0; tj < NTJ; ++tj) acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tj], acc[tj], 0, 0, 0);
    }
#pragma unroll
    for (int tj = 0; tj < NTJ; ++tj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = 16 * rb + 4 * j + fk, c = c0 + 16 * tj + fr;
        if (PHASE == 0) {
          if (a < b && 16 * tj + fr < tc) T1[(int64_t)a * b + c] = acc[tj][j];
        } else if (a < b && 16 * tj + fr < tc && a >= c) {
          const T val = (T)acc[tj][j];
          D[(int64_t)a * b + c] = val;
          D[(int64_t)c * b + a] = val;
        }
      }
  }
}

// L(c, n_i)^T = L_nn^{-1} V_ic[n_i, live_c] for the close views of big steps.
template <typename T, int NS, int W>
__global__ __launch_bounds__(NT) void k_trsm_big(LevelArgs<T> A, int32_t it0) {
  const Item item = A.items[it0 + xcd_swizzle(blockIdx.x, gridDim.x)];
  const Step st = A.steps[item.step];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const View v = A.views[item.view];
  const int bx = A.bsz[v.x];
  const int lc = v.proc ? A.rank[v.x] : bx;
  if (lc == 0) return;
  T* base = A.arena + A.slot_off[v.slot];
  const T* Lig = A.Li + A.u_off[i];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  constexpr int SW = W, LD = Strip<T, W>::LD;
  const int n4 = (n + 3) & ~3;
  for (int c0 = 0; c0 < lc; c0 += NS * SW) {
    const int tc = min(NS * SW, lc - c0);
    __syncthreads();
    for (int h = 0; h < NS; ++h)
      if (h * SW < tc)
        load_strip<T, W>(X + h * n4 * LD, base, v.trans, b, bx, r, n, c0 + h * SW, min(SW, tc - h * SW));
    __syncthreads();
    strip_product<T, 1, NS, W>(Lig, n, X, n, tc, base, v.trans, b, bx, r, c0);
  }
}

// Elimination of S_ii for steps with 64 < b_i <= BG_MAXB: blocked Cholesky in
// FP64 of the n_i x n_i trailing block (one workgroup per step, the matrix W
// in the step's scratch): per 64-column block the diagonal block is factored
// in LDS with its inverse (chol_inv_lds), the panel below is multiplied by
// L_kk^{-T} and the trailing lower triangle updated, 64 x 64 tiles on the FP64
// matrix cores.  L_nn^{-1} by block columns, Li_IJ = -L_II^{-1} sum_{K=J}^{I-1}
// L_IK Li_KJ (kept transposed in W's free upper triangle, the diagonal
// inverses after W); then the basis panel L^{-1} D(n_i, basis) and the factor
// are written as k_potrf writes them.
template <typename T>
size_t work_potrf_big(int bmax) {
  const size_t a = (size_t)2 * 64 * TLD * sizeof(double), s = work_strip_big<T>(bmax);
  return a > s ? a : s;
}

// C (64 x 64 in registers of the four wavefronts, rows 16 w..) += A B with
// A(row, k) and B(k, col) given by accessors, k < K.
template <typename FA, typename FB>
__device__ inline void tile_product(dbl4 acc[4], int K, FA fa, FB fb) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, fr = lane & 15, fk = lane >> 4;
  const int K4 = (K + 3) & ~3;
#pragma unroll 2
  for (int k0 = 0; k0 < K4; k0 += 4) {
    const int k = k0 + fk;
    const double av = k < K ? fa(16 * wv + fr, k) : 0.0;
    double bv[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) bv[tj] = k < K ? fb(k, 16 * tj + fr) : 0.0;
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tj], acc[tj], 0, 0, 0);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_potrf_big(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b <= 64 || b > BG_MAXB) return;
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  T* D = A.arena + A.slot_off[i];
  double* W = A.big + (int64_t)blockIdx.x * A.big_stride;   // n x n
  double* DI = W + (int64_t)n * n;                           // inverses of the diagonal blocks, 64 x 64 each
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = reinterpret_cast<double*>(smem_raw);
  double* X = S + 64 * TLD;
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = lane >> 4;
  if (tid == 0) bad = 0;
  for (int e = tid; e < n * n; e += NT) W[e] = (double)D[(int64_t)(r + e / n) * b + r + e % n];
  __syncthreads();
  const int nt = (n + 63) / 64;
  dbl4 acc[4];
  auto zero = [&]() {
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = dbl4{0.0, 0.0, 0.0, 0.0};
  };
  // ---- blocked right-looking Cholesky ----------------------------------------
  for (int kt = 0; kt < nt; ++kt) {
    const int kb = 64 * kt, nb = min(64, n - kb);
    for (int e = tid; e < 64 * 64; e += NT) {
      const int a = e >> 6, c = e & 63;
      S[a * TLD + c] = (a < nb && c < nb) ? W[(int64_t)(kb + a) * n + kb + c] : 0.0;
      X[a * TLD + c] = a == c ? 1.0 : 0.0;
    }
    __syncthreads();
    chol_inv_lds(S, X, nb, &bad);
    for (int e = tid; e < 64 * 64; e += NT) {
      const int a = e >> 6, c = e & 63;
      if (a < nb && c <= a) W[(int64_t)(kb + a) * n + kb + c] = S[a * TLD + c];
      DI[(int64_t)kt * 4096 + e] = (a < nb && c <= a) ? X[a * TLD + c] : 0.0;
    }
    __syncthreads();
    // panel: W[I, K] <- W[I, K] L_kk^{-T}; each wavefront its own 16 rows
    for (int i0 = kb + nb; i0 < n; i0 += 64) {
      zero();
      tile_product(acc, nb, [&](int row, int k) { return i0 + row < n ? W[(int64_t)(i0 + row) * n + kb + k] : 0.0; },
                   [&](int k, int col) { return col < nb ? X[col * TLD + k] : 0.0; });
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = i0 + 16 * wv + 4 * j + fk, col = 16 * tj + fr;
          if (row < n && col < nb) W[(int64_t)row * n + kb + col] = acc[tj][j];
        }
    }
    __syncthreads();
    // trailing lower triangle: W[I, J] -= P_I P_J^T, P = W[:, K]
    for (int ti = kt + 1; ti < nt; ++ti)
      for (int tjb = kt + 1; tjb <= ti; ++tjb) {
        const int i0 = 64 * ti, j0 = 64 * tjb;
        zero();
        tile_product(acc, nb, [&](int row, int k) { return i0 + row < n ? W[(int64_t)(i0 + row) * n + kb + k] : 0.0; },
                     [&](int k, int col) { return j0 + col < n ? W[(int64_t)(j0 + col) * n + kb + k] : 0.0; });
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int row = i0 + 16 * wv + 4 * j + fk, col = j0 + 16 * tj + fr;
            if (row < n && col < n && col <= row) W[(int64_t)row * n + col] -= acc[tj][j];
          }
      }
    __syncthreads();
  }
  // ---- L^{-1} by block columns (Li_IJ^T into W's upper triangle) ------------
  for (int jt = 0; jt < nt; ++jt) {
    for (int it = jt + 1; it < nt; ++it) {
      const int i0 = 64 * it, j0 = 64 * jt;
      const int ni = min(64, n - i0);
      // Z = sum_{K=J}^{I-1} L_IK Li_KJ
      zero();
      for (int kt = jt; kt < it; ++kt) {
        const int k0 = 64 * kt, nk = min(64, n - k0);
        if (kt == jt)
          tile_product(acc, nk, [&](int row, int k) { return row < ni ? W[(int64_t)(i0 + row) * n + k0 + k] : 0.0; },
                       [&](int k, int col) { return DI[(int64_t)jt * 4096 + k * 64 + col]; });
        else
          tile_product(acc, nk, [&](int row, int k) { return row < ni ? W[(int64_t)(i0 + row) * n + k0 + k] : 0.0; },
                       [&](int k, int col) { return j0 + col < n ? W[(int64_t)(j0 + col) * n + k0 + k] : 0.0; });
      }
      // Z into LDS, then Li_IJ = -L_II^{-1} Z
      __syncthreads();
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) S[(16 * wv + 4 * j + fk) * TLD + 16 * tj + fr] = acc[tj][j];
      __syncthreads();
      zero();
      tile_product(acc, ni, [&](int row, int k) { return DI[(int64_t)it * 4096 + row * 64 + k]; },
                   [&](int k, int col) { return S[k * TLD + col]; });
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 16 * wv + 4 * j + fk, c = 16 * tj + fr;
          if (a < ni && j0 + c < n) W[(int64_t)(j0 + c) * n + i0 + a] = -acc[tj][j];
        }
      __syncthreads();
    }
  }
  // ---- L_nn^{-1} (T), min pivot, error ---------------------------------------
  T* Lig = A.Li + A.u_off[i];
  for (int e = tid; e < n * n; e += NT) {
    const int j = e / n, k = e % n, jt = j >> 6, kt = k >> 6;
    double v = 0.0;
    if (k <= j) v = jt == kt ? DI[(int64_t)jt * 4096 + (j & 63) * 64 + (k & 63)] : W[(int64_t)k * n + j];
    Lig[e] = (T)v;
  }
  if (tid == 0) {
    double mp = 1e300;
    for (int k = 0; k < n; ++k) mp = fmin(mp, W[(int64_t)k * n + k]);
    A.minpiv[i] = mp;
    if (bad && atomicCAS(A.err, 0, 1) == 0) A.err[1] = i;
  }
  __syncthreads();   // L_nn^{-1} written (global, this workgroup)
  // ---- basis panel D(n, basis) <- L^{-1} D(n, basis), strips of 64 columns --
  T* Xs = reinterpret_cast<T*>(smem_raw);
  for (int c0 = 0; c0 < r; c0 += Strip<T>::SW) {
    const int tc = min(Strip<T>::SW, r - c0);
    __syncthreads();
    load_strip(Xs, D, 0, b, b, r, n, c0, tc);
    __syncthreads();
    strip_product<T, 1>(Lig, n, Xs, n, tc, D, 0, b, b, r, c0);
  }
  __syncthreads();
  // ---- the factor: rows n of D hold [L^{-1} D(n, basis) | L], D(basis, n) = 0
  for (int e = tid; e < n * n; e += NT) {
    const int j = e / n, c = e % n;
    D[(int64_t)(r + j) * b + r + c] = c <= j ? (T)W[(int64_t)j * n + c] : T(0);
  }
  for (int e = tid; e < r * n; e += NT) D[(int64_t)(e / n) * b + r + e % n] = T(0);
}

// ---------------------------------------------------------------------------
// Learned ranks by a capped rank-revealing factorization (rank_mode
// LEARNED_CAP, any block size): the MLP's width l = min(k + 8, b) caps the
// pivoted Cholesky of the far row's Gram matrix in the exact kernels
// (k_compress_gram, k_bg_eig); a capped step is kept only if the energy the
// cap leaves out cannot change the rank (lambda_{r+1} + bound <= theta^2),
// otherwise it is redone without the cap.  This kernel computes the features
// of every far row (Frobenius norms of the row and of its far blocks against
// theta, widths, counts, neighbour ranks: the same 16 as k_compress_rand) and
// evaluates the MLP: one workgroup per step.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_feat_mlp(LevelArgs<T> A, int32_t s0) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (A.rec && tid < REC_W) A.rec[(A.rec_off + i) * REC_W + tid] = tid < NFEAT ? 0.0f : -1.0f;
  // nothing to compress, or (capped ranks) a block the Gram kernels do not
  // take: no cap, and no features to compute
  if (st.nfar == 0 || b == 0 || (!A.feat_only && b > 128)) {
    if (tid == 0) A.lwidth[i] = b;
    return;
  }
  __shared__ double red[NT / WV];
  __shared__ double xf[NFEAT];
  __shared__ double hbuf[MLP_H];
  const double theta = *A.theta;
  double fro2 = 0.0, cmax2 = 0.0, bsum4 = 0.0, prs = 0.0, pss = 0.0;
  int ccnt = 0, wtot = 0, nproc = 0;
  for (int f = st.nclose; f < st.nclose + st.nfar; ++f) {
    const View v = A.views[st.view0 + f];
    const int bx = A.bsz[v.x];
    const int w = v.proc ? A.rank[v.x] : bx;
    const T* base = A.arena + A.slot_off[v.slot];
    wtot += w;
    if (v.proc) {
      ++nproc;
      prs += A.rank[v.x];
      pss += bx;
    }
    double s2 = 0.0;
    for (int e = tid; e < b * w; e += NT) {
      // the unit-stride index on consecutive threads for either storage
      const int a = v.trans ? e % b : e / w, c = v.trans ? e / b : e % w;
      const double x = (double)*view_ptr(base, v.trans, b, bx, a, c);
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    if (lane == 0) red[wv] = s2;
    __syncthreads();
    const double bn2 = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    fro2 += bn2;
    cmax2 = fmax(cmax2, bn2);
    ccnt += bn2 > theta * theta ? 1 : 0;
    bsum4 += bn2 * bn2;
  }
  if (tid == 0) {
    const double cmax = sqrt(cmax2), fro = sqrt(fro2);
    xf[0] = log2((double)b + 1.0);
    xf[1] = log2((double)wtot + 1.0);
    xf[2] = (double)A.level;
    xf[3] = (double)st.nfar;
    xf[4] = (double)st.nclose;
    xf[5] = clog10(fro, theta);
    xf[6] = clog10(sqrt(fro2 / max(b, 1)), theta);
    xf[7] = clog10(cmax, theta);
    xf[8] = clog10(sqrt(fro2 / max(wtot, 1)), theta);
    xf[9] = (double)ccnt / (double)max(st.nfar, 1);
    xf[10] = fro2 > 0.0 ? bsum4 / (fro2 * fro2) : 0.0;
    xf[11] = cmax2 > 0.0 ? fro2 / (cmax2 * st.nfar) : 0.0;
    xf[12] = (double)nproc / (double)max(st.nfar, 1);
    xf[13] = pss > 0.0 ? prs / pss : 0.0;
    xf[14] = b / 64.0;
    xf[15] = 1.0;
  }
  __syncthreads();
  if (A.rec && tid < NFEAT) A.rec[(A.rec_off + i) * REC_W + tid] = (float)xf[tid];
  if (A.feat_only || !A.mlp) {
    if (tid == 0) A.lwidth[i] = b;
    return;
  }
  if (wv == 0) {
    const float* P = A.mlp;
    double h = P[MLP_OFF_B1 + lane];
    for (int k = 0; k < NFEAT; ++k)
      h += (double)P[MLP_OFF_W1 + lane * NFEAT + k] * ((xf[k] - (double)P[MLP_OFF_MEAN + k]) / (double)P[MLP_OFF_STD + k]);
    hbuf[lane] = fmax(h, 0.0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double h2 = P[MLP_OFF_B2 + lane];
    for (int k = 0; k < MLP_H; ++k) h2 += (double)P[MLP_OFF_W2 + lane * MLP_H + k] * hbuf[k];
    h2 = fmax(h2, 0.0);
    const double z = wave_sum((double)P[MLP_OFF_W3 + lane] * h2) + (double)P[MLP_OFF_B3];
    if (lane == 0) {
      const double bz = z * b;
      const int k = (bz == bz) ? (int)fmin(fmax(ceil(bz), 0.0), (double)b) : b;
      A.lwidth[i] = min(k + SKETCH_OVERSAMPLE, b);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename T>
int32_t scratch_group(int bmax);
template <typename T>
static void launch(void (*kern)(LevelArgs<T>, int32_t, T*, int64_t), const LevelArgs<T>& A, int32_t start,
                   int32_t count, size_t work_elems, T* gscratch, hipStream_t stream, int bmax) {
  if (count <= 0) return;
  const size_t bytes = work_elems * sizeof(T);
  if (bytes <= max_lds_bytes()) {
    hipLaunchKernelGGL(kern, dim3(count), dim3(NT), bytes, stream, A, start, (T*)nullptr, (int64_t)0);
  } else {
    // the scratch holds scratch_group(bmax) slices: launch in chunks of that many
    const int32_t g = scratch_group<T>(bmax);
    for (int32_t c0 = 0; c0 < count; c0 += g)
      hipLaunchKernelGGL(kern, dim3(min(g, count - c0)), dim3(NT), 0, stream, A, start + c0, gscratch,
                         (int64_t)work_elems);
  }
}

template <typename T>
size_t work_compress(int bmax) {
  // FP64 work in units of T
  const size_t nd = (size_t)bmax * (bmax + 1) + (size_t)(bmax > QR_CH ? bmax : QR_CH) * (bmax + 1) +
                    (5 * (size_t)bmax > (size_t)NT ? 5 * (size_t)bmax : (size_t)NT) + 8;
  return nd * (sizeof(double) / sizeof(T));
}
template <typename T>
size_t work_rotate(int bmax) {
  return (size_t)bmax * (bmax + 1) + (size_t)bmax * (bmax > ROT_TC ? bmax + 1 : ROT_TC + 1);
}
template <typename T>
size_t work_potrf(int bmax) {
  return (size_t)2 * bmax * (bmax + 1);
}
template <typename T>
size_t work_trsm(int bmax) {
  return (size_t)bmax * (bmax + 1) + (size_t)bmax * (TRSM_TC + 1);
}
template <typename T>
size_t work_schur(int bmax) {
  return (size_t)bmax * (bmax + 1) + (size_t)bmax * (SCH_TC + 1);
}

template <typename T>
size_t factor_scratch_elems(int bmax) {
  size_t m = work_compress<T>(bmax);
  m = m > work_rotate<T>(bmax) ? m : work_rotate<T>(bmax);
  m = m > work_potrf<T>(bmax) ? m : work_potrf<T>(bmax);
  m = m > work_trsm<T>(bmax) ? m : work_trsm<T>(bmax);
  m = m > work_schur<T>(bmax) ? m : work_schur<T>(bmax);
  return m;
}

template <typename T>
int32_t scratch_group(int bmax) {
  const size_t per = factor_scratch_elems<T>(bmax) * sizeof(T);
  size_t g = ((size_t)4 << 30) / (per ? per : 1);   // at most 4 GiB of scratch
  if (g > 4096) g = 4096;
  if (g < 64) g = 64;
  return (int32_t)g;
}

template <typename T>
bool factor_needs_global(int bmax) {
  return factor_scratch_elems<T>(bmax) * sizeof(T) > max_lds_bytes();
}

// The exact compression of a wave (or, with A.lwidth, its capped first pass):
// the size classes in turn, the generic kernel for what they leave.  With
// retry = true only the steps flagged in big_fail are redone, uncapped, and the
// big-block Gram matrices are not formed again (a rejected step leaves its own
// intact).
template <typename T>
static void compress_pass(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gs, hipStream_t stream,
                          bool retry) {
  const int ns = w.s1 - w.s0;
  const size_t wg = work_compress_wg<T>() * sizeof(T), w128 = work_compress_wave<T, 128>() * sizeof(T);
  const size_t wgr = work_compress_gram<T, 64>(), wgr2 = work_compress_gram<T, 128>();
  const bool gram = sizeof(T) < sizeof(double) && wgr <= max_lds_bytes();
  const bool gram2 = gram && wgr2 <= max_lds_bytes();
  const bool bigc = A.big && work_bg_eig<T>() <= max_lds_bytes() &&
                    (size_t)2 * 64 * TLD * sizeof(double) <= max_lds_bytes();
  auto big_pass = [&](int small) {
    LevelArgs<T> C = A;
    C.small_by_wave = small;
    if (bigc && bmax >= BG_MIN) {
      // big blocks: Gram tiles on many workgroups, then one workgroup per
      // step; the generic kernel takes only what they leave (blocks above
      // BG_MAXB, Gram matrices whose rank cannot be settled within BG_MA pivots)
      // (the big-block kernels take no width cap, so a retry pass has
      // nothing to redo there: its flagged big steps go to the generic kernel)
      const int nt = (std::min(bmax, BG_MAXB) + 63) / 64;
      if (!retry) {
        const int ntile = nt * (nt + 1) / 2;
        hipLaunchKernelGGL(k_bg_gram<T>, dim3(ns * ntile), dim3(NT), (size_t)2 * 64 * TLD * sizeof(T), stream, A,
                           w.s0, ntile);
        hipLaunchKernelGGL(k_bg_eig<T>, dim3(ns), dim3(NT), work_bg_eig<T>(), stream, A, w.s0);
        hipLaunchKernelGGL(k_bg_cert<T>, dim3(ns), dim3(NT), (size_t)2 * 64 * TLD * sizeof(double), stream, A, w.s0);
        hipLaunchKernelGGL(k_bg_full<T>, dim3(ns), dim3(NT), 0, stream, A, w.s0);
      }
      C.big_retry = 1;
      C.need_exact = nullptr;
      C.lwidth = nullptr;
    }
    // (the first pass of LEARNED_CAP leaves the generic kernel to the retry)
    if (!A.lwidth || retry) launch<T>(k_compress<T>, C, w.s0, ns, work_compress<T>(bmax), gs, stream, bmax);
  };
  if (gram)
    hipLaunchKernelGGL((k_compress_gram<T, 64>), dim3(ns), dim3(NT), wgr, stream, A, w.s0);
  else if (!retry)
    hipLaunchKernelGGL(k_compress_wg<T>, dim3(ns), dim3(NT), wg, stream, A, w.s0);
  if (bmax > 64 && gram2) {
    hipLaunchKernelGGL((k_compress_gram<T, 128>), dim3(ns), dim3(NT), wgr2, stream, A, w.s0);
    if (bmax > 128) big_pass(128);
  } else if (bmax > 64) {
    const bool wave128 = w128 <= max_lds_bytes();
    if (wave128 && !retry) hipLaunchKernelGGL((k_compress_wave<T, 128>), dim3(ns), dim3(WV), w128, stream, A, w.s0);
    if (bmax > 128 || !wave128) big_pass(wave128 ? 128 : 64);
  }
}

template <typename T>
void launch_wave_compress(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gscratch, hipStream_t stream) {
  if (w.s1 <= w.s0) return;
  const int ns = w.s1 - w.s0;
  if (A.lwidth) {
    // learned ranks by a capped rank-revealing factorization: features and
    // MLP width, the capped pass, then the rejected steps without the cap
    hipLaunchKernelGGL(k_feat_mlp<T>, dim3(ns), dim3(NT), 0, stream, A, w.s0);
    compress_pass<T>(A, w, bmax, gscratch, stream, false);
    LevelArgs<T> R = A;
    R.lwidth = nullptr;
    R.need_exact = A.big_fail;
    compress_pass<T>(R, w, bmax, gscratch, stream, true);
    return;
  }
  if (A.feat_only) {
    // training records: the features of every far row (any block size), then
    // the exact compression of every step, which writes the labels
    LevelArgs<T> F = A;
    F.lwidth = A.need_exact;   // scratch for the widths (not used)
    hipLaunchKernelGGL(k_feat_mlp<T>, dim3(ns), dim3(NT), 0, stream, F, w.s0);
    LevelArgs<T> E = A;
    E.need_exact = nullptr;
    compress_pass<T>(E, w, bmax, gscratch, stream, false);
    return;
  }
  // learned ranks by sketches: the sketch kernel first; the exact kernels
  // then take only the steps it flags in need_exact
  if (A.mlp) hipLaunchKernelGGL(k_compress_rand<T>, dim3(ns), dim3(NT), work_compress_rand<T>(), stream, A, w.s0);
  compress_pass<T>(A, w, bmax, gscratch, stream, false);
}

template <typename T>
hipError_t launch_wave_rest(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gscratch, hipStream_t stream,
                            const SideStream* side) {
  hipError_t err = hipSuccess;
  auto keep = [&](hipError_t e) {
    if (err == hipSuccess) err = e;
  };
  T* gs = gscratch;
  const size_t wt = work_tiled<T>() * sizeof(T);
  const bool tiled = wt <= max_lds_bytes();
  LevelArgs<T> B = A;
  if (tiled) B.small_by_wave = 64;   // the generic kernels skip the steps the tiled ones take
  // steps of 65..BG_MAXB unknowns: tiled big-block kernels (strips of the
  // views in LDS, products on the FP64 matrix cores); the generic kernels then
  // take only larger blocks
  const size_t wsb = work_strip_big<T>(bmax);
  const bool big = tiled && bmax > 64 && A.big && wsb <= max_lds_bytes();
  LevelArgs<T> G = B;
  if (big) G.small_by_wave = BG_MAXB;
  const bool generic = !tiled || (bmax > 64 && (!big || bmax > BG_MAXB));
  B.items = A.rot;
  G.items = A.rot;
  const size_t wpb = work_potrf_big<T>(bmax);
  const bool ptiled = tiled && (size_t)PW4_LDS <= max_lds_bytes();
  const bool pbig = ptiled && bmax > 64 && big && wpb <= max_lds_bytes();
  // the diagonal blocks of the big steps (U_i^T D_i U_i, then their Cholesky
  // factor) depend on the compression only, the views' rotation touches no
  // diagonal block and neither touches the step scratch the other uses: with
  // a side stream the two run side by side, joined before the triangular
  // solves (not with compensation, which updates the diagonal blocks, nor when
  // generic kernels share the scratch)
  const bool fork = side && side->s && big && pbig && !generic && !A.compensate && w.s1 > w.s0;
  hipStream_t ds = fork ? side->s : stream;
  if (fork) {
    keep(hipEventRecord(side->fork, stream));
    keep(hipStreamWaitEvent(side->s, side->fork, 0));
  }
  if (big && w.s1 > w.s0) {
    const int nstrip = (std::min(bmax, BG_MAXB) + 31) / 32;
    const dim3 gd((unsigned)((w.s1 - w.s0) * nstrip));
    const size_t wsd = work_strip_big<T, 32>(bmax);
    hipLaunchKernelGGL((k_rot_big_diag<T, 0>), gd, dim3(NT), wsd, ds, B, w.s0, nstrip);
    hipLaunchKernelGGL((k_rot_big_diag<T, 1>), gd, dim3(NT), wsd, ds, B, w.s0, nstrip);
    if (fork) hipLaunchKernelGGL(k_potrf_big<T>, dim3(w.s1 - w.s0), dim3(NT), wpb, ds, B, w.s0);
  }
  if (fork) keep(hipEventRecord(side->join, ds));
  if (tiled && w.r1 > w.r0)
    hipLaunchKernelGGL(k_rotate_t<T>, dim3(w.r1 - w.r0), dim3(NT), wt, stream, B, w.r0);
  if (big && w.r1 > w.r0) {
    // (two strips per pass measured slower: the doubled LDS halves the
    // workgroups a compute unit holds, which hide the L2 latency of U_i)
    hipLaunchKernelGGL((k_rot_big<T, 1, SW_VIEW>), dim3(w.r1 - w.r0), dim3(NT), (work_strip_big<T, SW_VIEW>(bmax)),
                       stream, B, w.r0);
  }
  if (generic) launch<T>(k_rotate<T>, G, w.r0, w.r1 - w.r0, work_rotate<T>(bmax), gs, stream, bmax);
  if (A.compensate && w.s1 > w.s0)
    hipLaunchKernelGGL(k_compensate<T>, dim3(w.s1 - w.s0), dim3(NT), 0, stream, A, w.s0);
  if (ptiled && w.s1 > w.s0)
    hipLaunchKernelGGL(k_potrf_w<T>, dim3(w.s1 - w.s0), dim3(NT), PW4_LDS, stream, B, w.s0);
  if (!ptiled) {
    launch<T>(k_potrf<T>, A, w.s0, w.s1 - w.s0, work_potrf<T>(bmax), gs, stream, bmax);
  } else if (bmax > 64) {
    if (pbig && !fork && w.s1 > w.s0)
      hipLaunchKernelGGL(k_potrf_big<T>, dim3(w.s1 - w.s0), dim3(NT), wpb, stream, B, w.s0);
    if (!pbig || bmax > BG_MAXB)
      launch<T>(k_potrf<T>, pbig ? G : B, w.s0, w.s1 - w.s0, work_potrf<T>(bmax), gs, stream, bmax);
  }
  if (fork) keep(hipStreamWaitEvent(stream, side->join, 0));
  B.items = A.trsm;
  G.items = A.trsm;
  if (tiled && w.t1 > w.t0)
    hipLaunchKernelGGL(k_trsm_t<T>, dim3(w.t1 - w.t0), dim3(NT), wt, stream, B, w.t0);
  if (big && w.t1 > w.t0)
    hipLaunchKernelGGL((k_trsm_big<T, 1, Strip<T>::SW>), dim3(w.t1 - w.t0), dim3(NT), wsb, stream, B, w.t0);
  if (generic) launch<T>(k_trsm<T>, G, w.t0, w.t1 - w.t0, work_trsm<T>(bmax), gs, stream, bmax);
  return err;
}

// The Schur updates of a wave (after its triangular solves).
template <typename T>
void launch_wave_schur(const LevelArgs<T>& A, const WaveRange& w, int bmax, T* gscratch, hipStream_t stream) {
  T* gs = gscratch;
  const size_t wt = work_tiled<T>() * sizeof(T);
  const bool tiled = wt <= max_lds_bytes();
  LevelArgs<T> B = A;
  if (tiled) B.small_by_wave = 64;
  const size_t wsb = work_strip_big<T>(bmax);
  const bool big = tiled && bmax > 64 && A.big && wsb <= max_lds_bytes();
  LevelArgs<T> G = B;
  if (big) G.small_by_wave = BG_MAXB;
  const bool generic = !tiled || (bmax > 64 && (!big || bmax > BG_MAXB));
  if (tiled && w.p1 > w.p0) {
    if (A.bf16_schur && sizeof(T) == sizeof(float))
      hipLaunchKernelGGL(k_schur_bf16<T>, dim3(w.p1 - w.p0), dim3(NT), wt, stream, B, w.p0);
    else
      hipLaunchKernelGGL(k_schur_t<T>, dim3(w.p1 - w.p0), dim3(NT), wt, stream, B, w.p0);
  }
  if (big && w.p1 > w.p0) {
    if (A.bf16_schur && sizeof(T) == sizeof(float)) {
      // pairs with a narrow panel, then pairs of two wide ones (kernels of
      // their own: the wide one's registers would cost the narrow one occupancy)
      hipLaunchKernelGGL(k_schur_big_bf16<T>, dim3(w.p1 - w.p0), dim3(NT), wt, stream, B, w.p0);
      hipLaunchKernelGGL(k_schur_big_bf16w<T>, dim3(w.p1 - w.p0), dim3(NT), work_schur_big_bf16<T>(), stream, B,
                         w.p0);
    } else
      hipLaunchKernelGGL(k_schur_big<T>, dim3(w.p1 - w.p0), dim3(NT), wt, stream, B, w.p0);
  }
  if (generic) launch<T>(k_schur<T>, G, w.p0, w.p1 - w.p0, work_schur<T>(bmax), gs, stream, bmax);
}

template <typename T>
void launch_scatter_a0(T* arena, const double* vals, const int64_t* dst, int64_t nnz, hipStream_t stream) {
  int64_t blocks = (nnz + NT - 1) / NT;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_scatter_a0<T>, dim3((unsigned)blocks), dim3(NT), 0, stream, arena, vals, dst, nnz);
}

void launch_theta(const double* vals, const int64_t* diag_pos, int64_t n, double eps, double* out,
                  hipStream_t stream) {
  (void)hipMemsetAsync(out, 0, 2 * sizeof(double), stream);
  int64_t blocks = (n + NT - 1) / NT;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_theta_max, dim3((unsigned)blocks), dim3(NT), 0, stream, vals, diag_pos, n,
                     reinterpret_cast<unsigned long long*>(out + 1));
  hipLaunchKernelGGL(k_theta_fin, dim3(1), dim3(1), 0, stream, eps, out);
}

template <typename T>
void launch_gather_next(const Trans* items, int32_t nitems, const T* src, const int64_t* src_off,
                        const int32_t* bsz, const int32_t* rank, const int32_t* parent,
                        const int32_t* off_in_parent, T* dst, const int64_t* dst_off, const int32_t* bsz_next,
                        hipStream_t stream) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_gather_next<T>, dim3(nitems), dim3(NT), 0, stream, items, src, src_off, bsz, rank, parent,
                     off_in_parent, dst, dst_off, bsz_next);
}

template <typename T>
void launch_coarse_assemble(const int32_t* slot_p, const int32_t* slot_q, int32_t nslots, const T* arena,
                            const int64_t* slot_off, const int32_t* bsz, const int64_t* dof_off, double* Ad,
                            int64_t dim, hipStream_t stream) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_coarse_assemble<T>, dim3(nslots), dim3(NT), 0, stream, slot_p, slot_q, arena, slot_off, bsz,
                     dof_off, Ad, dim);
}

void launch_gj_inverse(double* Ad, int64_t dim, double* Pinv, double* W, double* R0, int32_t* err,
                       hipStream_t stream) {
  // Pinv holds two 64 x 64 pivot inverses: panel p uses half p % 2, and its
  // update kernel writes the next panel's into the other half
  const unsigned nt = (unsigned)((dim + GJ - 1) / GJ);
  const size_t lds = (size_t)2 * 64 * TLD * sizeof(double);
  if (dim > 0)
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(GJT), lds, stream, Ad, dim, (int64_t)0, (int)std::min<int64_t>(GJ, dim),
                       Pinv, err);
  int p = 0;
  for (int64_t k0 = 0; k0 < dim; k0 += GJ, ++p) {
    const int kb = (int)std::min<int64_t>(GJ, dim - k0);
    double* Pc = Pinv + (size_t)(p & 1) * GJ * GJ;
    double* Pn = k0 + kb < dim ? Pinv + (size_t)((p + 1) & 1) * GJ * GJ : nullptr;
    hipLaunchKernelGGL(k_gj_rows, dim3(nt), dim3(NT), lds, stream, (const double*)Ad, dim, k0, kb,
                       (const double*)Pc, W, R0);
    hipLaunchKernelGGL(k_gj_update, dim3(nt, nt), dim3(NT), lds, stream, Ad, dim, k0, kb, (const double*)Pc,
                       (const double*)W, (const double*)R0, Pn, err);
  }
}

#define CAE_INST(T)                                                                                         \
  template size_t factor_scratch_elems<T>(int);                                                            \
  template bool factor_needs_global<T>(int);                                                               \
  template int32_t scratch_group<T>(int);                                                                  \
  template void launch_wave_compress<T>(const LevelArgs<T>&, const WaveRange&, int, T*, hipStream_t);      \
  template hipError_t launch_wave_rest<T>(const LevelArgs<T>&, const WaveRange&, int, T*, hipStream_t,         \
                                         const SideStream*);                                                \
  template void launch_wave_schur<T>(const LevelArgs<T>&, const WaveRange&, int, T*, hipStream_t);         \
  template void launch_scatter_a0<T>(T*, const double*, const int64_t*, int64_t, hipStream_t);             \
  template void launch_gather_next<T>(const Trans*, int32_t, const T*, const int64_t*, const int32_t*,     \
                                      const int32_t*, const int32_t*, const int32_t*, T*, const int64_t*,  \
                                      const int32_t*, hipStream_t);                                        \
  template void launch_coarse_assemble<T>(const int32_t*, const int32_t*, int32_t, const T*, const int64_t*, \
                                          const int32_t*, const int64_t*, double*, int64_t, hipStream_t);
CAE_INST(double)
CAE_INST(float)

}  // namespace cae
