// HIP kernels (gfx950) of the preconditioner apply x = Q^T L^{-T} L^{-1} Q b
// (Proposition 2.2), of the product M x with the stored factor, of the dense
// remainder, and of FP64 PCG (SpMV, dot products, vector updates).
//
// Level vectors are FP64 with the layout y[(dof_off[i] + a) * nrhs + k]: the
// right-hand sides of one unknown are contiguous, so a block of b unknowns is
// one b x nrhs tile.  Factor entries of any precision are widened on load.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cae_internal.h"
#include "kernels.h"

namespace cae {

constexpr int NT = 256;
constexpr int RC = 16;   // right-hand sides per pass of a block kernel
// row stride (doubles) of the LDS vector tiles of the lean kernels: 144 bytes
// puts the four rows that the four threads of an output row read at once on
// different LDS banks
constexpr int RCP = RC + 2;

namespace {
size_t g_max_lds = 64 * 1024;
}
size_t max_lds_bytes() { return g_max_lds; }
void set_max_lds_bytes(size_t b) { g_max_lds = b; }

template <typename T>
__device__ inline double vget(const T* base, int trans, int bi, int bx, int a, int c) {
  return (double)(trans ? base[(int64_t)c * bi + a] : base[(int64_t)a * bx + c]);
}

// Forward block solve of one step: t = L_nn^{-1} y_i[n]; y_c -= L(c, n) t.
template <typename T>
__global__ __launch_bounds__(NT) void k_ap_fwd_generic(ApplyArgs<T> A, int32_t s0, double* y) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  const T* D = A.arena + A.slot_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* t = reinterpret_cast<double*>(smem_raw);    // n x RC
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < n * kc; e += NT) t[(e / kc) * RC + e % kc] = yi[(r + e / kc) * nrhs + k0 + e % kc];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const double d = (double)D[(int64_t)(r + k) * b + r + k];
      if (threadIdx.x < kc) t[k * RC + threadIdx.x] /= d;
      __syncthreads();
      const int m = n - k - 1;
      for (int e = threadIdx.x; e < m * kc; e += NT) {
        const int j = k + 1 + e / kc, c = e % kc;
        t[j * RC + c] -= (double)D[(int64_t)(r + j) * b + r + k] * t[k * RC + c];
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < n * kc; e += NT) yi[(r + e / kc) * nrhs + k0 + e % kc] = t[(e / kc) * RC + e % kc];
    // basis of i
    for (int e = threadIdx.x; e < r * kc; e += NT) {
      const int g = e / kc, c = e % kc;
      double s = 0;
      for (int j = 0; j < n; ++j) s += (double)D[(int64_t)(r + j) * b + g] * t[j * RC + c];
      yi[g * nrhs + k0 + c] -= s;
    }
    // close blocks
    for (int v = 0; v < st.nclose; ++v) {
      const View vw = A.views[st.view0 + v];
      const int bx = A.bsz[vw.x];
      const int lc = vw.proc ? A.rank[vw.x] : bx;
      const T* P = A.arena + A.slot_off[vw.slot];
      double* yx = y + A.dof_off[vw.x] * nrhs;
      for (int e = threadIdx.x; e < lc * kc; e += NT) {
        const int g = e / kc, c = e % kc;
        double s = 0;
        for (int j = 0; j < n; ++j) s += vget(P, vw.trans, b, bx, r + j, g) * t[j * RC + c];
        yx[g * nrhs + k0 + c] -= s;
      }
    }
  }
}

// Backward block solve of one step: z_n = L_nn^{-T} (u - sum_c L(c,n)^T z_c).
template <typename T>
__global__ __launch_bounds__(NT) void k_ap_bwd_generic(ApplyArgs<T> A, int32_t s0, double* y) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  const T* D = A.arena + A.slot_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* t = reinterpret_cast<double*>(smem_raw);    // n x RC
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < n * kc; e += NT) {
      const int j = e / kc, c = e % kc;
      double s = yi[(r + j) * nrhs + k0 + c];
      for (int g = 0; g < r; ++g) s -= (double)D[(int64_t)(r + j) * b + g] * yi[g * nrhs + k0 + c];
      for (int v = 0; v < st.nclose; ++v) {
        const View vw = A.views[st.view0 + v];
        const int bx = A.bsz[vw.x];
        const int lc = vw.proc ? A.rank[vw.x] : bx;
        const T* P = A.arena + A.slot_off[vw.slot];
        const double* yx = y + A.dof_off[vw.x] * nrhs;
        for (int g = 0; g < lc; ++g) s -= vget(P, vw.trans, b, bx, r + j, g) * yx[g * nrhs + k0 + c];
      }
      t[j * RC + c] = s;
    }
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
      const double d = (double)D[(int64_t)(r + k) * b + r + k];
      if (threadIdx.x < kc) t[k * RC + threadIdx.x] /= d;
      __syncthreads();
      for (int e = threadIdx.x; e < k * kc; e += NT) {
        const int j = e / kc, c = e % kc;
        t[j * RC + c] -= (double)D[(int64_t)(r + k) * b + r + j] * t[k * RC + c];
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < n * kc; e += NT) yi[(r + e / kc) * nrhs + k0 + e % kc] = t[(e / kc) * RC + e % kc];
  }
}

// ---------------------------------------------------------------------------
// Lean block-solve kernels: four threads share one output row and split the
// reduction index four ways, each keeping 16 FP64 accumulators (one per
// right-hand side of the pass); a reduce-scatter over the four lanes leaves
// each with the totals of four right-hand sides.  Factor entries are read
// straight from global memory, eight at a time per thread (each quarter
// walks its own addresses, consecutive rows on consecutive lanes), only the
// 16-wide vector tiles live in LDS, so a step needs 16 KB of LDS at b = 64
// and many steps run on one compute unit at once.
// ---------------------------------------------------------------------------
// Right-hand sides per pass R of the lean kernels: 16 (accumulators per
// thread), or 1 for a single right-hand side (no idle accumulators, the LDS
// vector tiles contiguous); RhsPass<R>::P is the row stride of those tiles.
template <int R>
struct RhsPass {
  static constexpr int P = R == 1 ? 1 : R + 2;
  static constexpr int NO = R == 1 ? 1 : 4;   // totals per lane after the reduce-scatter
};

template <int R>
__device__ inline void axpyR(double (&s)[R], double p, const double* v) {
#pragma unroll
  for (int k = 0; k < R; ++k) s[k] += p * v[k];
}

// s += sum over t = t0, t0 + 4, ... < tend of P[t * stride] V[t * P]: the
// panel entries loaded eight at a time (all in flight before the first is
// used), the LDS rows of V read only for t < tend.
template <int R, typename T>
__device__ inline void axpy_run(double (&s)[R], const T* P, int64_t stride, int t0, int tend, const double* V) {
  for (int t = t0; t < tend; t += 32) {
    T pv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int tu = t + 4 * u;
      // unconditional load (P[0] past the end), then zero: a predicated
      // load would be a branch per entry
      const T x = P[tu < tend ? (int64_t)tu * stride : 0];
      pv[u] = tu < tend ? x : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int tu = t + 4 * u;
      if (tu < tend) axpyR<R>(s, (double)pv[u], V + tu * RhsPass<R>::P);
    }
  }
}

// Sum of the R partial sums over the four lanes of a row (lanes 4 rl + q).
// R = 16: reduce-scattered, lane q returns in o[0..3] the totals of columns
// 4 q .. 4 q + 3 (12 exchanges instead of a 32-exchange butterfly); R = 1:
// every lane returns the total in o[0].
template <int R>
__device__ inline void quad_rs(const double (&s)[R], int q, double (&o)[RhsPass<R>::NO]) {
  if constexpr (R == 1) {
    double v = s[0];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    o[0] = v;
  } else {
    const bool hi2 = (q & 2) != 0, hi1 = (q & 1) != 0;
    double h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double send = hi2 ? s[j] : s[8 + j];
      h[j] = (hi2 ? s[8 + j] : s[j]) + __shfl_xor(send, 2, 64);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double send = hi1 ? h[j] : h[4 + j];
      o[j] = (hi1 ? h[4 + j] : h[j]) + __shfl_xor(send, 1, 64);
    }
  }
}

// y[4 q + j] (op)= o[j] for the columns 4 q + j < kc of one RHS row (y at
// column k0 of that row): two 16-byte accesses when the row chunk is whole;
// R = 1: lane q = 0 alone.
template <int R>
__device__ inline void store_out(double* y, int q, int kc, const double (&o)[RhsPass<R>::NO]) {
  if constexpr (R == 1) {
    if (q == 0) y[0] = o[0];
  } else {
    double* p = y + 4 * q;
    if (4 * q + 4 <= kc) {
      reinterpret_cast<double2*>(p)[0] = make_double2(o[0], o[1]);
      reinterpret_cast<double2*>(p)[1] = make_double2(o[2], o[3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 * q + j < kc) p[j] = o[j];
    }
  }
}
template <int R>
__device__ inline void sub_out(double* y, int q, int kc, const double (&o)[RhsPass<R>::NO]) {
  if constexpr (R == 1) {
    if (q == 0) y[0] -= o[0];
  } else {
    double* p = y + 4 * q;
    if (4 * q + 4 <= kc) {
      double2 a = reinterpret_cast<double2*>(p)[0], c = reinterpret_cast<double2*>(p)[1];
      a.x -= o[0];
      a.y -= o[1];
      c.x -= o[2];
      c.y -= o[3];
      reinterpret_cast<double2*>(p)[0] = a;
      reinterpret_cast<double2*>(p)[1] = c;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 * q + j < kc) p[j] -= o[j];
    }
  }
}
// The same for one row of an LDS vector tile (all R columns): set, or add
// sign * o.
template <int R>
__device__ inline void lds_set(double* row, int q, const double (&o)[RhsPass<R>::NO]) {
  if constexpr (R == 1) {
    if (q == 0) row[0] = o[0];
  } else {
    *reinterpret_cast<double2*>(row + 4 * q) = make_double2(o[0], o[1]);
    *reinterpret_cast<double2*>(row + 4 * q + 2) = make_double2(o[2], o[3]);
  }
}
template <int R>
__device__ inline void lds_add(double* row, int q, const double (&o)[RhsPass<R>::NO], double sign) {
  if constexpr (R == 1) {
    if (q == 0) row[0] += sign * o[0];
  } else {
    double2* tp = reinterpret_cast<double2*>(row + 4 * q);
    double2 a0 = tp[0], a1 = tp[1];
    a0.x += sign * o[0];
    a0.y += sign * o[1];
    a1.x += sign * o[2];
    a1.y += sign * o[3];
    tp[0] = a0;
    tp[1] = a1;
  }
}

// Y[t][0..R) = y[(row0 + t) * nrhs + k0 + k] (0 beyond kc), t < m, row
// stride RhsPass<R>::P; eight loads in flight per thread.
template <int R>
__device__ inline void load_vec_tile(double* Y, const double* y, int row0, int m, int nrhs, int k0, int kc) {
  constexpr int RP = RhsPass<R>::P;
  for (int e0 = 0; e0 < m * R; e0 += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + threadIdx.x + NT * u, t = e / R, k = e % R;
      v[u] = (e < m * R && k < kc) ? y[(int64_t)(row0 + t) * nrhs + k0 + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + threadIdx.x + NT * u;
      if (e < m * R) Y[(e / R) * RP + e % R] = v[u];
    }
  }
}

// Descriptors of the close views of a step, loaded by parallel threads into
// LDS before the panel loop: read per panel, they formed a chain of
// dependent scalar loads (view, then its block's size, rank and offsets)
// that the counters showed as the kernels' main wait.
constexpr int APV = 64;   // views staged (more are read directly)
struct ViewDesc {
  int64_t poff[APV];
  int64_t yoff[APV];
  int lc[APV];
  int bx[APV];
  int tr[APV];
};
template <typename T>
__device__ inline void stage_views(const ApplyArgs<T>& A, const Step& st, ViewDesc* vd) {
  for (int v = threadIdx.x; v < min(st.nclose, APV); v += NT) {
    const View vw = A.views[st.view0 + v];
    const int bx = A.bsz[vw.x];
    vd->poff[v] = A.slot_off[vw.slot];
    vd->yoff[v] = A.dof_off[vw.x] * A.nrhs;
    vd->lc[v] = vw.proc ? A.rank[vw.x] : bx;
    vd->bx[v] = bx;
    vd->tr[v] = vw.trans;
  }
}
template <typename T>
__device__ inline void view_desc(const ApplyArgs<T>& A, const Step& st, const ViewDesc* vd, int v, int64_t& poff,
                                 int64_t& yoff, int& lc, int& bx, int& tr) {
  if (v < APV) {
    poff = vd->poff[v];
    yoff = vd->yoff[v];
    lc = vd->lc[v];
    bx = vd->bx[v];
    tr = vd->tr[v];
  } else {
    const View vw = A.views[st.view0 + v];
    bx = A.bsz[vw.x];
    poff = A.slot_off[vw.slot];
    yoff = A.dof_off[vw.x] * A.nrhs;
    lc = vw.proc ? A.rank[vw.x] : bx;
    tr = vw.trans;
  }
}

template <typename T, int R>
__global__ __launch_bounds__(NT) void k_ap_rot2(ApplyArgs<T> A, double* y, int dir) {
  constexpr int RP = RhsPass<R>::P;
  const Step st = A.steps[blockIdx.x];
  if (st.nfar == 0) return;
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b == 0) return;
  const int nrhs = A.nrhs;
  const T* U = A.U + A.u_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Ys = reinterpret_cast<double*>(smem_raw);   // b x R
  const int rl = threadIdx.x >> 2, q = threadIdx.x & 3;
  for (int k0 = 0; k0 < nrhs; k0 += R) {
    const int kc = min(R, nrhs - k0);
    __syncthreads();
    load_vec_tile<R>(Ys, yi, 0, b, nrhs, k0, kc);
    __syncthreads();
    for (int a0 = 0; a0 < b; a0 += 64) {
      const int a = a0 + rl;
      double s[R];
#pragma unroll
      for (int k = 0; k < R; ++k) s[k] = 0.0;
      if (a < b) {
        if (dir == 0)
          axpy_run<R>(s, U + a, b, q, b, Ys);
        else
          axpy_run<R>(s, U + (int64_t)a * b, 1, q, b, Ys);
      }
      double o[RhsPass<R>::NO];
      quad_rs<R>(s, q, o);
      if (a < b) store_out<R>(yi + (int64_t)a * nrhs + k0, q, kc, o);
    }
  }
}

// Forward block solve of one step: t = L_nn^{-1} y_i[n], y_i[n] = t, and
// y_c -= L(c, n) t for the basis of i and (views != 0) every close block c;
// with views = 0 the close blocks are left to k_ap_fview.
template <typename T, int R>
__global__ __launch_bounds__(NT) void k_ap_fwd2(ApplyArgs<T> A, int32_t s0, double* y, int nmax, int views) {
  constexpr int RP = RhsPass<R>::P;
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* yn = reinterpret_cast<double*>(smem_raw);   // n x R
  double* tn = yn + (size_t)nmax * RP;                // n x R, row stride RP
  ViewDesc* vd = reinterpret_cast<ViewDesc*>(tn + (size_t)nmax * RP);
  const T* Li = A.Li + A.u_off[i];
  const T* D = A.arena + A.slot_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  const int rl = threadIdx.x >> 2, q = threadIdx.x & 3;
  stage_views(A, st, vd);
  for (int k0 = 0; k0 < nrhs; k0 += R) {
    const int kc = min(R, nrhs - k0);
    __syncthreads();
    load_vec_tile<R>(yn, yi, r, n, nrhs, k0, kc);
    __syncthreads();
    for (int row0 = 0; row0 < n; row0 += 64) {
      const int row = row0 + rl;
      double s[R];
#pragma unroll
      for (int k = 0; k < R; ++k) s[k] = 0.0;
      if (row < n) axpy_run<R>(s, Li + (int64_t)row * n, 1, q, row + 1, yn);
      double o[RhsPass<R>::NO];
      quad_rs<R>(s, q, o);
      if (row < n) {
        lds_set<R>(tn + row * RP, q, o);
        store_out<R>(yi + (int64_t)(r + row) * nrhs + k0, q, kc, o);
      }
    }
    __syncthreads();
    const int nv = views ? st.nclose : 0;
    for (int v = -1; v < nv; ++v) {
      const T* P;
      int trans, bx, lc;
      double* yx;
      if (v < 0) {
        P = D;
        trans = 0;
        bx = b;
        lc = r;
        yx = yi;
      } else {
        int64_t poff, yoff;
        view_desc(A, st, vd, v, poff, yoff, lc, bx, trans);
        P = A.arena + poff;
        yx = y + yoff;
      }
      for (int g0 = 0; g0 < lc; g0 += 64) {
        const int g = g0 + rl;
        double s[R];
#pragma unroll
        for (int k = 0; k < R; ++k) s[k] = 0.0;
        if (g < lc) {
          if (trans)
            axpy_run<R>(s, P + (int64_t)g * b + r, 1, q, n, tn);
          else
            axpy_run<R>(s, P + (int64_t)r * bx + g, bx, q, n, tn);
        }
        double o[RhsPass<R>::NO];
        quad_rs<R>(s, q, o);
        if (g < lc) sub_out<R>(yx + (int64_t)g * nrhs + k0, q, kc, o);
      }
    }
  }
}

// Backward block solve of one step: t = y_i[n] - sum_c L(c, n)^T z_c over the
// basis of i and the close blocks, then y_i[n] = L_nn^{-T} t.  With part the
// close blocks' products come precomputed (k_ap_bpart, maxclose slots of
// nmax x nrhs per step).
template <typename T, int R>
__global__ __launch_bounds__(NT) void k_ap_bwd2(ApplyArgs<T> A, int32_t s0, double* y, int nmax, const double* part,
                                                int maxclose) {
  constexpr int RP = RhsPass<R>::P;
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tn = reinterpret_cast<double*>(smem_raw);   // n x R
  double* zt = tn + (size_t)nmax * RP;                // 64 x R, row stride RP
  ViewDesc* vd = reinterpret_cast<ViewDesc*>(zt + (size_t)64 * RP);
  const T* Li = A.Li + A.u_off[i];
  const T* D = A.arena + A.slot_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  const int rl = threadIdx.x >> 2, q = threadIdx.x & 3;
  stage_views(A, st, vd);
  for (int k0 = 0; k0 < nrhs; k0 += R) {
    const int kc = min(R, nrhs - k0);
    __syncthreads();
    load_vec_tile<R>(tn, yi, r, n, nrhs, k0, kc);
    const int nv = part ? 0 : st.nclose;
    for (int v = -1; v < nv; ++v) {
      const T* P;
      int trans, bx, lc;
      const double* zx;
      if (v < 0) {
        P = D;
        trans = 0;
        bx = b;
        lc = r;
        zx = yi;
      } else {
        int64_t poff, yoff;
        view_desc(A, st, vd, v, poff, yoff, lc, bx, trans);
        P = A.arena + poff;
        zx = y + yoff;
      }
      for (int g0 = 0; g0 < lc; g0 += 64) {
        const int gc = min(64, lc - g0);
        __syncthreads();
        load_vec_tile<R>(zt, zx, g0, gc, nrhs, k0, kc);
        __syncthreads();
        for (int t0 = 0; t0 < n; t0 += 64) {
          const int t = t0 + rl;
          double s[R];
#pragma unroll
          for (int k = 0; k < R; ++k) s[k] = 0.0;
          if (t < n) {
            if (trans)
              axpy_run<R>(s, P + (int64_t)g0 * b + r + t, b, q, gc, zt);
            else
              axpy_run<R>(s, P + (int64_t)(r + t) * bx + g0, 1, q, gc, zt);
          }
          double o[RhsPass<R>::NO];
          quad_rs<R>(s, q, o);
          if (t < n) lds_add<R>(tn + t * RP, q, o, -1.0);
        }
      }
    }
    __syncthreads();
    if (part) {
      // the close blocks' products L(c, n)^T z_c from k_ap_bpart, subtracted
      // in view order (eight loads in flight per element)
      const double* pp = part + (int64_t)blockIdx.x * maxclose * nmax * nrhs;
      const int64_t pstride = (int64_t)nmax * nrhs;
      for (int e = threadIdx.x; e < n * R; e += NT) {
        const int t = e / R, k = e % R;
        if (k >= kc) continue;
        double acc = tn[t * RP + k];
        for (int v0 = 0; v0 < st.nclose; v0 += 8) {
          double pv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) pv[u] = v0 + u < st.nclose ? pp[(v0 + u) * pstride + t * nrhs + k0 + k] : 0.0;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (v0 + u < st.nclose) acc -= pv[u];
        }
        tn[t * RP + k] = acc;
      }
      __syncthreads();
    }
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int c = c0 + rl;
      double s[R];
#pragma unroll
      for (int k = 0; k < R; ++k) s[k] = 0.0;
      if (c < n) axpy_run<R>(s, Li + c, n, c + q, n, tn);
      double o[RhsPass<R>::NO];
      quad_rs<R>(s, q, o);
      if (c < n) store_out<R>(yi + (int64_t)(r + c) * nrhs + k0, q, kc, o);
    }
  }
}

// Forward update of one close block of one step (grid: steps x close views),
// after k_ap_fwd2 with views = 0 has left t = L_nn^{-1} y_i[n] in y_i[n]:
// y_c -= L(c, n) t.  Steps of one wave share no close block, so the
// workgroups of a launch write disjoint rows; a step's views run in parallel
// instead of one after another (the waves of the upper levels hold too few
// steps to hide that chain of memory round trips).
template <typename T, int R>
__global__ __launch_bounds__(NT) void k_ap_fview(ApplyArgs<T> A, int32_t s0, double* y, int nmax) {
  constexpr int RP = RhsPass<R>::P;
  const Step st = A.steps[s0 + blockIdx.x];
  const int v = blockIdx.y;
  if (v >= st.nclose) return;
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const View vw = A.views[st.view0 + v];
  const int bx = A.bsz[vw.x];
  const int lc = vw.proc ? A.rank[vw.x] : bx;
  if (lc <= 0) return;
  const int nrhs = A.nrhs;
  const T* P = A.arena + A.slot_off[vw.slot];
  const double* yi = y + A.dof_off[i] * nrhs;
  double* yx = y + A.dof_off[vw.x] * nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tn = reinterpret_cast<double*>(smem_raw);   // n x R, row stride RP
  const int rl = threadIdx.x >> 2, q = threadIdx.x & 3;
  for (int k0 = 0; k0 < nrhs; k0 += R) {
    const int kc = min(R, nrhs - k0);
    __syncthreads();
    load_vec_tile<R>(tn, yi, r, n, nrhs, k0, kc);
    __syncthreads();
    for (int g0 = 0; g0 < lc; g0 += 64) {
      const int g = g0 + rl;
      double s[R];
#pragma unroll
      for (int k = 0; k < R; ++k) s[k] = 0.0;
      if (g < lc) {
        if (vw.trans)
          axpy_run<R>(s, P + (int64_t)g * b + r, 1, q, n, tn);
        else
          axpy_run<R>(s, P + (int64_t)r * bx + g, bx, q, n, tn);
      }
      double o[RhsPass<R>::NO];
      quad_rs<R>(s, q, o);
      if (g < lc) sub_out<R>(yx + (int64_t)g * nrhs + k0, q, kc, o);
    }
  }
}

// Backward product of one close block of one step (grid: steps x close
// views): part = L(c, n)^T z_c (n x nrhs, zero when c has no live rows), in
// slot (step, view) of maxclose per step; k_ap_bwd2 subtracts them in view
// order.
template <typename T, int R>
__global__ __launch_bounds__(NT) void k_ap_bpart(ApplyArgs<T> A, int32_t s0, const double* y, double* part, int nmax,
                                                 int maxclose) {
  constexpr int RP = RhsPass<R>::P;
  const Step st = A.steps[s0 + blockIdx.x];
  const int v = blockIdx.y;
  if (v >= st.nclose) return;
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const View vw = A.views[st.view0 + v];
  const int bx = A.bsz[vw.x];
  const int lc = vw.proc ? A.rank[vw.x] : bx;
  const int nrhs = A.nrhs;
  const T* P = A.arena + A.slot_off[vw.slot];
  const double* zx = y + A.dof_off[vw.x] * nrhs;
  double* pp = part + ((int64_t)blockIdx.x * maxclose + v) * nmax * nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* pt = reinterpret_cast<double*>(smem_raw);   // n x R, row stride RP
  double* zt = pt + (size_t)nmax * RP;                // 64 x R, row stride RP
  const int rl = threadIdx.x >> 2, q = threadIdx.x & 3;
  for (int k0 = 0; k0 < nrhs; k0 += R) {
    const int kc = min(R, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < n * RP; e += NT) pt[e] = 0.0;
    for (int g0 = 0; g0 < lc; g0 += 64) {
      const int gc = min(64, lc - g0);
      __syncthreads();
      load_vec_tile<R>(zt, zx, g0, gc, nrhs, k0, kc);
      __syncthreads();
      for (int t0 = 0; t0 < n; t0 += 64) {
        const int t = t0 + rl;
        double s[R];
#pragma unroll
        for (int k = 0; k < R; ++k) s[k] = 0.0;
        if (t < n) {
          if (vw.trans)
            axpy_run<R>(s, P + (int64_t)g0 * b + r + t, b, q, gc, zt);
          else
            axpy_run<R>(s, P + (int64_t)(r + t) * bx + g0, 1, q, gc, zt);
        }
        double o[RhsPass<R>::NO];
        quad_rs<R>(s, q, o);
        if (t < n) lds_add<R>(pt + t * RP, q, o, 1.0);
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * R; e += NT) {
      const int t = e / R, k = e % R;
      if (k < kc) pp[t * nrhs + k0 + k] = pt[t * RP + k];
    }
  }
}

// w_i = Lcheck(:, n_i)^T z for every step (no ordering constraint).
template <typename T>
__global__ __launch_bounds__(NT) void k_mul_w(ApplyArgs<T> A, const double* z, double* w) {
  const Step st = A.steps[blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  const T* D = A.arena + A.slot_off[i];
  const double* zi = z + A.dof_off[i] * nrhs;
  double* wi = w + A.dof_off[i] * nrhs;
  for (int e = threadIdx.x; e < n * nrhs; e += NT) {
    const int j = e / nrhs, c = e % nrhs;
    double s = 0;
    for (int l = j; l < n; ++l) s += (double)D[(int64_t)(r + l) * b + r + j] * zi[(r + l) * nrhs + c];
    for (int g = 0; g < r; ++g) s += (double)D[(int64_t)(r + j) * b + g] * zi[g * nrhs + c];
    for (int v = 0; v < st.nclose; ++v) {
      const View vw = A.views[st.view0 + v];
      const int bx = A.bsz[vw.x];
      const int lc = vw.proc ? A.rank[vw.x] : bx;
      const T* P = A.arena + A.slot_off[vw.slot];
      const double* zx = z + A.dof_off[vw.x] * nrhs;
      for (int g = 0; g < lc; ++g) s += vget(P, vw.trans, b, bx, r + j, g) * zx[g * nrhs + c];
    }
    wi[(r + j) * nrhs + c] = s;
  }
}

// out += Lcheck(:, n_i) w_i for the steps of one wave.
template <typename T>
__global__ __launch_bounds__(NT) void k_mul_lw(ApplyArgs<T> A, int32_t s0, const double* w, double* out) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  const T* D = A.arena + A.slot_off[i];
  const double* wi = w + A.dof_off[i] * nrhs;
  double* oi = out + A.dof_off[i] * nrhs;
  for (int e = threadIdx.x; e < n * nrhs; e += NT) {
    const int j = e / nrhs, c = e % nrhs;
    double s = 0;
    for (int t = 0; t <= j; ++t) s += (double)D[(int64_t)(r + j) * b + r + t] * wi[(r + t) * nrhs + c];
    oi[(r + j) * nrhs + c] += s;
  }
  for (int e = threadIdx.x; e < r * nrhs; e += NT) {
    const int g = e / nrhs, c = e % nrhs;
    double s = 0;
    for (int t = 0; t < n; ++t) s += (double)D[(int64_t)(r + t) * b + g] * wi[(r + t) * nrhs + c];
    oi[g * nrhs + c] += s;
  }
  for (int v = 0; v < st.nclose; ++v) {
    const View vw = A.views[st.view0 + v];
    const int bx = A.bsz[vw.x];
    const int lc = vw.proc ? A.rank[vw.x] : bx;
    const T* P = A.arena + A.slot_off[vw.slot];
    double* ox = out + A.dof_off[vw.x] * nrhs;
    for (int e = threadIdx.x; e < lc * nrhs; e += NT) {
      const int g = e / nrhs, c = e % nrhs;
      double s = 0;
      for (int t = 0; t < n; ++t) s += vget(P, vw.trans, b, bx, r + t, g) * wi[(r + t) * nrhs + c];
      ox[g * nrhs + c] += s;
    }
  }
}

__global__ void k_to_next(const int64_t* dof_off, const int32_t* rank, const int32_t* parent,
                          const int32_t* off_in_parent, const int64_t* dof_off_next, int32_t nrhs, double* y,
                          double* ynext, int dir) {
  const int c = blockIdx.x;
  const int r = rank[c];
  if (r == 0) return;
  double* a = y + dof_off[c] * nrhs;
  double* b = ynext + (dof_off_next[parent[c]] + off_in_parent[c]) * nrhs;
  for (int e = threadIdx.x; e < r * nrhs; e += blockDim.x) {
    if (dir == 0)
      b[e] = a[e];
    else
      a[e] = b[e];
  }
}

// out = sign * A y, A dense row-major dim x dim, y/out dim x nrhs: eight rows
// per workgroup, 32 threads per row each summing every 32nd column for 16
// right-hand sides, then a shuffle reduction over the 32.
constexpr int MV_ROWS = 8;
__global__ __launch_bounds__(NT) void k_dense_mv(const double* A, int64_t dim, int32_t nrhs, const double* y,
                                                 double* out, double sign) {
  const int rl = threadIdx.x >> 5, part = threadIdx.x & 31;
  const int64_t row = (int64_t)blockIdx.x * MV_ROWS + rl;
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    double s[RC];
#pragma unroll
    for (int k = 0; k < RC; ++k) s[k] = 0.0;
    if (row < dim) {
      const double* Ar = A + row * dim;
      for (int64_t j = part; j < dim; j += 32) {
        const double a = Ar[j];
        const double* yj = y + j * nrhs + k0;
        if (kc == RC) {
#pragma unroll
          for (int k = 0; k < RC; ++k) s[k] += a * yj[k];
        } else {
#pragma unroll
          for (int k = 0; k < RC; ++k)
            if (k < kc) s[k] += a * yj[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RC; ++k)
      for (int o = 1; o < 32; o <<= 1) s[k] += __shfl_xor(s[k], o, 64);
    if (row < dim) {
#pragma unroll
      for (int k = 0; k < RC; ++k)
        if (part == k && k < kc) out[row * nrhs + k0 + k] = sign * s[k];
    }
  }
}

__global__ void k_perm_in(int64_t n, int32_t nrhs, const int32_t* perm, const double* x, int64_t ldx, double* y) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nrhs, k = e % nrhs;
    y[e] = x[perm[i] + k * ldx];
  }
}

__global__ void k_perm_out(int64_t n, int32_t nrhs, const int32_t* perm, const double* y, double* x, int64_t ldx) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nrhs, k = e % nrhs;
    x[perm[i] + k * ldx] = y[e];
  }
}

// ------------------------------------------------------------------ PCG ----
// y = A x for all right-hand sides: one thread per row, the row's entries
// read once per group of eight right-hand sides (the matrix is streamed
// nrhs / 8 times, not nrhs times).
// y = A x for nrhs columns, one thread per row, eight columns per pass.
__global__ void k_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                       int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy) {
  const int64_t i = xcd_swizzle(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
  for (int k0 = 0; k0 < nrhs; k0 += 8) {
    double s[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
      const double v = vals[e];
      const int64_t c = col_idx[e];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k0 + j < nrhs) s[j] += v * x[(int64_t)(k0 + j) * ldx + c];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k0 + j < nrhs) y[(int64_t)(k0 + j) * ldy + i] = s[j];
  }
}

constexpr int DOT_BLOCKS = 1024;
__global__ __launch_bounds__(NT) void k_dot_part(int64_t n, const double* a, int64_t lda, const double* b,
                                                 int64_t ldb, double* partial) {
  __shared__ double red[NT];
  const int k = blockIdx.y;
  const double* ak = a + k * lda;
  const double* bk = b + k * ldb;
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) s += ak[i] * bk[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[k * DOT_BLOCKS + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void k_dot_final(const double* partial, int nb, double* out) {
  __shared__ double red[NT];
  const int k = blockIdx.x;
  double s = 0;
  for (int e = threadIdx.x; e < nb; e += NT) s += partial[k * DOT_BLOCKS + e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

__global__ void k_pcg_xr(int64_t n, int32_t nrhs, const double* rz, const double* pq, const int32_t* active,
                         double* x, int64_t ldx, const double* p, double* r, const double* q) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n || !active[k]) return;
  const double alpha = rz[k] / pq[k];
  x[i + k * ldx] += alpha * p[i + k * n];
  r[i + k * n] -= alpha * q[i + k * n];
}

__global__ void k_pcg_beta(int32_t nrhs, double* rz, const double* rz_new, const int32_t* active, double* beta) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  beta[k] = active[k] ? rz_new[k] / rz[k] : 0.0;
  if (active[k]) rz[k] = rz_new[k];
}

__global__ void k_pcg_p(int64_t n, const int32_t* active, const double* beta, const double* z, double* p) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n || !active[k]) return;
  p[i + k * n] = z[i + k * n] + beta[k] * p[i + k * n];
}

// Segmented forms for the problems of a batch: one workgroup per (tile,
// column); a tile lies inside one segment, so its lane is uniform.
__global__ __launch_bounds__(NT) void k_seg_dot_part(SegTiles sg, const double* a, int64_t lda, const double* b,
                                                     int64_t ldb, double* partial) {
  __shared__ double red[NT];
  const int t = blockIdx.x, k = blockIdx.y;
  const double* ak = a + k * lda;
  const double* bk = b + k * ldb;
  double s = 0;
  for (int64_t i = sg.tb[t] + threadIdx.x; i < sg.te[t]; i += NT) s += ak[i] * bk[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)k * sg.ntiles + t] = red[0];
}

__global__ __launch_bounds__(NT) void k_seg_dot_final(SegTiles sg, const double* partial, double* out) {
  __shared__ double red[NT];
  const int sgm = blockIdx.x, k = blockIdx.y;
  double s = 0;
  for (int t = sg.sfirst[sgm] + threadIdx.x; t < sg.sfirst[sgm + 1]; t += NT) s += partial[(int64_t)k * sg.ntiles + t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k * sg.nseg + sgm] = red[0];
}

__global__ __launch_bounds__(NT) void k_seg_pcg_xr(SegTiles sg, int64_t n, const double* rz, const double* pq,
                                                   const int32_t* active, double* x, int64_t ldx, const double* p,
                                                   double* r, const double* q) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int lane = k * sg.nseg + sg.ts[t];
  if (!active[lane]) return;
  const double alpha = rz[lane] / pq[lane];
  for (int64_t i = sg.tb[t] + threadIdx.x; i < sg.te[t]; i += NT) {
    x[i + k * ldx] += alpha * p[i + k * n];
    r[i + k * n] -= alpha * q[i + k * n];
  }
}

__global__ __launch_bounds__(NT) void k_seg_pcg_p(SegTiles sg, int64_t n, const int32_t* active, const double* beta,
                                                  const double* z, double* p) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int lane = k * sg.nseg + sg.ts[t];
  if (!active[lane]) return;
  const double bt = beta[lane];
  for (int64_t i = sg.tb[t] + threadIdx.x; i < sg.te[t]; i += NT) p[i + k * n] = z[i + k * n] + bt * p[i + k * n];
}

// ---------------------------------------------------------------- MINRES ----
// Per-column scalars of preconditioned MINRES live on the device, st[f * nrhs
// + k] with field f below; only phibar (the preconditioned residual norm) is
// read back per iteration for the stopping test.
__global__ void k_mr_v(int64_t n, const int32_t* active, const double* st, int32_t nrhs, const double* y,
                       double* v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n || !active[k]) return;
  v[i + k * n] = y[i + k * n] / st[MR_BETA * nrhs + k];
}

// y -= c r with c = beta / oldb (which = 0) or alpha / beta (which = 1)
__global__ void k_mr_y(int64_t n, const int32_t* active, const double* st, int32_t nrhs, const double* r, double* y,
                       int which) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n || !active[k]) return;
  const double c = which == 0 ? st[MR_BETA * nrhs + k] / st[MR_OLDB * nrhs + k]
                              : st[MR_ALPHA * nrhs + k] / st[MR_BETA * nrhs + k];
  y[i + k * n] -= c * r[i + k * n];
}

__global__ void k_mr_scalars(int32_t nrhs, const int32_t* active, double* st) {
  const int k = threadIdx.x;
  if (k >= nrhs || !active[k]) return;
  double* f = st + k;
  const double alpha = f[MR_ALPHA * nrhs];
  const double beta = sqrt(fmax(f[MR_BSQ * nrhs], 0.0));
  const double cs = f[MR_CS * nrhs], sn = f[MR_SN * nrhs], dbar = f[MR_DBAR * nrhs];
  f[MR_OLDB * nrhs] = f[MR_BETA * nrhs];
  f[MR_BETA * nrhs] = beta;
  f[MR_OLDEPS * nrhs] = f[MR_EPSLN * nrhs];
  f[MR_DELTA * nrhs] = cs * dbar + sn * alpha;
  const double gbar = sn * dbar - cs * alpha;
  f[MR_EPSLN * nrhs] = sn * beta;
  f[MR_DBAR * nrhs] = -cs * beta;
  const double gamma = fmax(sqrt(gbar * gbar + beta * beta), 1e-300);
  f[MR_GAMMA * nrhs] = gamma;
  f[MR_CS * nrhs] = gbar / gamma;
  f[MR_SN * nrhs] = beta / gamma;
  const double phibar = f[MR_PHIBAR * nrhs];
  f[MR_PHI * nrhs] = (gbar / gamma) * phibar;
  f[MR_PHIBAR * nrhs] = (beta / gamma) * phibar;
}

// w_new = (v - oldeps w_prev2 - delta w_prev) / gamma into wout; x += phi w_new
__global__ void k_mr_wx(int64_t n, const int32_t* active, const double* st, int32_t nrhs, const double* v,
                        const double* wprev2, const double* wprev, double* wout, double* x, int64_t ldx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n || !active[k]) return;
  const double wn = (v[i + k * n] - st[MR_OLDEPS * nrhs + k] * wprev2[i + k * n] -
                     st[MR_DELTA * nrhs + k] * wprev[i + k * n]) /
                    st[MR_GAMMA * nrhs + k];
  wout[i + k * n] = wn;
  x[i + k * ldx] += st[MR_PHI * nrhs + k] * wn;
}

__global__ void k_copy_cols(int64_t n, const double* a, int64_t lda, double* b, int64_t ldb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i < n) b[i + k * ldb] = a[i + k * lda];
}

__global__ void k_fill(double* a, int64_t count, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    a[e] = v;
}

__global__ void k_residual(int64_t n, const double* b, int64_t ldb, double* r) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i < n) r[i + k * n] = b[i + k * ldb] - r[i + k * n];
}

// ------------------------------------------------------------ launchers ----
static unsigned grid1(int64_t work) {
  int64_t g = (work + NT - 1) / NT;
  if (g > 65535 * 4) g = 65535 * 4;
  return (unsigned)(g < 1 ? 1 : g);
}

// The lean kernels run with R = 1 right-hand side per pass for a single
// right-hand side, else with R = 16.
template <typename T>
void launch_ap_rotate(const ApplyArgs<T>& A, int32_t nsteps, double* y, int dir, int bmax, hipStream_t stream) {
  if (nsteps <= 0) return;
  if (A.nrhs == 1)
    hipLaunchKernelGGL((k_ap_rot2<T, 1>), dim3(nsteps), dim3(NT), (size_t)bmax * RhsPass<1>::P * sizeof(double), stream,
                       A, y, dir);
  else
    hipLaunchKernelGGL((k_ap_rot2<T, RC>), dim3(nsteps), dim3(NT), (size_t)bmax * RCP * sizeof(double), stream, A, y,
                       dir);
}
// Waves with fewer steps than split_steps run their close-block updates as
// one workgroup per (step, view) (k_ap_fview / k_ap_bpart).
template <typename T>
bool ap_split(const WaveRange& w, int bmax, int32_t split_steps) {
  const size_t lds = (size_t)2 * bmax * RCP * sizeof(double) + sizeof(ViewDesc);
  return w.s1 - w.s0 < split_steps && w.maxclose > 0 && lds <= max_lds_bytes();
}

size_t ap_part_elems(const WaveRange& w, int bmax, int nrhs) {
  return (size_t)(w.s1 - w.s0) * w.maxclose * bmax * nrhs;
}

template <typename T>
void launch_ap_fwd(const ApplyArgs<T>& A, const WaveRange& w, double* y, int bmax, int32_t split_steps,
                   hipStream_t stream) {
  const int32_t s0 = w.s0, s1 = w.s1;
  if (s1 <= s0) return;
  const size_t lds = (size_t)2 * bmax * RCP * sizeof(double) + sizeof(ViewDesc);
  if (lds <= max_lds_bytes()) {
    const bool split = ap_split<T>(w, bmax, split_steps);
    if (A.nrhs == 1) {
      const size_t l1 = (size_t)2 * bmax * RhsPass<1>::P * sizeof(double) + sizeof(ViewDesc);
      hipLaunchKernelGGL((k_ap_fwd2<T, 1>), dim3(s1 - s0), dim3(NT), l1, stream, A, s0, y, bmax, split ? 0 : 1);
      if (split)
        hipLaunchKernelGGL((k_ap_fview<T, 1>), dim3(s1 - s0, w.maxclose), dim3(NT),
                           (size_t)bmax * RhsPass<1>::P * sizeof(double), stream, A, s0, y, bmax);
    } else {
      hipLaunchKernelGGL((k_ap_fwd2<T, RC>), dim3(s1 - s0), dim3(NT), lds, stream, A, s0, y, bmax, split ? 0 : 1);
      if (split)
        hipLaunchKernelGGL((k_ap_fview<T, RC>), dim3(s1 - s0, w.maxclose), dim3(NT), (size_t)bmax * RCP * sizeof(double),
                           stream, A, s0, y, bmax);
    }
  } else {
    hipLaunchKernelGGL(k_ap_fwd_generic<T>, dim3(s1 - s0), dim3(NT), (size_t)bmax * RC * sizeof(double), stream, A,
                       s0, y);
  }
}
template <typename T>
void launch_ap_bwd(const ApplyArgs<T>& A, const WaveRange& w, double* y, int bmax, double* part,
                   int32_t split_steps, hipStream_t stream) {
  const int32_t s0 = w.s0, s1 = w.s1;
  if (s1 <= s0) return;
  const size_t lds = (size_t)(bmax + 64) * RCP * sizeof(double) + sizeof(ViewDesc);
  if (lds <= max_lds_bytes()) {
    const bool split = part != nullptr && ap_split<T>(w, bmax, split_steps);
    if (A.nrhs == 1) {
      const size_t l1 = (size_t)(bmax + 64) * RhsPass<1>::P * sizeof(double);
      if (split)
        hipLaunchKernelGGL((k_ap_bpart<T, 1>), dim3(s1 - s0, w.maxclose), dim3(NT), l1, stream, A, s0,
                           (const double*)y, part, bmax, (int)w.maxclose);
      hipLaunchKernelGGL((k_ap_bwd2<T, 1>), dim3(s1 - s0), dim3(NT), l1 + sizeof(ViewDesc), stream, A, s0, y, bmax,
                         split ? (const double*)part : (const double*)nullptr, (int)w.maxclose);
    } else {
      if (split)
        hipLaunchKernelGGL((k_ap_bpart<T, RC>), dim3(s1 - s0, w.maxclose), dim3(NT),
                           (size_t)(bmax + 64) * RCP * sizeof(double), stream, A, s0, (const double*)y, part, bmax,
                           (int)w.maxclose);
      hipLaunchKernelGGL((k_ap_bwd2<T, RC>), dim3(s1 - s0), dim3(NT), lds, stream, A, s0, y, bmax,
                         split ? (const double*)part : (const double*)nullptr, (int)w.maxclose);
    }
  } else {
    hipLaunchKernelGGL(k_ap_bwd_generic<T>, dim3(s1 - s0), dim3(NT), (size_t)bmax * RC * sizeof(double), stream, A,
                       s0, y);
  }
}
template <typename T>
void launch_mul_w(const ApplyArgs<T>& A, int32_t nsteps, const double* z, double* w, int bmax, hipStream_t stream) {
  if (nsteps <= 0) return;
  hipLaunchKernelGGL(k_mul_w<T>, dim3(nsteps), dim3(NT), 0, stream, A, z, w);
}
template <typename T>
void launch_mul_lw(const ApplyArgs<T>& A, int32_t s0, int32_t s1, const double* w, double* out, int bmax,
                   hipStream_t stream) {
  if (s1 <= s0) return;
  hipLaunchKernelGGL(k_mul_lw<T>, dim3(s1 - s0), dim3(NT), 0, stream, A, s0, w, out);
}

void launch_to_next(int32_t M, const int64_t* dof_off, const int32_t* rank, const int32_t* parent,
                    const int32_t* off_in_parent, const int64_t* dof_off_next, int32_t nrhs, const double* y,
                    double* ynext, int dir, hipStream_t stream) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_to_next, dim3(M), dim3(64), 0, stream, dof_off, rank, parent, off_in_parent, dof_off_next,
                     nrhs, const_cast<double*>(y), ynext, dir);
}

void launch_coarse_apply(const double* Aneg_inv, int64_t dim, int32_t nrhs, const double* y, double* out,
                         hipStream_t stream) {
  if (dim <= 0) return;
  hipLaunchKernelGGL(k_dense_mv, dim3((unsigned)((dim + MV_ROWS - 1) / MV_ROWS)), dim3(NT), 0, stream, Aneg_inv, dim, nrhs, y,
                     out, -1.0);
}
void launch_coarse_mul(const double* Ad, int64_t dim, int32_t nrhs, const double* y, double* out,
                       hipStream_t stream) {
  if (dim <= 0) return;
  hipLaunchKernelGGL(k_dense_mv, dim3((unsigned)((dim + MV_ROWS - 1) / MV_ROWS)), dim3(NT), 0, stream, Ad, dim, nrhs, y, out,
                     1.0);
}

void launch_perm_in(int64_t n, int32_t nrhs, const int32_t* perm, const double* x, int64_t ldx, double* y,
                    hipStream_t stream) {
  hipLaunchKernelGGL(k_perm_in, dim3(grid1(n * nrhs)), dim3(NT), 0, stream, n, nrhs, perm, x, ldx, y);
}
void launch_perm_out(int64_t n, int32_t nrhs, const int32_t* perm, const double* y, double* x, int64_t ldx,
                     hipStream_t stream) {
  hipLaunchKernelGGL(k_perm_out, dim3(grid1(n * nrhs)), dim3(NT), 0, stream, n, nrhs, perm, y, x, ldx);
}

void launch_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals, int32_t nrhs,
                 const double* x, int64_t ldx, double* y, int64_t ldy, hipStream_t stream) {
  hipLaunchKernelGGL(k_spmv, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, stream, n, row_ptr, col_idx, vals,
                     nrhs, x, ldx, y, ldy);
}

void launch_dots(int64_t n, int32_t nrhs, const double* a, int64_t lda, const double* b, int64_t ldb,
                 double* partial, double* out, hipStream_t stream) {
  int64_t nb = (n + NT - 1) / NT;
  if (nb > DOT_BLOCKS) nb = DOT_BLOCKS;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_dot_part, dim3((unsigned)nb, nrhs), dim3(NT), 0, stream, n, a, lda, b, ldb, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(nrhs), dim3(NT), 0, stream, (const double*)partial, (int)nb, out);
}

void launch_pcg_xr(int64_t n, int32_t nrhs, const double* rz, const double* pq, const int32_t* active,
                   double* x, int64_t ldx, const double* p, double* r, const double* q, hipStream_t stream) {
  hipLaunchKernelGGL(k_pcg_xr, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, nrhs, rz, pq, active,
                     x, ldx, p, r, q);
}

void launch_pcg_p(int64_t n, int32_t nrhs, double* rz, const double* rz_new, const int32_t* active,
                  const double* z, double* p, double* beta, hipStream_t stream) {
  hipLaunchKernelGGL(k_pcg_beta, dim3((unsigned)((nrhs + NT - 1) / NT)), dim3(NT), 0, stream, nrhs, rz, rz_new, active,
                     beta);
  hipLaunchKernelGGL(k_pcg_p, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, active,
                     (const double*)beta, z, p);
}

void launch_seg_dots(const SegTiles& sg, int32_t nrhs, const double* a, int64_t lda, const double* b, int64_t ldb,
                     double* partial, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_seg_dot_part, dim3((unsigned)sg.ntiles, nrhs), dim3(NT), 0, stream, sg, a, lda, b, ldb, partial);
  hipLaunchKernelGGL(k_seg_dot_final, dim3((unsigned)sg.nseg, nrhs), dim3(NT), 0, stream, sg, (const double*)partial,
                     out);
}

void launch_seg_pcg_xr(const SegTiles& sg, int64_t n, int32_t nrhs, const double* rz, const double* pq,
                       const int32_t* active, double* x, int64_t ldx, const double* p, double* r, const double* q,
                       hipStream_t stream) {
  hipLaunchKernelGGL(k_seg_pcg_xr, dim3((unsigned)sg.ntiles, nrhs), dim3(NT), 0, stream, sg, n, rz, pq, active, x, ldx,
                     p, r, q);
}

void launch_seg_pcg_p(const SegTiles& sg, int64_t n, int32_t nrhs, double* rz, const double* rz_new,
                      const int32_t* active, const double* z, double* p, double* beta, hipStream_t stream) {
  const int32_t L = nrhs * sg.nseg;
  hipLaunchKernelGGL(k_pcg_beta, dim3((unsigned)((L + NT - 1) / NT)), dim3(NT), 0, stream, L, rz, rz_new, active, beta);
  hipLaunchKernelGGL(k_seg_pcg_p, dim3((unsigned)sg.ntiles, nrhs), dim3(NT), 0, stream, sg, n, active,
                     (const double*)beta, z, p);
}

void launch_mr_v(int64_t n, int32_t nrhs, const int32_t* active, const double* st, const double* y, double* v,
                 hipStream_t stream) {
  hipLaunchKernelGGL(k_mr_v, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, active, st, nrhs, y, v);
}
void launch_mr_y(int64_t n, int32_t nrhs, const int32_t* active, const double* st, const double* r, double* y,
                 int which, hipStream_t stream) {
  hipLaunchKernelGGL(k_mr_y, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, active, st, nrhs, r, y,
                     which);
}
void launch_mr_scalars(int32_t nrhs, const int32_t* active, double* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_mr_scalars, dim3(1), dim3(NT), 0, stream, nrhs, active, st);
}
void launch_mr_wx(int64_t n, int32_t nrhs, const int32_t* active, const double* st, const double* v,
                  const double* wprev2, const double* wprev, double* wout, double* x, int64_t ldx,
                  hipStream_t stream) {
  hipLaunchKernelGGL(k_mr_wx, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, active, st, nrhs, v,
                     wprev2, wprev, wout, x, ldx);
}

void launch_copy_cols(int64_t n, int32_t nrhs, const double* a, int64_t lda, double* b, int64_t ldb,
                      hipStream_t stream) {
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, a, lda, b, ldb);
}

void launch_fill(double* a, int64_t count, double v, hipStream_t stream) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid1(count)), dim3(NT), 0, stream, a, count, v);
}

void launch_residual(int64_t n, int32_t nrhs, const double* b, int64_t ldb, double* r, hipStream_t stream) {
  hipLaunchKernelGGL(k_residual, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, b, ldb, r);
}

#define CAE_APPLY_INST(T)                                                                                        \
  template void launch_ap_rotate<T>(const ApplyArgs<T>&, int32_t, double*, int, int, hipStream_t);               \
  template void launch_ap_fwd<T>(const ApplyArgs<T>&, const WaveRange&, double*, int, int32_t, hipStream_t);   \
  template void launch_ap_bwd<T>(const ApplyArgs<T>&, const WaveRange&, double*, int, double*, int32_t,       \
                                 hipStream_t);                                                               \
  template bool ap_split<T>(const WaveRange&, int, int32_t);                                                   \
  template void launch_mul_w<T>(const ApplyArgs<T>&, int32_t, const double*, double*, int, hipStream_t);         \
  template void launch_mul_lw<T>(const ApplyArgs<T>&, int32_t, int32_t, const double*, double*, int, hipStream_t);
CAE_APPLY_INST(double)
CAE_APPLY_INST(float)

}  // namespace cae
