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

namespace {
size_t g_max_lds = 64 * 1024;
}
size_t max_lds_bytes() { return g_max_lds; }
void set_max_lds_bytes(size_t b) { g_max_lds = b; }

template <typename T>
__device__ inline double vget(const T* base, int trans, int bi, int bx, int a, int c) {
  return (double)(trans ? base[(int64_t)c * bi + a] : base[(int64_t)a * bx + c]);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_ap_rotate(ApplyArgs<T> A, double* y, int dir) {
  const Step st = A.steps[blockIdx.x];
  if (st.nfar == 0) return;                 // U_i = I
  const int i = st.blk;
  const int b = A.bsz[i];
  if (b == 0) return;
  const int nrhs = A.nrhs;
  const T* U = A.U + A.u_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Ys = reinterpret_cast<double*>(smem_raw);   // b x RC
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < b * kc; e += NT) Ys[(e / kc) * RC + e % kc] = yi[(e / kc) * nrhs + k0 + e % kc];
    __syncthreads();
    for (int e = threadIdx.x; e < b * kc; e += NT) {
      const int a = e / kc, k = e % kc;
      double s = 0;
      if (dir == 0)
        for (int l = 0; l < b; ++l) s += (double)U[(int64_t)l * b + a] * Ys[l * RC + k];
      else
        for (int l = 0; l < b; ++l) s += (double)U[(int64_t)a * b + l] * Ys[l * RC + k];
      yi[a * nrhs + k0 + k] = s;
    }
  }
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
// Block solves with the stored inverse L_nn^{-1} (computed at factorization):
// every step is a few small matrix products staged in LDS, with no sequential
// dependency inside the step.  Operand tiles are loaded with consecutive
// threads on consecutive addresses of the slot that holds them.
// ---------------------------------------------------------------------------
constexpr int PT = 64;          // panel column tile

struct ApLds {
  int ldl, ldp;
  size_t off_l, off_p, off_y, off_t, off_z, total;
};

template <typename T>
__host__ __device__ inline ApLds ap_layout(int bmax) {
  ApLds L;
  L.ldl = bmax + 1;
  L.ldp = PT + 1;
  size_t o = 0;
  L.off_l = o;
  o += (size_t)bmax * L.ldl * sizeof(T);
  o = (o + 15) & ~(size_t)15;
  L.off_p = o;
  o += (size_t)bmax * L.ldp * sizeof(T);
  o = (o + 15) & ~(size_t)15;
  L.off_y = o;
  o += (size_t)bmax * (RC + 1) * sizeof(double);
  L.off_t = o;
  o += (size_t)bmax * (RC + 1) * sizeof(double);
  L.off_z = o;
  o += (size_t)PT * (RC + 1) * sizeof(double);
  L.total = o;
  return L;
}

// Stage rows n (r..b-1) and columns [g0, g0+tc) of a panel view into Ps[t][g].
template <typename T>
__device__ inline void stage_panel(T* Ps, int ldp, const T* P, int trans, int b, int bx, int r, int n, int g0,
                                   int tc) {
  if (!trans) {
    for (int e = threadIdx.x; e < n * tc; e += NT) {
      const int t = e / tc, g = e % tc;
      Ps[t * ldp + g] = P[(int64_t)(r + t) * bx + g0 + g];
    }
  } else {   // slot rows are the panel columns: read along them
    for (int e = threadIdx.x; e < n * tc; e += NT) {
      const int g = e / n, t = e % n;
      Ps[t * ldp + g] = P[(int64_t)(g0 + g) * b + r + t];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_ap_fwd(ApplyArgs<T> A, int32_t s0, double* y, int bmax) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  const ApLds Lay = ap_layout<T>(bmax);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Ls = reinterpret_cast<T*>(smem_raw + Lay.off_l);
  T* Ps = reinterpret_cast<T*>(smem_raw + Lay.off_p);
  double* yn = reinterpret_cast<double*>(smem_raw + Lay.off_y);
  double* tn = reinterpret_cast<double*>(smem_raw + Lay.off_t);
  const int ldl = Lay.ldl, ldp = Lay.ldp, ldv = RC + 1;
  const T* Lig = A.Li + A.u_off[i];
  const T* D = A.arena + A.slot_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  for (int e = threadIdx.x; e < n * n; e += NT) Ls[(e / n) * ldl + e % n] = Lig[e];
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < n * kc; e += NT) yn[(e / kc) * ldv + e % kc] = yi[(r + e / kc) * nrhs + k0 + e % kc];
    __syncthreads();
    for (int e = threadIdx.x; e < n * kc; e += NT) {
      const int row = e / kc, k = e % kc;
      double s = 0;
      for (int c = 0; c <= row; ++c) s += (double)Ls[row * ldl + c] * yn[c * ldv + k];
      tn[row * ldv + k] = s;
      yi[(r + row) * nrhs + k0 + k] = s;
    }
    // panels: v = -1 is the basis of i (columns 0..r-1 of rows n of the diagonal block)
    for (int v = -1; v < st.nclose; ++v) {
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
        const View vw = A.views[st.view0 + v];
        bx = A.bsz[vw.x];
        lc = vw.proc ? A.rank[vw.x] : bx;
        P = A.arena + A.slot_off[vw.slot];
        trans = vw.trans;
        yx = y + A.dof_off[vw.x] * nrhs;
      }
      for (int g0 = 0; g0 < lc; g0 += PT) {
        const int tc = min(PT, lc - g0);
        __syncthreads();
        stage_panel(Ps, ldp, P, trans, b, bx, r, n, g0, tc);
        __syncthreads();
        for (int e = threadIdx.x; e < tc * kc; e += NT) {
          const int g = e / kc, k = e % kc;
          double s = 0;
          for (int t = 0; t < n; ++t) s += (double)Ps[t * ldp + g] * tn[t * ldv + k];
          yx[(g0 + g) * nrhs + k0 + k] -= s;
        }
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_ap_bwd(ApplyArgs<T> A, int32_t s0, double* y, int bmax) {
  const Step st = A.steps[s0 + blockIdx.x];
  const int i = st.blk;
  const int b = A.bsz[i];
  const int r = A.rank[i];
  const int n = b - r;
  if (n <= 0) return;
  const int nrhs = A.nrhs;
  const ApLds Lay = ap_layout<T>(bmax);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Ls = reinterpret_cast<T*>(smem_raw + Lay.off_l);
  T* Ps = reinterpret_cast<T*>(smem_raw + Lay.off_p);
  double* tn = reinterpret_cast<double*>(smem_raw + Lay.off_t);
  double* zt = reinterpret_cast<double*>(smem_raw + Lay.off_z);
  const int ldl = Lay.ldl, ldp = Lay.ldp, ldv = RC + 1;
  const T* Lig = A.Li + A.u_off[i];
  const T* D = A.arena + A.slot_off[i];
  double* yi = y + A.dof_off[i] * nrhs;
  for (int e = threadIdx.x; e < n * n; e += NT) Ls[(e / n) * ldl + e % n] = Lig[e];
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < n * kc; e += NT) tn[(e / kc) * ldv + e % kc] = yi[(r + e / kc) * nrhs + k0 + e % kc];
    for (int v = -1; v < st.nclose; ++v) {
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
        const View vw = A.views[st.view0 + v];
        bx = A.bsz[vw.x];
        lc = vw.proc ? A.rank[vw.x] : bx;
        P = A.arena + A.slot_off[vw.slot];
        trans = vw.trans;
        zx = y + A.dof_off[vw.x] * nrhs;
      }
      for (int g0 = 0; g0 < lc; g0 += PT) {
        const int tc = min(PT, lc - g0);
        __syncthreads();
        stage_panel(Ps, ldp, P, trans, b, bx, r, n, g0, tc);
        for (int e = threadIdx.x; e < tc * kc; e += NT) zt[(e / kc) * ldv + e % kc] = zx[(g0 + e / kc) * nrhs + k0 + e % kc];
        __syncthreads();
        for (int e = threadIdx.x; e < n * kc; e += NT) {
          const int t = e / kc, k = e % kc;
          double s = 0;
          for (int g = 0; g < tc; ++g) s += (double)Ps[t * ldp + g] * zt[g * ldv + k];
          tn[t * ldv + k] -= s;
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * kc; e += NT) {
      const int c = e / kc, k = e % kc;
      double s = 0;
      for (int row = c; row < n; ++row) s += (double)Ls[row * ldl + c] * tn[row * ldv + k];
      yi[(r + c) * nrhs + k0 + k] = s;
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

// out = sign * A y, A dense row-major dim x dim, y/out dim x nrhs.
constexpr int MV = 64;
__global__ __launch_bounds__(NT) void k_dense_mv(const double* A, int64_t dim, int32_t nrhs, const double* y,
                                                 double* out, double sign) {
  __shared__ double As[MV][MV + 1];
  __shared__ double Ys[MV][RC + 1];
  const int64_t i0 = (int64_t)blockIdx.x * MV;
  const int ti = (int)min<int64_t>(MV, dim - i0);
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int kc = min(RC, nrhs - k0);
    double acc[4] = {0, 0, 0, 0};   // outputs e = threadIdx.x + q*NT, q < 4 (64 x 16 tile)
    for (int64_t j0 = 0; j0 < dim; j0 += MV) {
      const int tj = (int)min<int64_t>(MV, dim - j0);
      __syncthreads();
      for (int e = threadIdx.x; e < ti * tj; e += NT) As[e / tj][e % tj] = A[(i0 + e / tj) * dim + j0 + e % tj];
      for (int e = threadIdx.x; e < tj * kc; e += NT) Ys[e / kc][e % kc] = y[(j0 + e / kc) * nrhs + k0 + e % kc];
      __syncthreads();
      for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < ti * kc) {
          const int a = e / kc, c = e % kc;
          double s = 0;
          for (int j = 0; j < tj; ++j) s += As[a][j] * Ys[j][c];
          acc[q] += s;
        }
      }
    }
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < ti * kc) out[(i0 + e / kc) * nrhs + k0 + e % kc] = sign * acc[q];
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
__global__ void k_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                       const double* x, int64_t ldx, double* y, int64_t ldy) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n) return;
  const double* xk = x + k * ldx;
  double s = 0;
  for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += vals[e] * xk[col_idx[e]];
  y[i + k * ldy] = s;
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
  const int k = threadIdx.x;
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

template <typename T>
void launch_ap_rotate(const ApplyArgs<T>& A, int32_t nsteps, double* y, int dir, int bmax, hipStream_t stream) {
  if (nsteps <= 0) return;
  hipLaunchKernelGGL(k_ap_rotate<T>, dim3(nsteps), dim3(NT), (size_t)bmax * RC * sizeof(double), stream, A, y, dir);
}
template <typename T>
void launch_ap_fwd(const ApplyArgs<T>& A, int32_t s0, int32_t s1, double* y, int bmax, hipStream_t stream) {
  if (s1 <= s0) return;
  const size_t lds = ap_layout<T>(bmax).total;
  if (lds <= max_lds_bytes())
    hipLaunchKernelGGL(k_ap_fwd<T>, dim3(s1 - s0), dim3(NT), lds, stream, A, s0, y, bmax);
  else
    hipLaunchKernelGGL(k_ap_fwd_generic<T>, dim3(s1 - s0), dim3(NT), (size_t)bmax * RC * sizeof(double), stream, A,
                       s0, y);
}
template <typename T>
void launch_ap_bwd(const ApplyArgs<T>& A, int32_t s0, int32_t s1, double* y, int bmax, hipStream_t stream) {
  if (s1 <= s0) return;
  const size_t lds = ap_layout<T>(bmax).total;
  if (lds <= max_lds_bytes())
    hipLaunchKernelGGL(k_ap_bwd<T>, dim3(s1 - s0), dim3(NT), lds, stream, A, s0, y, bmax);
  else
    hipLaunchKernelGGL(k_ap_bwd_generic<T>, dim3(s1 - s0), dim3(NT), (size_t)bmax * RC * sizeof(double), stream, A,
                       s0, y);
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
  hipLaunchKernelGGL(k_dense_mv, dim3((unsigned)((dim + MV - 1) / MV)), dim3(NT), 0, stream, Aneg_inv, dim, nrhs, y,
                     out, -1.0);
}
void launch_coarse_mul(const double* Ad, int64_t dim, int32_t nrhs, const double* y, double* out,
                       hipStream_t stream) {
  if (dim <= 0) return;
  hipLaunchKernelGGL(k_dense_mv, dim3((unsigned)((dim + MV - 1) / MV)), dim3(NT), 0, stream, Ad, dim, nrhs, y, out,
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
  hipLaunchKernelGGL(k_spmv, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, row_ptr, col_idx,
                     vals, x, ldx, y, ldy);
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
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(NT), 0, stream, nrhs, rz, rz_new, active, beta);
  hipLaunchKernelGGL(k_pcg_p, dim3((unsigned)((n + NT - 1) / NT), nrhs), dim3(NT), 0, stream, n, active,
                     (const double*)beta, z, p);
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
  template void launch_ap_fwd<T>(const ApplyArgs<T>&, int32_t, int32_t, double*, int, hipStream_t);              \
  template void launch_ap_bwd<T>(const ApplyArgs<T>&, int32_t, int32_t, double*, int, hipStream_t);              \
  template void launch_mul_w<T>(const ApplyArgs<T>&, int32_t, const double*, double*, int, hipStream_t);         \
  template void launch_mul_lw<T>(const ApplyArgs<T>&, int32_t, int32_t, const double*, double*, int, hipStream_t);
CAE_APPLY_INST(double)
CAE_APPLY_INST(float)

}  // namespace cae
