// HIP kernels (gfx950) of the rank-predicting MLP 16 -> 64 -> 64 -> 1 (ReLU)
// used by the learned-rank compression: feature statistics, forward pass,
// mean-squared-error gradient (one workgroup per 64 records, FP32, partial
// sums added into the gradient with atomics) and the Adam update.
//
// Records are REC_W floats: 16 features, then the label r/b (negative labels
// mark rows that are not training samples).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace cae {

namespace {
constexpr int MT = 256;
constexpr int SB = 64;          // records per workgroup in the gradient
constexpr int HL = MLP_H + 1;   // LDS row stride of the 64 x 64 layers
}

// mean and standard deviation of every feature over the rows with a label >= 0
__global__ __launch_bounds__(MT) void k_mlp_stats(const float* rec, int64_t n, float* P, int* nvalid) {
  __shared__ double s1[MT], s2[MT];
  __shared__ int cnt[MT];
  for (int f = 0; f < NFEAT; ++f) {
    double a = 0.0, q = 0.0;
    int c = 0;
    for (int64_t r = threadIdx.x; r < n; r += MT) {
      if (rec[r * REC_W + NFEAT] < 0.0f) continue;
      const double x = rec[r * REC_W + f];
      a += x;
      q += x * x;
      ++c;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = q;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int o = MT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        s1[threadIdx.x] += s1[threadIdx.x + o];
        s2[threadIdx.x] += s2[threadIdx.x + o];
        cnt[threadIdx.x] += cnt[threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int m = cnt[0];
      const double mu = m > 0 ? s1[0] / m : 0.0;
      const double var = m > 0 ? s2[0] / m - mu * mu : 0.0;
      P[MLP_OFF_MEAN + f] = (float)mu;
      P[MLP_OFF_STD + f] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
      if (f == 0) *nvalid = m;
    }
    __syncthreads();
  }
}

// z for every record, FP64 arithmetic on the FP32 parameters (the same
// evaluation as inside the compression kernel)
__global__ __launch_bounds__(MT) void k_mlp_predict(const float* P, const float* rec, int64_t n, float* z) {
  const int64_t r = blockIdx.x * (int64_t)MT + threadIdx.x;
  if (r >= n) return;
  double xn[NFEAT];
  for (int k = 0; k < NFEAT; ++k)
    xn[k] = ((double)rec[r * REC_W + k] - (double)P[MLP_OFF_MEAN + k]) / (double)P[MLP_OFF_STD + k];
  double h1[MLP_H];
  for (int j = 0; j < MLP_H; ++j) {
    double h = P[MLP_OFF_B1 + j];
    for (int k = 0; k < NFEAT; ++k) h += (double)P[MLP_OFF_W1 + j * NFEAT + k] * xn[k];
    h1[j] = h > 0.0 ? h : 0.0;
  }
  double out = P[MLP_OFF_B3];
  for (int j = 0; j < MLP_H; ++j) {
    double h = P[MLP_OFF_B2 + j];
    for (int k = 0; k < MLP_H; ++k) h += (double)P[MLP_OFF_W2 + j * MLP_H + k] * h1[k];
    out += (double)P[MLP_OFF_W3 + j] * (h > 0.0 ? h : 0.0);
  }
  z[r] = (float)out;
}

// loss = 0.5 / nvalid * sum (z - y)^2 over the valid records and its gradient
// (added into grad, loss_acc[0])
__global__ __launch_bounds__(MT) void k_mlp_grad(const float* P, const float* rec, int64_t n, float inv_n,
                                                 float* grad, float* loss_acc) {
  __shared__ float W1[MLP_H * NFEAT], W2[MLP_H * HL], b1[MLP_H], b2[MLP_H], w3[MLP_H], mu[NFEAT], sd[NFEAT];
  __shared__ float Xn[SB * (NFEAT + 1)], A1[SB * HL], A2[SB * HL], D[SB * HL], ys[SB], dz[SB];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * SB;
  for (int e = tid; e < MLP_H * NFEAT; e += MT) W1[e] = P[MLP_OFF_W1 + e];
  for (int e = tid; e < MLP_H * MLP_H; e += MT) W2[(e / MLP_H) * HL + e % MLP_H] = P[MLP_OFF_W2 + e];
  if (tid < MLP_H) {
    b1[tid] = P[MLP_OFF_B1 + tid];
    b2[tid] = P[MLP_OFF_B2 + tid];
    w3[tid] = P[MLP_OFF_W3 + tid];
  }
  if (tid < NFEAT) {
    mu[tid] = P[MLP_OFF_MEAN + tid];
    sd[tid] = P[MLP_OFF_STD + tid];
  }
  __syncthreads();
  for (int e = tid; e < SB * NFEAT; e += MT) {
    const int s = e / NFEAT, f = e % NFEAT;
    const int64_t r = r0 + s;
    Xn[s * (NFEAT + 1) + f] = r < n ? (rec[r * REC_W + f] - mu[f]) / sd[f] : 0.0f;
  }
  if (tid < SB) {
    const int64_t r = r0 + tid;
    ys[tid] = r < n ? rec[r * REC_W + NFEAT] : -1.0f;
  }
  __syncthreads();
  // forward: A1 = Xn W1^T + b1, A2 = relu(A1) W2^T + b2
  for (int e = tid; e < SB * MLP_H; e += MT) {
    const int s = e / MLP_H, j = e % MLP_H;
    float a = b1[j];
    for (int f = 0; f < NFEAT; ++f) a += W1[j * NFEAT + f] * Xn[s * (NFEAT + 1) + f];
    A1[s * HL + j] = a;
  }
  __syncthreads();
  for (int e = tid; e < SB * MLP_H; e += MT) {
    const int s = e / MLP_H, j = e % MLP_H;
    float a = b2[j];
    for (int k = 0; k < MLP_H; ++k) a += W2[j * HL + k] * fmaxf(A1[s * HL + k], 0.0f);
    A2[s * HL + j] = a;
  }
  __syncthreads();
  if (tid < SB) {
    float z = P[MLP_OFF_B3];
    for (int j = 0; j < MLP_H; ++j) z += w3[j] * fmaxf(A2[tid * HL + j], 0.0f);
    const bool ok = ys[tid] >= 0.0f;
    const float d = ok ? (z - ys[tid]) * inv_n : 0.0f;
    dz[tid] = d;
    if (ok) atomicAdd(loss_acc, 0.5f * (z - ys[tid]) * (z - ys[tid]) * inv_n);
  }
  __syncthreads();
  // output layer
  if (tid < MLP_H) {
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += fmaxf(A2[s * HL + tid], 0.0f) * dz[s];
    atomicAdd(grad + MLP_OFF_W3 + tid, g);
  } else if (tid == MLP_H) {
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += dz[s];
    atomicAdd(grad + MLP_OFF_B3, g);
  }
  // D = dA2
  for (int e = tid; e < SB * MLP_H; e += MT) {
    const int s = e / MLP_H, j = e % MLP_H;
    D[s * HL + j] = A2[s * HL + j] > 0.0f ? dz[s] * w3[j] : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < MLP_H * MLP_H; e += MT) {
    const int j = e / MLP_H, k = e % MLP_H;
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += D[s * HL + j] * fmaxf(A1[s * HL + k], 0.0f);
    atomicAdd(grad + MLP_OFF_W2 + e, g);
  }
  if (tid < MLP_H) {
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += D[s * HL + tid];
    atomicAdd(grad + MLP_OFF_B2 + tid, g);
  }
  // dA1 = (dA2 W2) * (A1 > 0), into A2's storage (A2 no longer needed)
  for (int e = tid; e < SB * MLP_H; e += MT) {
    const int s = e / MLP_H, k = e % MLP_H;
    float g = 0.0f;
    for (int j = 0; j < MLP_H; ++j) g += D[s * HL + j] * W2[j * HL + k];
    A2[s * HL + k] = A1[s * HL + k] > 0.0f ? g : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < MLP_H * NFEAT; e += MT) {
    const int k = e / NFEAT, f = e % NFEAT;
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += A2[s * HL + k] * Xn[s * (NFEAT + 1) + f];
    atomicAdd(grad + MLP_OFF_W1 + e, g);
  }
  if (tid < MLP_H) {
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += A2[s * HL + tid];
    atomicAdd(grad + MLP_OFF_B1 + tid, g);
  }
}

// Adam (Kingma and Ba) on the trainable entries (the normalisation is fixed)
__global__ void k_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, int step) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x + MLP_OFF_W1;
  if (e >= MLP_NPARAM) return;
  const float g = grad[e];
  const float mm = beta1 * m[e] + (1.0f - beta1) * g;
  const float vv = beta2 * v[e] + (1.0f - beta2) * g * g;
  m[e] = mm;
  v[e] = vv;
  const float mh = mm / (1.0f - powf(beta1, (float)step));
  const float vh = vv / (1.0f - powf(beta2, (float)step));
  P[e] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_mlp_zero(float* a, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] = 0.0f;
}

void launch_mlp_stats(const float* rec, int64_t n, float* P, int* nvalid, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_stats, dim3(1), dim3(MT), 0, s, rec, n, P, nvalid);
}
void launch_mlp_predict(const float* P, const float* rec, int64_t n, float* z, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)((n + MT - 1) / MT)), dim3(MT), 0, s, P, rec, n, z);
}
void launch_mlp_grad(const float* P, const float* rec, int64_t n, float inv_n, float* grad, float* loss,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_zero, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, grad, MLP_NPARAM);
  hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(64), 0, s, loss, 1);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((n + SB - 1) / SB)), dim3(MT), 0, s, P, rec, n, inv_n, grad, loss);
}
void launch_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, int step, hipStream_t s) {
  const int nt = MLP_NPARAM - MLP_OFF_W1;
  hipLaunchKernelGGL(k_mlp_adam, dim3((nt + 255) / 256), dim3(256), 0, s, P, grad, m, v, lr, 0.9f, 0.999f, 1e-8f,
                     step);
}
void launch_mlp_zero(float* a, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_zero, dim3((n + 255) / 256), dim3(256), 0, s, a, n);
}

}  // namespace cae
