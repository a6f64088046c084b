// Learned schedule cost model: a two-layer perceptron
//   h = relu(W1 x + b1)  (H hidden units),  y = w2 . h + b2
// predicting the log10 run time of a schedule on a graph (centred per
// pattern/graph group).  Training runs here in FP32 (forward, MSE loss,
// backward, Adam); inference runs with BF16 weights and inputs and FP32
// accumulation.  Parameters live in one FP32 device buffer laid out as
// [W1 (H x D, row-major), b1 (H), w2 (H), b2 (1)].
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "gz_internal.h"

namespace gz {
namespace mlp {

constexpr int TB = 256;

__device__ __forceinline__ float bf16_round(float x) {
  return __bfloat162float(__float2bfloat16(x));
}

// hpre[n][h] = sum_d W1[h][d] x[n][d] + b1[h]; one thread per (n, h)
template <bool BF16>
__global__ __launch_bounds__(TB) void k_hidden(const float* __restrict__ P,
                                               const float* __restrict__ X, int n, int D, int H,
                                               float* __restrict__ hpre) {
  const long long idx = (long long)blockIdx.x * TB + threadIdx.x;
  if (idx >= (long long)n * H) return;
  const int s = (int)(idx / H), h = (int)(idx % H);
  const float* w = P + (size_t)h * D;
  const float* x = X + (size_t)s * D;
  float acc = 0.0f;
  for (int d = 0; d < D; ++d) {
    const float wd = BF16 ? bf16_round(w[d]) : w[d];
    const float xd = BF16 ? bf16_round(x[d]) : x[d];
    acc = fmaf(wd, xd, acc);
  }
  const float b = P[(size_t)H * D + h];
  hpre[idx] = acc + (BF16 ? bf16_round(b) : b);
}

// y[n] = sum_h w2[h] relu(hpre[n][h]) + b2; one wave per sample
template <bool BF16>
__global__ __launch_bounds__(TB) void k_output(const float* __restrict__ P,
                                               const float* __restrict__ hpre, int n, int D,
                                               int H, float* __restrict__ y) {
  const int wave = (int)((blockIdx.x * TB + threadIdx.x) / 64);
  const int lane = threadIdx.x % 64;
  if (wave >= n) return;
  const float* w2 = P + (size_t)H * D + H;
  float acc = 0.0f;
  for (int h = lane; h < H; h += 64) {
    float a = fmaxf(hpre[(size_t)wave * H + h], 0.0f);
    if (BF16) a = bf16_round(a);
    const float w = BF16 ? bf16_round(w2[h]) : w2[h];
    acc = fmaf(w, a, acc);
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    const float b2 = P[(size_t)H * D + 2 * H];
    y[wave] = acc + (BF16 ? bf16_round(b2) : b2);
  }
}

// dy[n] = 2 (y[n] - t[n]) / n; loss partials
__global__ __launch_bounds__(TB) void k_dloss(const float* __restrict__ y,
                                              const float* __restrict__ t, int n,
                                              float* __restrict__ dy, float* __restrict__ loss) {
  const int i = blockIdx.x * TB + threadIdx.x;
  float e = 0.0f;
  if (i < n) {
    const float r = y[i] - t[i];
    dy[i] = 2.0f * r / (float)n;
    e = r * r / (float)n;
  }
  for (int o = 32; o >= 1; o >>= 1) e += __shfl_xor(e, o, 64);
  if ((threadIdx.x % 64) == 0) atomicAdd(loss, e);
}

// Output layer gradients: gw2[h] = sum_n dy relu(hpre), gb2 = sum_n dy;
// one workgroup per hidden unit h (h == H: the output bias).
__global__ __launch_bounds__(TB) void k_grad_out(const float* __restrict__ hpre,
                                                 const float* __restrict__ dy, int n, int D,
                                                 int H, float* __restrict__ G) {
  __shared__ float part[TB / 64];
  const int h = blockIdx.x;
  float acc = 0.0f;
  for (int s = threadIdx.x; s < n; s += TB)
    acc += dy[s] * (h < H ? fmaxf(hpre[(size_t)s * H + h], 0.0f) : 1.0f);
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x % 64) == 0) part[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < TB / 64; ++w) t += part[w];
    G[(size_t)H * D + H + h] = t;  // w2[h], or b2 when h == H
  }
}

// Hidden layer gradients: dh[n][h] = dy[n] w2[h] [hpre > 0];
// gW1[h][d] = sum_n dh x[n][d] (d < D), gb1[h] = sum_n dh (d == D).
// One thread per (h, d).
__global__ __launch_bounds__(TB) void k_grad_hidden(const float* __restrict__ P,
                                                    const float* __restrict__ X,
                                                    const float* __restrict__ hpre,
                                                    const float* __restrict__ dy, int n, int D,
                                                    int H, float* __restrict__ G) {
  const long long idx = (long long)blockIdx.x * TB + threadIdx.x;
  if (idx >= (long long)H * (D + 1)) return;
  const int h = (int)(idx / (D + 1)), d = (int)(idx % (D + 1));
  const float w2h = P[(size_t)H * D + H + h];
  float acc = 0.0f;
  for (int s = 0; s < n; ++s) {
    if (hpre[(size_t)s * H + h] > 0.0f) acc += dy[s] * w2h * (d < D ? X[(size_t)s * D + d] : 1.0f);
  }
  if (d < D) G[(size_t)h * D + d] = acc;
  else G[(size_t)H * D + h] = acc;
}

__global__ __launch_bounds__(TB) void k_adam(float* __restrict__ P, const float* __restrict__ G,
                                             float* __restrict__ m, float* __restrict__ v,
                                             long long np, float lr, float b1, float b2,
                                             float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i >= np) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_zero_f32(float* p, long long n) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

inline unsigned nblk(long long n) { return (unsigned)((n + TB - 1) / TB); }

}  // namespace mlp

long long mlp_param_count(int D, int H) { return (long long)H * D + 2LL * H + 1; }

#define GZ_MLP_HIP(call)                                                  \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return GZ_EDEVICE;                                                  \
    }                                                                     \
  } while (0)

// Forward pass into y[n]; `hpre` is caller scratch of n*H floats.
gz_status mlp_forward(const float* P, const float* X, int n, int D, int H, bool bf16,
                      float* hpre, float* y, hipStream_t st) {
  if (n <= 0) return GZ_OK;
  if (bf16) {
    hipLaunchKernelGGL(mlp::k_hidden<true>, dim3(mlp::nblk((long long)n * H)), dim3(mlp::TB), 0,
                       st, P, X, n, D, H, hpre);
    hipLaunchKernelGGL(mlp::k_output<true>, dim3(mlp::nblk((long long)n * 64)), dim3(mlp::TB),
                       0, st, P, hpre, n, D, H, y);
  } else {
    hipLaunchKernelGGL(mlp::k_hidden<false>, dim3(mlp::nblk((long long)n * H)), dim3(mlp::TB),
                       0, st, P, X, n, D, H, hpre);
    hipLaunchKernelGGL(mlp::k_output<false>, dim3(mlp::nblk((long long)n * 64)), dim3(mlp::TB),
                       0, st, P, hpre, n, D, H, y);
  }
  GZ_MLP_HIP(hipGetLastError());
  return GZ_OK;
}

// Loss and full gradient G of the MSE of the FP32 forward pass.  Scratch:
// hpre (n*H), y (n), dy (n), loss (1 float).
gz_status mlp_loss_grad(const float* P, const float* X, const float* t, int n, int D, int H,
                        float* G, float* hpre, float* y, float* dy, float* loss,
                        hipStream_t st) {
  gz_status rc = mlp_forward(P, X, n, D, H, false, hpre, y, st);
  if (rc) return rc;
  hipLaunchKernelGGL(mlp::k_zero_f32, dim3(1), dim3(mlp::TB), 0, st, loss, 1LL);
  hipLaunchKernelGGL(mlp::k_dloss, dim3(mlp::nblk(n)), dim3(mlp::TB), 0, st, y, t, n, dy, loss);
  hipLaunchKernelGGL(mlp::k_grad_out, dim3(H + 1), dim3(mlp::TB), 0, st, hpre, dy, n, D, H, G);
  hipLaunchKernelGGL(mlp::k_grad_hidden, dim3(mlp::nblk((long long)H * (D + 1))), dim3(mlp::TB),
                     0, st, P, X, hpre, dy, n, D, H, G);
  GZ_MLP_HIP(hipGetLastError());
  return GZ_OK;
}

gz_status mlp_adam(float* P, const float* G, float* m, float* v, int D, int H, float lr,
                   float b1, float b2, float eps, int step, hipStream_t st) {
  const long long np = mlp_param_count(D, H);
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp::k_adam, dim3(mlp::nblk(np)), dim3(mlp::TB), 0, st, P, G, m, v, np, lr,
                     b1, b2, eps, c1, c2);
  GZ_MLP_HIP(hipGetLastError());
  return GZ_OK;
}

}  // namespace gz
