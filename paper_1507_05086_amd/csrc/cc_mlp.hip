// cc_mlp.hip -- inference and training kernels of the learned eps policy:
// a 6 -> 64 -> 1 float32 network y = w2 . relu(W1 x + b1) + b2 that replaces
// the fixed eps of Algorithm 2's batch-size rule round by round.
//
// The hidden layer is exactly one wavefront wide, so every kernel maps lane
// j to hidden unit j: lane j keeps W1[j][0..5], b1[j] and w2[j] in
// registers, a sample is broadcast to the wave, the output is one wave
// reduction.  Training minimises L = mean_i (y_i - t_i)^2:
//   k_mlp_grad   each wave walks a fixed strided subset of the samples and
//                accumulates dL/dp per lane; a workgroup folds its waves in
//                LDS and writes one partial row (deterministic order);
//   k_mlp_adam   one workgroup sums the partial rows in order and applies
//                an Adam step with bias correction.
#include <mutex>

#include "cc_device.h"
#include "cc_launch.h"

namespace ccd {

constexpr int MLP_IN = 6, MLP_H = 64;
constexpr int MLP_P = MLP_H * MLP_IN + MLP_H + MLP_H + 1;  // 513
constexpr int MLP_ROW = MLP_P + 1;                         // partial row: grads + sum of squared residuals
constexpr int MLP_BS = 256;
constexpr int MLP_MAX_BLOCKS = 1024;  // workgroups of k_mlp_grad, and partial rows
constexpr int kMaxDevices = 64;

struct Unit {
  float w[MLP_IN], b1, w2;
};

__device__ inline Unit load_unit(const float *p, int j) {
  Unit u;
#pragma unroll
  for (int k = 0; k < MLP_IN; k++) u.w[k] = p[j * MLP_IN + k];
  u.b1 = p[MLP_H * MLP_IN + j];
  u.w2 = p[MLP_H * MLP_IN + MLP_H + j];
  return u;
}

__device__ inline float wave_fsum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ void __launch_bounds__(MLP_BS) k_mlp_forward(const float *p, const float *x, int n, float *y) {
  const int j = lane_id();
  const Unit u = load_unit(p, j);
  const float b2 = p[MLP_P - 1];
  const int gw = blockIdx.x * (MLP_BS / 64) + wave_id(), nw = gridDim.x * (MLP_BS / 64);
  for (int s = gw; s < n; s += nw) {
    float z = u.b1;
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) z = fmaf(u.w[k], x[(size_t)s * MLP_IN + k], z);
    const float h = z > 0.f ? z : 0.f;
    const float out = wave_fsum(u.w2 * h) + b2;
    if (j == 0) y[s] = out;
  }
}

__global__ void __launch_bounds__(MLP_BS) k_mlp_grad(const float *p, const float *x, const float *t, int n,
                                                     float *partial) {
  __shared__ float red[MLP_BS / 64][MLP_H][MLP_IN + 2];
  __shared__ float red_s[MLP_BS / 64][2];
  const int j = lane_id(), wv = wave_id();
  const Unit u = load_unit(p, j);
  const float b2 = p[MLP_P - 1];
  const float inv_n = n > 0 ? 2.f / (float)n : 0.f;
  float gw1[MLP_IN] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gb1 = 0.f, gw2 = 0.f, gb2 = 0.f, sq = 0.f;
  const int gw = blockIdx.x * (MLP_BS / 64) + wv, nw = gridDim.x * (MLP_BS / 64);
  for (int s = gw; s < n; s += nw) {
    float xs[MLP_IN];
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) xs[k] = x[(size_t)s * MLP_IN + k];
    float z = u.b1;
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) z = fmaf(u.w[k], xs[k], z);
    const float h = z > 0.f ? z : 0.f;
    const float r = wave_fsum(u.w2 * h) + b2 - t[s];
    const float dy = inv_n * r;
    gw2 = fmaf(dy, h, gw2);
    const float gz = z > 0.f ? dy * u.w2 : 0.f;
    gb1 += gz;
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) gw1[k] = fmaf(gz, xs[k], gw1[k]);
    gb2 += dy;
    sq = fmaf(r, r, sq);
  }
#pragma unroll
  for (int k = 0; k < MLP_IN; k++) red[wv][j][k] = gw1[k];
  red[wv][j][MLP_IN] = gb1;
  red[wv][j][MLP_IN + 1] = gw2;
  if (j == 0) {
    red_s[wv][0] = gb2;
    red_s[wv][1] = sq;
  }
  __syncthreads();
  float *row = partial + (size_t)blockIdx.x * MLP_ROW;
  for (int q = threadIdx.x; q < MLP_ROW; q += MLP_BS) {
    float acc = 0.f;
    for (int w = 0; w < MLP_BS / 64; w++) {
      if (q < MLP_H * MLP_IN) acc += red[w][q / MLP_IN][q % MLP_IN];
      else if (q < MLP_H * MLP_IN + MLP_H) acc += red[w][q - MLP_H * MLP_IN][MLP_IN];
      else if (q < MLP_P - 1) acc += red[w][q - MLP_H * MLP_IN - MLP_H][MLP_IN + 1];
      else acc += red_s[w][q - (MLP_P - 1)];
    }
    row[q] = acc;
  }
}

__global__ void __launch_bounds__(1024) k_mlp_adam(float *p, float *m, float *v, const float *partial, int nblk,
                                                   int n, long long step, float lr, float beta1, float beta2,
                                                   float eps, float *grad_out, float *loss_out) {
  const int q = threadIdx.x;
  if (q > MLP_P) return;
  float g = 0.f;
  for (int b = 0; b < nblk; b++) g += partial[(size_t)b * MLP_ROW + q];
  if (q == MLP_P) {
    if (loss_out) *loss_out = n > 0 ? g / (float)n : 0.f;
    return;
  }
  if (grad_out) grad_out[q] = g;
  if (lr > 0.f) {
    const float mq = beta1 * m[q] + (1.f - beta1) * g;
    const float vq = beta2 * v[q] + (1.f - beta2) * g * g;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.f - powf(beta1, (float)step));
    const float vh = vq / (1.f - powf(beta2, (float)step));
    p[q] -= lr * mh / (sqrtf(vh) + eps);
  }
}

// Partial gradient rows for callers that cannot allocate: one row per
// workgroup of k_mlp_grad, at most MLP_MAX_BLOCKS of them (about 2 MB).  Each
// device that runs the library holds its own copy until the process ends.
// Host code must never pass `scratch` itself to a kernel (on the host it is
// a stand-in, not a device address): mlp_scratch() looks up each device's
// address once, with hipGetSymbolAddress, and that address is what kernels
// get.  Every call on a device shares its copy, so calls that overlap on one
// device race.  k_mlp_grad writes every element of the rows it owns before
// k_mlp_adam reads them, so nothing needs clearing between calls.
static __device__ __align__(256) float scratch[MLP_MAX_BLOCKS * MLP_ROW];

hipError_t mlp_scratch(float **ptr, int *rows) {
  static std::mutex mu;
  static float *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<float *>(p);
  }
  *ptr = addr[dev];
  *rows = MLP_MAX_BLOCKS;
  return hipSuccess;
}

int mlp_grad_blocks(int n) {
  const int per_block = 16 * (MLP_BS / 64);  // about 16 samples per wave
  int b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > MLP_MAX_BLOCKS) b = MLP_MAX_BLOCKS;
  return b;
}

hipError_t launch_mlp_forward(const float *p, const float *x, int n, float *y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (n + (MLP_BS / 64) - 1) / (MLP_BS / 64);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(MLP_BS), 0, s, p, x, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_train_step(float *p, float *m, float *v, const float *x, const float *t, int n, long long step,
                                 float lr, float *partial, int nblk, float *grad, float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(MLP_BS), 0, s, p, x, t, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(576), 0, s, p, m, v, partial, nblk, n, step, lr, 0.9f, 0.999f, 1e-8f,
                     grad, loss);
  return hipGetLastError();
}

}  // namespace ccd
