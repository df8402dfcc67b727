// The learned planner's network: forward, backward, loss and optimiser kernels.
//
// The paper chooses its partition with a fixed rule (Section V) and finds
// that the best stream count depends on the device (Section VI: one stream
// instead of two on the Xeon Phi).  The learned planner predicts the run time
// of a candidate plan with a small regression network trained on timings the
// pipeline itself produces, and takes the candidate with the smallest
// prediction.
//
// Network (FP32): x (d) -> tanh(x W1 + b1) (H) -> tanh(. W2 + b2) (H) -> . W3 + b3.
// Loss: mean squared error over the batch, plus optionally (wd/2) times the
// sum of squares of the weight matrices (biases are not penalised).  Optimiser: Adam with bias
// correction (Kingma and Ba, 2015).  Parameters are one flat array:
// W1 (d x H, row-major), b1 (H), W2 (H x H), b2 (H), W3 (H x 1), b3 (1).
// Every reduction runs in a fixed order (per-thread strided partial sums, then
// a fixed LDS tree or wave butterfly), so results are deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ooc {
namespace {

// Y[r][j] = act(sum_i X[r][i] W[i][j] + b[j]); act = tanh or identity
__global__ __launch_bounds__(256) void dense_fwd(int64_t n, int din, int dout, const float* __restrict__ X,
                                                 const float* __restrict__ W, const float* __restrict__ b,
                                                 float* __restrict__ Y, int use_tanh) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * dout) return;
  const int64_t r = idx / dout;
  const int j = (int)(idx % dout);
  float acc = b[j];
  for (int i = 0; i < din; ++i) acc += X[r * din + i] * W[(int64_t)i * dout + j];
  Y[idx] = use_tanh ? tanhf(acc) : acc;
}

// loss = (1/n) sum (y - t)^2 (one thread), dY = 2 (y - t) / n
__global__ __launch_bounds__(256) void mse_grad(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                                                float* __restrict__ dy) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  dy[r] = 2.0f * (y[r] - t[r]) / (float)n;
}

// Sum of one value per thread over a 256-thread block in a fixed order (an LDS
// tree), so the result does not depend on scheduling.
__device__ double block_sum256(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  return red[0];
}

// loss = (1/n) sum (y - t)^2 (one block of 256 threads)
__global__ __launch_bounds__(256) void mse_loss(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                                                float* __restrict__ loss) {
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const double d = (double)y[r] - (double)t[r];
    acc += d * d;
  }
  acc = block_sum256(acc);
  if (threadIdx.x == 0) *loss = (float)(acc / (double)n);
}

// loss += (wd/2) * sum of squares of the weight matrices (one block of 256 threads)
__global__ __launch_bounds__(256) void l2_penalty(const float* __restrict__ W1, int64_t n1,
                                                  const float* __restrict__ W2, int64_t n2,
                                                  const float* __restrict__ W3, int64_t n3, float wd,
                                                  float* __restrict__ loss) {
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n1; i += 256) acc += (double)W1[i] * W1[i];
  for (int64_t i = threadIdx.x; i < n2; i += 256) acc += (double)W2[i] * W2[i];
  for (int64_t i = threadIdx.x; i < n3; i += 256) acc += (double)W3[i] * W3[i];
  acc = block_sum256(acc);
  if (threadIdx.x == 0) *loss = (float)((double)*loss + 0.5 * (double)wd * acc);
}

// dZ = dH * (1 - H^2) in place (tanh derivative from the stored activations)
__global__ __launch_bounds__(256) void tanh_bwd(int64_t count, const float* __restrict__ H, float* __restrict__ dH) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  dH[i] = dH[i] * (1.0f - H[i] * H[i]);
}

// dW[i][j] = sum_r X[r][i] dZ[r][j] + wd W[i][j]; db[j] = sum_r dZ[r][j].
// One wave per output (din*dout weights, then dout biases): lane l sums rows
// l, l+64, ..., then a fixed butterfly over the wave.
__global__ __launch_bounds__(256) void dense_wgrad(int64_t n, int din, int dout, const float* __restrict__ X,
                                                   const float* __restrict__ dZ, const float* __restrict__ W,
                                                   float wd, float* __restrict__ dW, float* __restrict__ db) {
  const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)din * dout;
  if (o >= nw + dout) return;  // the whole wave leaves together
  float acc = 0.f;
  if (o < nw) {
    const int i = (int)(o / dout), j = (int)(o % dout);
    for (int64_t r = lane; r < n; r += 64) acc += X[r * din + i] * dZ[r * dout + j];
  } else {
    const int j = (int)(o - nw);
    for (int64_t r = lane; r < n; r += 64) acc += dZ[r * dout + j];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    if (o < nw)
      dW[o] = acc + wd * W[o];
    else
      db[o - nw] = acc;
  }
}

// dX[r][i] = sum_j dZ[r][j] W[i][j]
__global__ __launch_bounds__(256) void dense_xgrad(int64_t n, int din, int dout, const float* __restrict__ dZ,
                                                   const float* __restrict__ W, float* __restrict__ dX) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * din) return;
  const int64_t r = idx / din;
  const int i = (int)(idx % din);
  float acc = 0.f;
  for (int j = 0; j < dout; ++j) acc += dZ[r * dout + j] * W[(int64_t)i * dout + j];
  dX[idx] = acc;
}

__global__ __launch_bounds__(256) void adam(int64_t count, float* __restrict__ p, const float* __restrict__ g,
                                            float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float mi = b1 * m[i] + (1.f - b1) * g[i];
  const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }

// Plain copy, 16 bytes per thread per step (for calibrating traffic counters).
__global__ __launch_bounds__(256) void copy16(int64_t n16, const double2* __restrict__ src, double2* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes % 16 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) return hipErrorInvalidValue;
  const int64_t n16 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(copy16, dim3(8192), dim3(256), 0, s, n16, static_cast<const double2*>(src),
                     static_cast<double2*>(dst));
  return hipGetLastError();
}

int64_t mlp_param_count(int d, int H) { return (int64_t)d * H + H + (int64_t)H * H + H + H + 1; }

int64_t mlp_scratch_floats(int64_t n, int d, int H) {
  // H1, H2, y, dy, dH2, dH1 (+ dX of layer 1 is not needed)
  return n * H * 4 + n * 2 + 16;
}

hipError_t launch_mlp_forward(int64_t n, int d, int H, const float* params, const float* X, float* scratch,
                              float* y_out, hipStream_t s) {
  const float* W1 = params;
  const float* b1 = W1 + (int64_t)d * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (int64_t)H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H;
  float* H1 = scratch;
  float* H2 = H1 + n * H;
  hipLaunchKernelGGL(dense_fwd, dim3(blocks(n * H)), dim3(256), 0, s, n, d, H, X, W1, b1, H1, 1);
  hipLaunchKernelGGL(dense_fwd, dim3(blocks(n * H)), dim3(256), 0, s, n, H, H, H1, W2, b2, H2, 1);
  hipLaunchKernelGGL(dense_fwd, dim3(blocks(n)), dim3(256), 0, s, n, H, 1, H2, W3, b3, y_out, 0);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(int64_t n, int d, int H, const float* params, const float* X, const float* t, float wd,
                           float* scratch, float* grad, float* loss, hipStream_t s) {
  const float* W1 = params;
  const float* b1 = W1 + (int64_t)d * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (int64_t)H * H;
  const float* W3 = b2 + H;
  float* gW1 = grad;
  float* gb1 = gW1 + (int64_t)d * H;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (int64_t)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H;
  float* H1 = scratch;
  float* H2 = H1 + n * H;
  float* dH2 = H2 + n * H;
  float* dH1 = dH2 + n * H;
  float* y = dH1 + n * H;
  float* dy = y + n;
  hipError_t e = launch_mlp_forward(n, d, H, params, X, scratch, y, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mse_loss, dim3(1), dim3(256), 0, s, n, y, t, loss);
  if (wd != 0.f)
    hipLaunchKernelGGL(l2_penalty, dim3(1), dim3(256), 0, s, W1, (int64_t)d * H, W2, (int64_t)H * H, W3, (int64_t)H, wd,
                       loss);
  hipLaunchKernelGGL(mse_grad, dim3(blocks(n)), dim3(256), 0, s, n, y, t, dy);
  // layer 3 (linear): dW3 = H2^T dy, db3 = sum dy, dH2 = dy W3^T
  hipLaunchKernelGGL(dense_wgrad, dim3(blocks(((int64_t)H + 1) * 64)), dim3(256), 0, s, n, H, 1, H2, dy, W3, wd, gW3, gb3);
  hipLaunchKernelGGL(dense_xgrad, dim3(blocks(n * H)), dim3(256), 0, s, n, H, 1, dy, W3, dH2);
  hipLaunchKernelGGL(tanh_bwd, dim3(blocks(n * H)), dim3(256), 0, s, n * H, H2, dH2);
  // layer 2
  hipLaunchKernelGGL(dense_wgrad, dim3(blocks(((int64_t)H * H + H) * 64)), dim3(256), 0, s, n, H, H, H1, dH2, W2, wd, gW2,
                     gb2);
  hipLaunchKernelGGL(dense_xgrad, dim3(blocks(n * H)), dim3(256), 0, s, n, H, H, dH2, W2, dH1);
  hipLaunchKernelGGL(tanh_bwd, dim3(blocks(n * H)), dim3(256), 0, s, n * H, H1, dH1);
  // layer 1
  hipLaunchKernelGGL(dense_wgrad, dim3(blocks(((int64_t)d * H + H) * 64)), dim3(256), 0, s, n, d, H, X, dH1, W1, wd, gW1,
                     gb1);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam, dim3(blocks(count)), dim3(256), 0, s, count, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace ooc
