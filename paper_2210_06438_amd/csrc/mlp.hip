// mlp.hip -- the cost model that picks the aggregation width: a 5-64-64-1
// FP32 perceptron with ReLU, trained on the GPU by these kernels (forward,
// row-wise backward, parameter gradients, MSE gradient, Adam).
//
// Parameters are one flat FP32 array of HYDRO_MLP_PARAMS values:
//   W1[64][5] b1[64] W2[64][64] b2[64] W3[64] b3
// y = W3 relu(W2 relu(W1 x + b1) + b2) + b3.
// Every reduction runs in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include "internal.hpp"

using hydro::api::fail;

namespace {

constexpr int kIn = HYDRO_MLP_INPUTS;
constexpr int kH = HYDRO_MLP_HIDDEN;
constexpr int kW1 = 0;
constexpr int kB1 = kW1 + kH * kIn;
constexpr int kW2 = kB1 + kH;
constexpr int kB2 = kW2 + kH * kH;
constexpr int kW3 = kB2 + kH;
constexpr int kB3 = kW3 + kH;
constexpr int kParams = kB3 + 1;
static_assert(kParams == HYDRO_MLP_PARAMS, "parameter count");
constexpr int kThreads = 256;

#define MLP_HIP(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(HYDRO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// One thread per row; the parameters are staged in LDS by each block.
__global__ void __launch_bounds__(kThreads)
    mlp_fwd(const float* __restrict__ p, const float* __restrict__ x, int rows,
            float* __restrict__ y, float* __restrict__ act) {
  __shared__ float sp[kParams];
  for (int i = threadIdx.x; i < kParams; i += kThreads) sp[i] = p[i];
  __syncthreads();
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= rows) return;
  float xi[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) xi[i] = x[r * kIn + i];
  float h1[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float s = sp[kB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) s = fmaf(sp[kW1 + j * kIn + i], xi[i], s);
    h1[j] = fmaxf(s, 0.0f);
  }
  float out = sp[kB3];
  for (int j = 0; j < kH; ++j) {
    float s = sp[kB2 + j];
#pragma unroll
    for (int k = 0; k < kH; ++k) s = fmaf(sp[kW2 + j * kH + k], h1[k], s);
    const float h2 = fmaxf(s, 0.0f);
    out = fmaf(sp[kW3 + j], h2, out);
    if (act) act[((size_t)rows + r) * kH + j] = h2;
  }
  if (act) {
#pragma unroll
    for (int j = 0; j < kH; ++j) act[(size_t)r * kH + j] = h1[j];
  }
  y[r] = out;
}

// Per row: dz2 = dy W3 [h2 > 0], dz1 = (W2^T dz2) [h1 > 0].
__global__ void __launch_bounds__(kThreads)
    mlp_bwd_rows(const float* __restrict__ p, const float* __restrict__ act,
                 const float* __restrict__ dy, int rows, float* __restrict__ dz) {
  __shared__ float sp[kParams];
  for (int i = threadIdx.x; i < kParams; i += kThreads) sp[i] = p[i];
  __syncthreads();
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= rows) return;
  const float g = dy[r];
  float z2[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    const float h2 = act[((size_t)rows + r) * kH + j];
    z2[j] = h2 > 0.0f ? g * sp[kW3 + j] : 0.0f;
    dz[((size_t)rows + r) * kH + j] = z2[j];
  }
  for (int k = 0; k < kH; ++k) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kH; ++j) s = fmaf(sp[kW2 + j * kH + k], z2[j], s);
    dz[(size_t)r * kH + k] = act[(size_t)r * kH + k] > 0.0f ? s : 0.0f;
  }
}

// One thread per parameter: sum over rows in row order.
__global__ void __launch_bounds__(kThreads)
    mlp_bwd_params(const float* __restrict__ x, const float* __restrict__ act,
                   const float* __restrict__ dz, const float* __restrict__ dy, int rows,
                   float* __restrict__ grad) {
  const int q = blockIdx.x * kThreads + threadIdx.x;
  if (q >= kParams) return;
  float s = 0.0f;
  if (q < kB1) {                       // W1[k][i]
    const int k = q / kIn, i = q % kIn;
    for (int r = 0; r < rows; ++r) s = fmaf(dz[(size_t)r * kH + k], x[r * kIn + i], s);
  } else if (q < kW2) {                // b1[k]
    const int k = q - kB1;
    for (int r = 0; r < rows; ++r) s += dz[(size_t)r * kH + k];
  } else if (q < kB2) {                // W2[j][k]
    const int j = (q - kW2) / kH, k = (q - kW2) % kH;
    for (int r = 0; r < rows; ++r)
      s = fmaf(dz[((size_t)rows + r) * kH + j], act[(size_t)r * kH + k], s);
  } else if (q < kW3) {                // b2[j]
    const int j = q - kB2;
    for (int r = 0; r < rows; ++r) s += dz[((size_t)rows + r) * kH + j];
  } else if (q < kB3) {                // W3[j]
    const int j = q - kW3;
    for (int r = 0; r < rows; ++r) s = fmaf(dy[r], act[((size_t)rows + r) * kH + j], s);
  } else {                             // b3
    for (int r = 0; r < rows; ++r) s += dy[r];
  }
  grad[q] = s;
}

// Mean squared error: loss = mean((y - t)^2); dy = 2 (y - t) / rows.
// One block; the loss is summed in a fixed tree order.
__global__ void __launch_bounds__(kThreads)
    mlp_mse(const float* __restrict__ y, const float* __restrict__ t, int rows,
            float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ float part[kThreads];
  float s = 0.0f;
  const float inv = 1.0f / (float)rows;
  for (int r = threadIdx.x; r < rows; r += kThreads) {
    const float e = y[r] - t[r];
    dy[r] = 2.0f * e * inv;
    s = fmaf(e, e, s);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = part[0] * inv;
}

// Adam (Kingma & Ba 2015) with bias correction, step t >= 1.
__global__ void __launch_bounds__(kThreads)
    mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
             float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
             float c2) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
  const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int blocks_for(int n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

extern "C" {

int hydro_mlp_forward(const float* params, const float* x, int32_t rows, float* y, float* act,
                      void* stream) {
  hydro::api::clear_error();
  if (rows < 0) return fail(HYDRO_EINVAL, "rows %d < 0", rows);
  if (rows == 0) return HYDRO_OK;
  if (!params || !x || !y) return fail(HYDRO_EINVAL, "NULL argument");
  hipLaunchKernelGGL(mlp_fwd, dim3(blocks_for(rows)), dim3(kThreads), 0, (hipStream_t)stream,
                     params, x, rows, y, act);
  MLP_HIP(hipGetLastError());
  return HYDRO_OK;
}

int hydro_mlp_backward(const float* params, const float* x, const float* act, const float* dy,
                       int32_t rows, float* scratch, float* grad, void* stream) {
  hydro::api::clear_error();
  if (rows < 1) return fail(HYDRO_EINVAL, "rows %d < 1", rows);
  if (!params || !x || !act || !dy || !scratch || !grad) return fail(HYDRO_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(mlp_bwd_rows, dim3(blocks_for(rows)), dim3(kThreads), 0, s, params, act, dy,
                     rows, scratch);
  MLP_HIP(hipGetLastError());
  hipLaunchKernelGGL(mlp_bwd_params, dim3(blocks_for(kParams)), dim3(kThreads), 0, s, x, act,
                     scratch, dy, rows, grad);
  MLP_HIP(hipGetLastError());
  return HYDRO_OK;
}

int hydro_mlp_mse(const float* y, const float* target, int32_t rows, float* dy, float* loss,
                  void* stream) {
  hydro::api::clear_error();
  if (rows < 1) return fail(HYDRO_EINVAL, "rows %d < 1", rows);
  if (!y || !target || !dy) return fail(HYDRO_EINVAL, "NULL argument");
  hipLaunchKernelGGL(mlp_mse, dim3(1), dim3(kThreads), 0, (hipStream_t)stream, y, target, rows,
                     dy, loss);
  MLP_HIP(hipGetLastError());
  return HYDRO_OK;
}

int hydro_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t n, float lr,
                   float beta1, float beta2, float eps, int32_t step, void* stream) {
  hydro::api::clear_error();
  if (n < 0 || step < 1) return fail(HYDRO_EINVAL, "n %d, step %d", n, step);
  if (n == 0) return HYDRO_OK;
  if (!params || !grad || !m || !v) return fail(HYDRO_EINVAL, "NULL argument");
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return fail(HYDRO_EINVAL, "bad Adam hyper-parameters");
  const float c1 = 1.0f - powf(beta1, (float)step);
  const float c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(mlp_adam, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, params,
                     grad, m, v, n, lr, beta1, beta2, eps, c1, c2);
  MLP_HIP(hipGetLastError());
  return HYDRO_OK;
}

}  // extern "C"
