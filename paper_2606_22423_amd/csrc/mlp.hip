// The strategy selector's network on the GPU: a 6 -> 64 -> 64 -> 8 MLP in
// fp32 with ReLU after the two hidden layers, its masked mean-squared-error
// gradient, and the Adam update (Kingma and Ba, 2015, Algorithm 1).
//
// Parameter vector (floats): W1 [64][6], b1 [64], W2 [64][64], b2 [64],
// W3 [8][64], b3 [8] -- 5128 values, row-major in that order.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scan_dev {

constexpr int kIn = 6, kHid = 64, kOut = 8;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid, kParams = kOffB3 + kOut;
static_assert(kParams == 5128, "parameter count");

// Forward pass: one wavefront per row, lane j computing hidden unit j of
// both layers and lanes 0-7 the outputs; the parameters are staged in LDS
// once per work-group (W2 transposed, so that lane j's reads of column i are
// consecutive).  Every sum is taken in the order of the definition (bias,
// then the inputs in index order, one fma each), as in a one-thread-per-row
// evaluation: the outputs do not depend on how rows are spread.  A row costs
// about 140 dependent fmas instead of 5000 in one thread.
constexpr int kFwdRowsPerWg = 4;

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ theta,
                                                          const float* __restrict__ X, uint32_t rows,
                                                          float* __restrict__ out) {
  __shared__ float w[kParams];  // W2 at kOffW2 transposed: w[kOffW2 + i * kHid + j] = W2[j][i]
  __shared__ float hb[kFwdRowsPerWg][2][kHid];
  for (int t = threadIdx.x; t < kParams; t += blockDim.x) {
    int src = t;
    if (t >= kOffW2 && t < kOffB2) {
      const int u = t - kOffW2;
      src = kOffW2 + (u % kHid) * kHid + u / kHid;
    }
    w[t] = theta[src];
  }
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t r = blockIdx.x * kFwdRowsPerWg + wave;
  const bool valid = r < rows;
  const uint32_t rr = valid ? r : 0u;  // rows >= 1: row 0 exists
  __syncthreads();
  // layer 1: unit `lane`
  float z = w[kOffB1 + lane];
#pragma unroll
  for (int c = 0; c < kIn; ++c) z = fmaf(w[kOffW1 + lane * kIn + c], X[(size_t)rr * kIn + c], z);
  hb[wave][0][lane] = fmaxf(z, 0.0f);
  __syncthreads();
  // layer 2: unit `lane`
  z = w[kOffB2 + lane];
#pragma unroll 16
  for (int i = 0; i < kHid; ++i) z = fmaf(w[kOffW2 + i * kHid + lane], hb[wave][0][i], z);
  hb[wave][1][lane] = fmaxf(z, 0.0f);
  __syncthreads();
  // outputs: lane q < 8
  if (lane < (uint32_t)kOut) {
    float o = w[kOffB3 + lane];
#pragma unroll 16
    for (int j = 0; j < kHid; ++j) o = fmaf(w[kOffW3 + lane * kHid + j], hb[wave][1][j], o);
    if (valid) out[(size_t)r * kOut + lane] = o;
  }
}

// Loss and gradient of sum_{i,j} m_ij (out_ij - y_ij)^2 * inv_denom for 32 rows
// per work-group; each work-group writes its partial gradient (kParams
// floats) and partial loss to its own slot, summed afterwards in a fixed
// order.  Per-row activations live in LDS; the outer-product reductions over
// the 32 rows are split across the 64 threads.
constexpr int kRowsPerWg = 32;

__global__ __launch_bounds__(64) void mlp_grad_kernel(const float* __restrict__ theta, const float* __restrict__ X,
                                                      const float* __restrict__ Y, const float* __restrict__ M,
                                                      uint32_t rows, float inv_denom, float* __restrict__ partials) {
  __shared__ float w[kParams];
  __shared__ float xs[kRowsPerWg][kIn];
  // rows padded by one float so per-row threads hit different LDS banks
  __shared__ float h1[kRowsPerWg][kHid + 1];
  __shared__ float h2[kRowsPerWg][kHid + 1];   // later reused for dz1
  __shared__ float dz2[kRowsPerWg][kHid + 1];
  __shared__ float dout[kRowsPerWg][kOut];
  __shared__ float lossv[kRowsPerWg];
  const int tid = threadIdx.x;
  for (int i = tid; i < kParams; i += blockDim.x) w[i] = theta[i];
  const uint32_t r0 = blockIdx.x * kRowsPerWg;
  for (int i = tid; i < kRowsPerWg * kIn; i += blockDim.x) {
    const uint32_t r = r0 + i / kIn;
    xs[i / kIn][i % kIn] = r < rows ? X[(size_t)r * kIn + i % kIn] : 0.0f;
  }
  __syncthreads();
  // forward + output error, one thread per row
  if (tid < kRowsPerWg) {
    const uint32_t r = r0 + tid;
    for (int j = 0; j < kHid; ++j) {
      float z = w[kOffB1 + j];
      for (int c = 0; c < kIn; ++c) z = fmaf(w[kOffW1 + j * kIn + c], xs[tid][c], z);
      h1[tid][j] = fmaxf(z, 0.0f);
    }
    float o[kOut];
    for (int q = 0; q < kOut; ++q) o[q] = w[kOffB3 + q];
    for (int j = 0; j < kHid; ++j) {
      float z = w[kOffB2 + j];
      for (int i = 0; i < kHid; ++i) z = fmaf(w[kOffW2 + j * kHid + i], h1[tid][i], z);
      const float a = fmaxf(z, 0.0f);
      h2[tid][j] = a;
      for (int q = 0; q < kOut; ++q) o[q] = fmaf(w[kOffW3 + q * kHid + j], a, o[q]);
    }
    float l = 0.0f;
    for (int q = 0; q < kOut; ++q) {
      float g = 0.0f;
      if (r < rows) {
        const float m = M[(size_t)r * kOut + q], d = o[q] - Y[(size_t)r * kOut + q];
        l += m * d * d;
        g = 2.0f * m * d * inv_denom;
      }
      dout[tid][q] = g;
    }
    lossv[tid] = l * inv_denom;
    // back through W3 and the second ReLU
    for (int j = 0; j < kHid; ++j) {
      float d = 0.0f;
      if (h2[tid][j] > 0.0f)
        for (int q = 0; q < kOut; ++q) d = fmaf(w[kOffW3 + q * kHid + j], dout[tid][q], d);
      dz2[tid][j] = d;
    }
  }
  __syncthreads();
  float* part = partials + (size_t)blockIdx.x * (kParams + 1);
  // gW3, gb3: 8 x 64 + 8 entries
  for (int e = tid; e < kOut * kHid; e += blockDim.x) {
    const int q = e / kHid, j = e % kHid;
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s = fmaf(dout[r][q], h2[r][j], s);
    part[kOffW3 + e] = s;
  }
  if (tid < kOut) {
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s += dout[r][tid];
    part[kOffB3 + tid] = s;
  }
  // gW2, gb2
  for (int e = tid; e < kHid * kHid; e += blockDim.x) {
    const int j = e / kHid, i = e % kHid;
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s = fmaf(dz2[r][j], h1[r][i], s);
    part[kOffW2 + e] = s;
  }
  {
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s += dz2[r][tid];
    part[kOffB2 + tid] = s;
  }
  __syncthreads();
  // dz1 = (W2^T dz2) * relu'(z1), written over h2 (no longer needed)
  if (tid < kRowsPerWg) {
    for (int i = 0; i < kHid; ++i) {
      float d = 0.0f;
      if (h1[tid][i] > 0.0f)
        for (int j = 0; j < kHid; ++j) d = fmaf(w[kOffW2 + j * kHid + i], dz2[tid][j], d);
      h2[tid][i] = d;
    }
  }
  __syncthreads();
  for (int e = tid; e < kHid * kIn; e += blockDim.x) {
    const int i = e / kIn, c = e % kIn;
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s = fmaf(h2[r][i], xs[r][c], s);
    part[kOffW1 + e] = s;
  }
  {
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s += h2[r][tid];
    part[kOffB1 + tid] = s;
  }
  if (tid == 0) {
    float s = 0.0f;
    for (int r = 0; r < kRowsPerWg; ++r) s += lossv[r];
    part[kParams] = s;
  }
}

// grad[i] = sum over work-groups of partials (fixed order); loss likewise.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partials, uint32_t nparts,
                                                         float* __restrict__ grad, float* __restrict__ loss) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > (uint32_t)kParams) return;
  float s = 0.0f;
  for (uint32_t p = 0; p < nparts; ++p) s += partials[(size_t)p * (kParams + 1) + i];
  if (i < (uint32_t)kParams) grad[i] = s;
  else if (loss) *loss = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, uint32_t count,
                                                   float lr, float beta1, float beta2, float eps, float bc1,
                                                   float bc2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * g;
  const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t launch_mlp_forward(const float* theta, const float* X, uint32_t rows, float* out, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((rows + kFwdRowsPerWg - 1) / kFwdRowsPerWg), dim3(64 * kFwdRowsPerWg),
                     0, st, theta, X, rows, out);
  return hipGetLastError();
}

uint32_t mlp_grad_partials(uint32_t rows) { return (rows + kRowsPerWg - 1) / kRowsPerWg; }

hipError_t launch_mlp_grad(const float* theta, const float* X, const float* Y, const float* M, uint32_t rows,
                           float inv_denom, float* partials, float* grad, float* loss, hipStream_t st) {
  const uint32_t np = mlp_grad_partials(rows);
  if (np == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(np), dim3(64), 0, st, theta, X, Y, M, rows, inv_denom, partials);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 1 + 255) / 256), dim3(256), 0, st, partials, np, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, uint32_t count, int step, float lr,
                       float beta1, float beta2, float eps, hipStream_t st) {
  const float bc1 = 1.0f - powf(beta1, (float)step), bc2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((count + 255) / 256), dim3(256), 0, st, theta, grad, m, v, count, lr, beta1,
                     beta2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace scan_dev
