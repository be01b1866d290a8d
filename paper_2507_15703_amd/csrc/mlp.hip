// Kernels of the spectrum surrogate (a small MLP): a BF16 matrix-core GEMM with FP32
// accumulation and a fused bias + GELU epilogue, the GELU derivative, column sums, an
// MSE loss with its gradient, Adam on FP32 master weights, and FP32 -> BF16 rounding.
//
// GEMM: C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]); Y = GELU(C) if act. A is FP32 in
// memory; B is BF16 or FP32. Operands are rounded to BF16 (round to nearest even) as they
// are loaded and multiplied on the matrix cores by v_mfma_f32_32x32x8_bf16 (FP32
// accumulation). Workgroup = 4 waves on a 64 x 64 tile of C, one 32 x 32 tile per wave.
// Operand layout of the 32x32x8 instruction (wave64): lane l supplies A[l % 32][4 (l / 32)
// + t] and B[4 (l / 32) + t][l % 32], t = 0..3; it receives D[8 (v / 4) + 4 (l / 32) + v % 4]
// [l % 32] in accumulator v = 0..15.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "mlp.hpp"

namespace cmbx {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (inputs are finite)
  return (short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

template <bool TA, bool TB, bool BBF>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const void* __restrict__ Bv, int ldb, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, int act, float* __restrict__ Y,
                                              int ldy) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int col0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int i = lane & 31;
  const int kq = 4 * (lane >> 5);
  f32x16 acc = {};
  const int ar = row0 + i, bc = col0 + i;
  for (int k0 = 0; k0 < K; k0 += 8) {
    bf16x4 a, b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + kq + t;
      float av = 0.f, bv = 0.f;
      if (ar < M && k < K) av = TA ? A[(size_t)k * lda + ar] : A[(size_t)ar * lda + k];
      if (bc < N && k < K) {
        const size_t idx = TB ? (size_t)bc * ldb + k : (size_t)k * ldb + bc;
        bv = BBF ? from_bf16(((const uint16_t*)Bv)[idx]) : ((const float*)Bv)[idx];
      }
      a[t] = to_bf16(av);
      b[t] = to_bf16(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int c = col0 + i;
  if (c >= N) return;
  const float bb = bias ? bias[c] : 0.f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = row0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (r < M) {
      const float z = acc[v] + bb;
      C[(size_t)r * ldc + c] = z;
      if (Y) Y[(size_t)r * ldy + c] = act ? gelu(z) : z;
    }
  }
}

__global__ void k_gelu_backward(const float* __restrict__ Z, const float* __restrict__ dY, float* __restrict__ dZ,
                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dZ[i] = dY[i] * gelu_grad(Z[i]);
}

__global__ void k_colsum(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + c];
  out[c] = s;
}

// dY = 2 (Y - T) / n; per-block partial sums of (Y - T)^2 / n into partial[blockIdx.x]
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                                             float* __restrict__ dY, float* __restrict__ partial) {
  __shared__ float red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float e = 0.f;
  if (i < n) {
    const float d = Y[i] - T[i];
    dY[i] = 2.0f * d / (float)n;
    e = d * d / (float)n;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ x, int n, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, uint16_t* __restrict__ wbf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  w[i] = wi;
  if (wbf) wbf[i] = (uint16_t)to_bf16(wi);
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (uint16_t)to_bf16(x[i]);
}

namespace {
dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }
}  // namespace

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  const dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64));
  const dim3 block(256);
#define CMBX_GEMM(TA, TB, BBF)                                                                              \
  hipLaunchKernelGGL((k_gemm<TA, TB, BBF>), grid, block, 0, s, g.M, g.N, g.K, g.A, g.lda, g.B, g.ldb, g.C, \
                     g.ldc, g.bias, g.act, g.Y, g.ldy)
  const int code = (g.transA ? 4 : 0) | (g.transB ? 2 : 0) | (g.b_bf16 ? 1 : 0);
  switch (code) {
    case 0: CMBX_GEMM(false, false, false); break;
    case 1: CMBX_GEMM(false, false, true); break;
    case 2: CMBX_GEMM(false, true, false); break;
    case 3: CMBX_GEMM(false, true, true); break;
    case 4: CMBX_GEMM(true, false, false); break;
    case 5: CMBX_GEMM(true, false, true); break;
    case 6: CMBX_GEMM(true, true, false); break;
    default: CMBX_GEMM(true, true, true); break;
  }
#undef CMBX_GEMM
  return hipGetLastError();
}

hipError_t launch_gelu_backward(const float* Z, const float* dY, float* dZ, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_backward, grid1(n), dim3(256), 0, s, Z, dY, dZ, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int rows, int cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, grid1(cols), dim3(256), 0, s, X, rows, cols, out);
  return hipGetLastError();
}

int64_t mse_partials(int64_t n) { return (n + 255) / 256; }

hipError_t launch_mse(const float* Y, const float* T, int64_t n, float* dY, float* partial, float* loss,
                      hipStream_t s) {
  const int64_t nb = mse_partials(n);
  hipLaunchKernelGGL(k_mse, dim3((unsigned)nb), dim3(256), 0, s, Y, T, n, dY, partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partial, (int)nb, loss);
  return hipGetLastError();
}

// Workspace of the allocation-free MSE: the per-block partial sums live in this file-scope
// array, one copy per device for the life of the process. In host code `scratch` names a
// host-side stand-in, never the device memory: only the address hipGetSymbolAddress
// returns for the current device is passed to kernels.
static __device__ __align__(256) float scratch[kMseScratchFloats];

hipError_t mse_scratch_address(float** out) {
  static std::mutex mu;
  static std::map<int, float*> addr;  // device -> address of that device's copy
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, static_cast<float*>(p)).first;
  }
  *out = it->second;
  return hipSuccess;
}

hipError_t launch_mse_noalloc(const float* Y, const float* T, int64_t n, float* dY, float* loss, hipStream_t s) {
  if (mse_partials(n) > kMseScratchFloats) return hipErrorInvalidValue;
  float* partial = nullptr;
  const hipError_t e = mse_scratch_address(&partial);
  if (e != hipSuccess) return e;
  // every partial k_sum reads is written by k_mse first: nothing to clear
  return launch_mse(Y, T, n, dY, partial, loss, s);
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, grid1(a.n), dim3(256), 0, s, a.w, a.m, a.v, a.g, a.n, a.lr, a.b1, a.b2, a.eps,
                     a.bc1, a.bc2, a.w_bf16);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, grid1(n), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

}  // namespace cmbx
