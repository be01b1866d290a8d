// Internal interface of the surrogate-network kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmbx {

struct GemmArgs {
  int M, N, K;
  const float* A;  // FP32, op(A) is M x K
  int lda, transA;
  const void* B;   // BF16 (b_bf16) or FP32, op(B) is K x N
  int ldb, transB, b_bf16;
  float* C;        // M x N pre-activation (bias added)
  int ldc;
  const float* bias;  // N values or nullptr
  int act;            // 1: Y = GELU(C); 0: Y = C
  float* Y;           // may be nullptr
  int ldy;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_gelu_backward(const float* Z, const float* dY, float* dZ, int64_t n, hipStream_t s);
hipError_t launch_colsum(const float* X, int rows, int cols, float* out, hipStream_t s);
int64_t mse_partials(int64_t n);
hipError_t launch_mse(const float* Y, const float* T, int64_t n, float* dY, float* partial, float* loss,
                      hipStream_t s);
// The same MSE with its partial sums in a static device array of kMseScratchFloats floats
// (no allocation, no workspace argument): n up to kMseScratchFloats * 256 values. Calls that
// overlap on one device share the array and race. hipErrorInvalidValue beyond the limit.
constexpr int64_t kMseScratchFloats = 65536;
hipError_t launch_mse_noalloc(const float* Y, const float* T, int64_t n, float* dY, float* loss, hipStream_t s);

struct AdamArgs {
  float *w, *m, *v;
  const float* g;
  int64_t n;
  float lr, b1, b2, eps, bc1, bc2;  // bc = 1 - beta^step
  uint16_t* w_bf16;                 // BF16 copy written after the update (may be nullptr)
};
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s);

}  // namespace cmbx
