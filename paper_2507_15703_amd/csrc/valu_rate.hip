// Calibration of the ALU roofline's peak: the rate at which the device issues plain
// 32-bit vector operations, one instruction kind at a time.
//
// Each thread runs CH independent chains of one operation (binary32 fma and add, xor,
// 32-bit mul_hi and mul_lo: the kinds the noise pass is made of) in a loop of ITERS
// iterations; the launch holds 8 workgroups of 256 threads per CU, so every SIMD has 8
// waves to pick from. The loop body is the CH operations and the scalar loop control, so
// the lane-operations per launch are blocks x threads x ITERS x CH. Prints one line per
// kind: ms per launch (mean of 5 after 2 warm-up launches, HIP events) and T lane-ops/s.
// The chains' results are summed into one output per thread so none is optimised away.
//
// Usage: valu_rate [CUs]   (default 256)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

namespace {

constexpr int CH = 8;
constexpr int ITERS = 4096;
constexpr int THREADS = 256;

template <int KIND>
__global__ __launch_bounds__(THREADS) void k_chain(float* __restrict__ out, float a, float b) {
  float f[CH];
  uint32_t u[CH];
  uint32_t k = __float_as_uint(a) | 1u;
  for (int c = 0; c < CH; ++c) {
    f[c] = threadIdx.x * 0.001f + c;
    u[c] = threadIdx.x + c + 12345u;
  }
  for (int i = 0; i < ITERS; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (KIND == 0) f[c] = __builtin_fmaf(f[c], a, b);
      if (KIND == 1) f[c] = f[c] + a;
      if (KIND == 2) u[c] = u[c] ^ k;
      if (KIND == 3) u[c] = __umulhi(u[c], k);
      if (KIND == 4) u[c] = u[c] * k;
    }
    // the operand (and, for xor, the chains) are opaque to the optimizer each iteration,
    // else xor and multiply chains fold into one operation by a combined constant
    asm volatile("" : "+s"(k));
    if (KIND == 2)
      for (int c = 0; c < CH; ++c) asm volatile("" : "+v"(u[c]));
  }
  float s = 0.0f;
  for (int c = 0; c < CH; ++c) s += KIND < 2 ? f[c] : (float)u[c];
  out[(size_t)blockIdx.x * THREADS + threadIdx.x] = s;
}

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

}  // namespace

int main(int argc, char** argv) {
  const int cus = argc > 1 ? std::atoi(argv[1]) : 256;
  if (cus < 1 || cus > 4096) {
    std::fprintf(stderr, "CUs must be in 1..4096\n");
    return 1;
  }
  const int blocks = cus * 8;
  float* out = nullptr;
  CHECK(hipMalloc(&out, (size_t)blocks * THREADS * sizeof(float)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  using Fn = void (*)(float*, float, float);
  const Fn fns[] = {k_chain<0>, k_chain<1>, k_chain<2>, k_chain<3>, k_chain<4>};
  const char* names[] = {"fma_f32", "add_f32", "xor_b32", "mul_hi_u32", "mul_lo_u32"};
  for (int j = 0; j < 5; ++j) {
    for (int w = 0; w < 2; ++w) hipLaunchKernelGGL(fns[j], dim3(blocks), dim3(THREADS), 0, 0, out, 1.0001f, 0.5f);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(fns[j], dim3(blocks), dim3(THREADS), 0, 0, out, 1.0001f, 0.5f);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= 5.0f;
    const double lane_ops = (double)blocks * THREADS * ITERS * CH;
    std::printf("%-11s %.4f ms per launch  %.2f T lane-ops/s\n", names[j], ms, lane_ops / (ms * 1e-3) / 1e12);
  }
  CHECK(hipFree(out));
  return 0;
}
