// HIP kernels of the hot path for gfx950: the three passes of the inverse 3-D FFT (the
// first fused with noise generation) and the sphere gather.
//
// Data layout (one realisation, plan precision T):
//   during the passes: complex [N][N][N/2] -- the half grid with its iz = 0 and iz = N/2
//     planes packed into column 0 as Z_0 + i Z_{N/2}. Both planes are Hermitian within
//     the plane, so after the x and y transforms they are real and column 0 holds their
//     two real 2-D transforms side by side. This keeps every line at N/2 columns.
//   after pass 3: real [N][N][N], z fastest -- the same bytes, in place.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "fft_device.hpp"
#include "kernels.hpp"
#include "noise_device.hpp"

namespace cmbx {

// ------------------------------------------------------------------ global accessors
// Column tile of a strided axis: element n of column q at p[n * stride + q].
template <typename T>
struct GlobalColIO {
  cpx<T>* p;
  size_t stride;
  __device__ __forceinline__ cpx<T> operator()(int q, int n) const { return p[(size_t)n * stride + q]; }
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const { p[(size_t)n * stride + q] = v; }
  // the tile is read and written in place, so all reads must finish before any write
  __device__ __forceinline__ void done() const { __syncthreads(); }
};

// Map footprint (layout in kernels.hpp): a column tile whose writes skip the rows n that
// no pixel stencil reads. `keep` is an LDS copy of the footprint's bytes for these rows,
// one byte per `1 << SHIFT` rows; NULL keeps every row.
template <typename T, int SHIFT>
struct KeptRowsColIO {
  GlobalColIO<T> g;
  const uint8_t* keep;
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const {
    if (!keep || keep[n >> SHIFT]) g(q, n, v);
  }
  __device__ __forceinline__ void done() const { g.done(); }
};

// Contiguous lines of length L: element n of line q at p[q * L + n].
template <typename T, int L>
struct GlobalLineIO {
  cpx<T>* p;
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const { p[(size_t)q * L + n] = v; }
  __device__ __forceinline__ void done() const {}
};

// The same, writing only the lines q that `keep` flags (a bit mask, or with more than 64
// lines per block an LDS byte array, NULL = every line), and of those only the elements n
// whose bit n / 16 is set in `zmask`. Element n holds the real outputs 2n and 2n + 1, so zmask flags
// blocks of 32 real outputs (whole 128-byte lines in FP32: partial-line writes cost more than they save).
template <typename T, int L, int LINES>
struct KeptLinesIO {
  cpx<T>* p;
  uint64_t keep;
  const uint8_t* keep_lds;
  uint64_t zmask;
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const {
    const bool line = LINES <= 64 ? ((keep >> q) & 1) != 0 : (!keep_lds || keep_lds[q] != 0);
    if (line && ((zmask >> (n >> 4)) & 1)) p[(size_t)q * L + n] = v;
  }
  __device__ __forceinline__ void done() const {}
};

// First stage of the z pass: the packed half line X_0 .. X_{M-1} (LDS, line-major) is
// turned into the M-point complex sequence
//   Z_k = (X_k + conj X_{M-k}) + i w^k (X_k - conj X_{M-k}),  w = exp(2 pi i / N),
//   Z_0 = (a + b) + i (a - b)   with X_0 = a, X_{N/2} = b (column 0 holds a + i b),
// whose inverse M-point DFT z_n gives the real outputs x_{2n} = Re z_n, x_{2n+1} = Im z_n.
template <typename T, int M, int LINES, int P = 0>
struct HalfToComplex {
  using Lds = LdsIO<T, M, LINES, false, P>;  // the tile's layout
  const cpx<T>* x;
  const cpx<T>* tw;  // N = 2M roots
  __device__ __forceinline__ cpx<T> operator()(int q, int k) const {
    const cpx<T> xk = x[Lds::index(q, k)];
    if (k == 0) return {xk.x + xk.y, xk.x - xk.y};
    const cpx<T> xc = conj(x[Lds::index(q, M - k)]);
    return (xk + xc) + mul_i(cmul(tw[k], xk - xc));
  }
  __device__ __forceinline__ void done() const { __syncthreads(); }
};

// ------------------------------------------------------------------ noise tables
// The binary32 Box-Muller tables (bmf layout), one copy per device, written by
// upload_noise_tables before the first single-precision plan runs there.
__device__ float g_bm_tab[bmf::kTabSize];

// LDS slots (complex units) the pass-x tile reserves for the tables: binary32 only.
template <typename T>
constexpr int tab_cpx() { return sizeof(T) == 4 ? bmf::kTabSize / 2 : 0; }

// ------------------------------------------------------------------ launch shapes
// threads per workgroup for `work` points in LDS: 512 from 4096 points (two butterflies
// per thread and stage or fewer), down to one wave for small tiles
constexpr int clamp_nt(int work) { return work >= 4096 ? 512 : work >= 2048 ? 256 : work >= 1024 ? 128 : 64; }

template <typename T, int N, int TZ>
struct XYShape {
  static constexpr int M = N / 2;
  static constexpr int NT = clamp_nt(N * TZ);
  static_assert(M % TZ == 0 && TZ % 2 == 0, "tile must divide N/2 and be even");
};

template <typename T, int N, int LINES>
struct ZShape {
  static constexpr int M = N / 2;
  static constexpr int NT = clamp_nt(LINES * M);
};

// ------------------------------------------------------------------ pass 1: noise + x
// Workgroup = (z tile zt of TZ packed columns, one iy). Generates the N x TZ tile of
// weighted modes in LDS (one Philox call per pair of neighbouring iz), then runs the
// length-N inverse transform along x and writes the tile's N rows of TZ columns (128 B for
// FP32 TZ = 16) to the strided x axis. smem: N TZ + N complex (tile, then twiddles), then
// for binary32 the Box-Muller tables. With a map footprint `fp`, only the rows ix of the
// x-planes that the map's stencils read are written (the transform itself is whole).
// LDS of the x pass after the tile: N twiddles, then for binary32 the Box-Muller tables.
template <typename T, int N, int TZ>
struct XLds {
  static constexpr int TW = N * TZ;                 // twiddles, in cpx<T>
  static constexpr int TAB = TW + N;                // binary32 tables
  static constexpr int SIZE = TAB + tab_cpx<T>();   // cpx<T> units
};

// Twiddles, binary32 tables and the footprint's plane flags into LDS (once per workgroup;
// the caller synchronises before the first tile).
template <typename T, int N, int TZ, int NT>
__device__ __forceinline__ void x_setup(cpx<T>* smem, const cpx<T>* __restrict__ twg,
                                        const uint8_t* __restrict__ fp, uint8_t* planes) {
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) smem[XLds<T, N, TZ>::TW + i] = twg[i];
  if constexpr (tab_cpx<T>() > 0) {
    float* tab = reinterpret_cast<float*>(smem + XLds<T, N, TZ>::TAB);
    for (int i = tid; i < bmf::kTabSize; i += NT) tab[i] = g_bm_tab[i];
  }
  if (fp)
    for (int i = tid; i < N; i += NT) planes[i] = fp[i];
}

// One tile: the modes of z tile zt (TZ packed columns) at row iy into LDS, the length-N
// inverse transform along x, and the rows written (with a map footprint, only the rows ix
// of the x-planes the map's stencils read; the transform itself is whole). Needs
// x_setup's LDS and no thread still reading the tile of an earlier call.
template <typename T, int N, int TZ, int NT, int P = 0>
__device__ __forceinline__ void x_tile(cpx<T>* smem, int zt, int iy, cpx<T>* __restrict__ buf,
                                       const T* __restrict__ wtab, uint32_t k0, uint32_t k1, int m_hi,
                                       const uint8_t* planes) {
  constexpr int M = N / 2;
  constexpr int PAIRS = TZ / 2;
  using Lds = LdsIO<T, N, TZ, true, P>;  // the tile's layout, as the transform reads it
  cpx<T>* tile = smem;
  const cpx<T>* tw = smem + XLds<T, N, TZ>::TW;
  const float* tab = tab_cpx<T>() > 0 ? reinterpret_cast<const float*>(smem + XLds<T, N, TZ>::TAB) : nullptr;
  const int tid = threadIdx.x;
  const int zc0 = zt * TZ;
  const T* wself = wtab + 3 * M * M + 1;
  const int fy2 = freq2(iy, N);
  if (zc0 == 0) {
    // column 0 packs the Hermitian planes iz = 0 and N/2; column 1 is iz = 1
    for (int ix = tid; ix < N; ix += NT) {
      const cpx<T> a = mode_value<T>(N, ix, iy, 0, k0, k1, wtab, wself, tab);
      const cpx<T> b = mode_value<T>(N, ix, iy, M, k0, k1, wtab, wself, tab);
      tile[Lds::index(0, ix)] = {a.x - b.y, a.y + b.x};  // Z_0 + i Z_{N/2}
      tile[Lds::index(1, ix)] = mode_value<T>(N, ix, iy, 1, k0, k1, wtab, wself, tab);
    }
  }
  // every other pair of columns (2p, 2p + 1) holds two generic modes drawn from one
  // Philox call. The two are neighbours in the column-fast tile (columns are its fastest
  // index), 16-byte aligned in binary32: one 16-byte store, which also runs the lanes'
  // stores over consecutive banks (two 8-byte stores met in pairs on a bank)
  auto store2 = [&](int pr, int ix, cpx<T> a, cpx<T> b) {
    cpx<T>* p = &tile[Lds::index(2 * pr, ix)];
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
    } else {
      p[0] = a;
      p[1] = b;
    }
  };
  auto pair = [&](int pr, int ix, int zc, int m0) {
    if (m0 > m_hi) {  // both modes beyond the spectrum's support: +0, no draw, no load
      store2(pr, ix, {T(0), T(0)}, {T(0), T(0)});
      return;
    }
    const int m1 = m0 + 2 * zc + 1;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)zc >> 1, (uint32_t)iy, (uint32_t)ix, 0u), k0, k1);
    store2(pr, ix, weighted<T>(wtab[m0], w.x, w.y, tab), weighted<T>(wtab[m1], w.z, w.w, tab));
  };
  if constexpr (NT % PAIRS == 0) {
    // a thread keeps its pair of columns over the rows it visits
    const int pr = tid % PAIRS;
    const int zc = zc0 + 2 * pr;
    if (zc != 0) {
      const int base = fy2 + zc * zc;
      for (int ix = tid / PAIRS; ix < N; ix += NT / PAIRS) pair(pr, ix, zc, freq2(ix, N) + base);
    }
  } else {
    for (int s = tid; s < N * PAIRS; s += NT) {
      const int pr = s % PAIRS;
      const int ix = s / PAIRS;
      const int zc = zc0 + 2 * pr;
      if (zc != 0) pair(pr, ix, zc, freq2(ix, N) + fy2 + zc * zc);
    }
  }
  __syncthreads();
  Lds first{tile};
  KeptRowsColIO<T, 0> last{{buf + (size_t)iy * M + zc0, (size_t)N * M}, planes};
  fft_run<T, N, TZ, NT, true, 1, 0, Lds, KeptRowsColIO<T, 0>, P>(tw, tile, first, last, tid);
}

// Largest s with s^2 <= d (d >= 0, below 2^24).
__device__ __forceinline__ int isqrt_floor(int d) {
  int s = (int)sqrtf((float)d);
  while (s * s > d) --s;
  while ((s + 1) * (s + 1) <= d) ++s;
  return s;
}

// floor(sqrt(d)) for 0 <= d < 2^22: the hardware square root is within an ulp of the
// root (below 2048), so the truncated value is off by at most one either way.
__device__ __forceinline__ int isqrt_small(int d) {
  int s = (int)__builtin_amdgcn_sqrtf((float)d);
  s -= s * s > d ? 1 : 0;
  s += (s + 1) * (s + 1) <= d ? 1 : 0;
  return s;
}

// Tiles of the x pass within the spectrum's support: z tile zt holds modes of nonzero
// weight only for rows with fy^2 + (zt TZ)^2 <= m_hi, i.e. |fy| <= R(zt): the rows
// 0 .. R and N - R .. N - 1, min(N, 2R + 1) of them (none if (zt TZ)^2 > m_hi).
__host__ __device__ constexpr int x_rows_in_support(int N, int TZ, int zt, int R) {
  return R < 0 ? 0 : (2 * R + 1 < N ? 2 * R + 1 : N);
}

// One pass-x workgroup per tile of the pipelined kernel (setup included).
template <typename T, int N, int TZ, int NT>
__device__ __forceinline__ void role_x(cpx<T>* smem, int zt, int iy, cpx<T>* __restrict__ buf,
                                       const T* __restrict__ wtab, const cpx<T>* __restrict__ twg, uint32_t k0,
                                       uint32_t k1, int m_hi, const uint8_t* __restrict__ fp) {
  // Every mode of the tile (the packed plane iz = N/2 included) beyond the spectrum's
  // support: its transform is zero, and pass y does not read those lines (it takes them
  // as zero), so the tile is left as it is.
  if (freq2(iy, N) + zt * TZ * zt * TZ > m_hi) return;
  __shared__ uint8_t planes[N];
  x_setup<T, N, TZ, NT>(smem, twg, fp, planes);
  __syncthreads();
  x_tile<T, N, TZ, NT>(smem, zt, iy, buf, wtab, k0, k1, m_hi, fp ? planes : nullptr);
}

// The thread's index, opaque to the optimizer: the y pass walks a work list and calls its
// transform in a loop, and without this the compiler keeps the per-thread addresses of
// every stage live across the loop (8 columns: 102 VGPRs instead of 47, 16 columns: 171
// instead of 80, halving occupancy). Recomputed per call they are cheap. (The z pass,
// whose blocks are small, runs faster with its addresses kept: it does not use this.)
__device__ __forceinline__ int opaque_tid() {
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  return tid;
}

// ------------------------------------------------------------------ pass 2: y
// Workgroup = (z tile zt, one ix): N rows (iy) of TZ columns, read, transformed along y,
// written back in place.
// After pass x the element (ix, iy, column zc) is zero wherever fy^2 + zc^2 exceeds the
// spectrum's last nonzero |f|^2 (every mode of that x-line had zero weight); the reader
// returns those zeros without loading them (pass x does not write them).
template <typename T, int N>
struct SupportColIO {
  GlobalColIO<T> g;
  int zc0, m_hi;
  __device__ __forceinline__ cpx<T> operator()(int q, int n) const {
    const int zc = zc0 + q;
    return freq2(n, N) + zc * zc > m_hi ? cpx<T>{T(0), T(0)} : g(q, n);
  }
  __device__ __forceinline__ void done() const { g.done(); }
};

// Raw buffer resource over `bytes` bytes at p (gfx9 descriptor word 3: 32-bit data
// format). Loads at an offset at or past `bytes` return zero without a memory access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ cpx<T> buffer_load_cpx(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
  else return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
}

// The same reader as SupportColIO for the column tile at zc0 of one plane, through a
// buffer resource on the plane: an element beyond the support is read at an offset past
// the plane (zero, no memory access) instead of under a branch, and the offsets are 32
// bits. The support test takes the row bound R of the thread's column (|fy| <= R, the
// floor root of m_hi - zc^2, -1 if that is negative), made once: every call of a thread
// is for its own column q = tid % TZ (column-fast tiles whose thread count is a multiple
// of TZ).
template <typename T, int N>
struct SupportBufCol {
  static constexpr int M = N / 2;
  __amdgpu_buffer_rsrc_t rs;
  int zc0, R;
  __device__ __forceinline__ SupportBufCol(const cpx<T>* plane, int zc0_, int m_hi, int q) : zc0(zc0_) {
    rs = buffer_rsrc(plane, (uint32_t)(N * M * sizeof(cpx<T>)));
    const int zc = zc0 + q;
    const int d = m_hi - zc * zc;  // (m_hi may be INT_MAX: no support bound)
    R = d < 0 ? -1 : d >= M * M ? M : isqrt_small(d);
  }
  __device__ __forceinline__ cpx<T> operator()(int q, int n) const {
    bool in;
    if constexpr ((N & (N - 1)) == 0) in = (int)((unsigned)(n + R) & (N - 1)) <= 2 * R;
    else in = n <= R || n >= N - R;
    const uint32_t off = in ? (uint32_t)(n * M + zc0 + q) * (uint32_t)sizeof(cpx<T>) : 0x80000000u;
    return buffer_load_cpx<T>(rs, off);
  }
  // the tile is read and written in place, so all reads must finish before any write
  __device__ __forceinline__ void done() const { __syncthreads(); }
};

// With a map footprint `fp`, x-planes that no stencil reads are skipped, and of the
// others only the 8-row blocks that some stencil reads are written.
template <typename T, int N, int TZ, int NT, int P = 0>
__device__ __forceinline__ void role_y(cpx<T>* smem, int zt, int ix, cpx<T>* __restrict__ buf,
                                       const cpx<T>* __restrict__ twg, int m_hi, const uint8_t* __restrict__ fp,
                                       bool load_tw = true) {
  constexpr int M = N / 2;
  constexpr int NB = footprint_blocks(N);
  cpx<T>* tile = smem;
  cpx<T>* tw = smem + N * TZ;
  const int tid = opaque_tid();
  // (the thread index is opaque: a loop over it is not reduced to one step by itself)
  if (load_tw) {
    if constexpr (N <= NT) {
      if (tid < N) tw[tid] = twg[tid];
    } else {
      for (int i = tid; i < N; i += NT) tw[i] = twg[i];
    }
  }
  // columns wholly beyond the support stay zero through pass y; pass z does not read them
  if (zt * TZ * zt * TZ > m_hi) return;
  if (fp && !fp[ix]) return;
  __shared__ uint8_t rows[NB];
  if (fp) {
    if constexpr (NB <= NT) {
      if (tid < NB) rows[tid] = fp[N + ix * NB + tid];
    } else {
      for (int i = tid; i < NB; i += NT) rows[i] = fp[N + ix * NB + i];
    }
  }
  __syncthreads();
  GlobalColIO<T> io{buf + (size_t)ix * N * M + zt * TZ, (size_t)M};
  KeptRowsColIO<T, 3> last{io, fp ? rows : nullptr};
  if constexpr (NT % TZ == 0) {
    SupportBufCol<T, N> first(buf + (size_t)ix * N * M, zt * TZ, m_hi, (int)((unsigned)tid % TZ));
    fft_run<T, N, TZ, NT, true, 1, 0, SupportBufCol<T, N>, KeptRowsColIO<T, 3>, P>(tw, tile, first, last, tid);
  } else {
    SupportColIO<T, N> first{io, zt * TZ, m_hi};
    fft_run<T, N, TZ, NT, true, 1, 0, SupportColIO<T, N>, KeptRowsColIO<T, 3>, P>(tw, tile, first, last, tid);
  }
}

// ------------------------------------------------------------------ pass 3: z (c2r)
// Workgroup = LINES consecutive (ix, iy) lines of N/2 complex, starting at line blk LINES;
// they are contiguous, so the block is loaded and stored with unit stride. Columns zc with
// zc^2 beyond the spectrum's last nonzero |f|^2 are zero after pass y (which does not
// write them) and are not read.
// With a map footprint `fp`, a block none of whose lines a stencil reads is skipped, and
// only the lines in 8-row blocks that some stencil reads are written (the others of a kept
// block are transformed from whatever pass y left there, and dropped), and of those only
// the 32-node z blocks that some stencil reads.
template <typename T, int N, int LINES, int NT, int P = 0>
__device__ __forceinline__ void role_z(cpx<T>* smem, int blk, cpx<T>* __restrict__ buf,
                                       const cpx<T>* __restrict__ twg, int m_hi, const uint8_t* __restrict__ fp) {
  constexpr int M = N / 2;
  constexpr int NB = footprint_blocks(N);
  cpx<T>* tile = smem;
  cpx<T>* tw = smem + LINES * M;
  const int tid = threadIdx.x;
  static_assert(footprint_zblocks(N) <= 64, "one bit per z block");
  // flags of the block's lines and of the z blocks as bit masks, built by every wave
  // from the footprint (identical in all waves, so the early return is uniform); blocks
  // of more than 64 lines keep their line flags in LDS
  uint64_t keep = ~0ull, zmask = ~0ull;
  __shared__ uint8_t keep_lds[LINES > 64 ? LINES : 1];
  if (fp) {
    const int lane = tid & 63;
    zmask = __ballot(lane < footprint_zblocks(N) && fp[footprint_z_offset(N) + lane] != 0);
    if constexpr (LINES <= 64) {
      const int l = blk * LINES + lane;
      keep = __ballot(lane < LINES && fp[N + (l / N) * NB + ((l % N) >> 3)] != 0);
      if (keep == 0) return;
    } else {
      int any = 0;
      for (int q = tid; q < LINES; q += NT) {
        const int l = blk * LINES + q;
        keep_lds[q] = fp[N + (l / N) * NB + ((l % N) >> 3)];
        any |= keep_lds[q];
      }
      if (!__syncthreads_or(any)) return;
    }
  }
  using Lds = LdsIO<T, M, LINES, false, P>;  // the tile's layout, as the transform reads it
  cpx<T>* g = buf + (size_t)blk * LINES * M;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  if constexpr (NT % M == 0) {
    // a thread meets one column only: its test is taken once, and its loads stay batched
    if ((tid % M) * (tid % M) > m_hi) {
      for (int i = tid; i < LINES * M; i += NT) tile[Lds::index(i / M, i % M)] = {T(0), T(0)};
    } else {
      for (int i = tid; i < LINES * M; i += NT) tile[Lds::index(i / M, i % M)] = g[i];
    }
  } else {
    for (int i = tid; i < LINES * M; i += NT) {
      const int zc = i % M;
      tile[Lds::index(i / M, zc)] = zc * zc > m_hi ? cpx<T>{T(0), T(0)} : g[i];
    }
  }
  __syncthreads();
  HalfToComplex<T, M, LINES, P> first{tile, tw};
  KeptLinesIO<T, M, LINES> last{g, keep, fp ? keep_lds : nullptr, zmask};
  fft_run<T, M, LINES, NT, false, 2, 0, HalfToComplex<T, M, LINES, P>, KeptLinesIO<T, M, LINES>, P>(tw, tile, first, last,
                                                                                                   tid);
}

// One workgroup per tile within the spectrum's support, listed by z tile (a prefix of the
// per-zt row counts, made in LDS; rows in the order 0 .. R, N - R .. N - 1): tiles beyond
// the support get no workgroup at all.
template <typename T, int N, int TZ, int P = 0>
__global__ __launch_bounds__((XYShape<T, N, TZ>::NT)) void k_pass_x(cpx<T>* __restrict__ buf,
                                                                 const T* __restrict__ wtab,
                                                                 const cpx<T>* __restrict__ twg,
                                                                 uint32_t k0, uint32_t k1, int m_hi,
                                                                 const uint8_t* __restrict__ fp) {
  constexpr int NT = XYShape<T, N, TZ>::NT;
  constexpr int T_ = N / 2 / TZ;  // z tiles
  __shared__ __align__(16) cpx<T> smem[XLds<T, N, TZ>::SIZE];
  __shared__ uint8_t planes[N];
  __shared__ int start[T_ + 1];   // first listed tile of each z tile
  __shared__ int radius[T_];      // R(zt)
  x_setup<T, N, TZ, NT>(smem, twg, fp, planes);
  for (int zt = threadIdx.x; zt < T_; zt += NT) {
    const int d = m_hi - zt * TZ * zt * TZ;
    radius[zt] = d < 0 ? -1 : isqrt_floor(d);
    start[zt + 1] = x_rows_in_support(N, TZ, zt, radius[zt]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    start[0] = 0;
    for (int zt = 0; zt < T_; ++zt) start[zt + 1] += start[zt];
  }
  __syncthreads();
  const int e = blockIdx.x;
  if (e >= start[T_]) return;  // (the grid is the host's count of the same tiles)
  int lo = 0, hi = T_ - 1;       // the z tile whose range holds e
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (start[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  const int k = e - start[lo], R = radius[lo];
  const int iy = k <= R ? k : N - (start[lo + 1] - start[lo] - k);
  x_tile<T, N, TZ, NT, P>(smem, lo, iy, buf, wtab, k0, k1, m_hi, fp ? planes : nullptr);
}

template <typename T, int N, int TZ, int P = 0>
__global__ __launch_bounds__((XYShape<T, N, TZ>::NT)) void k_pass_y(cpx<T>* __restrict__ buf,
                                                                 const cpx<T>* __restrict__ twg, int m_hi,
                                                                 const uint8_t* __restrict__ fp) {
  __shared__ cpx<T> smem[N * TZ + N];
  constexpr int T_ = N / 2 / TZ;  // column tiles per plane
  // whole field: the grid is (tile, plane), one pass of the loop; with a footprint a grid
  // of at most kZGrid workgroups walks (listed plane, tile) pairs, tiles beyond the
  // spectrum's support left out. One call site of the transform either way.
  int tiles = T_, count, e0, step;
  const uint32_t* plist = nullptr;
  if (fp) {
    const uint32_t* hdr = reinterpret_cast<const uint32_t*>(fp + footprint_list_offset(N));
    plist = hdr + kFootprintHeader + N * N;
    tiles = 0;
    while (tiles < T_ && tiles * TZ * tiles * TZ <= m_hi) ++tiles;
    count = (int)hdr[2] * tiles;
    e0 = blockIdx.x;
    step = gridDim.x;
  } else {
    e0 = blockIdx.y * T_ + blockIdx.x;
    count = e0 + 1;
    step = 1;
  }
  for (int e = e0; e < count; e += step) {
    const int zt = e % tiles, ix = plist ? (int)plist[e / tiles] : e / tiles;
    // the twiddles stay in LDS from one pair to the next (the tile lies below them)
    role_y<T, N, TZ, XYShape<T, N, TZ>::NT, P>(smem, zt, ix, buf, twg, m_hi, fp, e == e0);
    __syncthreads();  // the tile is reused by the next pair
  }
}

// The y pass over a map footprint's list with the next pair's loads in flight: a resident
// grid walks the (listed plane, tile within the support) pairs as k_pass_y does, and each
// workgroup issues the first stage's loads of its next pair into registers before it
// transforms the current one, whose inputs it loaded one turn earlier. Barriers inside
// the walk wait for LDS only (a full barrier would also wait for those loads). Same
// arithmetic and outputs as k_pass_y.
template <typename T, int SHIFT>
struct KeptRowsColLB {
  KeptRowsColIO<T, SHIFT> io;
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const { io(q, n, v); }
  // the next pair's row flags overwrite `keep`: every wave past its last use
  __device__ __forceinline__ void done() const { lds_barrier(); }
};

template <typename T, int N, int TZ, int P>
struct YWalk {
  static constexpr int NT = XYShape<T, N, TZ>::NT;
  static constexpr int R0 = stage_radix(N, 0, P);
  using Regs = cpx<T>[StageSlots<N, TZ, NT, R0>::PER][R0];
};

template <typename T, int N, int TZ, int P>
__device__ __forceinline__ void y_walk_load(cpx<T>* __restrict__ buf, const uint32_t* plist, int tiles, int m_hi,
                                            int e, typename YWalk<T, N, TZ, P>::Regs& v, int tid) {
  constexpr int M = N / 2;
  const int zt = e % tiles, ix = (int)plist[e / tiles];
  if constexpr (YWalk<T, N, TZ, P>::NT % TZ == 0) {
    SupportBufCol<T, N> src(buf + (size_t)ix * N * M, zt * TZ, m_hi, (int)((unsigned)tid % TZ));
    stage_inputs<T, N, TZ, YWalk<T, N, TZ, P>::NT, YWalk<T, N, TZ, P>::R0, true>(src, v, tid);
  } else {
    SupportColIO<T, N> src{{buf + (size_t)ix * N * M + zt * TZ, (size_t)M}, zt * TZ, m_hi};
    stage_inputs<T, N, TZ, YWalk<T, N, TZ, P>::NT, YWalk<T, N, TZ, P>::R0, true>(src, v, tid);
  }
}

// One pair on `cur` (loaded by the previous turn) while the next pair loads into `nxt`;
// false when the walk is over.
template <typename T, int N, int TZ, int P>
__device__ __forceinline__ bool y_walk_step(cpx<T>* smem, uint8_t* rows, cpx<T>* __restrict__ buf,
                                            const uint8_t* __restrict__ fp, const uint32_t* plist, int tiles,
                                            int count, int m_hi, int& e, typename YWalk<T, N, TZ, P>::Regs& cur,
                                            typename YWalk<T, N, TZ, P>::Regs& nxt) {
  constexpr int M = N / 2, NT = YWalk<T, N, TZ, P>::NT;
  constexpr int NB = footprint_blocks(N);
  const int tid = opaque_tid();
  const int en = e + (int)gridDim.x;
  if (en < count) y_walk_load<T, N, TZ, P>(buf, plist, tiles, m_hi, en, nxt, tid);
  const int zt = e % tiles, ix = (int)plist[e / tiles];
  for (int i = tid; i < NB; i += NT) rows[i] = fp[N + ix * NB + i];
  lds_barrier();  // the row flags (and the twiddles) in every wave; the tile is free
  KeptRowsColLB<T, 3> last{{{buf + (size_t)ix * N * M + zt * TZ, (size_t)M}, rows}};
  fft_run_from_regs<T, N, TZ, NT, true, 1, KeptRowsColLB<T, 3>, P, true>(smem + N * TZ, smem, cur, last, tid);
  e = en;
  return en < count;
}

template <typename T, int N, int TZ, int P = 0>
__global__ __launch_bounds__((XYShape<T, N, TZ>::NT), 4) void k_pass_y_walk(cpx<T>* __restrict__ buf,
                                                                      const cpx<T>* __restrict__ twg, int m_hi,
                                                                      const uint8_t* __restrict__ fp) {
  constexpr int NT = XYShape<T, N, TZ>::NT;
  constexpr int T_ = N / 2 / TZ;
  __shared__ cpx<T> smem[N * TZ + N];
  __shared__ uint8_t rows[footprint_blocks(N)];
  const uint32_t* hdr = reinterpret_cast<const uint32_t*>(fp + footprint_list_offset(N));
  const uint32_t* plist = hdr + kFootprintHeader + N * N;
  int tiles = 0;
  while (tiles < T_ && tiles * TZ * tiles * TZ <= m_hi) ++tiles;
  const int count = (int)hdr[2] * tiles;
  int e = blockIdx.x;
  if (e >= count) return;
  for (int i = threadIdx.x; i < N; i += NT) smem[N * TZ + i] = twg[i];
  typename YWalk<T, N, TZ, P>::Regs a, b;
  y_walk_load<T, N, TZ, P>(buf, plist, tiles, m_hi, e, a, threadIdx.x);
  // two pairs per turn, so that each names its register sets statically
  while (y_walk_step<T, N, TZ, P>(smem, rows, buf, fp, plist, tiles, count, m_hi, e, a, b) &&
         y_walk_step<T, N, TZ, P>(smem, rows, buf, fp, plist, tiles, count, m_hi, e, b, a)) {
  }
}

// Without a footprint one workgroup per block of LINES lines. With one, a grid of as many
// workgroups as the device holds at once walks the footprint's list of blocks that hold
// a read line (if the list was made for another block size, every block, each checked
// line by line).
constexpr int kZGrid = 1024;  // the y pass's walking grid (its tiles fit 2-4 per CU)

template <typename T, int N, int LINES, int P = 0>
__global__ __launch_bounds__((ZShape<T, N, LINES>::NT)) void k_pass_z(cpx<T>* __restrict__ buf,
                                                                   const cpx<T>* __restrict__ twg, int m_hi,
                                                                   const uint8_t* __restrict__ fp) {
  __shared__ cpx<T> smem[LINES * (N / 2) + N];
  constexpr int NBLK = N * N / LINES;
  const uint32_t* hdr = fp ? reinterpret_cast<const uint32_t*>(fp + footprint_list_offset(N)) : nullptr;
  const bool listed = hdr && hdr[0] == (uint32_t)LINES;
  // whole field: one pass of the loop, on this workgroup's own block (one call site of
  // the transform, so both cases run the same instructions)
  const int count = !fp ? (int)blockIdx.x + 1 : listed ? (int)hdr[1] : NBLK;
  for (int e = blockIdx.x; e < count; e += gridDim.x) {
    const int blk = listed ? (int)hdr[kFootprintHeader + e] : e;
    role_z<T, N, LINES, ZShape<T, N, LINES>::NT, P>(smem, blk, buf, twg, m_hi, fp);
    __syncthreads();  // the tile and the line flags are reused by the next block
  }
}

// ------------------------------------------------------------------ pass 3, streamed
// The z pass over a map footprint's block list with the next block's loads in flight
// while the current block is transformed: two LDS tiles, the next block copied from
// global memory straight into the idle one (global_load_lds, 16 B per lane, no
// registers), the transform's barriers LDS-only so that those copies are not waited for
// until the next block starts. Same arithmetic and outputs as k_pass_z.
typedef __attribute__((address_space(3))) void lds_void_t;

// First stage as HalfToComplex, on a tile copied whole: columns beyond the support hold
// whatever an earlier block left there and read as zero (what k_pass_z stores for them).
template <typename T, int M, int LINES, int P = 0>
struct HalfToComplexMasked {
  using Lds = LdsIO<T, M, LINES, false, P>;
  const cpx<T>* x;
  const cpx<T>* tw;
  int m_hi;
  __device__ __forceinline__ cpx<T> at(int q, int k) const {
    return k * k > m_hi ? cpx<T>{T(0), T(0)} : x[Lds::index(q, k)];
  }
  __device__ __forceinline__ cpx<T> operator()(int q, int k) const {
    const cpx<T> xk = at(q, k);
    if (k == 0) return {xk.x + xk.y, xk.x - xk.y};
    const cpx<T> xc = conj(at(q, M - k));
    return (xk + xc) + mul_i(cmul(tw[k], xk - xc));
  }
  __device__ __forceinline__ void done() const { lds_barrier(); }
};

// Binary32 transforms without a radix-16 stage only: those keep four waves per SIMD in
// registers (94 VGPRs at N = 512 with 4 x 8 x 8). Radix 16 or binary64 needed 160 and more
// and, held to 128, spilled: the streamed pass then ran at half the speed of k_pass_z.
template <typename T, int N, int LINES, int P>
constexpr bool z_streamable() {
  return sizeof(T) == 4 && max_radix(N / 2, P) <= 8 && LINES <= 64 &&
         ((size_t)LINES * (N / 2) * sizeof(cpx<T>)) % 1024 == 0;
}

// One block (LINES lines of M complex, contiguous in global memory and, in the same order,
// in the tile) into LDS: 1 KiB per wave instruction, 16 B per lane; a lane whose first
// column lies beyond the support loads nothing.
template <typename T, int M, int LINES, int NT>
__device__ __forceinline__ void z_block_to_lds(cpx<T>* tile, const cpx<T>* g, int m_hi) {
  constexpr int PER_LANE = 16 / (int)sizeof(cpx<T>);  // complex values per lane
  constexpr int PER_CHUNK = 64 * PER_LANE;
  constexpr int CHUNKS = LINES * M / PER_CHUNK;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < CHUNKS; c += NT / 64) {
    const int e = c * PER_CHUNK + lane * PER_LANE;
    const int col = e % M;
    if (col * col <= m_hi)
      __builtin_amdgcn_global_load_lds((const void*)(g + e), (lds_void_t*)(tile + c * PER_CHUNK), 16, 0, 0);
  }
}

// State of a workgroup's walk over the list: list entry e, its block, the next block and
// the flags of the current block's lines (lane q < LINES: line q).
struct ZWalk {
  int e, blk, blk1;
  uint32_t flag;  // the footprint byte of line lane (lanes past the block's lines: its last line)
};

// The footprint byte of line q of block blk (q < LINES), for the keep mask of the block.
template <int N, int LINES>
__device__ __forceinline__ uint32_t z_line_flag(const uint8_t* __restrict__ fp, int blk, int q) {
  constexpr int NB = footprint_blocks(N);
  const int l = blk * LINES + (q < LINES ? q : LINES - 1);
  return fp[N + (l / N) * NB + ((l % N) >> 3)];
}

// One block on `cur` (its copy issued by the previous step) while the next one streams
// into `nxt`. Returns false when the walk is over.
template <typename T, int N, int LINES, int P>
__device__ __forceinline__ bool z_stream_step(cpx<T>* cur, cpx<T>* nxt, const cpx<T>* tw, cpx<T>* __restrict__ buf,
                                              const uint8_t* __restrict__ fp, const uint32_t* hdr, bool listed,
                                              int count, int m_hi, uint64_t zmask, ZWalk& w) {
  constexpr int M = N / 2, NT = ZShape<T, N, LINES>::NT;
  const int lane = threadIdx.x & 63;
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this block's copy, flags and list entry are in
  lds_barrier();                       // ... in every wave, and no wave still reads nxt
  const uint64_t keep = __ballot(lane < LINES && w.flag != 0);
  const int en = w.e + (int)gridDim.x;
  const bool more = en < count;
  int blk2 = 0;
  uint32_t fn = 0;
  if (more) {
    if (en + (int)gridDim.x < count) blk2 = listed ? (int)hdr[kFootprintHeader + en + gridDim.x] : en + (int)gridDim.x;
    fn = z_line_flag<N, LINES>(fp, w.blk1, lane);  // read at the next step, after its wait
    z_block_to_lds<T, M, LINES, NT>(nxt, buf + (size_t)w.blk1 * LINES * M, m_hi);
  }
  HalfToComplexMasked<T, M, LINES, P> first{cur, tw, m_hi};
  KeptLinesIO<T, M, LINES> last{buf + (size_t)w.blk * LINES * M, keep, nullptr, zmask};
  fft_run<T, M, LINES, NT, false, 2, 0, HalfToComplexMasked<T, M, LINES, P>, KeptLinesIO<T, M, LINES>, P, true,
          LdsXorLines<T, M, LINES, true>>(tw, cur, first, last, threadIdx.x);
  w = {en, w.blk1, blk2, fn};
  return more;
}

template <typename T, int N, int LINES, int P = 0>
__global__ __launch_bounds__((ZShape<T, N, LINES>::NT), 4) void k_pass_z_stream(cpx<T>* __restrict__ buf,
                                                                          const cpx<T>* __restrict__ twg, int m_hi,
                                                                          const uint8_t* __restrict__ fp) {
  constexpr int M = N / 2, NT = ZShape<T, N, LINES>::NT;
  constexpr int NBLK = N * N / LINES;
  static_assert(z_streamable<T, N, LINES, P>(), "block of whole 1 KiB chunks, line flags in one wave");
  __shared__ __align__(16) cpx<T> tile0[LINES * M];
  __shared__ __align__(16) cpx<T> tile1[LINES * M];
  __shared__ cpx<T> tw[N];
  const uint32_t* hdr = reinterpret_cast<const uint32_t*>(fp + footprint_list_offset(N));
  const bool listed = hdr[0] == (uint32_t)LINES;  // else every block, each written line by line
  const int count = listed ? (int)hdr[1] : NBLK;
  ZWalk w;
  w.e = blockIdx.x;
  if (w.e >= count) return;
  const int lane = threadIdx.x & 63;
  const uint64_t zmask = __ballot(lane < footprint_zblocks(N) && fp[footprint_z_offset(N) + lane] != 0);
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  w.blk = listed ? (int)hdr[kFootprintHeader + w.e] : w.e;
  const int e1 = w.e + (int)gridDim.x;
  w.blk1 = e1 < count ? (listed ? (int)hdr[kFootprintHeader + e1] : e1) : 0;
  w.flag = z_line_flag<N, LINES>(fp, w.blk, lane);
  z_block_to_lds<T, M, LINES, NT>(tile0, buf + (size_t)w.blk * LINES * M, m_hi);
  // two steps per turn, so that each names its tiles statically: the compiler then sees
  // that the copies into one tile never alias the transform on the other
  while (z_stream_step<T, N, LINES, P>(tile0, tile1, tw, buf, fp, hdr, listed, count, m_hi, zmask, w) &&
         z_stream_step<T, N, LINES, P>(tile1, tile0, tw, buf, fp, hdr, listed, count, m_hi, zmask, w)) {
  }
}

// ------------------------------------------------------------------ debug noise
template <typename T>
__global__ void k_noise_debug(cpx<T>* __restrict__ out, int N, const T* __restrict__ wtab, uint32_t k0,
                              uint32_t k1) {
  const int M = N / 2;
  const int64_t total = (int64_t)N * N * (M + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int iz = (int)(i % (M + 1));
  const int64_t t = i / (M + 1);
  const int iy = (int)(t % N);
  const int ix = (int)(t / N);
  out[i] = mode_value<T>(N, ix, iy, iz, k0, k1, wtab, wtab + 3 * M * M + 1, g_bm_tab);
}

// ------------------------------------------------------------------ gather
// One thread per pixel. The position p = (r n + L/2) N/L and its floor are formed in FP64
// (no contraction, so CPU and GPU take the same integer decision); the fraction is then
// rounded to T, and weights and accumulation are in T. The 2 or 4 nodes per axis wrap
// modulo N.
template <typename T>
__device__ __forceinline__ void weights1d(T f, T* w, int interp) {
  if (interp == kTricubic) {
    w[0] = f * (T(-0.5) + f * (T(1.0) - T(0.5) * f));
    w[1] = T(1.0) + f * f * (T(-2.5) + T(1.5) * f);
    w[2] = f * (T(0.5) + f * (T(2.0) - T(1.5) * f));
    w[3] = f * f * (T(-0.5) + T(0.5) * f);
  } else {
    w[0] = T(1.0) - f;
    w[1] = f;
  }
}

__device__ __forceinline__ int wrap(int i, int N) { return i < 0 ? i + N : (i >= N ? i - N : i); }

// First stencil node i0 (before wrapping: -1 .. N-1) and fraction along each axis of the
// K-point stencil of pixel i. The gather and the map footprint both take their integer
// decisions here.
template <int K>
__device__ __forceinline__ void stencil_origin(int N, double scale, double3 obs, double r,
                                               const double* __restrict__ dirs, int64_t i, int i0[3],
                                               double frac[3]) {
#pragma clang fp contract(off)
  const double o[3] = {obs.x, obs.y, obs.z};
  // the three components loaded together, before the branches below
  const double n[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double p = (r * n[d] + o[d]) * scale;
    // any finite position is reduced modulo N; non-finite input samples node 0
    if (!(p > -1.0e9 && p < 1.0e9)) p = 0.0;
    const double fl = floor(p);
    int base = (int)fl;
    if ((unsigned)base >= (unsigned)N) {  // positions in the box need no reduction
      base %= N;
      base = base < 0 ? base + N : base;
    }
    i0[d] = base - (K == 4 ? 1 : 0);
    frac[d] = p - fl;
  }
}

// K taps of z, K times K lines: sum of w[0][a] w[1][b] w[2][c] f(i0 + (a, b, c)).
template <typename T, int K>
struct Taps {
  typedef T vec __attribute__((ext_vector_type(K), aligned(sizeof(T))));
};

template <typename T, int K, bool CONTIGUOUS>
__device__ __forceinline__ T stencil_sum(const T* __restrict__ field, int N, const int i0[3], const T (*w)[4]) {
  // element offsets in 32 bits (N^3 <= 2^30 for the largest compiled box, N = 1024): the
  // line (a, b) starts at xo[a] + yo[b]
  const uint32_t n = (uint32_t)N;
  uint32_t xo[K], yo[K], zo[K];
#pragma unroll
  for (int a = 0; a < K; ++a) xo[a] = (uint32_t)wrap(i0[0] + a, N) * (n * n);
#pragma unroll
  for (int b = 0; b < K; ++b) yo[b] = (uint32_t)wrap(i0[1] + b, N) * n;
#pragma unroll
  for (int c = 0; c < K; ++c) zo[c] = (uint32_t)wrap(i0[2] + c, N);
  // every tap is loaded before any is summed, so that the K x K line loads are in flight
  // together rather than one round trip after another
  T q[K][K][K];
#pragma unroll
  for (int a = 0; a < K; ++a) {
#pragma unroll
    for (int bb = 0; bb < K; ++bb) {
      const uint32_t line = xo[a] + yo[bb];
      if constexpr (CONTIGUOUS) {
        const typename Taps<T, K>::vec v =
            *reinterpret_cast<const typename Taps<T, K>::vec*>(field + (line + (uint32_t)i0[2]));
#pragma unroll
        for (int c = 0; c < K; ++c) q[a][bb][c] = v[c];
      } else {
#pragma unroll
        for (int c = 0; c < K; ++c) q[a][bb][c] = field[line + zo[c]];
      }
    }
  }
  T acc = 0;
#pragma unroll
  for (int a = 0; a < K; ++a) {
    T accb = 0;
#pragma unroll
    for (int bb = 0; bb < K; ++bb) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < K; ++c) s += w[2][c] * q[a][bb][c];
      accb += w[1][bb] * s;
    }
    acc += w[0][a] * accb;
  }
  return acc;
}

template <typename T, int K>
__device__ __forceinline__ void gather_pixel(const T* __restrict__ field, int N, double scale, double3 obs,
                                             double r, const double* __restrict__ dirs, int64_t i,
                                             T* __restrict__ out) {
  int i0[3];
  T w[3][4];
  {
    double frac[3];
    stencil_origin<K>(N, scale, obs, r, dirs, i, i0, frac);
#pragma unroll
    for (int d = 0; d < 3; ++d) weights1d<T>((T)frac[d], w[d], K == 4 ? kTricubic : kTrilinear);
  }
  // The K z taps of a line are contiguous unless the stencil wraps in z: then they are
  // read with vector loads of the taps alone (16 bytes for FP32 tricubic; the target
  // allows them at 4-byte alignment), else one by one. Both ways sum in the same order, and
  // no value outside the stencil is read (with a map footprint, cells beyond it are not
  // made).
  if (i0[2] >= 0 && i0[2] + K <= N)
    out[i] = stencil_sum<T, K, true>(field, N, i0, w);
  else
    out[i] = stencil_sum<T, K, false>(field, N, i0, w);
}

// Blocks are assigned so that each XCD's L2 serves a contiguous pixel range.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ field, int N, double scale, double3 obs,
                                                double r, const double* __restrict__ dirs, int64_t npix,
                                                T* __restrict__ out) {
  const int nb = gridDim.x;
  const int per = nb / 8;
  const int b = blockIdx.x;
  const int logical = (nb % 8 == 0) ? (b % 8) * per + b / 8 : b;
  const int64_t i = (int64_t)logical * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  gather_pixel<T, K>(field, N, scale, obs, r, dirs, i, out);
}

// ------------------------------------------------------------------ pixel order
// A record of the pixel order: the stencil's first node wrapped into the box, packed
// x << 20 | y << 10 | z (N <= 1024), and the fractions rounded to T as the gather rounds
// them. With the node wrapped, the z taps are contiguous exactly when z + K <= N (a first
// node at -1 wraps to N - 1), and the taps wrap to the same nodes.
template <typename T>
struct alignas(16) OrderRec {
  uint32_t node;
  T f[3];
};
static_assert(sizeof(OrderRec<float>) == 16 && sizeof(OrderRec<double>) == 32, "record sizes");

size_t pixel_order_record_bytes(int dtype) {
  return dtype == kF32 ? sizeof(OrderRec<float>) : sizeof(OrderRec<double>);
}

size_t pixel_order_bytes(int dtype, int64_t n_pix) {
  return (size_t)n_pix * (pixel_order_record_bytes(dtype) + sizeof(uint32_t));
}

__device__ __forceinline__ uint32_t spread3_10(uint32_t v) {
  uint32_t k = 0;
  for (int b = 0; b < 10; ++b) k |= ((v >> b) & 1u) << (3 * b);
  return k;
}

template <int K>
__device__ __forceinline__ void wrapped_node(int N, double scale, double3 obs, double r, const double* __restrict__ dirs,
                                             int64_t i, uint32_t c[3], double frac[3]) {
  int i0[3];
  stencil_origin<K>(N, scale, obs, r, dirs, i, i0, frac);
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = (uint32_t)wrap(i0[d], N);
}

// Key: the Morton code of the wrapped first node (x in the highest bit of each triple).
template <int K>
__global__ __launch_bounds__(256) void k_order_keys(int N, double scale, double3 obs, double r,
                                                    const double* __restrict__ dirs, int64_t npix,
                                                    uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  uint32_t c[3];
  double frac[3];
  wrapped_node<K>(N, scale, obs, r, dirs, i, c, frac);
  key[i] = (spread3_10(c[0]) << 2) | (spread3_10(c[1]) << 1) | spread3_10(c[2]);
  val[i] = (uint32_t)i;
}

// The records in sorted order.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_order_records(int N, double scale, double3 obs, double r,
                                                       const double* __restrict__ dirs, int64_t npix,
                                                       const uint32_t* __restrict__ sorted, OrderRec<T>* __restrict__ rec,
                                                       uint32_t* __restrict__ pix) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npix) return;
  const uint32_t i = sorted[j];
  uint32_t c[3];
  double frac[3];
  wrapped_node<K>(N, scale, obs, r, dirs, i, c, frac);
  OrderRec<T> o;
  o.node = (c[0] << 20) | (c[1] << 10) | c[2];
#pragma unroll
  for (int d = 0; d < 3; ++d) o.f[d] = (T)frac[d];
  rec[j] = o;
  pix[j] = i;
}

// Pixel pix[j] from record j, with the weights and the tap sum of gather_pixel.
template <typename T, int K>
__device__ __forceinline__ void gather_ordered_pixel(const T* __restrict__ field, int N,
                                                     const OrderRec<T>* __restrict__ rec,
                                                     const uint32_t* __restrict__ pix, int64_t j,
                                                     T* __restrict__ out) {
  const OrderRec<T> o = rec[j];
  const uint32_t p = pix[j];
  const int i0[3] = {(int)(o.node >> 20), (int)((o.node >> 10) & 1023u), (int)(o.node & 1023u)};
  T w[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) weights1d<T>(o.f[d], w[d], K == 4 ? kTricubic : kTrilinear);
  if (i0[2] + K <= N)
    out[p] = stencil_sum<T, K, true>(field, N, i0, w);
  else
    out[p] = stencil_sum<T, K, false>(field, N, i0, w);
}

// The gather in pixel order: thread j makes pixel pix[j] from record j.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_gather_ordered(const T* __restrict__ field, int N,
                                                        const OrderRec<T>* __restrict__ rec,
                                                        const uint32_t* __restrict__ pix, int64_t npix,
                                                        T* __restrict__ out) {
  const int nb = gridDim.x;
  const int per = nb / 8;
  const int b = blockIdx.x;
  const int logical = (nb % 8 == 0) ? (b % 8) * per + b / 8 : b;
  const int64_t j = (int64_t)logical * blockDim.x + threadIdx.x;
  if (j >= npix) return;
  gather_ordered_pixel<T, K>(field, N, rec, pix, j, out);
}

// Bits of the Morton key: 3 per level of the node coordinates in [0, N).
int order_key_bits(int N) {
  int bits = 0;
  while ((1 << (bits / 3)) < N) bits += 3;
  return bits;
}

hipError_t pixel_order_scratch_bytes(int N, int64_t n_pix, size_t* bytes) {
  size_t tmp = 0;
  const hipError_t e =
      sort_pairs_u32(nullptr, &tmp, nullptr, nullptr, nullptr, nullptr, n_pix, order_key_bits(N), nullptr);
  if (e != hipSuccess) return e;
  const size_t kv = ((size_t)n_pix * 16 + 255) / 256 * 256;
  *bytes = kv + tmp;
  return hipSuccess;
}

hipError_t launch_pixel_order(const PixelOrderArgs& a, hipStream_t s) {
  if (a.N > 1024 || a.n_pix < 1 || a.n_pix > ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const size_t n = (size_t)a.n_pix;
  const size_t kv = (n * 16 + 255) / 256 * 256;
  if (a.scratch_bytes < kv) return hipErrorInvalidValue;
  uint32_t* k_in = (uint32_t*)a.scratch;
  uint32_t* k_out = k_in + n;
  uint32_t* v_in = k_out + n;
  uint32_t* v_out = v_in + n;
  void* tmp = (char*)a.scratch + kv;
  size_t tmp_bytes = a.scratch_bytes - kv;
  const dim3 grid((unsigned)((n + 255) / 256));
  const double3 obs = make_double3(a.obs[0], a.obs[1], a.obs[2]);
  const bool cubic = a.interp == kTricubic;
  auto kk = cubic ? k_order_keys<4> : k_order_keys<2>;
  hipLaunchKernelGGL(kk, grid, dim3(256), 0, s, a.N, a.scale, obs, a.r, a.dirs, a.n_pix, k_in, v_in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int bits = order_key_bits(a.N);
  size_t need = 0;
  e = sort_pairs_u32(nullptr, &need, k_in, k_out, v_in, v_out, a.n_pix, bits, s);
  if (e != hipSuccess) return e;
  if (need > tmp_bytes) return hipErrorInvalidValue;
  e = sort_pairs_u32(tmp, &tmp_bytes, k_in, k_out, v_in, v_out, a.n_pix, bits, s);
  if (e != hipSuccess) return e;
  char* rec = (char*)a.order;
  uint32_t* pix = (uint32_t*)(rec + n * pixel_order_record_bytes(a.dtype));
  if (a.dtype == kF32) {
    auto k = cubic ? k_order_records<float, 4> : k_order_records<float, 2>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, a.N, a.scale, obs, a.r, a.dirs, a.n_pix, v_out,
                       (OrderRec<float>*)rec, pix);
  } else {
    auto k = cubic ? k_order_records<double, 4> : k_order_records<double, 2>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, a.N, a.scale, obs, a.r, a.dirs, a.n_pix, v_out,
                       (OrderRec<double>*)rec, pix);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ map footprint
// Mark what the K-point stencils of the pixels read: the 8-row block of line (ix, iy)
// and the 32-node z block (the x-planes are flagged from the row blocks afterwards, by
// k_zlist: every pixel would store into the same few bytes). Many threads store the same
// byte 1; nothing else writes it.
template <int K>
__global__ __launch_bounds__(256) void k_footprint(uint8_t* __restrict__ fp, int N, double scale, double3 obs,
                                                   double r, const double* __restrict__ dirs, int64_t npix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  int i0[3];
  double frac[3];
  stencil_origin<K>(N, scale, obs, r, dirs, i, i0, frac);
  const int nb = footprint_blocks(N);
  // z blocks: every pixel's few bytes are the same handful for the whole map, so a byte
  // already set is only read (stores from every thread to one cache line would queue)
  uint8_t* zb = fp + footprint_z_offset(N);
  int prevz = -1;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int b = wrap(i0[2] + c, N) >> 5;
    if (b != prevz && !zb[b]) zb[b] = 1;
    prevz = b;
  }
#pragma unroll
  for (int a = 0; a < K; ++a) {
    const int ix = wrap(i0[0] + a, N);
    int prev = -1;
#pragma unroll
    for (int b = 0; b < K; ++b) {
      const int blk = wrap(i0[1] + b, N) >> 3;
      if (blk != prev) fp[N + ix * nb + blk] = 1;
      prev = blk;
    }
  }
}

// Append `v` for the lanes with `need` to the list whose count is *count (one atomic per
// wave; the order among waves is not fixed).
__device__ __forceinline__ void wave_append(bool need, uint32_t v, uint32_t* count, uint32_t* list) {
  const uint64_t m = __ballot(need);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  if (need) list[base + __popcll(m & ((1ull << lane) - 1))] = v;
}

// The plane flags and the work lists: one thread per block of `lines` consecutive
// (ix, iy) lines -- a block that holds a line of a marked 8-row block goes to the z list
// -- and one per x-plane -- a plane with a marked row block is flagged and goes to the
// plane list.
__global__ __launch_bounds__(256) void k_zlist(uint8_t* __restrict__ fp, int N, int lines) {
  const int nb = footprint_blocks(N);
  const int nblk = N * N / lines;
  uint32_t* hdr = reinterpret_cast<uint32_t*>(fp + footprint_list_offset(N));
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) hdr[0] = (uint32_t)lines;
  bool need = false;
  if (b < nblk) {
    for (int l = b * lines; l < (b + 1) * lines && !need;) {
      const int iy = l % N;
      need = fp[N + (l / N) * nb + (iy >> 3)] != 0;
      l += min(8 - (iy & 7), N - iy);  // the next 8-row block, or the next plane's first
    }
  }
  wave_append(need, (uint32_t)b, &hdr[1], hdr + kFootprintHeader);
  bool plane = false;
  if (b < N) {
    // OR of the plane's row-block flags, all loads in flight together
    const uint8_t* row = fp + N + (size_t)b * nb;
    uint32_t any = 0;
#pragma unroll 16
    for (int k = 0; k < nb; ++k) any |= row[k];
    plane = any != 0;
    if (plane) fp[b] = 1;
  }
  wave_append(plane, (uint32_t)b, &hdr[2], hdr + kFootprintHeader + N * N);
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------ pipelined passes
// One launch runs the four stages of the hot path on four different realisations at once:
// pass x of item t, pass y of item t-1, pass z of item t-2 and the gather of item t-3.
// Each workgroup reads its (role, index) from a host-built schedule that interleaves the
// roles in proportion to their workgroup counts, so the ALU-bound noise workgroups share
// every CU with the HBM-bound transform and gather workgroups.
template <typename T>
struct PipeArgs {
  cpx<T>* bx;          // pass x output buffer
  const T* wtab_x;     // weights of the item in pass x
  uint32_t k0, k1;     // its seed words
  int m_hi_x, m_hi_y, m_hi_z;  // support bound of the items in passes x, y, z
  const uint8_t *fp_x, *fp_y, *fp_z;  // their map footprints (NULL: whole field)
  cpx<T>* by;          // pass y buffer
  cpx<T>* bz;          // pass z buffer
  const T* field_g;    // gather input field
  const double* dirs;  // gather directions
  const OrderRec<T>* rec;  // with fixed directions, the pixel order (records, indices), else NULL
  const uint32_t* pix;
  T* out;              // gather output
  int64_t npix;
  double r, scale;
  double3 obs;         // observer position in the box
  int cubic;
  const cpx<T>* tw;    // twiddles of this N
};

constexpr int kPipeNT = 256;

template <typename T, int N, int TX, int TY, int LZ>
struct PipeShape {
  static constexpr int M = N / 2;
  static constexpr int SX = N * TX + N + tab_cpx<T>(), SY = N * TY + N, SZ = LZ * M + N;
  static constexpr int SMEM = SX > SY ? (SX > SZ ? SX : SZ) : (SY > SZ ? SY : SZ);
};

template <typename T, int N, int TX, int TY, int LZ>
__global__ __launch_bounds__(kPipeNT) void k_pipeline(const uint32_t* __restrict__ sched, PipeArgs<T> a) {
  constexpr int M = N / 2;
  __shared__ __align__(16) cpx<T> smem[PipeShape<T, N, TX, TY, LZ>::SMEM];
  const uint32_t e = sched[blockIdx.x];
  const int role = (int)(e >> 30);
  const int idx = (int)(e & 0x3FFFFFFFu);
  if (role == 0) {
    role_x<T, N, TX, kPipeNT>(smem, idx % (M / TX), idx / (M / TX), a.bx, a.wtab_x, a.tw, a.k0, a.k1, a.m_hi_x, a.fp_x);
  } else if (role == 1) {
    const int zt = idx % (M / TY);
    int ix = idx / (M / TY);
    if (a.fp_y) {
      // with the item's plane list the index runs over (listed plane, tile)
      const uint32_t* hdr = reinterpret_cast<const uint32_t*>(a.fp_y + footprint_list_offset(N));
      if (ix >= (int)hdr[2]) return;
      ix = (int)hdr[kFootprintHeader + N * N + ix];
    }
    role_y<T, N, TY, kPipeNT>(smem, zt, ix, a.by, a.tw, a.m_hi_y, a.fp_y);
  } else if (role == 2) {
    int blk = idx;
    if (a.fp_z) {
      // with the item's z list (made for LZ) the index runs over the listed blocks
      const uint32_t* hdr = reinterpret_cast<const uint32_t*>(a.fp_z + footprint_list_offset(N));
      if (hdr[0] == (uint32_t)LZ) {
        if (idx >= (int)hdr[1]) return;
        blk = (int)hdr[kFootprintHeader + idx];
      }
    }
    role_z<T, N, LZ, kPipeNT>(smem, blk, a.bz, a.tw, a.m_hi_z, a.fp_z);
  } else {
    const int64_t i = (int64_t)idx * kPipeNT + threadIdx.x;
    if (i < a.npix) {
      if (a.rec) {
        if (a.cubic)
          gather_ordered_pixel<T, 4>(a.field_g, N, a.rec, a.pix, i, a.out);
        else
          gather_ordered_pixel<T, 2>(a.field_g, N, a.rec, a.pix, i, a.out);
      } else if (a.cubic) {
        gather_pixel<T, 4>(a.field_g, N, a.scale, a.obs, a.r, a.dirs, i, a.out);
      } else {
        gather_pixel<T, 2>(a.field_g, N, a.scale, a.obs, a.r, a.dirs, i, a.out);
      }
    }
  }
}

// ------------------------------------------------------------------ dispatch tables
namespace {

template <typename T>
constexpr int max_tz() { return sizeof(T) == 4 ? 16 : 8; }
constexpr int lds_budget() { return 72 * 1024; }

// default column tile: the largest even divisor of N/2 up to the type's maximum whose
// tile (plus twiddles) stays within the LDS budget
template <typename T>
constexpr int default_tz(int N) {
  for (int tz = max_tz<T>(); tz >= 2; tz -= 2)
    if ((N / 2) % tz == 0 && (N * tz + N) * 2 * (int)sizeof(T) <= lds_budget()) return tz;
  return 2;
}
// alternative tiles: half and a quarter of the default (kept even and dividing N/2)
constexpr int tz_choice(int d, int N, int k) {
  const int t = d >> k;
  return (t >= 2 && t % 2 == 0 && (N / 2) % t == 0) ? t : d;
}
// lines per z workgroup: about 2048 complex (FP64), dividing N^2. In FP32 smaller blocks
// (more workgroups per CU) ran the streamed pass faster: blocks of 1024 complex from
// N = 256 (eight per CU; N = 512 0.025 -> 0.021 ms with 2048, 0.020 with 1024; N = 256
// 0.0068 -> 0.0064 with 1024), 2048 below (N = 128 0.0048 -> 0.0044). Boxes of 3 x 2^k
// keep 4096 in FP32: a smaller block made N = 48's footprint maps stream, and the streamed
// kernel's radix-3 transform rounds differently from k_pass_z's (the whole field's), where
// maps made from the footprint must equal the whole field's
template <typename T>
constexpr int default_lines(int N) {
  const bool pow2 = (N & (N - 1)) == 0;
  const int target = (sizeof(T) == 8 ? 2048 : !pow2 ? 4096 : N >= 256 ? 1024 : 2048) / (N / 2);
  int l = 1;
  while (l * 2 <= target && (N * N) % (l * 2) == 0) l *= 2;
  return l;
}
// alternatives: twice (if the block stays within 8192 complex) and half the default
template <typename T>
constexpr int lines_choice(int N, int k) {
  const int d = default_lines<T>(N);
  if (k == 1) return (d * 2 * (N / 2) <= 8192 && (N * N) % (d * 2) == 0) ? d * 2 : d;
  if (k == 2) return d >= 2 ? d / 2 : d;
  return d;
}

using PassFn = hipError_t (*)(const FieldArgs&, hipStream_t);

// Tiles of the x pass within the support (as k_pass_x lists them), at least one.
inline int x_tiles_in_support(int N, int TZ, int m_hi) {
  int total = 0;
  for (int zt = 0; zt < N / 2 / TZ; ++zt) {
    const int d = m_hi - zt * TZ * zt * TZ;
    int R = -1;
    if (d >= 0) {
      R = (int)std::sqrt((double)d);
      while (R * R > d) --R;
      while ((R + 1) * (R + 1) <= d) ++R;
    }
    total += x_rows_in_support(N, TZ, zt, R);
  }
  return total > 0 ? total : 1;
}

template <typename T, int N, int TZ, int P = 0>
hipError_t run_x(const FieldArgs& a, hipStream_t s) {
  dim3 grid(x_tiles_in_support(N, TZ, a.m_hi));
  hipLaunchKernelGGL((k_pass_x<T, N, TZ, P>), grid, dim3(XYShape<T, N, TZ>::NT), 0, s, (cpx<T>*)a.buf,
                     (const T*)a.wtab, (const cpx<T>*)a.tw, a.k0, a.k1, a.m_hi, (const uint8_t*)a.fp);
  return hipGetLastError();
}
// Workgroups of `kernel` resident on the current device at once (occupancy x CUs; taken
// once per kernel, every device of a process being of one kind), 1024 if not known.
template <typename K>
int resident_grid(K kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess)
    return 1024;
  return per > 0 && cus > 0 ? per * cus : 1024;
}

template <typename T, int N, int TZ, int P = 0>
hipError_t run_y(const FieldArgs& a, hipStream_t s) {
  constexpr int NWG = N / 2 / TZ * N;
  if constexpr (P == 1) {
    // stage plan 1 walks the list with the next pair's loads in flight (k_pass_y_walk), on
    // as many workgroups as are resident; with stage plan 0 (which it would have to spill
    // at N = 256 and 512) the autotuner compares it against k_pass_y's plain walk
    if (a.fp) {
      static const int resident = resident_grid(k_pass_y_walk<T, N, TZ, P>, XYShape<T, N, TZ>::NT);
      hipLaunchKernelGGL((k_pass_y_walk<T, N, TZ, P>), dim3(resident), dim3(XYShape<T, N, TZ>::NT), 0, s,
                         (cpx<T>*)a.buf, (const cpx<T>*)a.tw, a.m_hi, (const uint8_t*)a.fp);
      return hipGetLastError();
    }
  }
  const dim3 grid = a.fp ? dim3(NWG > kZGrid ? kZGrid : NWG) : dim3(N / 2 / TZ, N);
  hipLaunchKernelGGL((k_pass_y<T, N, TZ, P>), grid, dim3(XYShape<T, N, TZ>::NT), 0, s, (cpx<T>*)a.buf,
                     (const cpx<T>*)a.tw, a.m_hi, (const uint8_t*)a.fp);
  return hipGetLastError();
}
template <typename T, int N, int LINES, int P = 0>
hipError_t run_z(const FieldArgs& a, hipStream_t s) {
  constexpr int NBLK = N * N / LINES;
  if constexpr (z_streamable<T, N, LINES, P>()) {
    // with a footprint: the streamed walk, as many workgroups as the device holds at once
    if (a.fp) {
      static const int resident = resident_grid(k_pass_z_stream<T, N, LINES, P>, ZShape<T, N, LINES>::NT);
      hipLaunchKernelGGL((k_pass_z_stream<T, N, LINES, P>), dim3(NBLK > resident ? resident : NBLK),
                         dim3(ZShape<T, N, LINES>::NT), 0, s, (cpx<T>*)a.buf, (const cpx<T>*)a.tw, a.m_hi,
                         (const uint8_t*)a.fp);
      return hipGetLastError();
    }
  }
  // a walking grid of what the device holds at once: a fixed one ran a second, partial
  // round of workgroups for blocks of 16 and 32 lines
  static const int resident = resident_grid(k_pass_z<T, N, LINES, P>, ZShape<T, N, LINES>::NT);
  dim3 grid(a.fp && NBLK > resident ? resident : NBLK);
  hipLaunchKernelGGL((k_pass_z<T, N, LINES, P>), grid, dim3(ZShape<T, N, LINES>::NT), 0, s, (cpx<T>*)a.buf,
                     (const cpx<T>*)a.tw, a.m_hi, (const uint8_t*)a.fp);
  return hipGetLastError();
}

// The x and y transforms of stacked layers (the 2-D passes of flat boxes): the y-pass
// kernel on `nlayers` planes (a transform along the middle axis of each), then the z-pass
// kernel on their nlayers N contiguous lines; neither skips anything.
using LayersFn = hipError_t (*)(void* buf, const void* tw, int nlayers, hipStream_t s);

template <typename T, int N, int TZ>
hipError_t run_y_layers(void* buf, const void* tw, int nlayers, hipStream_t s) {
  hipLaunchKernelGGL((k_pass_y<T, N, TZ>), dim3(N / 2 / TZ, nlayers), dim3(XYShape<T, N, TZ>::NT), 0, s,
                     (cpx<T>*)buf, (const cpx<T>*)tw, INT_MAX, (const uint8_t*)nullptr);
  return hipGetLastError();
}

template <typename T, int N, int LINES>
hipError_t run_z_layers(void* buf, const void* tw, int nlayers, hipStream_t s) {
  const int64_t lines = (int64_t)nlayers * N;
  if (lines % LINES) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_pass_z<T, N, LINES>), dim3((unsigned)(lines / LINES)), dim3(ZShape<T, N, LINES>::NT), 0, s,
                     (cpx<T>*)buf, (const cpx<T>*)tw, INT_MAX, (const uint8_t*)nullptr);
  return hipGetLastError();
}

constexpr int kChoices = 3;

using PipeFn = hipError_t (*)(const PipeLaunch&, hipStream_t);

template <typename T, int N, int TX, int TY, int LZ>
hipError_t run_pipe(const PipeLaunch& a, hipStream_t s) {
  PipeArgs<T> p{};
  p.bx = (cpx<T>*)a.bx;
  p.wtab_x = (const T*)a.wtab_x;
  p.k0 = a.k0;
  p.k1 = a.k1;
  p.by = (cpx<T>*)a.by;
  p.m_hi_x = a.m_hi_x;
  p.m_hi_y = a.m_hi_y;
  p.m_hi_z = a.m_hi_z;
  p.fp_x = (const uint8_t*)a.fp_x;
  p.fp_y = (const uint8_t*)a.fp_y;
  p.fp_z = (const uint8_t*)a.fp_z;
  p.bz = (cpx<T>*)a.bz;
  p.field_g = (const T*)a.field_g;
  p.dirs = a.dirs;
  if (a.order) {
    p.rec = (const OrderRec<T>*)a.order;
    p.pix = (const uint32_t*)((const char*)a.order + (size_t)a.npix * sizeof(OrderRec<T>));
  }
  p.out = (T*)a.out;
  p.npix = a.npix;
  p.r = a.r;
  p.scale = a.scale;
  p.obs = make_double3(a.obs[0], a.obs[1], a.obs[2]);
  p.cubic = a.cubic;
  p.tw = (const cpx<T>*)a.tw;
  hipLaunchKernelGGL((k_pipeline<T, N, TX, TY, LZ>), dim3(a.nblocks), dim3(kPipeNT), 0, s, a.sched, p);
  return hipGetLastError();
}

// pipelined tiles: half the default column tile (smaller LDS footprint, so more
// workgroups of mixed roles fit on a CU) and z blocks of about the same LDS size
template <typename T>
constexpr int pipe_lines(int N, int tx) {
  return (N * N) % (2 * tx) == 0 ? 2 * tx : default_lines<T>(N);
}

struct Entry {
  int dtype, N;
  int tz[kChoices];
  PassFn x[kChoices], y[kChoices];
  int lines[kChoices];
  PassFn z[kChoices];
  PassFn x1, y1, z1;     // the alternative stage plan (P = 1) at the default tiles, or nullptr

  int ptx, pty, plz;
  PipeFn pipe;
  LayersFn ylay;                   // layers' first transform, default column tile
  LayersFn zlay[kChoices + 1];     // layers' c2r, per z tile (lines[i]), then a tile dividing N
};

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

// Lengths with a second stage plan: a power-of-two part of at least 32 (smaller ones are
// one stage, whatever the plan).
constexpr bool alt_plan(int L) { return ilog2(pow2_part(L)) >= 5; }
template <typename T, int N, int TZ>
constexpr PassFn alt_x() {
  if constexpr (alt_plan(N)) return &run_x<T, N, TZ, 1>;
  else return nullptr;
}
template <typename T, int N, int TZ>
constexpr PassFn alt_y() {
  if constexpr (alt_plan(N)) return &run_y<T, N, TZ, 1>;
  else return nullptr;
}
template <typename T, int N, int LINES>
constexpr PassFn alt_z() {
  if constexpr (alt_plan(N / 2)) return &run_z<T, N, LINES, 1>;
  else return nullptr;
}

template <typename T, int N>
constexpr Entry make_entry() {
  constexpr int d = default_tz<T>(N);
  constexpr int t0 = d, t1 = tz_choice(d, N, 1), t2 = tz_choice(d, N, 2);
  constexpr int l0 = lines_choice<T>(N, 0), l1 = lines_choice<T>(N, 1), l2 = lines_choice<T>(N, 2);
  constexpr int px = t1, pz = pipe_lines<T>(N, t1);
  return Entry{sizeof(T) == 4 ? kF32 : kF64,
               N,
               {t0, t1, t2},
               {&run_x<T, N, t0>, &run_x<T, N, t1>, &run_x<T, N, t2>},
               {&run_y<T, N, t0>, &run_y<T, N, t1>, &run_y<T, N, t2>},
               {l0, l1, l2},
               {&run_z<T, N, l0>, &run_z<T, N, l1>, &run_z<T, N, l2>},
               alt_x<T, N, t0>(),
               alt_y<T, N, t0>(),
               alt_z<T, N, l0>(),
               px,
               px,
               pz,
               &run_pipe<T, N, px, px, pz>,
               &run_y_layers<T, N, t0>,
               {&run_z_layers<T, N, l0>, &run_z_layers<T, N, l1>, &run_z_layers<T, N, l2>,
                &run_z_layers<T, N, gcd_int(l0, N)>}};
}

#define CMBX_SIZES(T)                                                                                     \
  make_entry<T, 8>(), make_entry<T, 12>(), make_entry<T, 16>(), make_entry<T, 24>(), make_entry<T, 32>(), \
      make_entry<T, 48>(), make_entry<T, 64>(), make_entry<T, 96>(), make_entry<T, 128>(),                \
      make_entry<T, 192>(), make_entry<T, 256>(), make_entry<T, 384>(), make_entry<T, 512>(),             \
      make_entry<T, 768>(), make_entry<T, 1024>()

const Entry kTable[] = {CMBX_SIZES(float), CMBX_SIZES(double)};

const Entry* find(int dtype, int N) {
  for (const Entry& e : kTable)
    if (e.dtype == dtype && e.N == N) return &e;
  return nullptr;
}

int pick(const int* opts, int want) {
  if (want <= 0) return 0;
  for (int i = 0; i < kChoices; ++i)
    if (opts[i] == want) return i;
  return -1;
}

int distinct(const int* opts, int* out) {
  int n = 0;
  for (int i = 0; i < kChoices; ++i) {
    bool seen = false;
    for (int j = 0; j < n; ++j) seen = seen || out[j] == opts[i];
    if (!seen) out[n++] = opts[i];
  }
  return n;
}

}  // namespace

bool size_compiled(int N) { return find(kF32, N) != nullptr; }

int tile_xy_choices(int dtype, int N, int* out) {
  const Entry* e = find(dtype, N);
  return e ? distinct(e->tz, out) : 0;
}

int lines_z_choices(int dtype, int N, int* out) {
  const Entry* e = find(dtype, N);
  return e ? distinct(e->lines, out) : 0;
}

// The pass kernel for a tile choice and stage plan: plan 1 exists at the default tile only.
PassFn choose(const PassFn* fns, PassFn alt, int i, int plan) {
  if (i < 0) return nullptr;
  if (plan == 0) return fns[i];
  return i == 0 ? alt : nullptr;
}

hipError_t launch_pass_x(const FieldArgs& a, hipStream_t s) {
  const Entry* e = find(a.dtype, a.N);
  const PassFn f = e ? choose(e->x, e->x1, pick(e->tz, a.tile_x), a.plan_x) : nullptr;
  return f ? f(a, s) : hipErrorInvalidValue;
}
hipError_t launch_pass_y(const FieldArgs& a, hipStream_t s) {
  const Entry* e = find(a.dtype, a.N);
  const PassFn f = e ? choose(e->y, e->y1, pick(e->tz, a.tile_y), a.plan_y) : nullptr;
  return f ? f(a, s) : hipErrorInvalidValue;
}
hipError_t launch_pass_z(const FieldArgs& a, hipStream_t s) {
  const Entry* e = find(a.dtype, a.N);
  const PassFn f = e ? choose(e->z, e->z1, pick(e->lines, a.lines_z), a.plan_z) : nullptr;
  return f ? f(a, s) : hipErrorInvalidValue;
}

bool stage_plan_compiled(int dtype, int N, int which) {
  const Entry* e = find(dtype, N);
  if (!e) return false;
  return (which == 0 ? e->x1 : which == 1 ? e->y1 : e->z1) != nullptr;
}

bool pipeline_shape(int dtype, int N, int* tx, int* ty, int* lz) {
  const Entry* e = find(dtype, N);
  if (!e) return false;
  *tx = e->ptx;
  *ty = e->pty;
  *lz = e->plz;
  return true;
}

hipError_t launch_pipeline(const PipeLaunch& a, hipStream_t s) {
  const Entry* e = find(a.dtype, a.N);
  if (!e || a.nblocks < 1) return hipErrorInvalidValue;
  return e->pipe(a, s);
}

hipError_t launch_layers_c2c(int dtype, int N, void* buf, const void* tw, int nlayers, hipStream_t s) {
  const Entry* e = find(dtype, N);
  if (!e || nlayers < 1) return hipErrorInvalidValue;
  return e->ylay(buf, tw, nlayers, s);
}

hipError_t launch_layers_c2r(int dtype, int N, void* buf, const void* tw, int nlayers, hipStream_t s) {
  const Entry* e = find(dtype, N);
  if (!e || nlayers < 1) return hipErrorInvalidValue;
  for (int i = 0; i < kChoices; ++i)  // the first z tile that divides the layers' lines
    if (((int64_t)nlayers * N) % e->lines[i] == 0) return e->zlay[i](buf, tw, nlayers, s);
  return e->zlay[kChoices](buf, tw, nlayers, s);  // a tile that divides N
}

bool layers_supported(int dtype, int N, int nlayers) { return find(dtype, N) != nullptr && nlayers >= 1; }

hipError_t noise_table_address(const float** out) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_bm_tab));
  *out = static_cast<const float*>(p);
  return e;
}

// The device copy of the tables: the reciprocals 1 / c_j times 2^-23 (exact), which
// box_muller_f32 multiplies by the integer mi mod 2^16 instead of by m - c_j.
hipError_t upload_noise_tables(const float* host) {
  float dev[bmf::kTabSize];
  for (int i = 0; i < bmf::kTabSize; ++i) dev[i] = host[i];
  for (int j = 0; j < 128; ++j) dev[bmf::kTabInv + j] = std::ldexp(host[bmf::kTabInv + j], -23);
  return hipMemcpyToSymbol(HIP_SYMBOL(g_bm_tab), dev, sizeof(float) * bmf::kTabSize, 0, hipMemcpyHostToDevice);
}

hipError_t launch_noise_debug(int dtype, int N, void* out, const void* wtab, uint32_t k0, uint32_t k1,
                              hipStream_t s) {
  const int64_t total = (int64_t)N * N * (N / 2 + 1);
  const dim3 grid((unsigned)((total + 255) / 256));
  if (dtype == kF32)
    hipLaunchKernelGGL(k_noise_debug<float>, grid, dim3(256), 0, s, (cpx<float>*)out, N, (const float*)wtab, k0, k1);
  else
    hipLaunchKernelGGL(k_noise_debug<double>, grid, dim3(256), 0, s, (cpx<double>*)out, N, (const double*)wtab, k0,
                       k1);
  return hipGetLastError();
}

hipError_t launch_footprint(const FootprintArgs& a, hipStream_t s) {
  if (a.lines < 1 || (a.N * a.N) % a.lines) return hipErrorInvalidValue;
  const int64_t words = (int64_t)(footprint_list_offset(a.N) / 4) + kFootprintHeader;  // marks + header
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (uint32_t*)a.fp, words);
  const dim3 grid((unsigned)((a.n_pix + 255) / 256));
  if (a.interp == kTricubic)
    hipLaunchKernelGGL(k_footprint<4>, grid, dim3(256), 0, s, (uint8_t*)a.fp, a.N, a.scale, make_double3(a.obs[0], a.obs[1], a.obs[2]), a.r, a.dirs,
                       a.n_pix);
  else
    hipLaunchKernelGGL(k_footprint<2>, grid, dim3(256), 0, s, (uint8_t*)a.fp, a.N, a.scale, make_double3(a.obs[0], a.obs[1], a.obs[2]), a.r, a.dirs,
                       a.n_pix);
  const int threads = a.N * a.N / a.lines > a.N ? a.N * a.N / a.lines : a.N;  // per z block, and per plane
  hipLaunchKernelGGL(k_zlist, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, (uint8_t*)a.fp, a.N,
                     a.lines);
  return hipGetLastError();
}

int resolve_tile_xy(int dtype, int N, int tile) {
  const Entry* e = find(dtype, N);
  const int i = e ? pick(e->tz, tile) : -1;
  return i < 0 ? 0 : e->tz[i];
}

int resolve_lines_z(int dtype, int N, int lines_z) {
  const Entry* e = find(dtype, N);
  const int i = e ? pick(e->lines, lines_z) : -1;
  return i < 0 ? 0 : e->lines[i];
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  int64_t nb = (a.n_pix + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid((unsigned)nb);
  const bool cubic = a.interp == kTricubic;
  if (a.order) {
    const size_t n = (size_t)a.n_pix;
    const char* rec = (const char*)a.order;
    const uint32_t* pix = (const uint32_t*)(rec + n * pixel_order_record_bytes(a.dtype));
    if (a.dtype == kF32) {
      auto k = cubic ? k_gather_ordered<float, 4> : k_gather_ordered<float, 2>;
      hipLaunchKernelGGL(k, grid, dim3(256), 0, s, (const float*)a.field, a.N, (const OrderRec<float>*)rec, pix,
                         a.n_pix, (float*)a.out);
    } else {
      auto k = cubic ? k_gather_ordered<double, 4> : k_gather_ordered<double, 2>;
      hipLaunchKernelGGL(k, grid, dim3(256), 0, s, (const double*)a.field, a.N, (const OrderRec<double>*)rec, pix,
                         a.n_pix, (double*)a.out);
    }
    return hipGetLastError();
  }
  if (a.dtype == kF32) {
    auto k = cubic ? k_gather<float, 4> : k_gather<float, 2>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, (const float*)a.field, a.N, a.scale, make_double3(a.obs[0], a.obs[1], a.obs[2]), a.r, a.dirs, a.n_pix,
                       (float*)a.out);
  } else {
    auto k = cubic ? k_gather<double, 4> : k_gather<double, 2>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, (const double*)a.field, a.N, a.scale, make_double3(a.obs[0], a.obs[1], a.obs[2]), a.r, a.dirs,
                       a.n_pix, (double*)a.out);
  }
  return hipGetLastError();
}

}  // namespace cmbx
