// Column stage of flat boxes and the gather from stacked layers, for gfx950.
//
// Flat box N x N x M (Sec. II C, eq. finalpbox): the 3-D Fourier method (Sec. II D 1) draws
// every mode of the half grid in y and transforms along z first (this file), then along x
// and y (the layer passes of kernels.hip). The 2-D (hybrid) Fourier method (Sec. II D 2)
// draws, for every column (k_x, k_y), h correlated values S g at heights z_0 .. z_{h-1}
// from one precomputed factor S with S S^T = Gamma (this file), then runs the same x and y
// passes on its h layers.
#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "noise_device.hpp"
#include "slab.hpp"

namespace cmbx {
namespace {

__device__ __forceinline__ int fq(int i, int n) { return i <= n - i ? i : n - i; }

constexpr int slab_nt(int work) { return work >= 4096 ? 512 : work >= 2048 ? 256 : work >= 1024 ? 128 : 64; }
constexpr int kTabFloats = 768;  // binary32 Box-Muller tables (noise_device.hpp layout)

template <typename T>
__device__ __forceinline__ const float* stage_tab(float* lds, const float* __restrict__ g, int tid, int nt) {
  if constexpr (sizeof(T) == 4) {
    for (int i = tid; i < kTabFloats; i += nt) lds[i] = g[i];
    return lds;
  } else {
    return nullptr;
  }
}

// ------------------------------------------------------------------ flat box modes
// Mode (ix, iy, iz), iy = 0 .. N/2, of the half grid in y: Philox counter (iz >> 1, iy, ix, 2),
// words (x0, x1) for even iz and (x2, x3) for odd; generic modes half[row(s)][|fz|] (g_re + i g_im);
// on the planes iy = 0 and N/2 the mode and (-ix, -iz) are conjugate, the smaller ix M + iz
// drawn; the self-conjugate modes are real, full[2 c + (iz == M/2)] g_re with c the number
// of x, y indices equal to N/2. Zero weight: +0 (then conjugated like any value).
template <typename T>
__device__ __forceinline__ cpx<T> flat_mode(int N, int MZ, int ix, int iy, int iz, uint32_t k0, uint32_t k1,
                                            const int* __restrict__ sidx, const T* __restrict__ half,
                                            const T* __restrict__ full, const float* __restrict__ tab) {
  const int fx = fq(ix, N), fy = fq(iy, N), fz = fq(iz, MZ);
  int dx = ix, dz = iz;
  bool cj = false, self = false;
  if (iy == 0 || iy == N / 2) {
    const int px = ix == 0 ? 0 : N - ix, pz = iz == 0 ? 0 : MZ - iz;
    const int own = ix * MZ + iz, par = px * MZ + pz;
    if (own == par) {
      self = true;
    } else if (own > par) {
      dx = px;
      dz = pz;
      cj = true;
    }
  }
  const T w = self ? full[2 * ((ix == N / 2) + (iy == N / 2)) + (iz == MZ / 2)]
                   : half[(size_t)sidx[fx * fx + fy * fy] * (MZ / 2 + 1) + fz];
  if (w == T(0)) {
    const cpx<T> z = {T(0), T(0)};
    return cj ? conj(z) : z;
  }
  const uint2 wd = [&] {
    const uint4 q = philox4x32_10(make_uint4((uint32_t)dz >> 1, (uint32_t)iy, (uint32_t)dx, 2u), k0, k1);
    return (dz & 1) ? make_uint2(q.z, q.w) : make_uint2(q.x, q.y);
  }();
  T gr, gi;
  normal_pair(wd.x, wd.y, gr, gi, tab);
  if (self) return {w * gr, T(0)};
  const cpx<T> v = {w * gr, w * gi};
  return cj ? conj(v) : v;
}

// Element n of column q at p[n * stride + q] (the layers: n is the layer, q the packed y
// column), for the first ncols columns (a ragged last tile).
template <typename T>
struct ColumnWriter {
  cpx<T>* p;
  size_t stride;
  int ncols;
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const {
    if (q < ncols) p[(size_t)n * stride + q] = v;
  }
  __device__ __forceinline__ void done() const {}
};

// Workgroup = (ix, C consecutive packed y columns; the last tile of a row may hold fewer,
// the rest transform zeros and are not written): the C x MZ modes into LDS (one Philox
// call per pair of neighbouring iz; column 0 packs the planes iy = 0 and N/2 as A + i B),
// the length-MZ inverse transform along z, and layer n of every column written (C
// consecutive complex per layer).
template <typename T, int MZ, int C>
__global__ __launch_bounds__(slab_nt(MZ * C)) void k_flat_columns(cpx<T>* __restrict__ buf, int N,
                                                                  const int* __restrict__ sidx,
                                                                  const T* __restrict__ half,
                                                                  const T* __restrict__ full,
                                                                  const cpx<T>* __restrict__ twz, uint32_t k0,
                                                                  uint32_t k1, const float* __restrict__ bmg) {
  constexpr int NT = slab_nt(MZ * C);
  __shared__ cpx<T> tile[C * MZ];
  __shared__ cpx<T> tw[MZ];
  __shared__ float tabl[sizeof(T) == 4 ? kTabFloats : 1];
  using Lds = LdsIO<T, MZ, C, true>;
  const int tid = threadIdx.x;
  const int M2 = N / 2;
  const int tiles = (M2 + C - 1) / C;
  const int ix = blockIdx.x / tiles;
  const int c0 = (blockIdx.x % tiles) * C;
  const int ncols = M2 - c0 < C ? M2 - c0 : C;
  for (int i = tid; i < MZ; i += NT) tw[i] = twz[i];
  const float* tab = stage_tab<T>(tabl, bmg, tid, NT);
  __syncthreads();
  const int fx = fq(ix, N);
  for (int s = tid; s < C * (MZ / 2); s += NT) {
    const int q = s % C, pz = s / C;
    const int iyc = c0 + q, iz0 = 2 * pz;
    cpx<T> v[2];
    if (q >= ncols) {
      v[0] = v[1] = {T(0), T(0)};
    } else if (iyc == 0) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const cpx<T> a = flat_mode<T>(N, MZ, ix, 0, iz0 + t, k0, k1, sidx, half, full, tab);
        const cpx<T> b = flat_mode<T>(N, MZ, ix, M2, iz0 + t, k0, k1, sidx, half, full, tab);
        v[t] = {a.x - b.y, a.y + b.x};
      }
    } else {
      const T* row = half + (size_t)sidx[fx * fx + iyc * iyc] * (MZ / 2 + 1);
      const uint4 w = philox4x32_10(make_uint4((uint32_t)pz, (uint32_t)iyc, (uint32_t)ix, 2u), k0, k1);
      v[0] = weighted<T>(row[fq(iz0, MZ)], w.x, w.y, tab);
      v[1] = weighted<T>(row[fq(iz0 + 1, MZ)], w.z, w.w, tab);
    }
    tile[Lds::index(q, iz0)] = v[0];
    tile[Lds::index(q, iz0 + 1)] = v[1];
  }
  __syncthreads();
  Lds first{tile};
  ColumnWriter<T> last{buf + (size_t)ix * M2 + c0, (size_t)N * M2, ncols};
  fft_run<T, MZ, C, NT, true, 1, 0>(tw, tile, first, last, tid);
}

// Unpacked modes [N][N/2+1][M] (tests): one thread per mode.
template <typename T>
__global__ __launch_bounds__(256) void k_flat_modes_debug(cpx<T>* __restrict__ out, int N, int MZ,
                                                          const int* __restrict__ sidx, const T* __restrict__ half,
                                                          const T* __restrict__ full, uint32_t k0, uint32_t k1,
                                                          const float* __restrict__ bmg) {
  __shared__ float tabl[sizeof(T) == 4 ? kTabFloats : 1];
  const float* tab = stage_tab<T>(tabl, bmg, threadIdx.x, 256);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)N * (N / 2 + 1) * MZ;
  if (i >= total) return;
  const int iz = (int)(i % MZ);
  const int64_t t = i / MZ;
  const int iy = (int)(t % (N / 2 + 1));
  const int ix = (int)(t / (N / 2 + 1));
  out[i] = flat_mode<T>(N, MZ, ix, iy, iz, k0, k1, sidx, half, full, tab);
}

// ------------------------------------------------------------------ hybrid columns
// Column (ix, iy), iy = 0 .. N/2, of the 2-D method: h unit normal pairs, layer j from the
// Philox counter (j >> 1, iy, ix, 1) (words (x0, x1) for even j, (x2, x3) for odd), times
// the factor: v = F g with F the row's S / sqrt2 for a generic column, the real part only
// with S for the four self-conjugate columns; on the rows iy = 0 and N/2 the columns (ix)
// and (-ix) are conjugate, the smaller ix drawn. Sums over m in order, in T.
//
// One thread per (column, layer). Workgroup = the rows ix = g and N - g (one row for g = 0
// and N/2) and a block of columns: CB consecutive iy < N/2 (128-byte aligned rows of the
// packed layers), or, in the last block, the pair iy = 0 and N/2 whose packed sum A + i B
// is column 0 (column 0 is then written by the pair block only; with `unpacked` every
// (ix, iy) is written to its own place). The two rows share |k_x| and so every column's
// factor: each group of 2 HMAX threads loads one factor into registers, the loads stay in
// flight while the normal pairs are drawn, and the factors are then stored to LDS and read
// only there. Thread (q, r, c) draws the normal pair of layer q of column c in row r and
// forms row q of the factor times the column's pair vector.
template <typename T, int HMAX>
struct HybridShape {
  static constexpr int NT = 512;
  static constexpr int CB = NT / (2 * HMAX);  // columns per workgroup
  static constexpr int FS = HMAX * HMAX + 1;  // largest LDS stride of a factor
  static constexpr int PER = HMAX / 2;        // factor elements per thread
  static_assert(CB >= 2, "the packed pair shares a workgroup");
};

template <typename T, int HMAX>
__global__ __launch_bounds__(512) void k_hybrid_columns(cpx<T>* __restrict__ buf, int N, int h,
                                                        const int* __restrict__ sidx, const T* __restrict__ S,
                                                        const T* __restrict__ Sfull, uint32_t k0, uint32_t k1,
                                                        const float* __restrict__ bmg, int unpacked) {
  using Sh = HybridShape<T, HMAX>;
  constexpr int NT = Sh::NT, CB = Sh::CB;
  __shared__ float tabl[sizeof(T) == 4 ? kTabFloats : 1];
  __shared__ T fac[CB * Sh::FS];
  __shared__ T gr[HMAX][2][CB], gi[HMAX][2][CB];
  const int tid = threadIdx.x;
  const int M2 = N / 2;
  const int g = blockIdx.y;
  const int hh = h * h, fs = hh | 1;  // odd stride: the CB factors start in different banks
  const bool pairblk = (int)blockIdx.x == (M2 + CB - 1) / CB;
  // column iy of block position p; false if the position holds none
  auto column = [&](int p, int& iy) {
    if (pairblk) {
      iy = p == 0 ? 0 : M2;
      return p < 2;
    }
    iy = (int)blockIdx.x * CB + p;
    return iy < M2;
  };
  // the tables first: a wait for one of their loads would also wait for the factors'
  const float* tab = stage_tab<T>(tabl, bmg, tid, NT);
  const int fc = tid / (2 * HMAX), li = tid % (2 * HMAX);
  int fiy;
  const bool fload = column(fc, fiy);
  // self-conjugate columns: iy and ix = g both 0 or N/2 (without a column: any factor,
  // loaded and not stored); indices clamped into the factor, so no load waits on a branch
  const bool fself = (fiy == 0 || fiy == M2) && (g == 0 || g == M2);
  const T* src = !fload ? S
                 : fself ? Sfull + (size_t)((g == M2) + (fiy == M2)) * hh
                         : S + (size_t)sidx[g * g + fiy * fiy] * hh;
  T fv[Sh::PER];
#pragma unroll
  for (int k = 0; k < Sh::PER; ++k) {
    const int e = li + 2 * HMAX * k;
    fv[k] = src[e < hh ? e : hh - 1];
  }
  const int c = tid % CB, r = (tid / CB) & 1, q = tid / (2 * CB);
  int iy;
  const bool col = column(c, iy);
  const int ix = r ? N - g : g;
  const bool live = col && (r == 0 || (g > 0 && g < M2)) && q < h;
  const bool rowc = iy == 0 || iy == M2;
  const int px = ix == 0 ? 0 : N - ix;
  const bool self = rowc && ix == px;
  const bool flip = rowc && ix > px;
  lds_barrier();  // the staged tables (the factor loads stay in flight)
  T a = T(0), b = T(0);
  if (live) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)(q >> 1), (uint32_t)iy, (uint32_t)(flip ? px : ix), 1u), k0, k1);
    if (q & 1) normal_pair(w.z, w.w, a, b, tab);
    else normal_pair(w.x, w.y, a, b, tab);
  }
  if (fload) {
#pragma unroll
    for (int k = 0; k < Sh::PER; ++k)
      if (li + 2 * HMAX * k < hh) fac[fc * fs + li + 2 * HMAX * k] = fv[k];
  }
  gr[q][r][c] = a;
  gi[q][r][c] = b;
  __syncthreads();
  T ar = T(0), ai = T(0);
  if (live) {
    const T* F = fac + c * fs + q * h;
#pragma unroll
    for (int m = 0; m < HMAX; ++m) {
      if (m < h) {
        const T f = F[m];
        ar += f * gr[m][r][c];
        ai += f * gi[m][r][c];
      }
    }
  }
  const T vi = self ? T(0) : (flip ? -ai : ai);
  const int W = unpacked ? M2 + 1 : M2;
  const size_t at = ((size_t)q * N + ix) * W + iy;
  if (!pairblk) {  // uniform; packed column 0 comes from the pair block
    if (live && (unpacked || iy != 0)) buf[at] = {ar, vi};
    return;
  }
  if (unpacked) {  // uniform: (ix, 0) was written by the first block
    if (live && c == 1) buf[at] = {ar, vi};
    return;
  }
  __syncthreads();  // every thread has read the normals: gr, gi take the results
  gr[q][r][c] = ar;
  gi[q][r][c] = vi;
  __syncthreads();
  if (live && c == 0) buf[((size_t)q * N + ix) * W] = {ar - gi[q][r][1], vi + gr[q][r][1]};
}

// ------------------------------------------------------------------ layer gather
template <typename T>
__device__ __forceinline__ void keys_or_linear(T f, T* w, bool cubic) {
  if (cubic) {  // Keys cubic convolution, a = -1/2, at distances 1 + f, f, 1 - f, 2 - f
    w[0] = f * (T(-0.5) + f * (T(1.0) - T(0.5) * f));
    w[1] = T(1.0) + f * f * (T(-2.5) + T(1.5) * f);
    w[2] = f * (T(0.5) + f * (T(2.0) - T(1.5) * f));
    w[3] = f * f * (T(-0.5) + T(0.5) * f);
  } else {
    w[0] = T(1.0) - f;
    w[1] = f;
  }
}

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T, int K>
struct SlabTaps {
  typedef T vec __attribute__((ext_vector_type(K), aligned(sizeof(T))));
};

// One thread per pixel: p = (r n + o) (1 / dp) in FP64, floor(p) picks the stencil; x and y
// wrap modulo N; z wraps modulo nz, or (non-periodic layers) the pixel is NaN when its
// stencil leaves [0, nz). Weights and sums in T; the K taps along y (contiguous) are one
// vector load unless they wrap.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_slab_gather(const T* __restrict__ field, int N, int nz, int periodic,
                                                     double scale, double3 obs, double r,
                                                     const double* __restrict__ dirs, int64_t npix,
                                                     T* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npix) return;
  const double o[3] = {obs.x, obs.y, obs.z};
  int i0[3];
  T w[3][4];
  bool inside = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double p = (r * dirs[3 * i + d] + o[d]) * scale;
    if (!(p > -1.0e9 && p < 1.0e9)) p = 0.0;
    const double fl = floor(p);
    const int n = d < 2 ? N : nz;
    if (d < 2 || periodic) {
      int base = (int)fl % n;
      base = base < 0 ? base + n : base;
      i0[d] = base - (K == 4 ? 1 : 0);
    } else {
      i0[d] = (int)fl - (K == 4 ? 1 : 0);
      inside = i0[d] >= 0 && i0[d] + K <= nz;
    }
    keys_or_linear<T>((T)(p - fl), w[d], K == 4);
  }
  if (!inside) {
    out[i] = __builtin_nan("");
    return;
  }
  const bool contiguous = i0[1] >= 0 && i0[1] + K <= N;
  // every tap is loaded before any is summed: the K x K row loads are in flight together
  T q[K][K][K];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int iz = periodic ? wrapn(i0[2] + c, nz) : i0[2] + c;
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const T* row = field + ((size_t)iz * N + wrapn(i0[0] + a, N)) * N;
      if (contiguous) {
        const typename SlabTaps<T, K>::vec v = *reinterpret_cast<const typename SlabTaps<T, K>::vec*>(row + i0[1]);
#pragma unroll
        for (int b = 0; b < K; ++b) q[c][a][b] = v[b];
      } else {
#pragma unroll
        for (int b = 0; b < K; ++b) q[c][a][b] = row[wrapn(i0[1] + b, N)];
      }
    }
  }
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < K; ++c) {
    T accz = T(0);
#pragma unroll
    for (int a = 0; a < K; ++a) {
      T s = T(0);
#pragma unroll
      for (int b = 0; b < K; ++b) s += w[1][b] * q[c][a][b];
      accz += w[0][a] * s;
    }
    acc += w[2][c] * accz;
  }
  out[i] = acc;
}

// ------------------------------------------------------------------ direct gather
// The gather for few pixels without the layers' last transform: after the transform
// along x, line (z, x) of a layer holds the half spectrum along y, X_0 .. X_{N/2-1}
// (X_0 = a + i b packs the real X_0 = a and X_{N/2} = b), and the layer's value at y is its
// inverse DFT a + (-1)^y b + 2 sum_{k=1}^{N/2-1} (Re X_k cos(2 pi k y / N) - Im X_k sin(2 pi
// k y / N)) -- what the complex-to-real pass computes for every y, evaluated here only at
// the stencil's K rows (an output-pruned transform; the twiddles are the plan's N roots).
// Workgroup = one pixel, K waves; wave a takes the stencil's line x = i0x + a at each of the
// K layers: lane l takes the terms k = l, l + 64, ... (all its loads, line values and
// twiddles, issued before the first product), weights its K x K partial row sums by the y
// and z weights, and the wave's lanes are summed by shuffles; the waves' K sums are then
// weighted along x. The same weighted sum as k_slab_gather, in another order.
template <typename T, int K, int TMAX>
__global__ __launch_bounds__(64 * K) void k_slab_direct(const cpx<T>* __restrict__ layers, const cpx<T>* __restrict__ tw,
                                                         int N, int nz, int periodic, double scale, double3 obs, double r,
                                                         const double* __restrict__ dirs, int64_t npix, T* __restrict__ out) {
#pragma clang fp contract(off)
  // TMAX: terms per lane, 64 TMAX >= N / 2
  const int64_t i = blockIdx.x;
  if (i >= npix) return;
  __shared__ T part[K];  // the y- and z-weighted sum of the stencil's line x = i0x + a
  const int lane = threadIdx.x & 63, a = threadIdx.x >> 6;
  const double o[3] = {obs.x, obs.y, obs.z};
  const double n[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
  int i0[3];
  T w[3][4];
  bool inside = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double p = (r * n[d] + o[d]) * scale;
    if (!(p > -1.0e9 && p < 1.0e9)) p = 0.0;
    const double fl = floor(p);
    const int m = d < 2 ? N : nz;
    if (d < 2 || periodic) {
      int base = (int)fl % m;
      base = base < 0 ? base + m : base;
      i0[d] = base - (K == 4 ? 1 : 0);
    } else {
      i0[d] = (int)fl - (K == 4 ? 1 : 0);
      inside = i0[d] >= 0 && i0[d] + K <= nz;
    }
    keys_or_linear<T>((T)(p - fl), w[d], K == 4);
  }
  if (!inside) {  // uniform over the workgroup
    if (threadIdx.x == 0) out[i] = __builtin_nan("");
    return;
  }
  const int M = N / 2;
  const int x = wrapn(i0[0] + a, N);
  int y[K];
#pragma unroll
  for (int b = 0; b < K; ++b) y[b] = wrapn(i0[1] + b, N);
  const cpx<T>* line[K];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int z = periodic ? wrapn(i0[2] + c, nz) : i0[2] + c;
    line[c] = layers + ((size_t)z * N + x) * M;
  }
  // every load first: the lane's terms of the K lines and their twiddles w^(k y_b)
  cpx<T> X[TMAX][K], e[TMAX][K];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    const int k = lane + 64 * t;
    if (k < M) {
#pragma unroll
      for (int c = 0; c < K; ++c) X[t][c] = line[c][k];
#pragma unroll
      for (int b = 0; b < K; ++b) e[t][b] = tw[(k * y[b]) % N];
    }
  }
  T q = T(0);
#pragma unroll
  for (int c = 0; c < K; ++c) {
    T sc = T(0);
#pragma unroll
    for (int b = 0; b < K; ++b) {
      T acc = T(0);
#pragma unroll
      for (int t = 0; t < TMAX; ++t) {
        const int k = lane + 64 * t;
        if (k < M && k > 0) acc += X[t][c].x * e[t][b].x - X[t][c].y * e[t][b].y;
      }
      sc += w[1][b] * acc;
    }
    q += w[2][c] * sc;
  }
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  if (lane == 0) {
    // the terms k = 0 and N/2, packed in column 0: a + (-1)^y b
    T q0 = T(0);
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const cpx<T> X0 = line[c][0];
      T sc = T(0);
#pragma unroll
      for (int b = 0; b < K; ++b) sc += w[1][b] * (X0.x + ((y[b] & 1) ? -X0.y : X0.y));
      q0 += w[2][c] * sc;
    }
    part[a] = q0 + T(2) * q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = T(0);
#pragma unroll
    for (int aa = 0; aa < K; ++aa) acc += w[0][aa] * part[aa];
    out[i] = acc;
  }
}

template <typename T, int K>
hipError_t run_slab_direct_k(const SlabGatherArgs& a, const void* tw, hipStream_t s) {
  const int M = a.N / 2;
  auto k = M <= 64 ? k_slab_direct<T, K, 1> : M <= 128 ? k_slab_direct<T, K, 2> : M <= 256 ? k_slab_direct<T, K, 4>
                                                                                             : k_slab_direct<T, K, 8>;
  hipLaunchKernelGGL(k, dim3((unsigned)a.n_pix), dim3(64 * K), 0, s, (const cpx<T>*)a.field, (const cpx<T>*)tw, a.N,
                     a.nz, a.periodic_z, a.scale, make_double3(a.obs[0], a.obs[1], a.obs[2]), a.r, a.dirs, a.n_pix,
                     (T*)a.out);
  return hipGetLastError();
}

hipError_t run_slab_direct(const SlabGatherArgs& a, const void* tw, hipStream_t s) {
  const bool cubic = a.interp == 2;
  if (a.dtype == 1) return cubic ? run_slab_direct_k<float, 4>(a, tw, s) : run_slab_direct_k<float, 2>(a, tw, s);
  return cubic ? run_slab_direct_k<double, 4>(a, tw, s) : run_slab_direct_k<double, 2>(a, tw, s);
}

// ------------------------------------------------------------------ dispatch
template <typename T, int MZ>
constexpr int flat_cols() {
  // columns per workgroup: from 16 (FP32) / 8 (FP64), doubled up to 256 while the tile holds
  // fewer than 2048 modes (shallow boxes: four waves share the staged tables), halved while
  // the tile exceeds 64 KB
  int c = sizeof(T) == 4 ? 16 : 8;
  while (c < 256 && c * MZ < 2048) c *= 2;
  while (c > 1 && c * MZ * (int)sizeof(cpx<T>) > 65536) c /= 2;
  return c;
}

template <typename T, int MZ>
hipError_t run_flat(const SlabColumnsArgs& a, hipStream_t s) {
  constexpr int C = flat_cols<T, MZ>();
  const int tiles = (a.N / 2 + C - 1) / C;
  const T* half = (const T*)a.table;
  const T* full = half + (size_t)a.rows * (MZ / 2 + 1);
  hipLaunchKernelGGL((k_flat_columns<T, MZ, C>), dim3((unsigned)(a.N * tiles)), dim3(slab_nt(MZ * C)), 0, s,
                     (cpx<T>*)a.buf, a.N, a.sidx, half, full, (const cpx<T>*)a.twz, a.k0, a.k1, a.bm_tab);
  return hipGetLastError();
}

using FlatFn = hipError_t (*)(const SlabColumnsArgs&, hipStream_t);
struct FlatEntry {
  int M;
  FlatFn f32, f64;
};
#define CMBX_FLAT(MZ) FlatEntry{MZ, &run_flat<float, MZ>, &run_flat<double, MZ>}
const FlatEntry kFlat[] = {CMBX_FLAT(8),   CMBX_FLAT(12),  CMBX_FLAT(16),  CMBX_FLAT(24),  CMBX_FLAT(32),
                           CMBX_FLAT(48),  CMBX_FLAT(64),  CMBX_FLAT(96),  CMBX_FLAT(128), CMBX_FLAT(192),
                           CMBX_FLAT(256), CMBX_FLAT(384), CMBX_FLAT(512)};
#undef CMBX_FLAT

const FlatEntry* find_flat(int M) {
  for (const FlatEntry& e : kFlat)
    if (e.M == M) return &e;
  return nullptr;
}

template <typename T, int HMAX>
hipError_t run_hybrid_h(const SlabColumnsArgs& a, int unpacked, hipStream_t s) {
  const T* S = (const T*)a.table;
  const T* Sfull = S + (size_t)a.rows * a.h * a.h;
  using Sh = HybridShape<T, HMAX>;
  const int M2 = a.N / 2;
  const dim3 grid((unsigned)((M2 + Sh::CB - 1) / Sh::CB + 1), (unsigned)(M2 + 1));  // + the pair block
  hipLaunchKernelGGL((k_hybrid_columns<T, HMAX>), grid, dim3(Sh::NT), 0, s, (cpx<T>*)a.buf, a.N, a.h, a.sidx, S,
                     Sfull, a.k0, a.k1, a.bm_tab, unpacked);
  return hipGetLastError();
}

template <typename T>
hipError_t run_hybrid(const SlabColumnsArgs& a, int unpacked, hipStream_t s) {
  return a.h <= 16 ? run_hybrid_h<T, 16>(a, unpacked, s) : run_hybrid_h<T, kSlabMaxLayers>(a, unpacked, s);
}

}  // namespace

bool slab_depth_compiled(int M) { return find_flat(M) != nullptr; }

hipError_t launch_slab_columns(const SlabColumnsArgs& a, hipStream_t s) {
  if (a.method == kSlabHybrid) {
    if (a.h < 1 || a.h > kSlabMaxLayers) return hipErrorInvalidValue;
    return a.dtype == 1 ? run_hybrid<float>(a, 0, s) : run_hybrid<double>(a, 0, s);
  }
  const FlatEntry* e = find_flat(a.M);
  if (!e) return hipErrorInvalidValue;
  return a.dtype == 1 ? e->f32(a, s) : e->f64(a, s);
}

hipError_t launch_slab_columns_debug(const SlabColumnsArgs& a, hipStream_t s) {
  if (a.method == kSlabHybrid) {
    if (a.h < 1 || a.h > kSlabMaxLayers) return hipErrorInvalidValue;
    return a.dtype == 1 ? run_hybrid<float>(a, 1, s) : run_hybrid<double>(a, 1, s);
  }
  const int64_t total = (int64_t)a.N * (a.N / 2 + 1) * a.M;
  const dim3 grid((unsigned)((total + 255) / 256));
  const size_t hs = (size_t)a.rows * (a.M / 2 + 1);
  if (a.dtype == 1)
    hipLaunchKernelGGL(k_flat_modes_debug<float>, grid, dim3(256), 0, s, (cpx<float>*)a.buf, a.N, a.M, a.sidx,
                       (const float*)a.table, (const float*)a.table + hs, a.k0, a.k1, a.bm_tab);
  else
    hipLaunchKernelGGL(k_flat_modes_debug<double>, grid, dim3(256), 0, s, (cpx<double>*)a.buf, a.N, a.M, a.sidx,
                       (const double*)a.table, (const double*)a.table + hs, a.k0, a.k1, a.bm_tab);
  return hipGetLastError();
}

hipError_t launch_slab_gather(const SlabGatherArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n_pix + 255) / 256));
  const double3 o = make_double3(a.obs[0], a.obs[1], a.obs[2]);
  const bool cubic = a.interp == 2;
  if (a.dtype == 1) {
    auto k = cubic ? k_slab_gather<float, 4> : k_slab_gather<float, 2>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, (const float*)a.field, a.N, a.nz, a.periodic_z, a.scale, o, a.r,
                       a.dirs, a.n_pix, (float*)a.out);
  } else {
    auto k = cubic ? k_slab_gather<double, 4> : k_slab_gather<double, 2>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, (const double*)a.field, a.N, a.nz, a.periodic_z, a.scale, o, a.r,
                       a.dirs, a.n_pix, (double*)a.out);
  }
  return hipGetLastError();
}

hipError_t launch_slab_direct(const SlabGatherArgs& a, const void* tw, hipStream_t s) {
  return run_slab_direct(a, tw, s);
}

}  // namespace cmbx
