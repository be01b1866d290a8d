// C ABI of slab plans: flat N x N x M boxes with the 3-D Fourier method, and the 2-D
// (hybrid) Fourier method on h layers (see include/cmbx.h for the contract). Host side:
// argument checks, the FP64 per-column tables (weights, or the symmetric square roots of
// the column covariances by Jacobi eigendecomposition), and the launch sequence.
#include "../../include/cmbx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "host.hpp"
#include "kernels.hpp"
#include "slab.hpp"
#include "status.hpp"

struct cmbx_slab {
  int method = 0, N = 0, M = 0, h = 0, nz = 0;
  double dp = 0;
  int dtype = 0, batch = 0, device = 0;
  int interp = CMBX_TRILINEAR;
  int direct = CMBX_SLAB_DIRECT_AUTO;
  double obs[3] = {0, 0, 0};
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  void* field = nullptr;   // batch x nz x N^2 reals
  void* tw = nullptr;      // N roots
  void* twz = nullptr;     // M roots (flat)
  int* sidx = nullptr;     // device [2 (N/2)^2 + 1]
  void* table = nullptr;   // device per-column table (plan precision)
  int rows = 0;
  std::vector<int> sidx_host;
  std::vector<double> factors;  // hybrid: FP64 S per row, [rows][h][h]
  bool has_spectrum = false;
  size_t real_size() const { return dtype == CMBX_F32 ? 4 : 8; }
  size_t layers_bytes() const { return (size_t)nz * N * N * real_size(); }
};

namespace {

using cmbx::DeviceGuard;
using cmbx::fail;
using cmbx::ok;

constexpr double kTwoPi = 6.283185307179586;

int check(const cmbx_slab* s) { return s ? CMBX_OK : fail(CMBX_EINVAL, "slab is NULL"); }

// Rows of the per-column tables: every s = fx^2 + fy^2 with 0 <= fx, fy <= N/2, in
// increasing order; sidx[s] = its row or -1.
int make_rows(int N, std::vector<int>& sidx) {
  const int H = N / 2;
  sidx.assign(2 * H * H + 1, -1);
  for (int fx = 0; fx <= H; ++fx)
    for (int fy = 0; fy <= H; ++fy) sidx[fx * fx + fy * fy] = 0;
  int rows = 0;
  for (int& v : sidx)
    if (v == 0) v = rows++;
  return rows;
}

// P_box(s, fz) of eq. finalpbox in the fixed operation order: q = (s M^2 + fz^2 N^2) /
// (N^2 M^2), k = (2 pi / dp) sqrt(q), P_box = P_inf(k) ((c c) c) / (M N^2); 0 at k = 0.
double p_box(const cmbx_slab* p, int64_t s, int64_t fz, const double* kt, const double* pt, int64_t n) {
  if (s == 0 && fz == 0) return 0.0;
  const int64_t N = p->N, M = p->M;
  const double q = (double)(s * M * M + fz * fz * N * N) / (double)(N * N * M * M);
  const double c = kTwoPi / p->dp;
  const double k = c * std::sqrt(q);
  const double c3 = (c * c) * c / (double)(M * N * N);
  return cmbx::interp_p(kt, pt, n, k) * c3;
}

// Cyclic Jacobi eigendecomposition of a symmetric n x n matrix A (row-major, overwritten):
// plane rotations annihilate A_pq in row order, sweep after sweep, until every off-diagonal
// entry is below 1e-17 of the largest diagonal one (Golub & Van Loan, Matrix Computations,
// Sec. 8.5). w receives the eigenvalues, V (row-major) the eigenvectors as columns.
void jacobi(int n, std::vector<double>& A, std::vector<double>& V, std::vector<double>& w) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double dmax = 0.0, off = 0.0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(A[(size_t)i * n + i]));
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off = std::max(off, std::fabs(A[(size_t)p * n + q]));
    if (off <= 1e-17 * dmax || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// Symmetric square root S = V diag(sqrt(max(w, 0))) V^T of Gamma_jk = xi(|j - k|).
void sym_root(int h, const double* xi, double* S) {
  std::vector<double> A((size_t)h * h), V, w;
  for (int j = 0; j < h; ++j)
    for (int k = 0; k < h; ++k) A[(size_t)j * h + k] = xi[std::abs(j - k)];
  jacobi(h, A, V, w);
  for (int j = 0; j < h; ++j)
    for (int k = 0; k < h; ++k) {
      double acc = 0.0;
      for (int m = 0; m < h; ++m) acc += V[(size_t)j * h + m] * std::sqrt(std::max(w[m], 0.0)) * V[(size_t)k * h + m];
      S[(size_t)j * h + k] = acc;
    }
}

// Run f(i) for i in [0, n) on the host's threads.
template <class F>
void parallel_for(int n, F f) {
  const int nt = std::max(1, std::min<int>(std::thread::hardware_concurrency(), 32));
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&] {
      for (int i = next++; i < n; i = next++) f(i);
    });
  for (std::thread& th : pool) th.join();
}

template <typename T>
hipError_t upload(void* dst, const std::vector<double>& v) {
  std::vector<T> t(v.size());
  for (size_t i = 0; i < v.size(); ++i) t[i] = (T)v[i];
  return hipMemcpy(dst, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice);
}

int upload_roots(void* dst, int n, int dtype) {
  std::vector<double> re, im;
  cmbx::roots_of_unity(n, re, im);
  std::vector<double> v(2 * (size_t)n);
  for (int m = 0; m < n; ++m) v[2 * m] = re[m], v[2 * m + 1] = im[m];
  const hipError_t e = dtype == CMBX_F32 ? upload<float>(dst, v) : upload<double>(dst, v);
  return e == hipSuccess ? CMBX_OK : fail(CMBX_EHIP, "twiddle upload: %s", hipGetErrorString(e));
}

cmbx::SlabColumnsArgs columns_args(const cmbx_slab* p, uint64_t seed, void* buf, const float* bm) {
  cmbx::SlabColumnsArgs a{};
  a.dtype = p->dtype;
  a.method = p->method;
  a.N = p->N;
  a.M = p->M;
  a.h = p->h;
  a.buf = buf;
  a.sidx = p->sidx;
  a.table = p->table;
  a.rows = p->rows;
  a.twz = p->twz;
  a.k0 = (uint32_t)(seed & 0xffffffffu);
  a.k1 = (uint32_t)(seed >> 32);
  a.bm_tab = bm;
  return a;
}

int noise_table(const cmbx_slab* p, const float** bm) {
  *bm = nullptr;
  if (p->dtype != CMBX_F32) return CMBX_OK;
  HIP_TRY(cmbx::noise_table_address(bm));
  return CMBX_OK;
}

// The layers of one realisation into buf: the columns and the transform along x, then
// (unless `half`) the complex-to-real transform along y.
int enqueue_layers(const cmbx_slab* p, uint64_t seed, void* buf, hipStream_t s, bool half = false) {
  const float* bm = nullptr;
  if (int rc = noise_table(p, &bm)) return rc;
  HIP_TRY(cmbx::launch_slab_columns(columns_args(p, seed, buf, bm), s));
  HIP_TRY(cmbx::launch_layers_c2c(p->dtype, p->N, buf, p->tw, p->nz, s));
  if (!half) HIP_TRY(cmbx::launch_layers_c2r(p->dtype, p->N, buf, p->tw, p->nz, s));
  return CMBX_OK;
}

// Whether a map of n_pix pixels evaluates its stencils' rows directly from the layers'
// half spectra: the direct sums take K^2 N/2 terms per pixel, the complex-to-real pass and
// the gather about nz N^2 operations and two launches' latency; the direct way is taken
// while its terms stay below 2 nz N^2.
bool use_direct(const cmbx_slab* p, int64_t n_pix) {
  if (p->direct != CMBX_SLAB_DIRECT_AUTO) return p->direct == CMBX_SLAB_DIRECT_ALWAYS;
  const int64_t K = p->interp == CMBX_TRICUBIC ? 4 : 2;
  return n_pix * K * K * (p->N / 2) <= 2 * (int64_t)p->nz * p->N * p->N;
}

int enqueue_gather(const cmbx_slab* p, const void* layers, double r, const double* dirs, int64_t n_pix, void* out,
                   hipStream_t s, bool direct = false) {
  cmbx::SlabGatherArgs g{};
  g.dtype = p->dtype;
  g.interp = p->interp;
  g.N = p->N;
  g.nz = p->nz;
  g.periodic_z = p->method == CMBX_SLAB_FLAT ? 1 : 0;
  g.field = layers;
  g.scale = 1.0 / p->dp;
  for (int d = 0; d < 3; ++d) g.obs[d] = p->obs[d];
  g.r = r;
  g.dirs = dirs;
  g.n_pix = n_pix;
  g.out = out;
  if (direct) HIP_TRY(cmbx::launch_slab_direct(g, p->tw, s));
  else HIP_TRY(cmbx::launch_slab_gather(g, s));
  return CMBX_OK;
}

}  // namespace

extern "C" {

int cmbx_slab_create(int method, int N, int M, int h, double dp, int dtype, int batch, cmbx_slab** out) {
  if (!out) return fail(CMBX_EINVAL, "out is NULL");
  *out = nullptr;
  if (method != CMBX_SLAB_FLAT && method != CMBX_SLAB_HYBRID) return fail(CMBX_EINVAL, "unknown slab method %d", method);
  if (N < 8 || N > 1024 || N % 2) return fail(CMBX_EINVAL, "N = %d must be even and in [8, 1024]", N);
  if (M < 2 || M % 2 || M > 1 << 20) return fail(CMBX_EINVAL, "M = %d must be even and >= 2", M);
  if (!(dp > 0.0) || !std::isfinite(dp)) return fail(CMBX_EINVAL, "dp = %g must be positive and finite", dp);
  if (dtype != CMBX_F32 && dtype != CMBX_F64) return fail(CMBX_EINVAL, "unknown dtype %d", dtype);
  if (batch < 1) return fail(CMBX_EINVAL, "batch = %d must be >= 1", batch);
  if (method == CMBX_SLAB_FLAT) h = M;
  if (h < 1 || h > M || h > cmbx::kSlabMaxLayers && method == CMBX_SLAB_HYBRID)
    return fail(CMBX_EINVAL, "h = %d must be in [1, min(M, %d)]", h, cmbx::kSlabMaxLayers);
  if (!cmbx::is_2a3b(N) || !cmbx::size_compiled(N))
    return fail(CMBX_EUNSUPPORTED, "N = %d: compiled sizes are 2^a and 3 x 2^a in [8, 1024]", N);
  if (method == CMBX_SLAB_FLAT && !cmbx::slab_depth_compiled(M))
    return fail(CMBX_EUNSUPPORTED, "M = %d: compiled depths are 2^a and 3 x 2^a in [8, 512]", M);
  const int nz = method == CMBX_SLAB_FLAT ? M : h;
  if (!cmbx::layers_supported(dtype, N, nz))
    return fail(CMBX_EUNSUPPORTED, "%d layers of N = %d: no compiled line tile divides %d lines", nz, N, nz * N);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CMBX_EHIP, "no HIP device available");
  cmbx_slab* p = new cmbx_slab;
  p->method = method;
  p->N = N;
  p->M = M;
  p->h = h;
  p->nz = nz;
  p->dp = dp;
  p->dtype = dtype;
  p->batch = batch;
  p->obs[0] = p->obs[1] = 0.5 * N * dp;
  p->obs[2] = 0.5 * (nz - 1) * dp;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking);
  p->stream = p->own_stream;
  if (e == hipSuccess && cmbx::fault("alloc")) e = hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipMalloc(&p->field, p->layers_bytes() * batch);
  if (e == hipSuccess) e = hipMalloc(&p->tw, (size_t)N * 2 * p->real_size());
  if (e == hipSuccess && method == CMBX_SLAB_FLAT) e = hipMalloc(&p->twz, (size_t)M * 2 * p->real_size());
  p->rows = make_rows(N, p->sidx_host);
  if (e == hipSuccess) e = hipMalloc(&p->sidx, p->sidx_host.size() * sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpy(p->sidx, p->sidx_host.data(), p->sidx_host.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && dtype == CMBX_F32) e = cmbx::ensure_noise_tables(p->device);
  if (e != hipSuccess) {
    const int code = e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP;
    const char* msg = hipGetErrorString(e);
    cmbx_slab_destroy(p);
    return fail(code, "slab allocation (N = %d, layers = %d, batch = %d): %s", N, nz, batch, msg);
  }
  int rc = upload_roots(p->tw, N, dtype);
  if (rc == CMBX_OK && method == CMBX_SLAB_FLAT) rc = upload_roots(p->twz, M, dtype);
  if (rc != CMBX_OK) {
    const std::string msg = cmbx::err_msg();
    cmbx_slab_destroy(p);
    return fail(rc, "%s", msg.c_str());
  }
  *out = p;
  return ok();
}

int cmbx_slab_destroy(cmbx_slab* p) {
  if (!p) return ok();
  DeviceGuard g(p->device);
  if (p->own_stream) (void)hipStreamSynchronize(p->own_stream);
  if (p->stream && p->stream != p->own_stream) (void)hipStreamSynchronize(p->stream);
  for (void* d : {p->field, p->tw, p->twz, (void*)p->sidx, p->table})
    if (d) (void)hipFree(d);
  if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
  delete p;
  return ok();
}

int cmbx_slab_set(cmbx_slab* p, int key, int64_t value) {
  if (int rc = check(p)) return rc;
  switch (key) {
    case CMBX_OPT_INTERP:
      if (value != CMBX_TRILINEAR && value != CMBX_TRICUBIC) return fail(CMBX_EINVAL, "unknown interpolant %lld", (long long)value);
      p->interp = (int)value;
      return ok();
    case CMBX_OPT_STREAM:
      p->stream = value == -1 ? p->own_stream : (hipStream_t)(intptr_t)value;
      return ok();
    case CMBX_SLAB_OPT_DIRECT:
      if (value != CMBX_SLAB_DIRECT_AUTO && value != CMBX_SLAB_DIRECT_NEVER && value != CMBX_SLAB_DIRECT_ALWAYS)
        return fail(CMBX_EINVAL, "unknown direct-evaluation mode %lld", (long long)value);
      p->direct = (int)value;
      return ok();
    default:
      return fail(CMBX_EINVAL, "option %d does not apply to slabs", key);
  }
}

int cmbx_slab_observer(cmbx_slab* p, double x, double y, double z) {
  if (int rc = check(p)) return rc;
  if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return fail(CMBX_EINVAL, "observer must be finite");
  p->obs[0] = x;
  p->obs[1] = y;
  p->obs[2] = z;
  return ok();
}

int cmbx_slab_cap_observer(const cmbx_slab* p, double r, double z_min, double* xyz) {
  if (int rc = check(p)) return rc;
  if (!xyz) return fail(CMBX_EINVAL, "xyz is NULL");
  if (!(r > 0.0) || !std::isfinite(r)) return fail(CMBX_EINVAL, "r = %g must be positive and finite", r);
  if (!(z_min >= -1.0 && z_min <= 1.0)) return fail(CMBX_EINVAL, "z_min = %g must lie in [-1, 1]", z_min);
  const double c = 0.5 * p->N * p->dp;
  xyz[0] = c;
  xyz[1] = c;
  xyz[2] = 0.5 * (p->nz - 1) * p->dp - r * (1.0 + z_min) / 2.0;
  return ok();
}

int cmbx_slab_spectrum(cmbx_slab* p, const double* k, const double* P, int64_t n) {
  if (int rc = check(p)) return rc;
  if (!k || !P) return fail(CMBX_EINVAL, "k and P_inf must be non-NULL host arrays");
  if (n < 2) return fail(CMBX_EINVAL, "n = %lld must be >= 2", (long long)n);
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(k[i]) || k[i] < 0) return fail(CMBX_EINVAL, "k[%lld] = %g must be finite and >= 0", (long long)i, k[i]);
    if (!std::isfinite(P[i]) || P[i] < 0) return fail(CMBX_EINVAL, "P_inf[%lld] = %g must be finite and >= 0", (long long)i, P[i]);
    if (i > 0 && !(k[i] > k[i - 1])) return fail(CMBX_EINVAL, "k must be strictly increasing (index %lld)", (long long)i);
  }
  DeviceGuard g(p->device);
  HIP_TRY(hipStreamSynchronize(p->stream));
  const int H = p->N / 2;
  const int64_t smax = 2ll * H * H;
  std::vector<int64_t> s_of_row(p->rows);
  for (int64_t s = 0; s <= smax; ++s)
    if (p->sidx_host[s] >= 0) s_of_row[p->sidx_host[s]] = s;
  const int self_s[3] = {0, H * H, 2 * H * H};
  std::vector<double> tab;
  if (p->method == CMBX_SLAB_FLAT) {
    // sqrt(P_box / 2) per (row, fz), then sqrt(P_box) at the six self-conjugate (s, fz)
    const int nf = p->M / 2 + 1;
    tab.resize((size_t)p->rows * nf + 6);
    for (int r = 0; r < p->rows; ++r)
      for (int fz = 0; fz < nf; ++fz) tab[(size_t)r * nf + fz] = std::sqrt(p_box(p, s_of_row[r], fz, k, P, n) * 0.5);
    for (int c = 0; c < 3; ++c)
      for (int t = 0; t < 2; ++t) tab[(size_t)p->rows * nf + 2 * c + t] = std::sqrt(p_box(p, self_s[c], t ? p->M / 2 : 0, k, P, n));
  } else {
    // Gamma of each row from xi(d) = sum over the M values of fz of P_box e^{2 pi i fz d / M}
    // = P(0) + 2 sum_{0 < fz < M/2} P(fz) cos(2 pi fz d / M) + P(M/2) (-1)^d; S its root
    const int h = p->h, M = p->M;
    p->factors.assign((size_t)p->rows * h * h, 0.0);
    parallel_for(p->rows, [&](int r) {
      std::vector<double> pz(M / 2 + 1), xi(h);
      for (int fz = 0; fz <= M / 2; ++fz) pz[fz] = p_box(p, s_of_row[r], fz, k, P, n);
      for (int d = 0; d < h; ++d) {
        double acc = pz[0];
        for (int fz = 1; fz < M / 2; ++fz) acc += 2.0 * pz[fz] * std::cos(kTwoPi * (double)((int64_t)fz * d % M) / M);
        acc += (d % 2 ? -1.0 : 1.0) * pz[M / 2];
        xi[d] = acc;
      }
      sym_root(h, xi.data(), &p->factors[(size_t)r * h * h]);
    });
    const double inv_sqrt2 = 1.0 / std::sqrt(2.0);
    tab.resize((size_t)(p->rows + 3) * h * h);
    for (size_t i = 0; i < (size_t)p->rows * h * h; ++i) tab[i] = p->factors[i] * inv_sqrt2;
    for (int c = 0; c < 3; ++c)
      std::copy_n(&p->factors[(size_t)p->sidx_host[self_s[c]] * h * h], (size_t)h * h, &tab[(size_t)(p->rows + c) * h * h]);
  }
  if (p->table) (void)hipFree(p->table);
  p->table = nullptr;
  p->has_spectrum = false;
  hipError_t e = hipMalloc(&p->table, tab.size() * p->real_size());
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "slab table: %s", hipGetErrorString(e));
  e = p->dtype == CMBX_F32 ? upload<float>(p->table, tab) : upload<double>(p->table, tab);
  if (e != hipSuccess) return fail(CMBX_EHIP, "slab table upload: %s", hipGetErrorString(e));
  p->has_spectrum = true;
  return ok();
}

int cmbx_slab_simulate(cmbx_slab* p, uint64_t seed, double r, const double* dirs, int64_t n_pix, void* out) {
  if (int rc = check(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set: call cmbx_slab_spectrum first");
  if (!(r > 0.0) || !std::isfinite(r)) return fail(CMBX_EINVAL, "r = %g must be positive and finite", r);
  if (n_pix < 1 || n_pix > (int64_t)1 << 31) return fail(CMBX_EINVAL, "n_pix = %lld out of range", (long long)n_pix);
  if (!dirs || !out) return fail(CMBX_EINVAL, "dirs and out must be non-NULL device pointers");
  DeviceGuard g(p->device);
  const bool direct = use_direct(p, n_pix);
  for (int b = 0; b < p->batch; ++b) {
    char* buf = (char*)p->field + (size_t)b * p->layers_bytes();
    if (int rc = enqueue_layers(p, seed + (uint64_t)b, buf, p->stream, direct)) return rc;
    if (int rc = enqueue_gather(p, buf, r, dirs, n_pix, (char*)out + (size_t)b * n_pix * p->real_size(), p->stream,
                                direct))
      return rc;
  }
  return ok();
}

int cmbx_slab_debug_layers(cmbx_slab* p, uint64_t seed, void* layers) {
  if (int rc = check(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!layers) return fail(CMBX_EINVAL, "layers is NULL");
  DeviceGuard g(p->device);
  if (int rc = enqueue_layers(p, seed, layers, p->stream)) return rc;
  return ok();
}

int cmbx_slab_debug_columns(cmbx_slab* p, uint64_t seed, void* cols) {
  if (int rc = check(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!cols) return fail(CMBX_EINVAL, "cols is NULL");
  DeviceGuard g(p->device);
  const float* bm = nullptr;
  if (int rc = noise_table(p, &bm)) return rc;
  HIP_TRY(cmbx::launch_slab_columns_debug(columns_args(p, seed, cols, bm), p->stream));
  return ok();
}

int cmbx_slab_factor(const cmbx_slab* p, int64_t s, double* S) {
  if (int rc = check(p)) return rc;
  if (p->method != CMBX_SLAB_HYBRID) return fail(CMBX_EINVAL, "only hybrid slabs have column factors");
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!S || s < 0 || s >= (int64_t)p->sidx_host.size() || p->sidx_host[s] < 0)
    return fail(CMBX_EINVAL, "s = %lld is not fx^2 + fy^2 with 0 <= fx, fy <= N/2", (long long)s);
  const size_t hh = (size_t)p->h * p->h;
  std::copy_n(&p->factors[(size_t)p->sidx_host[s] * hh], hh, S);
  return ok();
}

int cmbx_slab_info(const cmbx_slab* p, int* N, int* M, int* nz, double* dp, void** layers) {
  if (int rc = check(p)) return rc;
  if (N) *N = p->N;
  if (M) *M = p->M;
  if (nz) *nz = p->nz;
  if (dp) *dp = p->dp;
  if (layers) *layers = p->field;
  return ok();
}

int cmbx_box_size(double b, double theta_max, double size_factor, double R, int* N, int* M, double* dp) {
  if (!N || !M || !dp) return fail(CMBX_EINVAL, "box_size: NULL output");
  if (!(b > 0) || !(theta_max > 0) || !(size_factor > 0) || !(R > 0) || !std::isfinite(b) || !std::isfinite(theta_max) ||
      !std::isfinite(size_factor) || !std::isfinite(R))
    return fail(CMBX_EINVAL, "box_size: arguments must be positive and finite");
  const double d = 0.85 * R * b / 5.0;
  const double width = 2.0 * R * std::sin(std::min(theta_max, M_PI / 2)) / d;
  const double height = R * (1.0 - std::cos(theta_max)) / d;
  const double n = size_factor * std::ldexp(1.0, (int)std::ceil(std::log2(2.0 * width)));
  const double m = size_factor * std::ldexp(1.0, (int)std::ceil(std::log2(2.0 * height)));
  if (!(n >= 1 && n < 2e9 && m >= 1 && m < 2e9)) return fail(CMBX_EINVAL, "box_size: the box is out of range");
  *N = (int)std::lround(n);
  *M = (int)std::lround(m);
  *dp = d;
  return ok();
}

}  // extern "C"
