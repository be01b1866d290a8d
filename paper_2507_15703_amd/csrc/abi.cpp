// C ABI of the box simulator: argument checking, plans, host FP64 tables, and the launch
// sequences of the hot path (see include/cmbx.h for the contract of every entry point).
#include "../../include/cmbx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "linalg.hpp"
#include "mlp.hpp"
#include "host.hpp"
#include "status.hpp"

struct cmbx_plan {
  int N = 0;
  double L = 0;
  double obs[3] = {0, 0, 0};  // observer position in the box (set to the centre at creation)
  int dtype = 0;
  int batch = 0;
  int device = 0;
  int interp = CMBX_TRILINEAR;
  int tile_x = 0;  // 0 = compiled default
  int tile_y = 0;
  int lines_z = 0;
  int plan_x = 0;  // FFT stage plan per pass (1: the alternative, with the default tile only)
  int plan_y = 0;
  int plan_z = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  void* field = nullptr;   // batch x N^3 reals
  void* tw = nullptr;      // N complex roots of unity
  void* wtab = nullptr;    // 3 (N/2)^2 + 1 half weights, then 4 full weights
  int m_hi = 0;            // largest |f|^2 of nonzero half weight in the current table
  void* fp = nullptr;      // map footprint of the last simulate_patch call
  bool prune = true;       // maps make only the part of the field their stencils read
  bool fixed_dirs = false; // the caller keeps the directions at a given address unchanged
  // what fp (or ord) was last made from (reused while fixed_dirs holds and every key is
  // the same)
  struct PixKey {
    bool valid = false;
    double r = 0;
    const double* dirs = nullptr;
    int64_t n_pix = 0;
    int lines = 0, interp = 0;
    double obs[3] = {0, 0, 0};
  };
  PixKey fp_key;
  // with fixed directions, the gather's pixel order (made once per key; room for
  // ord_cap pixels) and the work space it is sorted in
  void* ord = nullptr;
  int64_t ord_cap = 0;
  void* ord_scratch = nullptr;
  size_t ord_scratch_bytes = 0;
  PixKey ord_key;
  bool has_spectrum = false;
  size_t real_size() const { return dtype == CMBX_F32 ? 4 : 8; }
  size_t field_bytes() const { return (size_t)N * N * N * real_size(); }
  int64_t wtab_len() const { return 3ll * (N / 2) * (N / 2) + 1 + 4; }
};

struct cmbx_ensemble {
  // lane 0 runs on the caller's stream; lane i > 0 on streams[i - 1], forked from and
  // joined back into the caller's stream at every launch
  std::vector<hipGraph_t> graph;
  std::vector<hipGraphExec_t> exec;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  std::vector<void*> dev;  // rotating workspaces and the schedule
  std::vector<void*> fps;  // one map footprint per realisation whose plan prunes, and one
                           // pixel order per realisation whose plan fixes the directions
  std::vector<int> modes;  // execution mode chosen per (precision, N) group
  // support bound each plan had when its kernels were captured (they skip what lies beyond)
  std::vector<std::pair<const cmbx_plan*, int>> bounds;
  int device = 0;
};

namespace cmbx {

std::string& err_msg() {
  thread_local std::string msg;
  return msg;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  err_msg() = buf;
  return code;
}

int ok() {
  err_msg().clear();
  return CMBX_OK;
}

}  // namespace cmbx

namespace cmbx {

bool is_2a3b(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// exp(2 pi i m / N) in extended precision, rounded to double, for m = 0 .. N-1
void roots_of_unity(int N, std::vector<double>& re, std::vector<double>& im) {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  re.resize(N);
  im.resize(N);
  for (int m = 0; m < N; ++m) {
    // the full angle in long double (64-bit significand) rounded once to double; the
    // quarter turns are set exactly below
    const long double ang = two_pi * (long double)m / (long double)N;
    re[m] = (double)cosl(ang);
    im[m] = (double)sinl(ang);
    if (4 * m % N == 0) {
      const int q = 4 * m / N;
      re[m] = q == 0 ? 1.0 : q == 2 ? -1.0 : 0.0;
      im[m] = q == 1 ? 1.0 : q == 3 ? -1.0 : 0.0;
    }
  }
}

// P_inf at k: linear between nodes, zero outside [k[0], k[n-1]] (same operations and
// order as the specification: i = last node with k_i <= k, clamped to n-2).
double interp_p(const double* kt, const double* pt, int64_t n, double k) {
  if (!(k >= kt[0] && k <= kt[n - 1])) return 0.0;
  int64_t i = (int64_t)(std::upper_bound(kt, kt + n, k) - kt) - 1;
  i = std::min<int64_t>(std::max<int64_t>(i, 0), n - 2);
  const double d = k - kt[i];
  const double h = kt[i + 1] - kt[i];
  const double t = d / h;
  const double dp = pt[i + 1] - pt[i];
  const double prod = dp * t;
  return pt[i] + prod;
}

// Fault injection for tests of the error paths: the environment variable CMBX_FAULT holds
// a comma-separated list of sites ("alloc": plan allocation, "capture": ensemble graph
// capture, "launch": ensemble launch) that then fail as the runtime would.
bool fault(const char* site) {
  const char* e = std::getenv("CMBX_FAULT");
  if (!e || !*e) return false;
  const std::string list = std::string(",") + e + ",";
  return list.find(std::string(",") + site + ",") != std::string::npos;
}

// The binary32 Box-Muller tables (layout in noise_device.hpp): each entry the binary64
// value of its definition rounded once to binary32.
void fill_noise_tables(float* t) {
  for (int j = 0; j < 128; ++j) {
    const double c = 1.0 + j / 128.0;
    t[j] = (float)std::log(j >= 54 ? c / 2.0 : c);
    t[128 + j] = (float)(1.0 / c);
  }
  const double step = 2.0 * M_PI / 256.0;
  for (int k = 0; k < 256; ++k) {
    const double ang = (k + 0.5) * step;
    t[256 + k] = (float)std::sin(ang);
    t[512 + k] = (float)std::cos(ang);
  }
}

// Upload the tables to the current device once per process.
hipError_t ensure_noise_tables(int device) {
  static std::mutex mu;
  static std::set<int> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count(device)) return hipSuccess;
  std::vector<float> t(cmbx::kNoiseTableSize);
  fill_noise_tables(t.data());
  const hipError_t e = cmbx::upload_noise_tables(t.data());
  if (e == hipSuccess) done.insert(device);
  return e;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != dev) (void)hipSetDevice(dev);
}

DeviceGuard::~DeviceGuard() {
  if (prev >= 0) (void)hipSetDevice(prev);
}

}  // namespace cmbx

namespace {

using cmbx::fail;
using cmbx::ok;
using cmbx::DeviceGuard;
using cmbx::ensure_noise_tables;
using cmbx::fault;
using cmbx::fill_noise_tables;
using cmbx::interp_p;
using cmbx::is_2a3b;
using cmbx::roots_of_unity;

// Returns the largest |f|^2 whose half weight is not zero: the passes skip what lies beyond.
template <typename T>
int fill_weights(const cmbx_plan* p, const double* kt, const double* pt, int64_t n, std::vector<T>& out) {
  // P_box = P_inf (2 pi / L)^3 (eq. finalpbox, cubic box); half = sqrt(P_box / 2),
  // full = sqrt(P_box) at |f|^2 = c (N/2)^2, c = 0..3; P_box(0) = 0.
  const int M = p->N / 2;
  const int64_t mmax = 3ll * M * M;
  const double c = 6.283185307179586 / p->L;
  const double c3 = c * c * c;
  out.assign(mmax + 1 + 4, T(0));
  std::vector<double> pbox(mmax + 1);
  for (int64_t m = 0; m <= mmax; ++m) {
    const double k = c * std::sqrt((double)m);
    const double pi = interp_p(kt, pt, n, k);
    pbox[m] = m == 0 ? 0.0 : pi * c3;
    out[m] = (T)std::sqrt(pbox[m] * 0.5);
  }
  for (int cc = 0; cc < 4; ++cc) out[mmax + 1 + cc] = (T)std::sqrt(pbox[(int64_t)cc * M * M]);
  int64_t hi = mmax;
  while (hi > 0 && out[hi] == T(0)) --hi;
  return (int)hi;
}

int check_plan(const cmbx_plan* p) {
  if (!p) return fail(CMBX_EINVAL, "plan is NULL");
  return CMBX_OK;
}

cmbx::FieldArgs field_args(const cmbx_plan* p, uint64_t seed, void* buf) {
  cmbx::FieldArgs a{};  // value-initialised: every pointer not set below is NULL (fp: the whole field)
  a.dtype = p->dtype;
  a.N = p->N;
  a.buf = buf;
  a.wtab = p->wtab;
  a.tw = p->tw;
  a.k0 = (uint32_t)(seed & 0xffffffffu);
  a.k1 = (uint32_t)(seed >> 32);
  a.m_hi = p->m_hi;
  a.tile_x = p->tile_x;
  a.tile_y = p->tile_y;
  a.lines_z = p->lines_z;
  a.plan_x = p->plan_x;
  a.plan_y = p->plan_y;
  a.plan_z = p->plan_z;
  return a;
}

// The field of one realisation in buf: the whole field, or with a map footprint `fp` only
// the part that footprint marks (what the map's stencils read).
int enqueue_field(const cmbx_plan* p, uint64_t seed, void* buf, hipStream_t s, const void* fp = nullptr) {
  cmbx::FieldArgs a = field_args(p, seed, buf);
  a.fp = fp;
  HIP_TRY(cmbx::launch_pass_x(a, s));
  HIP_TRY(cmbx::launch_pass_y(a, s));
  HIP_TRY(cmbx::launch_pass_z(a, s));
  return CMBX_OK;
}

// Shell radius: with the observer at the box centre the whole sphere must lie in the box,
// 0 < r < L/2; with the observer moved only the cap has to (the caller's part: the box is
// periodic and any position is reduced into it), so r need only be positive and finite.
int check_radius(const cmbx_plan* p, double r) {
  const double h = 0.5 * p->L;
  const bool centred = p->obs[0] == h && p->obs[1] == h && p->obs[2] == h;
  if (centred && !(r > 0.0 && r < h)) return fail(CMBX_EINVAL, "r = %g must satisfy 0 < r < L/2 = %g", r, h);
  if (!(r > 0.0 && std::isfinite(r))) return fail(CMBX_EINVAL, "r = %g must be positive and finite", r);
  return CMBX_OK;
}

int enqueue_gather(const cmbx_plan* p, const void* field, double r, const double* dirs, int64_t n_pix, void* out,
                   hipStream_t s, const void* order = nullptr) {
  cmbx::GatherArgs g{};
  g.order = order;
  g.dtype = p->dtype;
  g.interp = p->interp;
  g.N = p->N;
  g.field = field;
  g.scale = (double)p->N / p->L;
  for (int d = 0; d < 3; ++d) g.obs[d] = p->obs[d];
  g.r = r;
  g.dirs = dirs;
  g.n_pix = n_pix;
  g.out = out;
  HIP_TRY(cmbx::launch_gather(g, s));
  return CMBX_OK;
}

// The map footprint of (r, dirs) in fp, with the z-pass work list for blocks of `lines`
// lines (0: the plan's own z tile).
int enqueue_footprint(const cmbx_plan* p, void* fp, double r, const double* dirs, int64_t n_pix, hipStream_t s,
                      int lines = 0) {
  cmbx::FootprintArgs f{};
  f.interp = p->interp;
  f.N = p->N;
  f.lines = lines > 0 ? lines : cmbx::resolve_lines_z(p->dtype, p->N, p->lines_z);
  f.fp = fp;
  f.scale = (double)p->N / p->L;
  for (int d = 0; d < 3; ++d) f.obs[d] = p->obs[d];
  f.r = r;
  f.dirs = dirs;
  f.n_pix = n_pix;
  HIP_TRY(cmbx::launch_footprint(f, s));
  return CMBX_OK;
}

// The gather's pixel order of (r, dirs) in `order` (pixel_order_bytes), sorted in
// `scratch` (pixel_order_scratch_bytes bytes).
int enqueue_pixel_order(const cmbx_plan* p, void* order, void* scratch, size_t scratch_bytes, double r,
                        const double* dirs, int64_t n_pix, hipStream_t s) {
  cmbx::PixelOrderArgs a{};
  a.dtype = p->dtype;
  a.interp = p->interp;
  a.N = p->N;
  a.scale = (double)p->N / p->L;
  for (int d = 0; d < 3; ++d) a.obs[d] = p->obs[d];
  a.r = r;
  a.dirs = dirs;
  a.n_pix = n_pix;
  a.order = order;
  a.scratch = scratch;
  a.scratch_bytes = scratch_bytes;
  HIP_TRY(cmbx::launch_pixel_order(a, s));
  return CMBX_OK;
}

cmbx_plan::PixKey pix_key(const cmbx_plan* p, double r, const double* dirs, int64_t n_pix, int lines) {
  cmbx_plan::PixKey k;
  k.valid = true;
  k.r = r;
  k.dirs = dirs;
  k.n_pix = n_pix;
  k.lines = lines;
  k.interp = p->interp;
  for (int d = 0; d < 3; ++d) k.obs[d] = p->obs[d];
  return k;
}

bool same_key(const cmbx_plan::PixKey& a, const cmbx_plan::PixKey& b) {
  return a.valid && b.valid && a.r == b.r && a.dirs == b.dirs && a.n_pix == b.n_pix && a.lines == b.lines &&
         a.interp == b.interp && a.obs[0] == b.obs[0] && a.obs[1] == b.obs[1] && a.obs[2] == b.obs[2];
}

// With fixed directions: the plan's pixel order of (r, dirs), made on stream s if the key
// changed, and returned (NULL without fixed directions, or when s is being captured and
// the order would have to be made: the gather then reads the directions).
int plan_pixel_order(cmbx_plan* p, double r, const double* dirs, int64_t n_pix, hipStream_t s, const void** out) {
  *out = nullptr;
  if (!p->fixed_dirs) return CMBX_OK;
  const cmbx_plan::PixKey k = pix_key(p, r, dirs, n_pix, 0);
  if (!same_key(p->ord_key, k)) {
    p->ord_key.valid = false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return CMBX_OK;
    size_t sb = 0;
    HIP_TRY(cmbx::pixel_order_scratch_bytes(p->N, n_pix, &sb));
    if (n_pix > p->ord_cap) {
      if (p->ord) HIP_TRY(hipFree(p->ord));
      p->ord = nullptr;
      p->ord_cap = 0;
      const hipError_t e = hipMalloc(&p->ord, cmbx::pixel_order_bytes(p->dtype, n_pix));
      if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "pixel order: %s",
                                       hipGetErrorString(e));
      p->ord_cap = n_pix;
    }
    if (sb > p->ord_scratch_bytes) {
      if (p->ord_scratch) HIP_TRY(hipFree(p->ord_scratch));
      p->ord_scratch = nullptr;
      p->ord_scratch_bytes = 0;
      const hipError_t e = hipMalloc(&p->ord_scratch, sb);
      if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "pixel order: %s",
                                       hipGetErrorString(e));
      p->ord_scratch_bytes = sb;
    }
    if (int rc = enqueue_pixel_order(p, p->ord, p->ord_scratch, p->ord_scratch_bytes, r, dirs, n_pix, s)) return rc;
    p->ord_key = k;
  }
  *out = p->ord;
  return CMBX_OK;
}

int check_patch_args(const cmbx_plan* p, double r, const double* dirs, int64_t n_pix, const void* out) {
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set: call cmbx_spectrum_table first");
  if (int rc = check_radius(p, r)) return rc;
  if (n_pix < 1) return fail(CMBX_EINVAL, "n_pix = %lld must be >= 1", (long long)n_pix);
  if (n_pix > (int64_t)1 << 31) return fail(CMBX_EINVAL, "n_pix = %lld exceeds 2^31", (long long)n_pix);
  if (!dirs || !out) return fail(CMBX_EINVAL, "dirs and out must be non-NULL device pointers");
  return CMBX_OK;
}

// Launch the whole hot path for every realisation of the plan on stream s.
int enqueue_patch(cmbx_plan* p, uint64_t seed, double r, const double* dirs, int64_t n_pix, void* out,
                  hipStream_t s) {
  // the realisations share their pixels, hence one footprint; with fixed directions it
  // is made once and reused while the pixels' key stays the same
  if (p->prune) {
    const int lines = cmbx::resolve_lines_z(p->dtype, p->N, p->lines_z);
    auto& k = p->fp_key;
    const bool same = p->fixed_dirs && k.valid && k.r == r && k.dirs == dirs && k.n_pix == n_pix &&
                      k.lines == lines && k.interp == p->interp && k.obs[0] == p->obs[0] &&
                      k.obs[1] == p->obs[1] && k.obs[2] == p->obs[2];
    if (!same) {
      k.valid = false;
      if (int rc = enqueue_footprint(p, p->fp, r, dirs, n_pix, s)) return rc;
      k = {p->fixed_dirs, r, dirs, n_pix, lines, p->interp, {p->obs[0], p->obs[1], p->obs[2]}};
    }
  }
  const void* order = nullptr;
  if (int rc = plan_pixel_order(p, r, dirs, n_pix, s, &order)) return rc;
  for (int b = 0; b < p->batch; ++b) {
    char* buf = (char*)p->field + (size_t)b * p->field_bytes();
    int rc = enqueue_field(p, seed + (uint64_t)b, buf, s, p->prune ? p->fp : nullptr);
    if (rc) return rc;
    rc = enqueue_gather(p, buf, r, dirs, n_pix, (char*)out + (size_t)b * n_pix * p->real_size(), s, order);
    if (rc) return rc;
  }
  return CMBX_OK;
}

}  // namespace

extern "C" {

int cmbx_plan_box(int N, double L, int dtype, int batch, cmbx_plan** out) {
  if (!out) return fail(CMBX_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 8 || N > 1024 || N % 2) return fail(CMBX_EINVAL, "N = %d must be even and in [8, 1024]", N);
  if (!(L > 0.0) || !std::isfinite(L)) return fail(CMBX_EINVAL, "L = %g must be positive and finite", L);
  if (dtype != CMBX_F32 && dtype != CMBX_F64) return fail(CMBX_EINVAL, "unknown dtype %d", dtype);
  if (batch < 1) return fail(CMBX_EINVAL, "batch = %d must be >= 1", batch);
  if (!is_2a3b(N) || !cmbx::size_compiled(N))
    return fail(CMBX_EUNSUPPORTED, "N = %d: compiled sizes are 2^a and 3 x 2^a in [8, 1024]", N);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CMBX_EHIP, "no HIP device available");
  cmbx_plan* p = new cmbx_plan;
  p->N = N;
  p->L = L;
  p->obs[0] = p->obs[1] = p->obs[2] = 0.5 * L;
  p->dtype = dtype;
  p->batch = batch;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking);
  p->stream = p->own_stream;
  if (e == hipSuccess && fault("alloc")) e = hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipMalloc(&p->field, p->field_bytes() * batch);
  if (e == hipSuccess) e = hipMalloc(&p->tw, (size_t)N * 2 * p->real_size());
  if (e == hipSuccess) e = hipMalloc(&p->wtab, (size_t)p->wtab_len() * p->real_size());
  if (e == hipSuccess) e = hipMalloc(&p->fp, cmbx::footprint_bytes(N));
  if (e == hipSuccess && dtype == CMBX_F32) e = ensure_noise_tables(p->device);
  if (e != hipSuccess) {
    const int code = (e == hipErrorOutOfMemory) ? CMBX_ENOMEM : CMBX_EHIP;
    const std::string msg = hipGetErrorString(e);
    cmbx_plan_destroy(p);
    return fail(code, "plan allocation (N = %d, batch = %d): %s", N, batch, msg.c_str());
  }
  std::vector<double> re, im;
  roots_of_unity(N, re, im);
  if (dtype == CMBX_F32) {
    std::vector<float> t(2 * N);
    for (int m = 0; m < N; ++m) t[2 * m] = (float)re[m], t[2 * m + 1] = (float)im[m];
    e = hipMemcpy(p->tw, t.data(), t.size() * 4, hipMemcpyHostToDevice);
  } else {
    std::vector<double> t(2 * N);
    for (int m = 0; m < N; ++m) t[2 * m] = re[m], t[2 * m + 1] = im[m];
    e = hipMemcpy(p->tw, t.data(), t.size() * 8, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    cmbx_plan_destroy(p);
    return fail(CMBX_EHIP, "twiddle upload: %s", hipGetErrorString(e));
  }
  *out = p;
  return ok();
}

int cmbx_plan_destroy(cmbx_plan* p) {
  if (!p) return ok();
  DeviceGuard g(p->device);
  if (p->own_stream) (void)hipStreamSynchronize(p->own_stream);
  if (p->stream && p->stream != p->own_stream) (void)hipStreamSynchronize(p->stream);
  if (p->field) (void)hipFree(p->field);
  if (p->tw) (void)hipFree(p->tw);
  if (p->wtab) (void)hipFree(p->wtab);
  if (p->fp) (void)hipFree(p->fp);
  if (p->ord) (void)hipFree(p->ord);
  if (p->ord_scratch) (void)hipFree(p->ord_scratch);
  if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
  delete p;
  return ok();
}

int cmbx_plan_observer(cmbx_plan* p, double x, double y, double z) {
  if (int rc = check_plan(p)) return rc;
  if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
    return fail(CMBX_EINVAL, "observer position must be finite");
  p->obs[0] = x;
  p->obs[1] = y;
  p->obs[2] = z;
  return ok();
}

int cmbx_plan_cap_observer(const cmbx_plan* p, double r, double z_min, double* xyz) {
  if (int rc = check_plan(p)) return rc;
  if (!xyz) return fail(CMBX_EINVAL, "xyz is NULL");
  if (!(r > 0.0) || !std::isfinite(r)) return fail(CMBX_EINVAL, "r = %g must be positive and finite", r);
  if (!(z_min >= -1.0 && z_min <= 1.0)) return fail(CMBX_EINVAL, "z_min = %g must lie in [-1, 1]", z_min);
  const double h = 0.5 * p->L;
  xyz[0] = h;
  xyz[1] = h;
  xyz[2] = h - r * (1.0 + z_min) / 2.0;
  return ok();
}

int cmbx_plan_set(cmbx_plan* p, int key, int64_t value) {
  if (int rc = check_plan(p)) return rc;
  int opts[4];
  switch (key) {
    case CMBX_OPT_INTERP:
      if (value != CMBX_TRILINEAR && value != CMBX_TRICUBIC) return fail(CMBX_EINVAL, "unknown interpolant %lld", (long long)value);
      p->interp = (int)value;
      return ok();
    case CMBX_OPT_PRUNE:
      if (value != 0 && value != 1) return fail(CMBX_EINVAL, "prune = %lld must be 0 or 1", (long long)value);
      p->prune = value == 1;
      return ok();
    case CMBX_OPT_FIXED_DIRS:
      if (value != 0 && value != 1) return fail(CMBX_EINVAL, "fixed_dirs = %lld must be 0 or 1", (long long)value);
      p->fixed_dirs = value == 1;
      p->fp_key.valid = false;  // setting it (again) makes the next call rebuild the footprint
      p->ord_key.valid = false;  // and the pixel order
      return ok();
    case CMBX_OPT_STREAM:
      p->stream = value == -1 ? p->own_stream : (hipStream_t)(intptr_t)value;
      return ok();
    case CMBX_OPT_TILE_XY:
    case CMBX_OPT_TILE_X:
    case CMBX_OPT_TILE_Y: {
      const int n = cmbx::tile_xy_choices(p->dtype, p->N, opts);
      if (value != 0 && std::find(opts, opts + n, (int)value) == opts + n)
        return fail(CMBX_EINVAL, "tile %lld not compiled for N = %d", (long long)value, p->N);
      if (key != CMBX_OPT_TILE_Y) p->tile_x = (int)value;
      if (key != CMBX_OPT_TILE_X) p->tile_y = (int)value;
      // stage plan 1 exists at the default tile only: another tile takes plan 0
      if (value != 0 && value != opts[0]) {
        if (key != CMBX_OPT_TILE_Y) p->plan_x = 0;
        if (key != CMBX_OPT_TILE_X) p->plan_y = 0;
      }
      return ok();
    }
    case CMBX_OPT_LINES_Z: {
      const int n = cmbx::lines_z_choices(p->dtype, p->N, opts);
      if (value != 0 && std::find(opts, opts + n, (int)value) == opts + n)
        return fail(CMBX_EINVAL, "z lines %lld not compiled for N = %d", (long long)value, p->N);
      p->lines_z = (int)value;
      if (value != 0 && value != opts[0]) p->plan_z = 0;  // plan 1 is compiled at the default tile only
      return ok();
    }
    case CMBX_OPT_PLAN_X:
    case CMBX_OPT_PLAN_Y:
    case CMBX_OPT_PLAN_Z: {
      const int which = key - CMBX_OPT_PLAN_X;
      if (value != 0 && value != 1) return fail(CMBX_EINVAL, "stage plan %lld must be 0 or 1", (long long)value);
      if (value == 1 && !cmbx::stage_plan_compiled(p->dtype, p->N, which))
        return fail(CMBX_EINVAL, "N = %d has one stage plan for pass %d", p->N, which);
      if (value == 1) {  // plan 1 is compiled at the default tile: the pass's tile becomes that
        const int t = which == 2 ? cmbx::resolve_lines_z(p->dtype, p->N, 0) : cmbx::resolve_tile_xy(p->dtype, p->N, 0);
        (which == 0 ? p->tile_x : which == 1 ? p->tile_y : p->lines_z) = t;
      }
      (which == 0 ? p->plan_x : which == 1 ? p->plan_y : p->plan_z) = (int)value;
      return ok();
    }
    default:
      return fail(CMBX_EINVAL, "unknown option key %d", key);
  }
}

int cmbx_plan_get(const cmbx_plan* p, int key, int64_t* value) {
  if (int rc = check_plan(p)) return rc;
  if (!value) return fail(CMBX_EINVAL, "value is NULL");
  switch (key) {
    case CMBX_OPT_INTERP: *value = p->interp; break;
    case CMBX_OPT_TILE_X: *value = cmbx::resolve_tile_xy(p->dtype, p->N, p->tile_x); break;
    case CMBX_OPT_TILE_Y: *value = cmbx::resolve_tile_xy(p->dtype, p->N, p->tile_y); break;
    case CMBX_OPT_LINES_Z: *value = cmbx::resolve_lines_z(p->dtype, p->N, p->lines_z); break;
    case CMBX_OPT_PRUNE: *value = p->prune ? 1 : 0; break;
    case CMBX_OPT_FIXED_DIRS: *value = p->fixed_dirs ? 1 : 0; break;
    case CMBX_OPT_PLAN_X: *value = p->plan_x; break;
    case CMBX_OPT_PLAN_Y: *value = p->plan_y; break;
    case CMBX_OPT_PLAN_Z: *value = p->plan_z; break;
    default: return fail(CMBX_EINVAL, "option %d cannot be read back", key);
  }
  return ok();
}

int cmbx_plan_info(const cmbx_plan* p, int* N, double* L, int* dtype, int* batch, void** field) {
  if (int rc = check_plan(p)) return rc;
  if (N) *N = p->N;
  if (L) *L = p->L;
  if (dtype) *dtype = p->dtype;
  if (batch) *batch = p->batch;
  if (field) *field = p->field;
  return ok();
}

int cmbx_spectrum_table(cmbx_plan* p, const double* k, const double* P, int64_t n) {
  if (int rc = check_plan(p)) return rc;
  if (!k || !P) return fail(CMBX_EINVAL, "k and P_inf must be non-NULL host arrays");
  if (n < 2) return fail(CMBX_EINVAL, "n = %lld must be >= 2", (long long)n);
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(k[i]) || k[i] < 0) return fail(CMBX_EINVAL, "k[%lld] = %g must be finite and >= 0", (long long)i, k[i]);
    if (!std::isfinite(P[i]) || P[i] < 0) return fail(CMBX_EINVAL, "P_inf[%lld] = %g must be finite and >= 0", (long long)i, P[i]);
    if (i > 0 && !(k[i] > k[i - 1])) return fail(CMBX_EINVAL, "k must be strictly increasing (index %lld)", (long long)i);
  }
  DeviceGuard g(p->device);
  hipError_t e;
  int hi = 0;
  // the table is uploaded synchronously with respect to the plan's stream
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return fail(CMBX_EHIP, "stream sync: %s", hipGetErrorString(e));
  if (p->dtype == CMBX_F32) {
    std::vector<float> w;
    hi = fill_weights(p, k, P, n, w);
    e = hipMemcpy(p->wtab, w.data(), w.size() * 4, hipMemcpyHostToDevice);
  } else {
    std::vector<double> w;
    hi = fill_weights(p, k, P, n, w);
    e = hipMemcpy(p->wtab, w.data(), w.size() * 8, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return fail(CMBX_EHIP, "weight table upload: %s", hipGetErrorString(e));
  p->m_hi = hi;
  p->has_spectrum = true;
  return ok();
}

int cmbx_simulate_patch(cmbx_plan* p, uint64_t seed, double r, const double* dirs, int64_t n_pix, void* out) {
  if (int rc = check_plan(p)) return rc;
  if (int rc = check_patch_args(p, r, dirs, n_pix, out)) return rc;
  DeviceGuard g(p->device);
  if (int rc = enqueue_patch(p, seed, r, dirs, n_pix, out, p->stream)) return rc;
  return ok();
}

int cmbx_debug_noise(cmbx_plan* p, uint64_t seed, void* halfgrid) {
  if (int rc = check_plan(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!halfgrid) return fail(CMBX_EINVAL, "halfgrid is NULL");
  DeviceGuard g(p->device);
  HIP_TRY(cmbx::launch_noise_debug(p->dtype, p->N, halfgrid, p->wtab, (uint32_t)(seed & 0xffffffffu),
                                   (uint32_t)(seed >> 32), p->stream));
  return ok();
}

int cmbx_debug_field(cmbx_plan* p, uint64_t seed, void* field) {
  if (int rc = check_plan(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!field) return fail(CMBX_EINVAL, "field is NULL");
  DeviceGuard g(p->device);
  if (int rc = enqueue_field(p, seed, field, p->stream)) return rc;
  return ok();
}

int cmbx_debug_passes(cmbx_plan* p, uint64_t seed, int npasses, void* buf) {
  if (int rc = check_plan(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!buf) return fail(CMBX_EINVAL, "buf is NULL");
  if (npasses < 1 || npasses > 3) return fail(CMBX_EINVAL, "npasses = %d must be 1, 2 or 3", npasses);
  DeviceGuard g(p->device);
  const cmbx::FieldArgs a = field_args(p, seed, buf);
  HIP_TRY(cmbx::launch_pass_x(a, p->stream));
  if (npasses >= 2) HIP_TRY(cmbx::launch_pass_y(a, p->stream));
  if (npasses >= 3) HIP_TRY(cmbx::launch_pass_z(a, p->stream));
  return ok();
}

int cmbx_debug_gather(cmbx_plan* p, const void* field, double r, const double* dirs, int64_t n_pix, void* out) {
  if (int rc = check_plan(p)) return rc;
  if (!field) return fail(CMBX_EINVAL, "field is NULL");
  if ((uintptr_t)field % 16 != 0) return fail(CMBX_EINVAL, "field must be 16-byte aligned");
  if (int rc = check_radius(p, r)) return rc;
  if (n_pix < 1 || n_pix > (int64_t)1 << 31) return fail(CMBX_EINVAL, "bad n_pix %lld", (long long)n_pix);
  if (!dirs || !out) return fail(CMBX_EINVAL, "dirs and out must be non-NULL");
  DeviceGuard g(p->device);
  if (int rc = enqueue_gather(p, field, r, dirs, n_pix, out, p->stream)) return rc;
  return ok();
}

int cmbx_healpix_cap(int64_t nside, double z_min, double* dirs, int64_t capacity, int64_t* n_pix, void* stream) {
  if (!n_pix) return fail(CMBX_EINVAL, "healpix_cap: n_pix is NULL");
  if (nside < 1 || nside > cmbx::kHealpixMaxNside)
    return fail(CMBX_EINVAL, "healpix_cap: nside = %lld must be in [1, %lld]", (long long)nside,
                (long long)cmbx::kHealpixMaxNside);
  if (std::isnan(z_min)) return fail(CMBX_EINVAL, "healpix_cap: z_min is NaN");
  const int64_t count = cmbx::healpix_cap_count(nside, z_min);
  *n_pix = count;
  if (!dirs) return ok();
  if (capacity < count)
    return fail(CMBX_EINVAL, "healpix_cap: capacity %lld < %lld pixels", (long long)capacity, (long long)count);
  HIP_TRY(cmbx::launch_healpix_cap(nside, count, dirs, (hipStream_t)stream));
  return ok();
}

int cmbx_pixel_covariance(const double* dirs, int64_t n_pix, const double* cl, int lmax, double* gamma,
                          void* stream) {
  if (!dirs || !cl || !gamma) return fail(CMBX_EINVAL, "pixel_covariance: NULL pointer");
  if (n_pix < 1 || n_pix > cmbx::kCovMaxPixels)
    return fail(CMBX_EINVAL, "pixel_covariance: n_pix = %lld must be in [1, %lld]", (long long)n_pix,
                (long long)cmbx::kCovMaxPixels);
  if (lmax < 0 || lmax > cmbx::kCovMaxL)
    return fail(CMBX_EINVAL, "pixel_covariance: lmax = %d must be in [0, %d]", lmax, cmbx::kCovMaxL);
  HIP_TRY(cmbx::launch_pixel_cov(dirs, n_pix, cl, lmax, gamma, (hipStream_t)stream));
  return ok();
}

int cmbx_cholesky(double* A, int64_t n, int64_t lda, double shift, int64_t* info, void* stream) {
  if (!A || n < 1 || lda < n) return fail(CMBX_EINVAL, "cholesky: need A != NULL, n >= 1, lda >= n");
  if (!std::isfinite(shift)) return fail(CMBX_EINVAL, "cholesky: shift must be finite");
  HIP_TRY(cmbx::launch_cholesky(A, n, lda, shift, info, (hipStream_t)stream));
  return ok();
}

int cmbx_whiten(const double* L, int64_t n, int64_t ldl, double* B, int64_t nrhs, int64_t ldb, void* stream) {
  if (!L || !B || n < 1 || nrhs < 1 || ldl < n || ldb < n)
    return fail(CMBX_EINVAL, "whiten: need non-NULL L, B, n, nrhs >= 1 and leading dimensions >= n");
  HIP_TRY(cmbx::launch_trsm_rows(L, n, ldl, B, nrhs, ldb, (hipStream_t)stream));
  return ok();
}

int cmbx_gemm_nt_sub(int64_t m, int64_t n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double* C, int64_t ldc, int lower, void* stream) {
  if (!A || !B || !C || m < 1 || n < 1 || k < 1 || k > cmbx::kCholPanel || lda < k || ldb < k || ldc < n)
    return fail(CMBX_EINVAL, "gemm_nt_sub: bad sizes or NULL operand (k must be 1 .. %d)", cmbx::kCholPanel);
  HIP_TRY(cmbx::launch_gemm_nt_sub(m, n, k, A, lda, B, ldb, C, ldc, lower ? 1 : 0, (hipStream_t)stream));
  return ok();
}

int64_t cmbx_footprint_bytes(int N) {
  if (N < 8 || N > 1024) return fail(CMBX_EINVAL, "N = %d must be in [8, 1024]", N);
  return (int64_t)cmbx::footprint_bytes(N);
}

int cmbx_debug_footprint(cmbx_plan* p, double r, const double* dirs, int64_t n_pix, void* fp) {
  if (int rc = check_plan(p)) return rc;
  if (int rc = check_radius(p, r)) return rc;
  if (n_pix < 1 || n_pix > (int64_t)1 << 31) return fail(CMBX_EINVAL, "bad n_pix %lld", (long long)n_pix);
  if (!dirs || !fp) return fail(CMBX_EINVAL, "dirs and fp must be non-NULL");
  if ((uintptr_t)fp % 4 != 0) return fail(CMBX_EINVAL, "fp must be 4-byte aligned");
  DeviceGuard g(p->device);
  if (int rc = enqueue_footprint(p, fp, r, dirs, n_pix, p->stream)) return rc;
  return ok();
}

namespace {

// One realisation to simulate inside an ensemble.
struct Item {
  const cmbx_plan* plan;
  int slot;  // batch slot of the plan's workspace (chained mode)
  uint64_t seed;
  double r;
  const double* dirs;
  int64_t n_pix;
  void* out;
  int lane = 0;  // chained mode: the graph (and stream) the item runs in
  void* fp = nullptr;  // its map footprint if its plan prunes
  bool fixed = false;  // its plan fixes the directions: fp is made at creation, not in the graph
  void* ord = nullptr; // with fixed directions, the gather's pixel order (made at creation)
};

// Interleave the roles' workgroups in proportion to their counts (largest-deficit
// order), so every stretch of the launch carries the same mix of roles.
void interleave(const int64_t cnt[4], std::vector<uint32_t>& sched) {
  int64_t total = 0, issued[4] = {0, 0, 0, 0};
  for (int r = 0; r < 4; ++r) total += cnt[r];
  for (int64_t pos = 0; pos < total; ++pos) {
    int best = -1;
    double bd = -1e300;
    for (int r = 0; r < 4; ++r) {
      if (issued[r] >= cnt[r]) continue;
      const double d = (double)cnt[r] * (double)(pos + 1) / (double)total - (double)issued[r];
      if (d > bd) bd = d, best = r;
    }
    sched.push_back(((uint32_t)best << 30) | (uint32_t)issued[best]);
    ++issued[best];
  }
}

// A group of items of one (precision, N) and what each execution mode needs.
struct Group {
  int dtype = 0, N = 0;
  std::vector<Item> items;
  std::vector<void*> bufs;              // pipelined: rotating workspaces (owned)
  std::vector<cmbx::PipeLaunch> pipe;   // pipelined launches (sched = offset until upload)
  std::vector<size_t> sched_off;
  int mode = CMBX_ENS_CHAINED;
};

int enqueue_group(const Group& gr, int mode, const uint32_t* dsched, hipStream_t s, int lane) {
  if (mode == CMBX_ENS_CHAINED) {
    for (const Item& it : gr.items) {
      if (lane >= 0 && it.lane != lane) continue;
      char* buf = (char*)it.plan->field + (size_t)it.slot * it.plan->field_bytes();
      if (it.fp && !it.fixed)
        if (int rc = enqueue_footprint(it.plan, it.fp, it.r, it.dirs, it.n_pix, s)) return rc;
      if (int rc = enqueue_field(it.plan, it.seed, buf, s, it.fp)) return rc;
      if (int rc = enqueue_gather(it.plan, buf, it.r, it.dirs, it.n_pix, it.out, s, it.ord)) return rc;
    }
    return CMBX_OK;
  }
  if (lane > 0) return CMBX_OK;  // pipelined groups run in lane 0
  int tx = 0, ty = 0, lz = 0;
  if (!cmbx::pipeline_shape(gr.dtype, gr.N, &tx, &ty, &lz)) return fail(CMBX_EUNSUPPORTED, "no pipelined kernel");
  for (const Item& it : gr.items)
    if (it.fp && !it.fixed)
      if (int rc = enqueue_footprint(it.plan, it.fp, it.r, it.dirs, it.n_pix, s, lz)) return rc;
  for (size_t i = 0; i < gr.pipe.size(); ++i) {
    cmbx::PipeLaunch a = gr.pipe[i];
    a.sched = dsched + gr.sched_off[i];
    HIP_TRY(cmbx::launch_pipeline(a, s));
  }
  return CMBX_OK;
}

// The footprints of the items whose plans fix the directions, for each group's mode (its
// plan's z tile chained, the pipelined kernel's otherwise), made now on a stream of their
// own and waited for: the graphs then do not remake them at every launch.
int make_fixed_footprints(const std::vector<Group>& groups) {
  bool any = false;
  for (const Group& gr : groups)
    for (const Item& it : gr.items) any = any || (it.fp && it.fixed);
  if (!any) return CMBX_OK;
  hipStream_t st = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  int rc = CMBX_OK;
  for (const Group& gr : groups) {
    int tx = 0, ty = 0, lz = 0;
    if (gr.mode != CMBX_ENS_CHAINED && !cmbx::pipeline_shape(gr.dtype, gr.N, &tx, &ty, &lz)) lz = 0;
    for (const Item& it : gr.items)
      if (rc == CMBX_OK && it.fp && it.fixed)
        rc = enqueue_footprint(it.plan, it.fp, it.r, it.dirs, it.n_pix, st, gr.mode == CMBX_ENS_CHAINED ? 0 : lz);
  }
  const hipError_t e = hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (rc != CMBX_OK) return rc;
  if (e != hipSuccess) return fail(CMBX_EHIP, "fixed footprints: %s", hipGetErrorString(e));
  return CMBX_OK;
}

// The pixel orders of the items whose plans fix the directions (chained mode's gathers
// read them), made on a stream of their own in one shared work space and waited for.
int make_fixed_orders(const std::vector<Group>& groups) {
  size_t sb = 0;
  for (const Group& gr : groups)
    for (const Item& it : gr.items)
      if (it.ord) {
        size_t b = 0;
        HIP_TRY(cmbx::pixel_order_scratch_bytes(it.plan->N, it.n_pix, &b));
        sb = std::max(sb, b);
      }
  if (sb == 0) return CMBX_OK;
  void* scratch = nullptr;
  hipError_t e = hipMalloc(&scratch, sb);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "pixel orders: %s", hipGetErrorString(e));
  hipStream_t st = nullptr;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  int rc = CMBX_OK;
  for (const Group& gr : groups)
    for (const Item& it : gr.items)
      if (e == hipSuccess && rc == CMBX_OK && it.ord)
        rc = enqueue_pixel_order(it.plan, it.ord, scratch, sb, it.r, it.dirs, it.n_pix, st);
  if (st) {
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
    (void)hipStreamDestroy(st);
  }
  (void)hipFree(scratch);
  if (rc != CMBX_OK) return rc;
  if (e != hipSuccess) return fail(CMBX_EHIP, "pixel orders: %s", hipGetErrorString(e));
  return CMBX_OK;
}

// Capture the groups (each in its chosen mode, or all in `force` if >= 0; only group
// `only` if >= 0; only the items of `lane` if >= 0) into a graph.
int capture(const std::vector<Group>& groups, const uint32_t* dsched, int only, int force, int lane,
            hipGraph_t* graph, hipGraphExec_t* exec) {
  if (fault("capture")) return fail(CMBX_EHIP, "ensemble capture: injected fault (CMBX_FAULT)");
  hipStream_t cap = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  int rc = CMBX_OK;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  for (size_t gi = 0; e == hipSuccess && rc == CMBX_OK && gi < groups.size(); ++gi) {
    if (only >= 0 && (int)gi != only) continue;
    rc = enqueue_group(groups[gi], force >= 0 ? force : groups[gi].mode, dsched, cap, lane);
  }
  hipGraph_t gph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(cap, &gph);
  if (e == hipSuccess) e = e_end;
  (void)hipStreamDestroy(cap);
  if (rc == CMBX_OK && e == hipSuccess) e = hipGraphInstantiate(exec, gph, nullptr, nullptr, 0);
  if (rc != CMBX_OK || e != hipSuccess) {
    if (gph) (void)hipGraphDestroy(gph);
    if (rc != CMBX_OK) return rc;
    return fail(CMBX_EHIP, "ensemble capture: %s", hipGetErrorString(e));
  }
  *graph = gph;
  return CMBX_OK;
}

// Split the chained items over up to `want` lanes by plan, largest work first into the
// lightest lane. Returns the number of lanes used: at most the number of chained plans
// (1: everything in lane 0).
int assign_lanes(std::vector<Group>& groups, int want) {
  std::vector<const cmbx_plan*> plans;
  std::vector<double> cost;
  for (Group& gr : groups) {
    for (Item& it : gr.items) {
      it.lane = 0;
      if (gr.mode != CMBX_ENS_CHAINED) continue;
      size_t k = 0;
      while (k < plans.size() && plans[k] != it.plan) ++k;
      if (k == plans.size()) plans.push_back(it.plan), cost.push_back(0.0);
      cost[k] += (double)it.plan->N * it.plan->N * it.plan->N + (double)it.n_pix;
    }
  }
  const int nl = std::min<int>(want, (int)plans.size());
  if (nl < 2) return 1;
  std::vector<size_t> order(plans.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<double> load(nl, 0.0);
  std::vector<int> lane_of(plans.size(), 0);
  for (size_t k : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lane_of[k] = l;
    load[l] += cost[k];
  }
  for (Group& gr : groups)
    for (Item& it : gr.items) {
      if (gr.mode != CMBX_ENS_CHAINED) continue;
      size_t k = 0;
      while (plans[k] != it.plan) ++k;
      it.lane = lane_of[k];
    }
  return nl;
}

void clear_lanes(cmbx_ensemble* en) {
  for (hipGraphExec_t x : en->exec)
    if (x) (void)hipGraphExecDestroy(x);
  for (hipGraph_t gph : en->graph)
    if (gph) (void)hipGraphDestroy(gph);
  for (hipStream_t st : en->streams)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : en->done)
    if (ev) (void)hipEventDestroy(ev);
  if (en->fork) (void)hipEventDestroy(en->fork);
  en->exec.clear();
  en->graph.clear();
  en->streams.clear();
  en->done.clear();
  en->fork = nullptr;
}

// Capture `lanes` graphs (lane 0 also holds the pipelined groups) and their streams.
int build_lanes(cmbx_ensemble* en, const std::vector<Group>& groups, const uint32_t* dsched, int lanes) {
  for (int l = 0; l < lanes; ++l) {
    hipGraph_t gph = nullptr;
    hipGraphExec_t ex = nullptr;
    if (int rc = capture(groups, dsched, -1, -1, lanes == 1 ? -1 : l, &gph, &ex)) return rc;
    en->graph.push_back(gph);
    en->exec.push_back(ex);
  }
  if (lanes > 1) {
    HIP_TRY(hipEventCreateWithFlags(&en->fork, hipEventDisableTiming));
    for (int l = 1; l < lanes; ++l) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      en->streams.push_back(st);
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      en->done.push_back(ev);
    }
  }
  return CMBX_OK;
}

// Lane 0 on s; the other lanes forked from s onto their streams and joined back into s.
int launch_lanes(cmbx_ensemble* en, hipStream_t s) {
  const size_t nl = en->exec.size();
  if (nl > 1) HIP_TRY(hipEventRecord(en->fork, s));
  for (size_t i = 1; i < nl; ++i) {
    HIP_TRY(hipStreamWaitEvent(en->streams[i - 1], en->fork, 0));
    HIP_TRY(hipGraphLaunch(en->exec[i], en->streams[i - 1]));
    HIP_TRY(hipEventRecord(en->done[i - 1], en->streams[i - 1]));
  }
  HIP_TRY(hipGraphLaunch(en->exec[0], s));
  for (size_t i = 1; i < nl; ++i) HIP_TRY(hipStreamWaitEvent(s, en->done[i - 1], 0));
  return CMBX_OK;
}

// Average milliseconds of an ensemble's launch over 16 launches after three warm-ups
// (-1 on error).
double time_ensemble(cmbx_ensemble* en) {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double ms = -1.0;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess) {
    int rc = CMBX_OK;
    for (int i = 0; rc == CMBX_OK && i < 3; ++i) rc = launch_lanes(en, s);
    hipError_t e = rc == CMBX_OK ? hipEventRecord(e0, s) : hipErrorUnknown;
    for (int i = 0; e == hipSuccess && rc == CMBX_OK && i < 16; ++i) rc = launch_lanes(en, s);
    if (e == hipSuccess && rc == CMBX_OK) e = hipEventRecord(e1, s);
    if (e == hipSuccess && rc == CMBX_OK) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess && rc == CMBX_OK && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / 16.0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  return ms;
}

// Average milliseconds of a graph over three launches after two warm-ups (-1 on error).
double time_graph(hipGraphExec_t exec) {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double ms = -1.0;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess) {
    hipError_t e = hipSuccess;
    for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; e == hipSuccess && i < 3; ++i) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / 3.0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  return ms;
}

}  // namespace

int cmbx_ensemble_create(const cmbx_job* jobs, int n_jobs, int mode, cmbx_ensemble** out) {
  if (!out) return fail(CMBX_EINVAL, "out is NULL");
  *out = nullptr;
  const int lanes_flag = (mode >> 8) & 7;  // lanes asked for, 0 = auto
  mode &= ~0x700;
  if (mode != CMBX_ENS_AUTO && mode != CMBX_ENS_CHAINED && mode != CMBX_ENS_PIPELINED)
    return fail(CMBX_EINVAL, "unknown ensemble mode %d", mode);
  if (lanes_flag > CMBX_ENS_MAX_LANES)
    return fail(CMBX_EINVAL, "%d lanes asked for; at most %d", lanes_flag, CMBX_ENS_MAX_LANES);
  if (!jobs || n_jobs < 1) return fail(CMBX_EINVAL, "need at least one job");
  for (int j = 0; j < n_jobs; ++j) {
    if (!jobs[j].plan) return fail(CMBX_EINVAL, "job %d has no plan", j);
    if (int rc = check_patch_args(jobs[j].plan, jobs[j].r, jobs[j].dirs, jobs[j].n_pix, jobs[j].out)) {
      cmbx::err_msg() = "job " + std::to_string(j) + ": " + cmbx::err_msg();
      return rc;
    }
    if (jobs[j].plan->device != jobs[0].plan->device) return fail(CMBX_EINVAL, "all jobs must be on one device");
  }
  DeviceGuard g(jobs[0].plan->device);
  // Realisations grouped by (precision, N), in job order.
  std::vector<Group> groups;
  std::map<std::pair<int, int>, size_t> index;
  for (int j = 0; j < n_jobs; ++j) {
    const cmbx_plan* p = jobs[j].plan;
    const auto key = std::make_pair(p->dtype, p->N);
    if (!index.count(key)) {
      index[key] = groups.size();
      groups.emplace_back();
      groups.back().dtype = p->dtype;
      groups.back().N = p->N;
    }
    Group& gr = groups[index[key]];
    for (int b = 0; b < p->batch; ++b)
      gr.items.push_back(Item{p, b, jobs[j].seed + (uint64_t)b, jobs[j].r, jobs[j].dirs, jobs[j].n_pix,
                              (char*)jobs[j].out + (size_t)b * jobs[j].n_pix * p->real_size()});
  }
  // Within a group the chained mode runs items one after another in their plans'
  // workspaces; a plan used by two jobs is fine there (they run in order).
  cmbx_ensemble* en = new cmbx_ensemble;
  en->device = jobs[0].plan->device;
  for (int j = 0; j < n_jobs; ++j) en->bounds.emplace_back(jobs[j].plan, jobs[j].plan->m_hi);
  auto bail = [&](int code, const std::string& msg) {
    clear_lanes(en);
    for (void* d : en->dev) (void)hipFree(d);
    for (void* d : en->fps) (void)hipFree(d);
    delete en;
    return code == CMBX_OK ? CMBX_OK : fail(code, "%s", msg.c_str());
  };
  // a footprint per realisation of a pruning plan, made inside the graph at every launch
  // (from the pixel directions as they are then)
  for (Group& gr : groups)
    for (Item& it : gr.items) {
      if (!it.plan->prune) continue;
      void* f = nullptr;
      const hipError_t e = hipMalloc(&f, cmbx::footprint_bytes(it.plan->N));
      if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "ensemble footprints");
      en->fps.push_back(f);
      it.fp = f;
      it.fixed = it.plan->fixed_dirs;
    }
  // with fixed directions, a pixel order per realisation for the chained gathers
  for (Group& gr : groups)
    for (Item& it : gr.items) {
      if (!it.plan->fixed_dirs) continue;
      void* o = nullptr;
      const hipError_t e = hipMalloc(&o, cmbx::pixel_order_bytes(it.plan->dtype, it.n_pix));
      if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "ensemble pixel orders");
      en->fps.push_back(o);
      it.ord = o;
    }
  // fixed footprints and orders are valid before any launch (the timing launches of auto
  // mode included)
  if (int rc = make_fixed_footprints(groups)) return bail(rc, cmbx::err_msg());
  if (int rc = make_fixed_orders(groups)) return bail(rc, cmbx::err_msg());
  std::vector<uint32_t> sched;
  if (mode != CMBX_ENS_CHAINED) {
    for (Group& gr : groups) {
      const int N = gr.N, M = N / 2;
      const cmbx_plan* p0 = gr.items[0].plan;
      int tx, ty, lz;
      if (!cmbx::pipeline_shape(gr.dtype, N, &tx, &ty, &lz)) return bail(CMBX_EUNSUPPORTED, "no pipelined kernel");
      const int n = (int)gr.items.size();
      const int nbuf = n < 4 ? n : 4;
      gr.bufs.assign(nbuf, nullptr);
      for (int i = 0; i < nbuf; ++i) {
        const hipError_t e = hipMalloc(&gr.bufs[i], p0->field_bytes());
        if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? CMBX_ENOMEM : CMBX_EHIP, "ensemble workspace");
        en->dev.push_back(gr.bufs[i]);
      }
      for (int t = 0; t < n + 3; ++t) {
        const int ix = t, iy = t - 1, iz = t - 2, ig = t - 3;
        int64_t cnt[4] = {0, 0, 0, 0};
        cmbx::PipeLaunch a{};
        a.dtype = gr.dtype;
        a.N = N;
        a.tw = p0->tw;
        if (ix < n) {
          cnt[0] = (int64_t)(M / tx) * N;
          a.bx = gr.bufs[ix % nbuf];
          a.wtab_x = gr.items[ix].plan->wtab;
          a.m_hi_x = gr.items[ix].plan->m_hi;
          a.fp_x = gr.items[ix].fp;
          a.k0 = (uint32_t)(gr.items[ix].seed & 0xffffffffu);
          a.k1 = (uint32_t)(gr.items[ix].seed >> 32);
        }
        if (iy >= 0 && iy < n) {
          cnt[1] = (int64_t)(M / ty) * N;
          a.by = gr.bufs[iy % nbuf];
          a.m_hi_y = gr.items[iy].plan->m_hi;
          a.fp_y = gr.items[iy].fp;
        }
        if (iz >= 0 && iz < n) {
          cnt[2] = (int64_t)N * N / lz;
          a.bz = gr.bufs[iz % nbuf];
          a.m_hi_z = gr.items[iz].plan->m_hi;
          a.fp_z = gr.items[iz].fp;
        }
        if (ig >= 0 && ig < n) {
          const Item& it = gr.items[ig];
          cnt[3] = (it.n_pix + cmbx::kPipeThreads - 1) / cmbx::kPipeThreads;
          a.field_g = gr.bufs[ig % nbuf];
          a.dirs = it.dirs;
          a.order = it.ord;
          a.out = it.out;
          a.npix = it.n_pix;
          a.r = it.r;
          a.scale = (double)N / it.plan->L;
          for (int d = 0; d < 3; ++d) a.obs[d] = it.plan->obs[d];
          a.cubic = it.plan->interp == CMBX_TRICUBIC;
        }
        gr.sched_off.push_back(sched.size());
        interleave(cnt, sched);
        a.nblocks = (int)(sched.size() - gr.sched_off.back());
        gr.pipe.push_back(a);
      }
    }
  }
  uint32_t* dsched = nullptr;
  if (!sched.empty()) {
    hipError_t e = hipMalloc((void**)&dsched, sched.size() * sizeof(uint32_t));
    if (e != hipSuccess) return bail(CMBX_ENOMEM, "ensemble schedule");
    en->dev.push_back(dsched);
    e = hipMemcpy(dsched, sched.data(), sched.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(CMBX_EHIP, std::string("schedule upload: ") + hipGetErrorString(e));
  }
  for (Group& gr : groups) gr.mode = mode == CMBX_ENS_AUTO ? CMBX_ENS_CHAINED : mode;
  if (mode == CMBX_ENS_AUTO) {
    // time each group alone in both modes and keep the faster
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      double t[2] = {-1.0, -1.0};
      const int modes[2] = {CMBX_ENS_CHAINED, CMBX_ENS_PIPELINED};
      for (int k = 0; k < 2; ++k) {
        hipGraph_t gph = nullptr;
        hipGraphExec_t ex = nullptr;
        if (int rc = capture(groups, dsched, (int)gi, modes[k], -1, &gph, &ex)) return bail(rc, cmbx::err_msg());
        t[k] = time_graph(ex);
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(gph);
        if (t[k] < 0) return bail(CMBX_EHIP, "ensemble autotune launch failed");
      }
      groups[gi].mode = t[1] < t[0] ? CMBX_ENS_PIPELINED : CMBX_ENS_CHAINED;
    }
  }
  // Lanes: the chained items are split by plan (items of one plan share its workspace and
  // stay in one lane) into up to CMBX_ENS_MAX_LANES graphs that run on as many streams.
  std::vector<int> chosen;
  for (const Group& gr : groups) chosen.push_back(gr.mode);
  auto set_modes = [&](const std::vector<int>& m, int want) {
    for (size_t gi = 0; gi < groups.size(); ++gi) groups[gi].mode = m[gi];
    return assign_lanes(groups, want);  // lanes usable
  };
  if (mode != CMBX_ENS_AUTO || lanes_flag != 0) {
    const int lanes = set_modes(chosen, lanes_flag > 0 ? lanes_flag : 1);
    if (int rc = make_fixed_footprints(groups)) return bail(rc, cmbx::err_msg());
    if (int rc = build_lanes(en, groups, dsched, lanes)) return bail(rc, cmbx::err_msg());
  } else {
    // AUTO: time the whole ensemble in each candidate -- the modes chosen per group, and
    // every group chained (the chains of different plans then overlap, which a group
    // timed alone does not show), on 1 .. CMBX_ENS_MAX_LANES lanes -- keep the fastest
    struct Cand {
      std::vector<int> modes;
      int lanes;
    };
    std::vector<Cand> cands;
    const std::vector<int> all_chained(groups.size(), CMBX_ENS_CHAINED);
    for (const std::vector<int>* m : {(const std::vector<int>*)&chosen, &all_chained}) {
      if (m == &all_chained && all_chained == chosen) break;
      for (int want = 1; want <= CMBX_ENS_MAX_LANES; ++want) {
        const int got = set_modes(*m, want);
        if (got == want && !(m == &all_chained && want == 1)) cands.push_back({*m, want});
      }
    }
    // six sweeps over every candidate, in alternating order, each candidate scored by the
    // median of its six times: the candidates are a few percent apart, as much as the clock
    // drifts over a sweep, and a best-of-sweeps score favoured the candidates of widest
    // spread (more lanes: four had timed level with two and then ran 5-7 % slower in steady
    // state; re-timing only the two fastest of the first sweep had kept a candidate that
    // lost by 5 %)
    constexpr int kSweeps = 6;
    std::vector<std::vector<double>> ts(cands.size());
    auto time_cand = [&](size_t c) -> int {
      set_modes(cands[c].modes, cands[c].lanes);
      clear_lanes(en);
      if (int rc = build_lanes(en, groups, dsched, cands[c].lanes)) return rc;
      const double t = time_ensemble(en);
      if (t < 0) return fail(CMBX_EHIP, "ensemble timing failed");
      ts[c].push_back(t);
      return CMBX_OK;
    };
    size_t best = 0;
    if (cands.size() > 1) {
      for (int round = 0; round < kSweeps; ++round)
        for (size_t c = 0; c < cands.size(); ++c)
          if (int rc = time_cand(round % 2 ? cands.size() - 1 - c : c)) return bail(rc, cmbx::err_msg());
      std::vector<double> tc(cands.size());
      for (size_t c = 0; c < cands.size(); ++c) {
        std::sort(ts[c].begin(), ts[c].end());
        tc[c] = 0.5 * (ts[c][kSweeps / 2 - 1] + ts[c][kSweeps / 2]);
      }
      for (size_t c = 1; c < cands.size(); ++c)
        if (tc[c] < tc[best]) best = c;
      // within 1 % of the fastest the fewest lanes win, but two rather than one where two
      // exist: one lane runs the chains strictly one after another, and where it timed
      // level with two at creation, two ran 2-4 % faster in steady state (and one 1 %
      // slower than the plans on their own streams)
      const double fastest = tc[best];
      int two = 0;
      for (const Cand& cd : cands) two |= cd.lanes == 2;
      auto rank = [&](int lanes) { return two && lanes == 1 ? 3 : lanes; };
      for (size_t c = 0; c < cands.size(); ++c)
        if (tc[c] <= 1.01 * fastest && rank(cands[c].lanes) < rank(cands[best].lanes)) best = c;
    }
    set_modes(cands[best].modes, cands[best].lanes);
    clear_lanes(en);
    if (int rc = make_fixed_footprints(groups)) return bail(rc, cmbx::err_msg());
    if (int rc = build_lanes(en, groups, dsched, cands[best].lanes)) return bail(rc, cmbx::err_msg());
  }
  bool any_pipe = false;
  for (const Group& gr : groups) {
    en->modes.push_back(gr.mode);
    any_pipe = any_pipe || gr.mode == CMBX_ENS_PIPELINED;
  }
  if (!any_pipe) {
    // the rotating workspaces and the schedule are not used by the chosen graph
    for (void* d : en->dev) (void)hipFree(d);
    en->dev.clear();
  }
  *out = en;
  return ok();
}

int cmbx_ensemble_modes(const cmbx_ensemble* en, int* modes, int cap) {
  if (!en) return fail(CMBX_EINVAL, "ensemble is NULL");
  const int n = (int)en->modes.size();
  for (int i = 0; modes && i < n && i < cap; ++i) modes[i] = en->modes[i];
  return n;
}

int cmbx_noise_tables(float* out, int cap) {
  if (!out || cap < cmbx::kNoiseTableSize)
    return fail(CMBX_EINVAL, "noise tables need a buffer of %d floats", cmbx::kNoiseTableSize);
  fill_noise_tables(out);
  return cmbx::kNoiseTableSize;
}

int cmbx_ensemble_lanes(const cmbx_ensemble* en) {
  if (!en) return fail(CMBX_EINVAL, "ensemble is NULL");
  return (int)en->exec.size();
}

int cmbx_ensemble_launch(cmbx_ensemble* en, void* stream) {
  if (!en) return fail(CMBX_EINVAL, "ensemble is NULL");
  if (fault("launch")) return fail(CMBX_EHIP, "ensemble launch: injected fault (CMBX_FAULT)");
  for (const auto& b : en->bounds)
    if (b.first->m_hi > b.second)
      return fail(CMBX_ESTATE, "a plan's spectrum now reaches |f|^2 = %d, beyond the %d its kernels were captured with: "
                  "create the ensemble again", b.first->m_hi, b.second);
  DeviceGuard g(en->device);
  if (int rc = launch_lanes(en, (hipStream_t)stream)) return rc;
  return ok();
}

int cmbx_ensemble_destroy(cmbx_ensemble* en) {
  if (!en) return ok();
  DeviceGuard g(en->device);
  (void)hipDeviceSynchronize();
  clear_lanes(en);
  for (void* d : en->dev) (void)hipFree(d);
  for (void* d : en->fps) (void)hipFree(d);
  delete en;
  return ok();
}

int cmbx_time_passes(cmbx_plan* p, uint64_t seed, double r, const double* dirs, int64_t n_pix, void* out, int reps,
                     double* ms) {
  if (int rc = check_plan(p)) return rc;
  if (int rc = check_patch_args(p, r, dirs, n_pix, out)) return rc;
  if (reps < 1 || !ms) return fail(CMBX_EINVAL, "reps must be >= 1 and ms non-NULL");
  DeviceGuard g(p->device);
  cmbx::FieldArgs a = field_args(p, seed, p->field);
  // the passes as cmbx_simulate_patch runs them: with the map's footprint if the plan
  // prunes (made once, before the timed launches)
  if (p->prune) {
    p->fp_key.valid = false;
    if (int rc = enqueue_footprint(p, p->fp, r, dirs, n_pix, p->stream)) return rc;
    a.fp = p->fp;
  }
  // and the gather in the pixel order if the plan fixes the directions
  const void* order = nullptr;
  if (int rc = plan_pixel_order(p, r, dirs, n_pix, p->stream, &order)) return rc;
  // per kernel: one untimed launch, then the timed ones between two events; the first
  // timed launch is queued while the untimed one runs, so the host's submission delay
  // after an event is not counted as kernel time
  hipEvent_t ev[8] = {};
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  int rc = CMBX_OK;
  hipError_t e = hipSuccess;
  auto launch = [&](int k) -> int {
    if (k == 3) return enqueue_gather(p, p->field, r, dirs, n_pix, out, p->stream, order);
    const hipError_t he = k == 0 ? cmbx::launch_pass_x(a, p->stream)
                          : k == 1 ? cmbx::launch_pass_y(a, p->stream)
                                   : cmbx::launch_pass_z(a, p->stream);
    return he == hipSuccess ? CMBX_OK : fail(CMBX_EHIP, "pass %d launch: %s", k, hipGetErrorString(he));
  };
  for (int k = 0; k < 4 && e == hipSuccess && rc == CMBX_OK; ++k) {
    rc = launch(k);
    if (rc == CMBX_OK) e = hipEventRecord(ev[2 * k], p->stream);
    for (int i = 0; e == hipSuccess && rc == CMBX_OK && i < reps; ++i) rc = launch(k);
    if (e == hipSuccess && rc == CMBX_OK) e = hipEventRecord(ev[2 * k + 1], p->stream);
  }
  if (e == hipSuccess && rc == CMBX_OK) e = hipEventSynchronize(ev[7]);
  for (int i = 0; e == hipSuccess && rc == CMBX_OK && i < 4; ++i) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
    ms[i] = (double)t / reps;
  }
  for (auto& ee : ev) (void)hipEventDestroy(ee);
  if (rc != CMBX_OK) return rc;
  if (e != hipSuccess) return fail(CMBX_EHIP, "pass timing: %s", hipGetErrorString(e));
  return ok();
}

int cmbx_tile_choices(int dtype, int N, int which, int* out) {
  if (!out || (which != 0 && which != 1)) return 0;
  int tmp[4];
  const int n = which == 0 ? cmbx::tile_xy_choices(dtype, N, tmp) : cmbx::lines_z_choices(dtype, N, tmp);
  for (int i = 0; i < n; ++i) out[i] = tmp[i];
  return n;
}

namespace {

// The autotuner; with dirs (and a pruning plan) it times the passes as a map of those
// pixels makes them: from the footprint, its z list rebuilt for each z tile tried.
int autotune(cmbx_plan* p, int reps, int* best, double* ms, double r, const double* dirs, int64_t n_pix) {
  if (int rc = check_plan(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (reps < 1) return fail(CMBX_EINVAL, "reps = %d must be >= 1", reps);
  DeviceGuard g(p->device);
  const bool pruned = dirs != nullptr && p->prune;
  int tz[4], ln[4];
  const int ntz = cmbx::tile_xy_choices(p->dtype, p->N, tz);
  const int nln = cmbx::lines_z_choices(p->dtype, p->N, ln);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  cmbx::FieldArgs a = field_args(p, 0x5eedull, p->field);
  if (pruned) a.fp = p->fp;
  int fp_lines = -1;
  // the footprint with the z list for the z tile in `a` (made before the timed launches)
  auto prepare = [&]() -> int {
    if (!pruned) return CMBX_OK;
    const int lines = cmbx::resolve_lines_z(p->dtype, p->N, a.lines_z);
    if (lines == fp_lines) return CMBX_OK;
    p->fp_key.valid = false;
    if (int rc = enqueue_footprint(p, p->fp, r, dirs, n_pix, p->stream, lines)) return rc;
    fp_lines = lines;
    return CMBX_OK;
  };
  auto launch = [&](int which) {
    return which == 0 ? cmbx::launch_pass_x(a, p->stream)
           : which == 1 ? cmbx::launch_pass_y(a, p->stream)
                        : cmbx::launch_pass_z(a, p->stream);
  };
  // average ms of `reps` launches of the passes first .. last (after one warm-up round),
  // or a negative value on error
  auto time_passes = [&](int first, int last) -> double {
    hipError_t e = hipSuccess;
    for (int w = first; e == hipSuccess && w <= last; ++w) e = launch(w);
    if (e == hipSuccess) e = hipEventRecord(e0, p->stream);
    for (int i = 0; e == hipSuccess && i < reps; ++i)
      for (int w = first; e == hipSuccess && w <= last; ++w) e = launch(w);
    if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    return e == hipSuccess ? (double)t / reps : -1.0;
  };
  int* opt[3] = {&a.tile_x, &a.tile_y, &a.lines_z};
  int* optp[3] = {&a.plan_x, &a.plan_y, &a.plan_z};
  int pick[3] = {p->tile_x, p->tile_y, p->lines_z};
  int pickp[3] = {p->plan_x, p->plan_y, p->plan_z};
  double tbest[3] = {0, 0, 0};
  bool bad = false;
  // Each shape is judged by the whole x -> y -> z chain, not by its own kernel alone: a
  // pass's write pattern changes what the next pass pays (narrow x tiles time as fast as
  // wide ones in isolation but slow pass y down). Coordinate descent, two sweeps, over each
  // pass's compiled choices: every tile with stage plan 0, and the default tile with the
  // alternative stage plan 1 where there is one.
  for (int sweep = 0; sweep < 2 && !bad; ++sweep) {
    for (int which = 0; which < 3 && !bad; ++which) {
      const int n = which == 2 ? nln : ntz;
      const int* vals = which == 2 ? ln : tz;
      const int ncand = n + (cmbx::stage_plan_compiled(p->dtype, p->N, which) ? 1 : 0);
      double best_t = 1e300;
      for (int i = 0; i < ncand && !bad; ++i) {
        for (int o = 0; o < 3; ++o) *opt[o] = pick[o], *optp[o] = pickp[o];
        *opt[which] = i < n ? vals[i] : vals[0];
        *optp[which] = i < n ? 0 : 1;
        if (prepare() != CMBX_OK) {
          bad = true;
          break;
        }
        const double t = time_passes(0, 2);
        if (t < 0) bad = true;
        else if (t < best_t) best_t = t, pick[which] = *opt[which], pickp[which] = *optp[which];
      }
    }
  }
  for (int o = 0; o < 3; ++o) *opt[o] = pick[o], *optp[o] = pickp[o];
  if (!bad && prepare() != CMBX_OK) bad = true;
  for (int which = 0; which < 3 && !bad; ++which) {
    tbest[which] = time_passes(which, which);
    if (tbest[which] < 0) bad = true;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (bad) return fail(CMBX_EHIP, "autotune launch failed: %s", hipGetErrorString(hipGetLastError()));
  p->tile_x = pick[0];
  p->tile_y = pick[1];
  p->lines_z = pick[2];
  p->plan_x = pickp[0];
  p->plan_y = pickp[1];
  p->plan_z = pickp[2];
  for (int i = 0; i < 3; ++i) {
    if (best) best[i] = pick[i];
    if (ms) ms[i] = tbest[i];
  }
  return ok();
}

}  // namespace

int cmbx_plan_autotune(cmbx_plan* p, int reps, int* best, double* ms) {
  return autotune(p, reps, best, ms, 0.0, nullptr, 0);
}

int cmbx_plan_autotune_patch(cmbx_plan* p, int reps, double r, const double* dirs, int64_t n_pix, int* best,
                             double* ms) {
  if (int rc = check_plan(p)) return rc;
  if (int rc = check_radius(p, r)) return rc;
  if (n_pix < 1 || n_pix > (int64_t)1 << 31) return fail(CMBX_EINVAL, "bad n_pix %lld", (long long)n_pix);
  if (!dirs) return fail(CMBX_EINVAL, "dirs must be a non-NULL device pointer");
  return autotune(p, reps, best, ms, r, dirs, n_pix);
}

int cmbx_enqueue_stage(cmbx_plan* p, int stage, uint64_t seed, void* buf, double r, const double* dirs,
                       int64_t n_pix, void* out, void* stream) {
  if (int rc = check_plan(p)) return rc;
  if (!p->has_spectrum) return fail(CMBX_ESTATE, "no spectrum set");
  if (!buf || (uintptr_t)buf % 16 != 0) return fail(CMBX_EINVAL, "buf must be a 16-byte aligned device pointer");
  if (stage < 0 || stage > 3) return fail(CMBX_EINVAL, "stage = %d must be 0..3", stage);
  if (stage == 3)
    if (int rc = check_patch_args(p, r, dirs, n_pix, out)) return rc;
  DeviceGuard g(p->device);
  hipStream_t s = (hipStream_t)stream;
  const cmbx::FieldArgs a = field_args(p, seed, buf);
  switch (stage) {
    case 0: HIP_TRY(cmbx::launch_pass_x(a, s)); break;
    case 1: HIP_TRY(cmbx::launch_pass_y(a, s)); break;
    case 2: HIP_TRY(cmbx::launch_pass_z(a, s)); break;
    default:
      if (int rc = enqueue_gather(p, buf, r, dirs, n_pix, out, s)) return rc;
  }
  return ok();
}

int cmbx_mlp_gemm(int M, int N, int K, const float* A, int lda, int transA, const void* B, int ldb, int transB,
                  int b_bf16, float* C, int ldc, const float* bias, int act, float* Y, int ldy, void* stream) {
  if (M < 1 || N < 1 || K < 1) return fail(CMBX_EINVAL, "gemm sizes must be >= 1 (M=%d N=%d K=%d)", M, N, K);
  if (!A || !B || !C) return fail(CMBX_EINVAL, "gemm operands must be non-NULL");
  if (lda < (transA ? M : K) || ldb < (transB ? K : N) || ldc < N || (Y && ldy < N))
    return fail(CMBX_EINVAL, "gemm leading dimension shorter than a row");
  cmbx::GemmArgs g{M, N, K, A, lda, transA ? 1 : 0, B, ldb, transB ? 1 : 0, b_bf16 ? 1 : 0, C, ldc, bias, act ? 1 : 0,
                   Y, ldy};
  HIP_TRY(cmbx::launch_gemm(g, (hipStream_t)stream));
  return ok();
}

int cmbx_mlp_gelu_backward(const float* Z, const float* dY, float* dZ, int64_t n, void* stream) {
  if (!Z || !dY || !dZ || n < 1) return fail(CMBX_EINVAL, "gelu_backward: bad arguments");
  HIP_TRY(cmbx::launch_gelu_backward(Z, dY, dZ, n, (hipStream_t)stream));
  return ok();
}

int cmbx_mlp_colsum(const float* X, int rows, int cols, float* out, void* stream) {
  if (!X || !out || rows < 1 || cols < 1) return fail(CMBX_EINVAL, "colsum: bad arguments");
  HIP_TRY(cmbx::launch_colsum(X, rows, cols, out, (hipStream_t)stream));
  return ok();
}

int64_t cmbx_mlp_mse_partials(int64_t n) { return n < 1 ? 0 : cmbx::mse_partials(n); }

int cmbx_mlp_mse(const float* Y, const float* T, int64_t n, float* dY, float* partial, float* loss, void* stream) {
  if (!Y || !T || !dY || !partial || !loss || n < 1) return fail(CMBX_EINVAL, "mse: bad arguments");
  if (cmbx::mse_partials(n) > (1 << 24)) return fail(CMBX_EINVAL, "mse: n too large");
  HIP_TRY(cmbx::launch_mse(Y, T, n, dY, partial, loss, (hipStream_t)stream));
  return ok();
}

int cmbx_mlp_mse_noalloc(const float* Y, const float* T, int64_t n, float* dY, float* loss, void* stream) {
  if (!Y || !T || !dY || !loss || n < 1) return fail(CMBX_EINVAL, "mse_noalloc: bad arguments");
  if (n > CMBX_MSE_NOALLOC_MAX)
    return fail(CMBX_EINVAL, "mse_noalloc: n = %lld exceeds the static workspace's limit %lld", (long long)n,
                (long long)CMBX_MSE_NOALLOC_MAX);
  static_assert(CMBX_MSE_NOALLOC_MAX == cmbx::kMseScratchFloats * 256, "limit of the static workspace");
  HIP_TRY(cmbx::launch_mse_noalloc(Y, T, n, dY, loss, (hipStream_t)stream));
  return ok();
}

int cmbx_mlp_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float beta1, float beta2, float eps,
                  int step, uint16_t* w_bf16, void* stream) {
  if (!w || !m || !v || !g || n < 1 || step < 1) return fail(CMBX_EINVAL, "adam: bad arguments");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return fail(CMBX_EINVAL, "adam: betas must be in [0, 1) and eps > 0");
  cmbx::AdamArgs a{w, m, v, g, n, lr, beta1, beta2, eps, 1.f - std::pow(beta1, (float)step),
                   1.f - std::pow(beta2, (float)step), w_bf16};
  HIP_TRY(cmbx::launch_adam(a, (hipStream_t)stream));
  return ok();
}

int cmbx_bf16_round(const float* x, uint16_t* y, int64_t n, void* stream) {
  if (!x || !y || n < 1) return fail(CMBX_EINVAL, "bf16_round: bad arguments");
  HIP_TRY(cmbx::launch_to_bf16(x, y, n, (hipStream_t)stream));
  return ok();
}

const char* cmbx_last_error(void) { return cmbx::err_msg().c_str(); }

const char* cmbx_version(void) { return "cmbx 0.1.0 (gfx950)"; }

}  // extern "C"
