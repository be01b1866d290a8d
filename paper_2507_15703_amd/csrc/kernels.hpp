// Internal interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmbx {

enum { kF32 = 1, kF64 = 2 };
enum { kTrilinear = 1, kTricubic = 2 };

// Box sizes with compiled kernels: N = 2^a 3^b, 8 <= N <= 1024, N/2 also 2^a 3^b.
bool size_compiled(int N);

// Tile choices compiled for (dtype, N). Returns the count written (<= 4); [0] is the default.
int tile_xy_choices(int dtype, int N, int* out);
int lines_z_choices(int dtype, int N, int* out);

// Map footprint: what the interpolation stencils of one map's pixels read. Bytes [0, N):
// x-plane ix is read; then for each ix the footprint_blocks(N) bytes of its 8-row blocks:
// some line (ix, iy) with iy / 8 = block is read; then at footprint_z_offset(N) the
// footprint_zblocks(N) bytes of the 32-node z blocks: some node iz with iz / 32 = block
// is read. 1 = read, 0 = not. Then, 4-byte aligned at footprint_list_offset(N), the work
// lists: a header of four words (the z block size `lines` the z list was made for, the z
// list's count, the plane list's count, 0), the z list -- the indices of the blocks of
// `lines` consecutive (ix, iy) lines that hold a read line, room for N^2 -- and the plane
// list -- the x-planes read, room for N; both in no particular order.
constexpr int footprint_blocks(int N) { return (N + 7) / 8; }
constexpr int footprint_zblocks(int N) { return (N + 31) / 32; }
constexpr size_t footprint_z_offset(int N) { return (size_t)N * (1 + footprint_blocks(N)); }
constexpr size_t footprint_list_offset(int N) { return (footprint_z_offset(N) + footprint_zblocks(N) + 3) & ~(size_t)3; }
constexpr int kFootprintHeader = 4;  // words before the z list
constexpr size_t footprint_bytes(int N) {
  return footprint_list_offset(N) + 4 * (kFootprintHeader + (size_t)N * N + (size_t)N);
}

struct FootprintArgs {
  int interp, N;
  int lines;           // z block (lines per z workgroup) the work list is for
  void* fp;            // footprint_bytes(N), cleared and filled by the launch
  double scale;        // N / L
  double obs[3];       // observer position in the box (L / 2 each: the centre)
  double r;
  const double* dirs;  // [n_pix][3]
  int64_t n_pix;
};
// Three kernels: clear the marks and the list header, mark every pixel's stencil, list
// the z blocks and the planes.
hipError_t launch_footprint(const FootprintArgs& a, hipStream_t s);
// Lines per z workgroup that launch_pass_z uses for (dtype, N) and a lines_z option
// (0 = default); 0 if not compiled.
int resolve_lines_z(int dtype, int N, int lines_z);
// Columns per x/y workgroup for a tile option (0 = default); 0 if not compiled.
int resolve_tile_xy(int dtype, int N, int tile);

struct FieldArgs {
  int dtype, N;
  void* buf;           // N^3 reals, in place (complex N x N x N/2 during the passes)
  const void* wtab;    // sqrt(P_box/2) for |f|^2 = 0 .. 3 (N/2)^2, then sqrt(P_box) x 4
  const void* tw;      // N roots exp(2 pi i m / N), complex, plan precision
  uint32_t k0, k1;     // Philox key (seed words)
  int m_hi;            // largest |f|^2 of nonzero weight: the passes skip what lies beyond
  const void* fp;      // map footprint: only what it marks is made (NULL = the whole field)
  int tile_x, tile_y, lines_z;  // 0 = compiled default
  int plan_x, plan_y, plan_z;   // FFT stage plan of each pass: 0, or 1 (the default tile only)
};
// Whether pass `which` (0 x, 1 y, 2 z) of (dtype, N) has the alternative stage plan 1.
bool stage_plan_compiled(int dtype, int N, int which);

// Pass 1: noise + weights + Hermitian planes + inverse FFT along x.
hipError_t launch_pass_x(const FieldArgs& a, hipStream_t s);
// Pass 2: inverse FFT along y.
hipError_t launch_pass_y(const FieldArgs& a, hipStream_t s);
// Pass 3: complex-to-real inverse FFT along z (unpacks the iz = 0 / N/2 column).
hipError_t launch_pass_z(const FieldArgs& a, hipStream_t s);

// Stacked layers [nlayers][N][N/2] complex (plan precision), in place: c2c transforms
// along the middle axis of every layer (launch_layers_c2c), then c2r transforms of the
// nlayers N contiguous lines of N/2 complex, column 0 packing the rows of frequency 0 and
// N/2, into N reals each (launch_layers_c2r). tw: the N roots exp(2 pi i m / N).
// layers_supported: N is compiled (any nlayers >= 1).
hipError_t launch_layers_c2c(int dtype, int N, void* buf, const void* tw, int nlayers, hipStream_t s);
hipError_t launch_layers_c2r(int dtype, int N, void* buf, const void* tw, int nlayers, hipStream_t s);
bool layers_supported(int dtype, int N, int nlayers);
// Device address of the binary32 Box-Muller tables on the current device.
hipError_t noise_table_address(const float** out);

// Number of binary32 Box-Muller table entries and their upload to the current device
// (before the first single-precision field there; the values never change).
constexpr int kNoiseTableSize = 768;
hipError_t upload_noise_tables(const float* host);

// Unpacked weighted half grid [N][N][N/2+1] (tests).
hipError_t launch_noise_debug(int dtype, int N, void* out, const void* wtab, uint32_t k0, uint32_t k1,
                              hipStream_t s);

struct GatherArgs {
  int dtype, interp, N;
  const void* field;   // [N][N][N] reals
  double scale;        // N / L
  double obs[3];       // observer position in the box
  double r;
  const double* dirs;  // [n_pix][3]
  int64_t n_pix;
  void* out;           // [n_pix]
  const void* order = nullptr;  // the pixel order of (r, dirs) if made (dirs are then not read)
};
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);

// Pixel order of a map whose directions stay fixed: the pixels sorted by the Morton code
// of their stencil's first node (wrapped into the box), each with that node and its
// fractions, so that the threads of a gather wave read the same few field lines. The same
// integer decisions and fractions as the gather's own (stencil_origin), so a map gathered
// in this order is bit-identical. Layout: n_pix records of pixel_order_record_bytes(dtype)
// (packed node x << 20 | y << 10 | z, then the three fractions in the plan's precision),
// then n_pix uint32 pixel indices.
size_t pixel_order_record_bytes(int dtype);
size_t pixel_order_bytes(int dtype, int64_t n_pix);
// Work space of launch_pixel_order (keys and values to sort and the sort's own storage).
hipError_t pixel_order_scratch_bytes(int N, int64_t n_pix, size_t* bytes);
struct PixelOrderArgs {
  int dtype, interp, N;
  double scale, obs[3], r;
  const double* dirs;
  int64_t n_pix;
  void* order;    // pixel_order_bytes(dtype, n_pix)
  void* scratch;  // pixel_order_scratch_bytes(N, n_pix), 256-byte aligned
  size_t scratch_bytes;
};
hipError_t launch_pixel_order(const PixelOrderArgs& a, hipStream_t s);
// Stable sort of n (key, value) pairs by the low `bits` bits of the keys (pixel_order.hip).
hipError_t sort_pairs_u32(void* tmp, size_t* tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, int64_t n, int bits, hipStream_t s);

// HEALPix RING pixel centres of the polar cap: the number of pixels in the rings with
// z >= z_min (host only), and their unit directions, [count][3] FP64, for resolution n.
int64_t healpix_cap_count(int64_t n, double z_min);
hipError_t launch_healpix_cap(int64_t n, int64_t count, double* dirs, hipStream_t s);
constexpr int64_t kHealpixMaxNside = int64_t(1) << 20;

// Pixel covariance Gamma [n][n] FP64 of unit directions dirs [n][3] for C_l, l = 0 .. lmax
// (all device memory); n <= kCovMaxPixels (the grid's y extent), lmax <= kCovMaxL.
hipError_t launch_pixel_cov(const double* dirs, int64_t n, const double* cl, int lmax, double* gamma,
                            hipStream_t s);
constexpr int64_t kCovMaxPixels = int64_t(65535) * 16;
constexpr int kCovMaxL = 1 << 16;

// Pipelined launch: one workgroup per schedule entry (role << 30 | index), role 0 = pass x
// (tile index zt + (N/2/tx) iy), 1 = pass y (zt + (N/2/ty) ix), 2 = pass z (line block of
// lz lines), 3 = gather (pixel block of 256). Each role works on its own buffer.
struct PipeLaunch {
  int dtype, N;
  const uint32_t* sched;
  int nblocks;
  void* bx;
  const void* wtab_x;
  uint32_t k0, k1;
  int m_hi_x, m_hi_y, m_hi_z;
  const void *fp_x, *fp_y, *fp_z;
  void* by;
  void* bz;
  const void* field_g;
  const double* dirs;
  const void* order = nullptr;  // the gather item's pixel order (pixel_order_bytes), or NULL
  void* out;
  int64_t npix;
  double r, scale;
  double obs[3];
  int cubic;
  const void* tw;
};
hipError_t launch_pipeline(const PipeLaunch& a, hipStream_t s);
// Tile shapes of the pipelined kernel for (dtype, N); false if N is not compiled.
bool pipeline_shape(int dtype, int N, int* tx, int* ty, int* lz);
constexpr int kPipeThreads = 256;

}  // namespace cmbx
