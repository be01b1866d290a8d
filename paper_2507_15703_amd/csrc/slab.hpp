// Internal interface of the flat-box kernels (slab.hip): the column stage of the 3-D
// Fourier method on an N x N x M box and of the 2-D (hybrid) Fourier method, and the
// gather from stacked layers. The 2-D inverse transforms of the layers are
// launch_layers_c2c / launch_layers_c2r (kernels.hpp).
//
// Layers: [nz][N][N/2] complex during the passes (column 0 packs the rows of y frequency
// 0 and N/2 as A + i B, both Hermitian in x), [nz][N][N] real after them (y fastest).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmbx {

enum { kSlabFlat = 1, kSlabHybrid = 2 };  // the 3-D method on N x N x M; the 2-D method on h layers
constexpr int kSlabMaxLayers = 32;         // h of the 2-D method

// Rows of a per-column table: s = fx^2 + fy^2 (0 <= fx, fy <= N/2) -> sidx[s], the row of
// that s (-1 if s is not such a sum).
struct SlabColumnsArgs {
  int dtype, method, N, M, h;
  void* buf;              // layers [nz][N][N/2] complex (nz = M flat, h hybrid), or the debug layout
  const int* sidx;        // [2 (N/2)^2 + 1]
  const void* table;      // flat: sqrt(P_box/2) [rows][M/2+1], then sqrt(P_box) at the six
                          //   self-conjugate (s, fz); hybrid: S/sqrt2 [rows][h][h], then S [3][h][h]
                          //   at s = 0, (N/2)^2, 2 (N/2)^2 (S the symmetric root of Gamma)
  int rows;
  const void* twz;        // flat: M roots exp(2 pi i m / M)
  uint32_t k0, k1;        // Philox key
  const float* bm_tab;    // binary32 Box-Muller tables on the device
};
// The column stage into the packed layers.
hipError_t launch_slab_columns(const SlabColumnsArgs& a, hipStream_t s);
// Debug layouts (unpacked): flat: the modes [N][N/2+1][M] before the z transform;
// hybrid: the correlated columns [h][N][N/2+1].
hipError_t launch_slab_columns_debug(const SlabColumnsArgs& a, hipStream_t s);
// M with a compiled z transform (flat boxes).
bool slab_depth_compiled(int M);

struct SlabGatherArgs {
  int dtype, interp, N, nz;
  int periodic_z;        // 1: z wraps modulo nz (the flat box); 0: NaN where a stencil leaves [0, nz)
  const void* field;     // [nz][N][N] reals
  double scale;          // 1 / dp
  double obs[3];
  double r;
  const double* dirs;    // [n_pix][3]
  int64_t n_pix;
  void* out;
};
hipError_t launch_slab_gather(const SlabGatherArgs& a, hipStream_t s);
// The same map from the layers after the transform along x only (complex [nz][N][N/2],
// packed column 0), each stencil row's value evaluated directly from its line's half
// spectrum with the N roots tw: for maps of few pixels, in place of the complex-to-real
// pass and the gather.
hipError_t launch_slab_direct(const SlabGatherArgs& a, const void* tw, hipStream_t s);

}  // namespace cmbx
