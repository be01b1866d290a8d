// The sort behind the gather's pixel order (kernels.hpp): rocPRIM's device radix sort of
// (Morton key, pixel index) pairs. It runs once per (plan, directions) when the directions
// stay fixed, outside the hot path; a translation unit of its own keeps its templates out
// of the kernels' build.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "kernels.hpp"

namespace cmbx {

hipError_t sort_pairs_u32(void* tmp, size_t* tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, int64_t n, int bits, hipStream_t s) {
  size_t b = *tmp_bytes;
  const hipError_t e =
      rocprim::radix_sort_pairs(tmp, b, keys_in, keys_out, vals_in, vals_out, (size_t)n, 0u, (unsigned)bits, s);
  *tmp_bytes = b;
  return e;
}

}  // namespace cmbx
