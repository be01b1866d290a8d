// Host-side helpers shared by the C ABI sources: size checks, FP64 tables, the binary32
// Box-Muller tables on the device, fault injection for tests, and a device guard.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace cmbx {

// n = 2^a 3^b
bool is_2a3b(int n);
// exp(2 pi i m / N), m = 0 .. N-1, from long double sin/cos, rounded once to double;
// the quarter turns exact
void roots_of_unity(int N, std::vector<double>& re, std::vector<double>& im);
// P_inf at k: linear between table nodes, zero outside [k[0], k[n-1]]
double interp_p(const double* kt, const double* pt, int64_t n, double k);
// CMBX_FAULT lists `site`: the caller fails there as the runtime would (tests only)
bool fault(const char* site);
// the 768 binary32 Box-Muller table entries (layout in noise_device.hpp)
void fill_noise_tables(float* t);
// upload those tables to `device` (the current device) once per process
hipError_t ensure_noise_tables(int device);

// Makes `dev` current for a scope and restores the previous device after it.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

}  // namespace cmbx
