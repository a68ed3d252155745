#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace mpoevo {

// Device status bits kept per handle (sticky until read by the host).
enum : int { kStatusNotConverged = 1, kStatusBarrierTimeout = 2, kStatusNonFinite = 4 };

struct SvdPlan {
  int m, n;        // Theta is m x n
  bool on_theta;   // one-sided Jacobi on the columns of Theta (n <= m) or of Theta^dag
  int mx, nx;      // column length and number of columns of the Jacobi matrix X
  int b, nb, np;   // block width, number of blocks (even), padded column count
  int H;           // column height in the work buffer: mx rows of X, then np rows of V
  size_t lds;      // dynamic LDS bytes of the Jacobi kernel
  size_t ws;       // workspace bytes
};

// LDS budget of the Jacobi kernel (bytes); the workspace size depends on it, so it is a
// build constant rather than a device query (device_init checks that the device provides it).
constexpr size_t kSvdLdsBytes = 128 * 1024;

// Plan for an m x n truncation given the LDS capacity per workgroup.
SvdPlan svd_plan(int m, int n, size_t lds_cap = kSvdLdsBytes);

// Largest workspace of any plan with m, n <= maxdim (memoised).
size_t svd_ws_bound(int maxdim);

// One-time kernel attribute setup (dynamic LDS above the default limit).
hipError_t svd_configure();

// FP64 SVD + truncation (see `truncate` in mpoevo.h). `status` points to the handle's device
// status word. Writes A_out (m x kcap), B_out (kcap x n) with kcap = min(Dmax, m, n).
hipError_t svd_truncate(const SvdPlan& p, const double2* theta, int Dmax, double cutoff,
                        int direction, double2* A_out, double2* B_out, int* k_dev,
                        double* disc_dev, double* norm_dev, double* sigma_dev, void* ws,
                        int* status, hipStream_t st);

}  // namespace mpoevo
