#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace mpoevo {

// Device status bits kept per handle (sticky until read by the host).
enum : int { kStatusNotConverged = 1, kStatusBarrierTimeout = 2, kStatusNonFinite = 4 };

struct SvdPlan {
  int m, n;        // Theta is m x n
  int direction;   // 0: keep U (A = U_k, B = S V_k^dag); 1: keep V (A = U_k S, B = V_k^dag)
  int xconj;       // 0: X = Theta; 1: X = Theta^dag
  int acc;         // accumulate the column rotations Q (nx x nx) of X
  int mx, nx;      // X is mx x nx (column length, number of columns)
  int rank_max;    // min(m, n)
  int rmax;        // rows per lane of the Jacobi kernel (mx <= 64 rmax)
  int b, nb, np;   // block width, number of blocks (even), padded column count
  int qr;          // Jacobi runs on R^dag of the column-pivoted QR X Pi = Q R
  int frows;       // rows in the rounding floor 8 eps sqrt(frows) ||X||_F: X's rows
  int np_alloc;    // columns of the per-column arrays (>= np, and >= the Jacobi phase's np with qr)
  size_t aux_elems;  // (qr) elements of the buffer holding R^dag
  double accept;   // a sweep whose largest relative inner product is at most this is the last
                   // (0: only the sweep that finds every pair below the rounding tolerance)
  int threads;     // threads per Jacobi workgroup (one pair per wave)
  size_t lds;      // dynamic LDS bytes of the Jacobi kernel
  size_t ws;       // workspace bytes
  int split_ok;    // the products of the truncation may split K (their scratch ends the workspace)
};

// Early end of the Jacobi iteration for bond matrices formed by FP32 contractions (relative
// rounding about 1e-7): cyclic Jacobi converges quadratically, so after a sweep whose largest
// relative inner product was mu the columns are orthogonal to about mu^2 <= 1e-9, far below what
// the input determines, and the sweep that would only confirm it is skipped.
constexpr double kSvdAcceptFp32 = 3e-5;

// LDS budget of the Jacobi kernel (bytes); the workspace size depends on it, so it is a
// build constant rather than a device query (device_init checks that the device provides it).
constexpr size_t kSvdLdsBytes = 128 * 1024;
// Dynamic LDS of the pivoted-QR factorisation at its largest size: 16 columns of 512 rows.
constexpr size_t kQrLdsBytes = 16 * 16 * 512;

// Plan for an m x n truncation in the given direction. want_basis: the call will ask for the
// preconditioner of the next truncation (rectangular Theta then accumulates Q).
SvdPlan svd_plan(int m, int n, int direction, bool want_basis = false,
                 size_t lds_cap = kSvdLdsBytes);

// Plan for an m x n truncation preconditioned by a column-pivoted QR: X = Theta^dag
// (direction 0) or Theta (direction 1), X Pi = Q R (R upper trapezoidal, min(rows, cols) x
// cols), one-sided Jacobi on R^dag, whose normalised converged columns with rows permuted by Pi
// are X's right singular vectors, i.e. the factor the direction keeps. For Theta whose singular
// values spread over many decades (the first truncation of a bond in a time step) this converges
// in about 8 sweeps where Jacobi on X needs 25-40.
SvdPlan svd_plan_qr(int m, int n, int direction, size_t lds_cap = kSvdLdsBytes);
// Whether the pivoted-QR plan applies: max(m, n) <= 512.
bool svd_qr_ok(int m, int n, int direction);

// The plan with products that never split K: its workspace drops the split-K scratch
// (kGemmScratchBytes), so that several small truncations can run side by side in one buffer.
SvdPlan svd_plan_unsplit(SvdPlan p);

// Largest workspace of any plan with m, n <= maxdim (memoised).
size_t svd_ws_bound(int maxdim);

// One-time kernel attribute setup (dynamic LDS above the default limit).
hipError_t svd_configure();

// FP64 SVD + truncation (see `truncate` in mpoevo.h). Preconditioning (square Theta, or a plan
// made with want_basis; ignored otherwise): with `warm` (nx x nx unitary P, column j at
// warm + j nx) Jacobi starts from X P instead of X, which has the same singular values and left
// singular vectors; a P close to X's right singular vectors leaves X P nearly orthogonal and
// saves most sweeps. With `basis_out` the unitary for the next truncation of the same bond is
// written there in the same layout: for square Theta the normalised converged columns (or the
// identity when some column is at the rounding floor), i.e. X's left singular vectors, which
// precondition the opposite-direction visit; for rectangular Theta (same orientation on every
// visit) the accumulated P Q, i.e. X's right singular vectors. `warm` and `basis_out` may be
// the same buffer. `status` points to the handle's device
// status words. Writes A_out (m x kcap), B_out (kcap x n) with kcap = min(Dmax, m, n).
// Optional profiling: the Jacobi launch is bracketed by ev0 / ev1 (both or neither) and its
// sweep count is stored at sweeps_dev (device int, nullable).
// coop: launch the Jacobi kernel cooperatively (the runtime then guarantees that its workgroups
// are resident together, and runs it alone on the device). With coop false it is an ordinary
// launch that can overlap work on other streams; the caller must keep the workgroups of all
// Jacobi launches in flight at once within what the device holds together (one per compute
// unit), and the kernel's bounded waits turn a violation into a barrier-timeout status.
// blocks_dev (device int, nullable): the number of column blocks the Jacobi rounds took (trailing
// blocks of columns at the rounding floor are left out; see svd_sweep_flop).
// complete_dev (device int, nullable): 1 when every singular value lies clearly above the
// rounding floor (X numerically of full column rank), else 0; a square basis_out then needs
// the costly completion of its columns.
hipError_t svd_truncate(const SvdPlan& p, const double2* theta, int Dmax, double cutoff,
                        double2* A_out, double2* B_out, int* k_dev, double* disc_dev,
                        double* norm_dev, double* sigma_dev, void* ws, int* status,
                        hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                        int* sweeps_dev = nullptr, const double2* warm = nullptr,
                        double2* basis_out = nullptr, bool coop = true, int* complete_dev = nullptr,
                        int* blocks_dev = nullptr);

// FP64 Householder QR of X = Theta (plan of svd_plan_qr with direction 1: Theta m x n, m >= n) or
// X = Theta^dag (direction 0: Theta m x n, n >= m), without pivoting, blocked in panels of 16
// columns (one workgroup per panel, compact-WY block reflectors), written out as the explicit thin
// Q (mx x nx, orthonormal columns spanning X's column space when X has full column rank; an
// orthonormal completion otherwise): adjoint false: out = Q row-major (mx x nx); adjoint true:
// out = Q^dag row-major (nx x mx). For the one-site fit: Theta = its local tensor (rows (a', s'),
// columns b') with direction 1 gives the left-orthonormal site; Theta (rows a', columns (s', b'))
// with direction 0 and adjoint true gives the right-orthonormal site. ws: the plan's workspace
// (p.ws bytes). coop: cooperative launch (the panels' workgroups wait on each other).
hipError_t qr_isometry(const SvdPlan& p, const double2* theta, double2* out, bool adjoint, void* ws,
                       int* status, hipStream_t st, bool coop);

// Workgroups of the Jacobi launch of a plan.
inline int svd_grid(const SvdPlan& p) { return p.nb / 2; }

// Algorithmic flops of one Jacobi sweep of a plan over nb column blocks (the plan's own when
// nb <= 0), 36 mx per column pair visit: 16 mx for the three inner products, 20 mx for the
// rotation of the two columns.
double svd_sweep_flop(const SvdPlan& p, int nb = 0);
// The plan the Jacobi iteration of a truncation runs on: the plan itself, or for the pivoted-QR
// plan that of R^dag (nx x min(mx, nx)).
SvdPlan svd_jacobi_plan(const SvdPlan& p);
// Host function of the Jacobi kernel instance a plan launches (names profiled launches).
const void* svd_jacobi_kernel_ptr(const SvdPlan& p);

}  // namespace mpoevo
