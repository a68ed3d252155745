// FP64 SVD of the projected two-site tensor by one-sided (Hestenes) Jacobi, and the truncation
// of the two-site update (keep k <= Dmax singular values, split as U | S V^dag or U S | V^dag).
//
// Orientation. Jacobi orthogonalises the columns of X by plane rotations from the right,
// X Q = (columns sigma_j x_j), Q unitary. A rectangular Theta is oriented so that X has
// min(m, n) columns (X = Theta when m > n, X = Theta^dag when m < n); a square one by the sweep
// direction (left-to-right keeps U: X = Theta; right-to-left keeps V: X = Theta^dag). The kept
// factor is either the normalised converged columns of X, or, when it lies on the other side
// (rectangular Theta), the accumulated rotation Q itself; both are orthonormal to rounding. The
// other factor is the exact projection (S V^dag = U^dag Theta, or U S = Theta V) on the FP64
// matrix cores.
//
// Preconditioning. Starting from X P instead of X, with P a unitary close to X's right singular
// vectors, leaves the singular values and left singular vectors unchanged and X P nearly
// orthogonal, so Jacobi ends in a few sweeps. The truncation of a bond leaves such a P for the
// next truncation of the same bond: the normalised columns (square Theta; they are the singular
// vectors on the side the next, opposite-direction visit multiplies) or the accumulated P Q
// (rectangular Theta, same orientation every visit).
//
// Numerically zero columns: a column whose norm is at the rounding level of the matrix,
// floor = 8 eps sqrt(mx) ||Theta||_F, only carries cancellation noise; rotating it against a
// large column regenerates noise of its own size, so pairs with such a column are not rotated
// and those singular values are treated as zero (never kept). Every other pair is rotated until
// |x^dag y| <= tol |x| |y|, so the normalised kept columns are orthonormal to tol.
//
// Parallel schedule: the np columns are cut into nb blocks of b columns; a round pairs the
// blocks (round-robin), one workgroup per block pair holds its 2b columns in LDS, one wave per
// column pair with both columns in registers. The first round of a sweep visits every pair of
// its 2b columns (so every pair inside a block is visited once per sweep), the other rounds
// only the b x b pairs across their two blocks: each pair of columns is rotated exactly once
// per sweep. A workgroup starts a round once the two workgroups that wrote its blocks in the
// previous round have published (point-to-point flags of the cooperative launch); every sweep
// ends with a wait for all workgroups, after which a sweep whose largest relative inner product
// is below tol (or below kAccept) ends the iteration.

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "dev_common.h"
#include "svd.h"

namespace mpoevo {
namespace {

constexpr int kMaxSweeps = 60;
constexpr int kMaxGrid = 256;      // workgroups of a Jacobi launch (nb / 2 <= 256)
constexpr double kAccept = 1e-13;  // columns this orthogonal need no further sweep
constexpr double kEps = 2.220446049250313e-16;
constexpr int kMaxDim = 1024;      // largest m, n of a truncation
// Largest n of a truncation preconditioned by the pivoted QR.
constexpr int kQrMaxDim = 512;
constexpr unsigned long long kBarrierTimeoutTicks = 300000000ull;  // 3 s of the 100 MHz clock

struct SvdWs {  // carved from the caller's workspace
  double2* X;           // [np][mx] column-major
  double2* Q;           // [np][nx] accumulated rotation (plans with acc), else null
  double* sigma;        // [np]
  int* perm;            // [np]
  unsigned* bar;        // [2] timeout flag
  unsigned* flags;      // [kMaxGrid] barrier generation reached by each workgroup
  unsigned* sweep_max;  // [kMaxSweeps] bits of the largest |x^dag y| / (|x| |y|) of a sweep
  int* k_shared;        // [0] kept rank, [1] columns form a complete basis
  double2* aux;         // [np][mx] (plans with qr) Jacobi input R^dag after the pivoted QR of X
  int* qperm;           // [np] (qr) column pivots: column j of X Pi is column qperm[j] of X
  int* pinv;            // [np] (qr) inverse pivots
  unsigned long long* qkeys;  // [2][kMaxGrid] (qr) each workgroup's published candidate (step, norm, column)
  double* qrefl;        // [2][kMaxGrid][8] (qr) each candidate's reflector: tau, 1 / (alpha - beta), beta
  double2* qcol;        // [2][nb / 2][mx] (qr) each workgroup's candidate column
  int* qsteps;          // [1] (qr) steps taken (fewer than min(mx, nx) when the rest is exactly zero)
  void* gemm;           // split-K scratch of the products (kGemmScratchBytes)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t ws_bytes(int mx, int nx, int np, bool acc, bool qr, int np_alloc, size_t aux_elems) {
  return align256(sizeof(double2) * (size_t)mx * np) +
         (acc ? align256(sizeof(double2) * (size_t)nx * np) : 0) + align256(sizeof(double) * np_alloc) +
         align256(sizeof(int) * np_alloc) + 256 + sizeof(unsigned) * kMaxGrid +
         align256(sizeof(unsigned) * kMaxSweeps) + 256 +
         (qr ? align256(sizeof(double2) * aux_elems) + 2 * align256(sizeof(int) * np) +
                   align256(2 * sizeof(unsigned long long) * kMaxGrid) + align256(16 * sizeof(double) * kMaxGrid) +
                   align256(2 * sizeof(double2) * (size_t)mx * np) + 256
              : 0) +
         kGemmScratchBytes;
}

SvdWs carve(const SvdPlan& p, void* ws) {
  unsigned char* base = static_cast<unsigned char*>(ws);
  SvdWs w;
  size_t off = 0;
  w.X = reinterpret_cast<double2*>(base + off);
  off += align256(sizeof(double2) * (size_t)p.mx * p.np);
  w.Q = nullptr;
  if (p.acc) {
    w.Q = reinterpret_cast<double2*>(base + off);
    off += align256(sizeof(double2) * (size_t)p.nx * p.np);
  }
  w.sigma = reinterpret_cast<double*>(base + off);
  off += align256(sizeof(double) * p.np_alloc);
  w.perm = reinterpret_cast<int*>(base + off);
  off += align256(sizeof(int) * p.np_alloc);
  w.bar = reinterpret_cast<unsigned*>(base + off);
  off += 256;
  w.flags = reinterpret_cast<unsigned*>(base + off);
  off += sizeof(unsigned) * kMaxGrid;
  w.sweep_max = reinterpret_cast<unsigned*>(base + off);
  off += align256(sizeof(unsigned) * kMaxSweeps);
  w.k_shared = reinterpret_cast<int*>(base + off);
  off += 256;
  w.aux = nullptr;
  w.qperm = w.pinv = nullptr;
  w.qkeys = nullptr;
  w.qrefl = nullptr;
  w.qcol = nullptr;
  w.qsteps = nullptr;
  if (p.qr) {
    w.aux = reinterpret_cast<double2*>(base + off);
    off += align256(sizeof(double2) * p.aux_elems);
    w.qperm = reinterpret_cast<int*>(base + off);
    off += align256(sizeof(int) * p.np);
    w.pinv = reinterpret_cast<int*>(base + off);
    off += align256(sizeof(int) * p.np);
    w.qkeys = reinterpret_cast<unsigned long long*>(base + off);
    off += align256(2 * sizeof(unsigned long long) * kMaxGrid);
    w.qrefl = reinterpret_cast<double*>(base + off);
    off += align256(16 * sizeof(double) * kMaxGrid);
    w.qcol = reinterpret_cast<double2*>(base + off);
    off += align256(2 * sizeof(double2) * (size_t)p.mx * p.np);  // nb / 2 <= np columns
    w.qsteps = reinterpret_cast<int*>(base + off);
    off += 256;
  }
  w.gemm = base + off;
  return w;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Lane exchange of a double through the data-parallel-primitives network (no LDS access).
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  int lo = static_cast<int>(b & 0xffffffffll), hi = static_cast<int>(b >> 32);
  // every lane reads a lane of its own row (quad permutations, row mirrors), so no lane keeps its
  // old value and none needs initialising
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Sum over the 64 lanes, identical in every lane (each step adds the same two numbers in both
// partner lanes): pair lanes within quads, then halves of 8, rows of 16, then across rows.
// x + (x of the partner row, rows paired 0-1 and 2-3) in every lane: v_permlane16_swap exchanges
// the odd rows of one operand with the even rows of the other, so swapping x with itself leaves
// the two rows of a pair in the two results, whose sum is the pair's sum.
__device__ inline double row_pair_sum(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(b), hi = static_cast<unsigned>(b >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h[0]) << 32) | l[0])) +
         __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h[1]) << 32) | l[1]));
}
// x + (x of the other half of the wave) in every lane (v_permlane32_swap, the same way).
__device__ inline double half_pair_sum(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(b), hi = static_cast<unsigned>(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h[0]) << 32) | l[0])) +
         __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h[1]) << 32) | l[1]));
}

__device__ inline void wave_sum2(double& a, double& b) {
  a += dpp_move<0xB1>(a); b += dpp_move<0xB1>(b);
  a += dpp_move<0x4E>(a); b += dpp_move<0x4E>(b);
  a += dpp_move<0x141>(a); b += dpp_move<0x141>(b);
  a += dpp_move<0x140>(a); b += dpp_move<0x140>(b);
  a = row_pair_sum(a); b = row_pair_sum(b);
  a = half_pair_sum(a); b = half_pair_sum(b);
}

template <int R>
__device__ inline double sq_norm_part(const double2 (&u)[R]) {
  double a = 0.0;
#pragma unroll
  for (int t = 0; t < R; ++t) a = fma(u[t].x, u[t].x, fma(u[t].y, u[t].y, a));
  return a;
}

// 1/sqrt(x) to full double precision: the hardware estimate plus two Newton steps.
__device__ inline double rsqrt_d(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r;
}

// Round-robin pairing of n (even) items: round r in 0..n-2, pair index k in 0..n/2-1.
__device__ inline void rr_pair(int r, int k, int n, int& x, int& y) {
  x = (r + k) % (n - 1);
  y = (k == 0) ? (n - 1) : (r - k + n - 1) % (n - 1);
}

// X = Theta (xconj 0) or Theta^dag (xconj 1), zero padding columns; Q = P (the preconditioner,
// nx x nx, column j at P + j nx) or the identity, zero padding columns; clear the state.
// With copy == 0 the first nx columns of X are left to the preconditioning product.
__global__ void svd_init_kernel(const double2* __restrict__ theta, SvdPlan p, SvdWs w, int copy,
                                const double2* __restrict__ P) {
  const long long total = (long long)p.mx * p.np;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long first = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (long long idx = first; idx < total; idx += stride) {
    const int j = (int)(idx / p.mx), row = (int)(idx % p.mx);
    if (j < p.nx && !copy) continue;
    double2 v{0.0, 0.0};
    if (j < p.nx) {
      if (p.xconj == 0) v = theta[(long long)row * p.n + j];
      else {
        const double2 t = theta[(long long)j * p.n + row];
        v = double2{t.x, -t.y};
      }
    }
    w.X[idx] = v;
  }
  if (p.acc) {
    const long long qtotal = (long long)p.nx * p.np;
    for (long long idx = first; idx < qtotal; idx += stride) {
      const int j = (int)(idx / p.nx), row = (int)(idx % p.nx);
      double2 v{0.0, 0.0};
      if (j < p.nx) v = P ? P[idx] : double2{row == j ? 1.0 : 0.0, 0.0};
      w.Q[idx] = v;
    }
  }
  if (blockIdx.x == 0) {
    if (p.qr) {
      for (int i = threadIdx.x; i < 2 * kMaxGrid; i += blockDim.x) w.qkeys[i] = 0ull;
      if (threadIdx.x == 0) *w.qsteps = 0;
    }
    if (threadIdx.x < 3) w.bar[threadIdx.x] = 0u;
    for (int i = threadIdx.x; i < kMaxSweeps; i += blockDim.x) w.sweep_max[i] = 0u;
    for (int i = threadIdx.x; i < kMaxGrid; i += blockDim.x) w.flags[i] = 0u;
  }
}

// Synchronisation between the workgroups of the cooperative launch, without a shared counter
// (whose atomics serialise): workgroup g publishes in flags[g] the number of rounds it has
// completed (release); a workgroup that needs the blocks written in the previous round waits
// for the flags of the two workgroups that wrote them (acquire), and at the end of a sweep every
// workgroup waits for all flags. A wait longer than the timeout (or another workgroup's timeout)
// sets bar[2] and makes every waiting workgroup return false; all workgroups then leave the sweep
// loop. The waits poll with relaxed loads and acquire once, by a fence after the flags are seen
// (an acquiring load in the poll would invalidate the L2 cache on every iteration).

// Waits until flags[j] >= gen for j = f0, f1 (nblocks < 0) or for every j < nblocks.
__device__ bool wait_flags(unsigned* flags, unsigned* bar, int f0, int f1, int nblocks, unsigned gen) {
  __shared__ int timed_out;
  if (threadIdx.x == 0) timed_out = 0;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const unsigned long long t0 = wall_clock64();
    bool fail = false;
    while (true) {
      int mine = 1;
      if (nblocks < 0) {
        if (lane == 0) mine = __hip_atomic_load(&flags[f0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gen;
        if (lane == 1) mine = __hip_atomic_load(&flags[f1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gen;
      } else {
        for (int j = lane; j < nblocks; j += 64)
          mine &= __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gen;
      }
      if (__all(mine)) break;
      if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > kBarrierTimeoutTicks) {
        fail = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (fail && lane == 0) {
      __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      timed_out = 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // pairs with the release stores seen
  }
  __syncthreads();
  return timed_out == 0;
}

// The pair index of round r of the round-robin over n blocks that holds block blk.
__device__ inline int rr_owner(int r, int blk, int n) {
  if (blk == n - 1) return 0;
  const int k1 = ((blk - r) % (n - 1) + (n - 1)) % (n - 1);  // blk in the first slot
  if (k1 < n / 2) return k1;
  return ((r - blk) % (n - 1) + (n - 1)) % (n - 1);          // blk in the second slot
}

// One Jacobi rotation of the column pair (u, v) held in registers (RMAX rows per lane), given
// their squared norms a = |u|^2, bb = |v|^2: the inner product g = u^dag v, the rotation that
// makes the pair orthogonal, applied in place (and to the pair's columns of the accumulated
// rotation, qu and qv, when ACC). The norms follow the rotation exactly in exact arithmetic,
// |u'|^2 = a - t |g|, |v'|^2 = bb + t |g|; when either loses more than 31/32 of its value
// (cancellation) both are recomputed from the columns. Returns whether the pair was rotated;
// raises wave_max (wave-uniform) to the pair's squared relative inner product |g|^2 / (a bb).
template <int RMAX, bool ACC>
__device__ inline bool jacobi_pair(double2 (&u)[RMAX], double2 (&v)[RMAX], double2 (&qu)[RMAX],
                                   double2 (&qv)[RMAX], double& a, double& bb, int lane,
                                   double floor2, double tol2, double& wave_max) {
  double gr = 0.0, gi = 0.0;
#pragma unroll
  for (int t = 0; t < RMAX; ++t) {
    gr = fma(u[t].x, v[t].x, fma(u[t].y, v[t].y, gr));
    gi = fma(u[t].x, v[t].y, fma(-u[t].y, v[t].x, gi));
  }
  wave_sum2(gr, gi);
  const double g2 = fma(gr, gr, gi * gi);  // |g|^2
  const double ab = a * bb;
  const bool live = fmin(a, bb) > floor2;
  if (live && ab > 0.0) wave_max = fmax(wave_max, g2 * __builtin_amdgcn_rcp(ab));
  if (!(live && g2 > tol2 * ab)) return false;
  // The rotation [[c, -s e], [s conj(e), c]] (e = conj(g) / |g|) with tan(2 theta) =
  // 2 |g| / (bb - a), |theta| <= pi/4, from two reciprocal square roots and no division:
  // rho = sqrt((bb - a)^2 + 4 |g|^2), cos^2 = (1 + |bb - a| / rho) / 2,
  // s e = sr conj(g) and s conj(e) = sr g with sr = sign(bb - a) / (rho cos), t |g| = sr |g|^2 / cos.
  const double dab = bb - a;
  const double r1 = rsqrt_d(fma(dab, dab, 4.0 * g2));
  const double c2 = fma(0.5 * fabs(dab), r1, 0.5);
  const double rc = rsqrt_d(c2);
  const double c = c2 * rc;
  const double sr = (dab >= 0.0 ? r1 : -r1) * rc;
  const double pr = sr * gr, pi = sr * gi;
#pragma unroll
  for (int tt = 0; tt < RMAX; ++tt) {
    const double2 un{c * u[tt].x - (pr * v[tt].x + pi * v[tt].y), c * u[tt].y - (pr * v[tt].y - pi * v[tt].x)};
    v[tt] = double2{(pr * u[tt].x - pi * u[tt].y) + c * v[tt].x, (pr * u[tt].y + pi * u[tt].x) + c * v[tt].y};
    u[tt] = un;
  }
  if (ACC) {
#pragma unroll
    for (int tt = 0; tt < RMAX; ++tt) {
      const double2 un{c * qu[tt].x - (pr * qv[tt].x + pi * qv[tt].y), c * qu[tt].y - (pr * qv[tt].y - pi * qv[tt].x)};
      qv[tt] = double2{(pr * qu[tt].x - pi * qu[tt].y) + c * qv[tt].x, (pr * qu[tt].y + pi * qu[tt].x) + c * qv[tt].y};
      qu[tt] = un;
    }
  }
  const double tg = sr * g2 * rc;  // t |g|
  const double an = a - tg, bn = bb + tg;
  if (an < 0.03125 * a || bn < 0.03125 * bb) {  // wave-uniform: all lanes hold the same values
    double x = sq_norm_part(u), y = sq_norm_part(v);
    wave_sum2(x, y);
    a = x;
    bb = y;
  } else {
    a = an;
    bb = bn;
  }
  return true;
}

template <int R>
__device__ inline void load_col(double2 (&u)[R], const double2* c, int lane, int len) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = lane + 64 * t;
    u[t] = row < len ? c[row] : double2{0.0, 0.0};
  }
}

template <int R>
__device__ inline void store_col(const double2 (&u)[R], double2* c, int lane, int len) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = lane + 64 * t;
    if (row < len) c[row] = u[t];
  }
}

// One-sided Jacobi sweeps. RMAX = rows per lane (mx <= 64 RMAX; with ACC also nx <= mx). Launched
// with nb / 2 workgroups of 64 b threads that must all be resident together (a cooperative
// launch, or an ordinary one whose caller bounds the load); dynamic LDS holds the 2b columns of X
// (mx rows each) followed, with ACC, by the same 2b columns of Q (nx rows each).
template <int RMAX, bool ACC>
__global__ __launch_bounds__(RMAX <= 8 ? 512 : 256) void svd_jacobi_kernel(SvdPlan p, SvdWs w,
                                                                          double tol, int* status,
                                                                          int* sweeps_out, int* blocks_out) {
  extern __shared__ double2 cols[];  // [2b][mx] then (ACC) [2b][nx]
  __shared__ unsigned wg_max;        // bits of a non-negative float: integer order = value order
  __shared__ double floor2_sh;
  __shared__ int nbe_sh;
  __shared__ double nrm[2 * 16];     // squared norms of the 2b columns held in LDS (b <= 16)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int two_b = 2 * p.b, mx = p.mx, nx = p.nx;
  double2* qcols = cols + two_b * mx;
  if (tid == 0) {  // squared rounding floor from the initial column norms (fixed order)
    double fro2 = 0.0;
    for (int j = 0; j < p.nx; ++j) fro2 += w.sigma[j];
    const double fl = 8.0 * kEps * sqrt((double)p.frows);
    floor2_sh = fl * fl * fro2;
  }
  __syncthreads();
  const double floor2 = floor2_sh;
  // A column at the rounding floor is never rotated (a pair needs both columns above it), so its
  // norm never changes: trailing blocks made only of columns clearly below it (half the floor,
  // so that no column the pair test would take is left out; the tail of R^dag after the pivoted
  // QR of a numerically rank-deficient matrix) are left out of the rounds altogether, with the
  // same result. Every workgroup finds the same block count nbe.
  if (wave == 0) {
    int last = -1;
    for (int j = lane; j < nx; j += 64)
      if (w.sigma[j] > 0.5 * floor2) last = j;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off, 64));
    if (lane == 0) {
      int nbe = max((last + p.b) / p.b, 2);
      nbe += nbe & 1;
      nbe_sh = min(nbe, p.nb);
    }
  }
  __syncthreads();
  const int nbe = nbe_sh;
  const unsigned nblk = nbe / 2;
  if (blockIdx.x >= nblk) return;  // (block 0 always takes part and reports)
  const double tol2 = tol * tol;
  bool ok = true;
  int sweep = 0;
  unsigned gen = 0;
  // The verdict on sweep s is read in the second pairing step (r = 1) of sweep s + 1, after a
  // wait for every workgroup to have finished sweep s: by then the slower workgroups have mostly
  // caught up, so no workgroup idles at the end of each sweep. A converged sweep thus keeps the
  // rotations of the next sweep's first pairing step (pairs below tol are not rotated; the others
  // only further). With a single pairing step per sweep, and after the last allowed sweep, the
  // verdict is read at once.
  const int rounds = nbe - 1;
  auto converged = [&](int s) {
    const double mxr = (double)__uint_as_float(
        __hip_atomic_load(&w.sweep_max[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    return mxr <= tol || mxr <= kAccept || mxr <= p.accept;
  };
  bool conv = false;
  int done_sweeps = 0;
  for (; sweep < kMaxSweeps && ok && !conv; ++sweep) {
    for (int r = 0; r < rounds && ok; ++r) {
      int bp, bq;
      rr_pair(r, blockIdx.x, nbe, bp, bq);
      // the two blocks were written in the previous round by the workgroups that held them
      if (r > 0 || sweep > 0) {
        const int rp = r > 0 ? r - 1 : rounds - 1;
        if (!(ok = wait_flags(w.flags, w.bar, rr_owner(rp, bp, nbe), rr_owner(rp, bq, nbe), -1, gen)))
          break;
      }
      if (r == 1 && sweep > 0) {  // the previous sweep's verdict
        if (!(ok = wait_flags(w.flags, w.bar, 0, 0, (int)nblk, (unsigned)(sweep * rounds)))) break;
        if (converged(sweep - 1)) {
          conv = true;
          break;
        }
      }
      const int gx = bp * p.b + wave, gy = bq * p.b + wave;  // this wave's two global columns
      const int pk = wave;
      // Cross rounds (r > 0): wave k keeps column k of the first block in registers from its
      // global load to its global store and meets the columns of the second block (in LDS) in
      // turn. The first round of a sweep holds every column in LDS and also visits the pairs
      // inside each block.
      double2 u[RMAX], qu[RMAX];
      double na = 0.0;
      if (wave < p.b) {  // global -> registers (own column) / LDS (the second block's column)
        double2 v[RMAX];
        load_col(u, w.X + (long long)gx * mx, lane, mx);
        load_col(v, w.X + (long long)gy * mx, lane, mx);
        if (r == 0) store_col(u, cols + wave * mx, lane, mx);
        store_col(v, cols + (p.b + wave) * mx, lane, mx);
        double nb = sq_norm_part(v);
        na = sq_norm_part(u);
        wave_sum2(na, nb);
        if (lane == 0) {
          nrm[wave] = na;
          nrm[p.b + wave] = nb;
        }
        if (ACC) {
          load_col(qu, w.Q + (long long)gx * nx, lane, nx);
          load_col(v, w.Q + (long long)gy * nx, lane, nx);
          if (r == 0) store_col(qu, qcols + wave * nx, lane, nx);
          store_col(v, qcols + (p.b + wave) * nx, lane, nx);
        }
      }
      if (tid == 0) wg_max = 0u;
      __syncthreads();
      double wave_max = 0.0;  // largest squared relative inner product this wave met (uniform)
      if (r == 0) {
        for (int ir = 0; ir < two_b - 1; ++ir) {
          if (pk < p.b) {
            int x, y;
            rr_pair(ir, pk, two_b, x, y);
            double2 uu[RMAX], v[RMAX], quu[RMAX], qv[RMAX];
            load_col(uu, cols + x * mx, lane, mx);
            load_col(v, cols + y * mx, lane, mx);
            if (ACC) {
              load_col(quu, qcols + x * nx, lane, nx);
              load_col(qv, qcols + y * nx, lane, nx);
            }
            double a = nrm[x], bb = nrm[y];
            if (jacobi_pair<RMAX, ACC>(uu, v, quu, qv, a, bb, lane, floor2, tol2, wave_max)) {
              store_col(uu, cols + x * mx, lane, mx);
              store_col(v, cols + y * mx, lane, mx);
              if (lane == 0) {
                nrm[x] = a;
                nrm[y] = bb;
              }
              if (ACC) {
                store_col(quu, qcols + x * nx, lane, nx);
                store_col(qv, qcols + y * nx, lane, nx);
              }
            }
          }
          __syncthreads();
        }
        if (pk < p.b) {  // the first block's columns back into registers for the store below
          load_col(u, cols + pk * mx, lane, mx);
          if (ACC) load_col(qu, qcols + pk * nx, lane, nx);
        }
      } else {
        for (int ir = 0; ir < p.b; ++ir) {
          if (pk < p.b) {
            int y = pk + ir;
            y = p.b + (y >= p.b ? y - p.b : y);
            double2 v[RMAX], qv[RMAX];
            load_col(v, cols + y * mx, lane, mx);
            if (ACC) load_col(qv, qcols + y * nx, lane, nx);
            double nb = nrm[y];
            if (jacobi_pair<RMAX, ACC>(u, v, qu, qv, na, nb, lane, floor2, tol2, wave_max)) {
              store_col(v, cols + y * mx, lane, mx);
              if (ACC) store_col(qv, qcols + y * nx, lane, nx);
              if (lane == 0) nrm[y] = nb;
            }
          }
          __syncthreads();
        }
      }
      if (lane == 0 && wave_max > 0.0)
        atomicMax(&wg_max, __float_as_uint(sqrtf((float)fmin(wave_max, 1.0))));
      if (wave < p.b) {  // registers / LDS -> global (the LDS columns are final after the last barrier)
        double2 v[RMAX];
        store_col(u, w.X + (long long)gx * mx, lane, mx);
        load_col(v, cols + (p.b + wave) * mx, lane, mx);
        store_col(v, w.X + (long long)gy * mx, lane, mx);
        if (ACC) {
          store_col(qu, w.Q + (long long)gx * nx, lane, nx);
          load_col(v, qcols + (p.b + wave) * nx, lane, nx);
          store_col(v, w.Q + (long long)gy * nx, lane, nx);
        }
      }
      __syncthreads();  // every wave's share of wg_max (and of the global stores, for the release)
      if (tid == 0) {
        if (wg_max) atomicMax(&w.sweep_max[sweep], wg_max);
        __hip_atomic_store(&w.flags[blockIdx.x], ++gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ++gen;
      }
    }
    if (!ok || conv) break;
    done_sweeps = sweep + 1;
    if (rounds == 1 || sweep + 1 == kMaxSweeps) {  // the verdict at once
      if (!(ok = wait_flags(w.flags, w.bar, 0, 0, (int)nblk, gen))) break;
      conv = converged(sweep);
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    atomicMax(&status[1], done_sweeps);
    if (sweeps_out) *sweeps_out = done_sweeps;
    if (blocks_out) *blocks_out = nbe;
    if (!ok) atomicOr(status, kStatusBarrierTimeout);
    else if (!conv) {
      atomicOr(status, kStatusNotConverged);
      atomicMax(reinterpret_cast<unsigned*>(&status[2]), w.sweep_max[kMaxSweeps - 1]);
    }
  }
}

// sigma_j = |X[:, j]| (squared if `squared`) for j < nx (one wave per column).
__global__ void svd_norms_kernel(SvdPlan p, SvdWs w, int* status, int squared) {
  const int j = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= p.nx) return;
  const double2* c = w.X + (long long)j * p.mx;
  double s = 0.0;
  for (int row = lane; row < p.mx; row += 64) s = fma(c[row].x, c[row].x, fma(c[row].y, c[row].y, s));
  s = wave_sum(s);
  if (lane == 0) {
    const double sg = squared ? s : sqrt(s);
    if (!isfinite(sg)) atomicOr(status, kStatusNonFinite);
    w.sigma[j] = sg;
  }
}

// Rank the singular values (descending, ties by index), choose k, write the statistics.
// One workgroup of 1024 threads; nx <= 1024.
__global__ __launch_bounds__(1024) void svd_select_kernel(SvdPlan p, SvdWs w, int kcap,
                                                          double cutoff, int* k_dev,
                                                          double* disc_dev, double* norm_dev,
                                                          double* sigma_dev, int* complete_dev) {
  __shared__ double sig[1024];
  __shared__ int rank_of[1024];
  __shared__ double red[1024];
  __shared__ double kept_part[1024];
  __shared__ int cnt[1024];
  const int t = threadIdx.x;
  const int r = p.nx;
  sig[t] = (t < r) ? w.sigma[t] : -1.0;
  __syncthreads();
  if (t < r) {
    const double s = sig[t];
    int rk = 0;
    for (int i = 0; i < r; ++i) rk += (sig[i] > s || (sig[i] == s && i < t)) ? 1 : 0;
    rank_of[t] = rk;
    w.perm[rk] = t;
    if (sigma_dev && rk < p.rank_max) sigma_dev[rk] = s;
  }
  __syncthreads();
  double smax = 0.0, fro2 = 0.0;
  for (int i = 0; i < r; ++i) {
    smax = fmax(smax, sig[i]);
    fro2 += sig[i] * sig[i];
  }
  const double floor_abs = 8.0 * kEps * sqrt((double)p.frows) * sqrt(fro2);
  const double thr = fmax(cutoff * smax, floor_abs);
  // every column clearly above the rounding floor: the normalised columns form a complete
  // orthonormal basis (used to precondition the next truncation at the same bond)
  cnt[t] = (t < r && !(sig[t] > 2.0 * floor_abs)) ? 1 : 0;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) cnt[t] += cnt[t + off];
    __syncthreads();
  }
  const bool complete = cnt[0] == 0;
  __syncthreads();
  cnt[t] = (t < r && sig[t] > 0.0 && sig[t] > thr) ? 1 : 0;
  red[t] = 0.0;
  __syncthreads();
  if (t < r) red[rank_of[t]] = sig[t] * sig[t];
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) cnt[t] += cnt[t + off];
    __syncthreads();
  }
  int k = cnt[0];
  k = k < 1 ? 1 : (k > kcap ? kcap : k);
  kept_part[t] = (t < k) ? red[t] : 0.0;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) {
      red[t] += red[t + off];
      kept_part[t] += kept_part[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double tot = red[0], kept = kept_part[0];
    w.k_shared[0] = k;
    w.k_shared[1] = complete ? 1 : 0;
    if (complete_dev) *complete_dev = complete ? 1 : 0;
    if (k_dev) *k_dev = k;
    if (disc_dev) *disc_dev = tot > 0.0 ? fmax(0.0, (tot - kept) / tot) : 0.0;
    if (norm_dev) *norm_dev = sqrt(kept);
  }
}

// The kept isometry in descending order of sigma, zero beyond k. Source column j: the
// normalised converged column X[:, j] / sigma_j (from_q 0, length mx) or the accumulated
// rotation's column Q[:, j] (from_q 1, length nx); its length is m (direction 0) or n (1).
// Direction 0 -> A_out[i][r] = src[perm r][i] (m x kcap); direction 1 -> B_out[r][c] =
// conj(src[perm r][c]) (kcap x n).
__global__ void svd_isometry_kernel(SvdPlan p, SvdWs w, int kcap, double2* out, int from_q) {
  const int k = w.k_shared[0];
  const int len = p.direction == 0 ? p.m : p.n;
  const int ld = from_q ? p.nx : p.mx;
  const double2* src = from_q ? w.Q : w.X;
  const long long total = (long long)len * kcap;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int i, rr;
    if (p.direction == 0) { i = (int)(idx / kcap); rr = (int)(idx % kcap); }
    else { rr = (int)(idx / len); i = (int)(idx % len); }
    double2 v{0.0, 0.0};
    if (rr < k) {
      const int j = w.perm[rr];
      const double2 x = src[(long long)j * ld + (w.pinv ? w.pinv[i] : i)];
      if (from_q) v = x;
      else {
        const double s = w.sigma[j];
        if (s > 0.0) v = double2{x.x / s, x.y / s};
      }
      if (p.direction == 1) v.y = -v.y;
    }
    out[idx] = v;
  }
}

// Unitary basis of the column space of X (square X only) when every column is above the
// rounding floor: out[j][row] = X[j][row] / sigma_j. Otherwise left to svd_complete_kernel.
__global__ void svd_basis_kernel(SvdPlan p, SvdWs w, double2* out) {
  if (!w.k_shared[1]) return;
  const long long total = (long long)p.mx * p.nx;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / p.mx), row = (int)(idx % p.mx);
    const double inv = 1.0 / w.sigma[j];
    const double2 x = w.X[(long long)j * p.mx + (w.pinv ? w.pinv[row] : row)];
    out[idx] = double2{x.x * inv, x.y * inv};
  }
}

__device__ inline double2 cmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

// Sum of a complex value over the 64 lanes of a wave, in every lane.
__device__ inline double2 wave_csum(double2 v) {
  wave_sum2(v.x, v.y);
  return v;
}

// One wave applies I - f v v^dag (v[j] = 1, v[i] = a[i] below) to the columns c0 .. cend-1 (at
// most four, processed together so that their loads overlap) of the n-row matrix at base.
__device__ inline void reflect_cols(const double2* a, double2 f, int j, int n, double2* base, int c0,
                                    int cend, int lane) {
  constexpr int G = 4;
  double2* col[G];
  double2 acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    col[q] = base + (long long)(c0 + q) * n;
    acc[q] = (c0 + q < cend && lane == 0) ? col[q][j] : double2{0.0, 0.0};
  }
  for (int i = j + 1 + lane; i < n; i += 64) {
    const double2 v = a[i];
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (c0 + q < cend) {
        const double2 pr = cmulc(v, col[q][i]);
        acc[q].x += pr.x;
        acc[q].y += pr.y;
      }
  }
  double2 fq[G];
#pragma unroll
  for (int q = 0; q < G; ++q) fq[q] = (c0 + q < cend) ? cmul(f, wave_csum(acc[q])) : double2{0.0, 0.0};
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (c0 + q < cend) col[q][j] = double2{col[q][j].x - fq[q].x, col[q][j].y - fq[q].y};
  }
  for (int i = j + 1 + lane; i < n; i += 64) {
    const double2 v = a[i];
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (c0 + q < cend) {
        const double2 d = cmul(v, fq[q]);
        col[q][i] = double2{col[q][i].x - d.x, col[q][i].y - d.y};
      }
  }
}

// The square case with columns at the rounding floor (X numerically rank-deficient, rank r < n):
// a complete unitary whose first r columns are the normalised columns above the floor, U_r, and
// whose other n - r columns are an orthonormal basis of the orthogonal complement of span(U_r),
// taken from the Householder QR U_r = Q R (U_r = H_0 ... H_{r-1} [R; 0], the complement being
// Q's columns r .. n-1, built by applying H_{r-1}, ..., H_0 to the last n - r unit vectors).
// X's storage holds U_r during the factorisation (X is no longer needed). One workgroup of 1024
// threads; each wave takes whole columns.
constexpr int kCompleteThreads = 1024;
__global__ __launch_bounds__(kCompleteThreads) void svd_complete_kernel(SvdPlan p, SvdWs w, double2* out) {
  if (w.k_shared[1]) return;
  const int n = p.nx;  // == p.mx
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kCompleteThreads / 64;
  __shared__ int pos[kMaxDim];      // output column of X's column j
  __shared__ int scan[kCompleteThreads];
  __shared__ double2 tau[kMaxDim];
  __shared__ double floor_sh;
  if (tid == 0) {
    double fro2 = 0.0;
    for (int j = 0; j < n; ++j) fro2 += w.sigma[j] * w.sigma[j];
    floor_sh = 8.0 * kEps * sqrt((double)p.frows) * sqrt(fro2);
  }
  __syncthreads();
  // rank of each good column among the good ones (columns j = tid, tid + 1024 never needed: n <= 1024)
  const bool good = tid < n && w.sigma[tid] > 2.0 * floor_sh;
  scan[tid] = good ? 1 : 0;
  __syncthreads();
  for (int off = 1; off < kCompleteThreads; off <<= 1) {  // inclusive scan
    const int v = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  const int r = scan[kCompleteThreads - 1];
  if (tid < n) pos[tid] = good ? scan[tid] - 1 : r + (tid + 1 - scan[tid]) - 1;
  __syncthreads();
  if (r == 0) {  // nothing above the floor: the identity
    for (long long idx = tid; idx < (long long)n * n; idx += kCompleteThreads)
      out[idx] = double2{(idx / n) == (idx % n) ? 1.0 : 0.0, 0.0};
    return;
  }
  // U_r -> A (column-major n x r in X's storage, column pos[j]); also the first r output columns
  double2* A = w.X;
  for (long long idx = tid; idx < (long long)n * n; idx += kCompleteThreads) {
    const int j = (int)(idx / n), row = (int)(idx % n);
    if (w.sigma[j] > 2.0 * floor_sh) {
      const double inv = 1.0 / w.sigma[j];
      const double2 x = w.X[(long long)j * n + (w.pinv ? w.pinv[row] : row)];
      const double2 u{x.x * inv, x.y * inv};
      out[(long long)pos[j] * n + row] = u;
    }
  }
  __syncthreads();
  for (long long idx = tid; idx < (long long)n * r; idx += kCompleteThreads) A[idx] = out[idx];
  __syncthreads();
  // Householder QR of A: reflector j (v_j = 1 at row j, A[i][j] below), A := H_j^dag A
  for (int j = 0; j < r; ++j) {
    double2* a = A + (long long)j * n;
    if (wave == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < n; i += 64) s = fma(a[i].x, a[i].x, fma(a[i].y, a[i].y, s));
      double dummy = 0.0;
      wave_sum2(s, dummy);
      const double2 al = a[j];
      double2 t{0.0, 0.0};
      if (s > 0.0 || al.y != 0.0) {
        const double xn = sqrt(fma(al.x, al.x, fma(al.y, al.y, s)));
        const double beta = al.x >= 0.0 ? -xn : xn;
        t = double2{(beta - al.x) / beta, -al.y / beta};
        // scale = 1 / (alpha - beta)
        const double2 d{al.x - beta, al.y};
        const double dn = 1.0 / fma(d.x, d.x, d.y * d.y);
        const double2 sc{d.x * dn, -d.y * dn};
        for (int i = j + 1 + lane; i < n; i += 64) a[i] = cmul(a[i], sc);
        if (lane == 0) a[j] = double2{beta, 0.0};
      }
      if (lane == 0) tau[j] = t;
    }
    __syncthreads();
    const double2 tj = tau[j];
    if (tj.x != 0.0 || tj.y != 0.0)  // H_j^dag = I - conj(tau) v v^dag
      for (int c = j + 1 + 4 * wave; c < r; c += 4 * nwaves)
        reflect_cols(a, double2{tj.x, -tj.y}, j, n, A, c, r, lane);
    __syncthreads();
  }
  // complement: E = [0; I_{n-r}] in output columns r .. n-1, then E := H_{r-1} ... then H_0
  for (long long idx = tid; idx < (long long)n * (n - r); idx += kCompleteThreads) {
    const int c = (int)(idx / n), row = (int)(idx % n);
    out[(long long)(r + c) * n + row] = double2{row == r + c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int j = r - 1; j >= 0; --j) {
    const double2 tj = tau[j];
    if (tj.x != 0.0 || tj.y != 0.0)  // H_j = I - tau v v^dag
      for (int c = r + 4 * wave; c < n; c += 4 * nwaves)
        reflect_cols(A + (long long)j * n, tj, j, n, out, c, n, lane);
    __syncthreads();
  }
}

// Largest value over the 64 lanes, in every lane (the lane-exchange pattern of wave_sum2).
__device__ inline double wave_max1(double a) {
  a = fmax(a, dpp_move<0xB1>(a));
  a = fmax(a, dpp_move<0x4E>(a));
  a = fmax(a, dpp_move<0x141>(a));
  a = fmax(a, dpp_move<0x140>(a));
  const unsigned long long b1 = static_cast<unsigned long long>(__double_as_longlong(a));
  auto l1 = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(b1), static_cast<unsigned>(b1), false, false);
  auto h1 = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(b1 >> 32), static_cast<unsigned>(b1 >> 32), false, false);
  a = fmax(__longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h1[0]) << 32) | l1[0])),
           __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h1[1]) << 32) | l1[1])));
  const unsigned long long b2 = static_cast<unsigned long long>(__double_as_longlong(a));
  auto l2 = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(b2), static_cast<unsigned>(b2), false, false);
  auto h2 = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(b2 >> 32), static_cast<unsigned>(b2 >> 32), false, false);
  return fmax(__longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h2[0]) << 32) | l2[0])),
              __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h2[1]) << 32) | l2[1])));
}

// Candidate keys of the pivoted QR, one 64-bit word per workgroup and step: bits 63..44 the step
// (plus one), 43..12 the high word of the candidate's squared norm (a non-negative double, so its
// bit pattern orders like its value; 20 mantissa bits decide the pivot), 11..0 4095 minus its
// column. The largest key below the step field is the pivot: largest norm, ties to the smallest
// column; a key with norm field 0 offers no candidate.
__device__ inline unsigned long long qr_key(unsigned step, double norm2, int column) {
  const unsigned hi = norm2 > 0.0 ? (unsigned)((unsigned long long)__double_as_longlong(norm2) >> 32) : 0u;
  return ((unsigned long long)step << 44) | ((unsigned long long)hi << 12) | (unsigned long long)(4095 - column);
}
constexpr unsigned long long kQrKeyMask = (1ull << 44) - 1;

// Waits until every workgroup's key carries step `step` (or later) and returns in every thread the
// largest key (step field removed), or ~0 on a timeout (bounded like wait_flags).
__device__ unsigned long long wait_keys(unsigned long long* keys, unsigned* bar, int nblocks, unsigned step) {
  __shared__ unsigned long long best_sh;
  __shared__ int timed_out;
  if (threadIdx.x == 0) timed_out = 0;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const unsigned long long t0 = wall_clock64();
    unsigned long long best = 0;
    bool fail = false;
    while (true) {
      int mine = 1;
      best = 0;
      for (int k = lane; k < nblocks; k += 64) {
        const unsigned long long key = __hip_atomic_load(&keys[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        mine &= (unsigned)(key >> 44) >= step;
        best = max(best, key & kQrKeyMask);
      }
      if (__all(mine)) break;
      if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > kBarrierTimeoutTicks) {
        fail = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = max(best, (unsigned long long)__shfl_xor((long long)best, off, 64));
    if (fail && lane == 0) {
      __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      timed_out = 1;
    }
    if (lane == 0) best_sh = best;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // pairs with the release stores seen
  }
  __syncthreads();
  return timed_out ? ~0ull : best_sh;
}

// Householder QR with column pivoting of X (mx x nx, column-major; min(mx, nx) steps): at step j the
// remaining column of largest norm becomes column j (pivots kept as a permutation), its reflector
// H_j = I - tau v v^dag (v_j = 1) zeroes it below row j, and H_j^dag is applied to the remaining
// columns. Spread over the Jacobi grid's workgroups (launched together, like the Jacobi
// kernel): workgroup g keeps columns [g C, g C + C) (C = 2b <= 16) of X in LDS, one wave per
// column. Per step j wave 0 takes the workgroup's remaining column of largest norm, forms its
// reflector, publishes the column (rows j..) and the reflector, then a key with its norm and
// index (release), and waits for all other keys; the largest key names the pivot, whose column and
// reflector every wave then loads to apply H_j^dag to its own column and recompute its norm below
// row j; the owner's wave records the pivot and R(j, j). One exchange per step, and the keys
// carry the choice, so no wave reads the candidates separately. Two buffers (by the parity of j)
// keep consecutive steps apart. At the end each workgroup writes its columns back:
// R(r, c) = X[qperm[c]][r] for r <= c. Waits are bounded (barrier-timeout status).
// RM: rows per lane (mx <= 64 RM).
constexpr int kQrThreads = 1024;
template <int RM>
__global__ __launch_bounds__(kQrThreads) void svd_qrcp_grid_kernel(SvdPlan p, SvdWs w, int* status) {
  extern __shared__ double2 slab[];  // [C][mx] columns
  __shared__ double nrm2[16];
  __shared__ int done[16];
  __shared__ unsigned long long key_sh;
  __shared__ double stop2_sh;
  const int m = p.mx, n = p.nx, C = 2 * p.b, nwg = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c_lo = g * C;
  double2* X = w.X;
  if (tid == 0) {  // from the squared column norms of X (w.sigma), summed in a fixed order
    double fro2 = 0.0;
    for (int c = 0; c < n; ++c) fro2 += w.sigma[c];
    const double fl = 4.0 * kEps * sqrt((double)p.frows);  // half the Jacobi rounding floor
    stop2_sh = fl * fl * fro2;
  }
  for (long long idx = tid; idx < (long long)C * m; idx += blockDim.x) {
    const int k = (int)(idx / m), i = (int)(idx % m);
    slab[idx] = c_lo + k < n ? X[(long long)(c_lo + k) * m + i] : double2{0.0, 0.0};
  }
  __syncthreads();
  if (wave < C) {
    double sq = 0.0, dummy = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double2 x = slab[(long long)wave * m + i];
      sq = fma(x.x, x.x, fma(x.y, x.y, sq));
    }
    wave_sum2(sq, dummy);
    if (lane == 0) {
      nrm2[wave] = sq;
      done[wave] = c_lo + wave < n ? 0 : 1;
    }
  }
  bool ok = true;
  int j = 0;
  const int jmax = min(m, n);  // a wide X has rank <= mx
  for (; j < jmax && ok; ++j) {
    const int par = j & 1;
    __syncthreads();  // norms and done flags of the previous step
    if (wave == 0) {  // this workgroup's candidate: its column (rows j..), reflector and key
      const double mine = (lane < C && !done[lane]) ? nrm2[lane] : -1.0;
      const double wmax = wave_max1(mine);
      const unsigned long long hit = __ballot(mine == wmax);
      const int kk = hit ? __builtin_ctzll(hit) : 0;  // (no hit only for a NaN norm)
      const double2* src = slab + (long long)kk * m;
      double2* dst = w.qcol + ((long long)par * nwg + g) * m;
      double sq = 0.0, dummy = 0.0;
      for (int i = j + lane; i < m; i += 64) {
        const double2 x = src[i];
        dst[i] = x;
        if (i > j) sq = fma(x.x, x.x, fma(x.y, x.y, sq));
      }
      wave_sum2(sq, dummy);
      if (lane == 0) {
        const double2 al = src[j];
        double2 tv{0.0, 0.0}, sc{0.0, 0.0};
        double beta = al.x;
        if (sq > 0.0 || al.y != 0.0) {
          const double xn = sqrt(fma(al.x, al.x, fma(al.y, al.y, sq)));
          beta = al.x >= 0.0 ? -xn : xn;
          const double rb = 1.0 / beta;
          tv = double2{(beta - al.x) * rb, -al.y * rb};
          const double2 d{al.x - beta, al.y};
          const double dn = 1.0 / fma(d.x, d.x, d.y * d.y);
          sc = double2{d.x * dn, -d.y * dn};  // 1 / (alpha - beta): v_i = x_i sc below row j
        }
        double* r = w.qrefl + ((long long)par * kMaxGrid + g) * 8;
        r[0] = tv.x;
        r[1] = tv.y;
        r[2] = sc.x;
        r[3] = sc.y;
        r[4] = beta;
        key_sh = qr_key((unsigned)(j + 1), wmax, c_lo + kk);
      }
    }
    // keys by parity too: a workgroup writes this slot again only after every workgroup has
    // published the next step, i.e. has finished reading this one
    unsigned long long* keys = w.qkeys + par * kMaxGrid;
    __syncthreads();  // wave 0's stores before the release
    if (tid == 0) __hip_atomic_store(&keys[g], key_sh, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long best = wait_keys(keys, w.bar, nwg, (unsigned)(j + 1));
    if (best == ~0ull) {
      ok = false;
      break;
    }
    // The remaining columns (at most n - j, each of squared norm at most the largest, which the
    // key holds to 20 mantissa bits) together below half the rounding floor: their part below
    // row j is left out of R (a change of X below the floor, which the Jacobi iteration does
    // not resolve) and the factorisation ends. The same test everywhere; exact zeros included.
    {
      const double bn = __longlong_as_double((long long)(((best >> 12) & 0xffffffffull) << 32));
      if (bn * (double)(n - j) <= stop2_sh) break;
    }
    if (wave >= C) continue;
    const int c = 4095 - (int)(best & 4095), gg = c / C;  // the pivot and its workgroup
    const int k = wave;
    const bool mine_pivot = gg == g && c - c_lo == k;
    const double* r = w.qrefl + ((long long)par * kMaxGrid + gg) * 8;
    if (mine_pivot) {  // R(j, j) and the pivot
      if (lane == 0) {
        slab[(long long)k * m + j] = double2{r[4], 0.0};
        done[k] = 1;
        w.qperm[j] = c;
      }
      continue;
    }
    if (done[k]) continue;
    const double2 tv{r[0], r[1]}, sc{r[2], r[3]};
    // the pivot column below row j and this wave's column (rows j..)
    const double2* pc = w.qcol + ((long long)par * nwg + gg) * m;
    double2 x[RM], col[RM];
    double dr = 0.0, di = 0.0;
#pragma unroll
    for (int t = 0; t < RM; ++t) {
      const int row = lane + 64 * t;
      x[t] = (row > j && row < m) ? pc[row] : double2{0.0, 0.0};
      col[t] = (row >= j && row < m) ? slab[(long long)k * m + row] : double2{0.0, 0.0};
      // conj(x) col
      dr = fma(x[t].x, col[t].x, fma(x[t].y, col[t].y, dr));
      di = fma(x[t].x, col[t].y, fma(-x[t].y, col[t].x, di));
    }
    wave_sum2(dr, di);
    // s = v^dag col = col_j + conj(sc) sum_{i>j} conj(x_i) col_i;  H_j^dag col = col - v conj(tau) s
    const double2 cj = slab[(long long)k * m + j];
    const double2 s{cj.x + sc.x * dr + sc.y * di, cj.y + sc.x * di - sc.y * dr};
    const double2 f = cmul(double2{tv.x, -tv.y}, s);
    const double2 fs = cmul(sc, f);  // v_i conj(tau) s = x_i (sc f) below row j
    double nq = 0.0, dummy = 0.0;
#pragma unroll
    for (int t = 0; t < RM; ++t) {
      const int row = lane + 64 * t;
      if (row == j) col[t] = double2{col[t].x - f.x, col[t].y - f.y};
      else if (row > j && row < m) {
        const double2 d = cmul(x[t], fs);
        col[t] = double2{col[t].x - d.x, col[t].y - d.y};
        nq = fma(col[t].x, col[t].x, fma(col[t].y, col[t].y, nq));
      }
    }
#pragma unroll
    for (int t = 0; t < RM; ++t) {
      const int row = lane + 64 * t;
      if (row >= j && row < m) slab[(long long)k * m + row] = col[t];
    }
    wave_sum2(nq, dummy);
    if (lane == 0) nrm2[k] = nq;
  }
  if (!ok) {
    if (tid == 0) atomicOr(status, kStatusBarrierTimeout);
    return;
  }
  __syncthreads();
  for (long long idx = tid; idx < (long long)C * m; idx += blockDim.x) {
    const int k = (int)(idx / m), i = (int)(idx % m);
    if (c_lo + k < n) X[(long long)(c_lo + k) * m + i] = slab[idx];
  }
  if (g == 0 && tid == 0) *w.qsteps = j;
}

// Pivots of the columns never chosen (all exactly zero below the last step) in increasing order,
// and the inverse permutation. One workgroup.
__global__ __launch_bounds__(1024) void svd_qrperm_kernel(SvdPlan p, SvdWs w) {
  __shared__ int used[kMaxDim];
  const int n = p.nx, j0 = min(max(*w.qsteps, 0), n);
  for (int c = threadIdx.x; c < n; c += blockDim.x) used[c] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < j0; j += blockDim.x) {
    const int q = w.qperm[j];
    if (q >= 0 && q < n) used[q] = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int j = j0;
    for (int c = 0; c < n && j < n; ++c)
      if (!used[c]) w.qperm[j++] = c;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) w.pinv[c] = c;  // (a complete permutation overwrites all)
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int q = w.qperm[j];
    if (q >= 0 && q < n) w.pinv[q] = j;
  }
}

// Blocked Householder QR without pivoting of X (mx x nx, column-major in q.X, nx <= mx <= 512),
// written out as the explicit thin Q (one-site updates: only the column space matters, any
// orthonormal basis of it gives the same fitted state). One launch of G = ceil(nx / P) panel
// workgroups (P = kQbPanel columns each) followed by ceil(mx / 16) row workgroups, all of 16 waves.
// Panel workgroup g owns the columns [P g, P g + P), one wave per column (the other waves only
// meet the barriers), each column in its wave's registers (lane l, register i: row l + 64 i). For
// k = 0 .. g - 1 it waits for panel k (flag) and applies B_k^dag = H_{P-1}^dag ... H_0^dag to its
// columns, reflector by reflector (V_k staged in LDS: one pass over V, where the compact-WY form
// B_k^dag = I - V_k T_k^dag V_k^dag takes two and an exchange between the waves); panel g - 1 it
// takes kQbGroup reflectors at a time, as that panel publishes them, so that most of this update
// overlaps its factorisation. Then it factorises its panel with P Householder steps (H_j = I - tau_j v_j
// v_j^dag, v_j(j) = 1, H_j^dag zeroes column j below row j): at step j the wave of column j + 1
// takes H_j^dag and forms the next reflector at once, handing it to the other waves through LDS
// (two buffers, one barrier per column) and writing it to the panel's column of q.X (zeros above
// the diagonal, 1 on it); after every kQbGroup-th reflector their taus are written and a flag
// raised (release, only when a next panel exists), at the end all P taus (q.tau, 0 for the columns
// past nx: identity reflectors) and the panel flag. Panels of 8 columns: the column step has fewer
// waves reading each reflector and sharing the SIMDs than with 16, and the chain of panel
// hand-offs stays short (0.45 ms per 512 x 256 QR against 0.53 ms with 16 and 0.71 ms with 4);
// groups of 2 reflectors leave less of the previous panel for after its last flag (0.43 ms
// against 0.45 ms with groups of 4).
// Row workgroup b owns rows [16 b, 16 b + 16) of P_Q = B_0 B_1 ... B_{G-1} (one wave per row, the
// row in registers: lane l, register i: column l + 64 i). It starts from the identity and, as panel
// k is published, takes P_Q <- P_Q B_k = P_Q H_0 ... H_{P-1} (reflector by reflector: P_Q -= tau
// (P_Q v) v^dag); Q = P_Q [I; 0] is P_Q's first nx columns. The rows follow the panels one update
// behind, so Q is complete one update after the last panel.
// out (adjoint 0): Q row-major (mx x nx); (adjoint 1): Q^dag row-major (nx x mx). Waits are
// bounded (barrier-timeout status).
constexpr int kQbThreads = 1024;
constexpr int kQbRows = 8;    // entries of a 512-long column (or row) per lane
constexpr int kQbPanel = 8;   // columns per panel workgroup (one wave each; at most 16)
constexpr int kQbGroup = 2;                 // reflectors per group a panel publishes for the next one (>= 2)
constexpr int kQbQuarters = kQbPanel / kQbGroup;  // groups per panel
// Workspace of the blocked QR: X (mx x kQbPanel G, column-major, the columns past nx zero), the
// panels' taus (G x kQbPanel), G panel flags, an abort word, then kQbQuarters G flags (panel g's
// reflectors 4 q .. 4 q + 3 published).
struct QbWs {
  double2* X;
  double2* tau;
  unsigned* flags;
};
size_t qb_bytes(int mx, int G) {
  return align256(sizeof(double2) * (size_t)mx * kQbPanel * G) + align256(sizeof(double2) * kQbPanel * (size_t)G) +
         align256(sizeof(unsigned) * (size_t)((1 + kQbQuarters) * G + 1));
}
QbWs qb_carve(int mx, int G, void* ws) {
  unsigned char* base = static_cast<unsigned char*>(ws);
  QbWs q;
  q.X = reinterpret_cast<double2*>(base);
  base += align256(sizeof(double2) * (size_t)mx * kQbPanel * G);
  q.tau = reinterpret_cast<double2*>(base);
  base += align256(sizeof(double2) * kQbPanel * (size_t)G);
  q.flags = reinterpret_cast<unsigned*>(base);
  return q;
}

// X = Theta (xconj 0) or Theta^dag (xconj 1) into the blocked QR's workspace; flags cleared.
__global__ void qb_init_kernel(const double2* __restrict__ theta, SvdPlan p, QbWs q, int G) {
  const long long total = (long long)p.mx * kQbPanel * G;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / p.mx), row = (int)(idx % p.mx);
    double2 v{0.0, 0.0};
    if (j < p.nx) {
      if (p.xconj == 0) v = theta[(long long)row * p.n + j];
      else {
        const double2 t = theta[(long long)j * p.n + row];
        v = double2{t.x, -t.y};
      }
    }
    q.X[idx] = v;
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < (1 + kQbQuarters) * G + 1; i += blockDim.x) q.flags[i] = 0u;
}

__global__ __launch_bounds__(kQbThreads) void qr_blocked_kernel(SvdPlan p, QbWs q, double2* __restrict__ out,
                                                               int adjoint, int* status) {
  // vs: a panel's V (16 x 512) staged for an update; during a factorisation its first 1024 entries
  // hold the two reflector buffers; at the end of a row workgroup, the transposed rows
  extern __shared__ double2 vs[];
  __shared__ double2 tk[16];  // a staged panel's taus
  __shared__ double2 tau_s[16];
  __shared__ int abort_s;
  const int m = p.mx, n = p.nx, G = (n + kQbPanel - 1) / kQbPanel;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double2* X = q.X;
  unsigned* flags = q.flags;
  unsigned* abort_word = q.flags + G;
  unsigned* qflags = q.flags + G + 1;
  if (tid == 0) abort_s = 0;

  auto wait_flag = [&](unsigned* f) -> bool {
    if (tid == 0) {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > kBarrierTimeoutTicks) {
          __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          abort_s = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return abort_s == 0;
  };
  // reflectors a0 .. a0 + na - 1 of panel k (rows from kQbPanel k on; the rows above are zero)
  // into vs[a][r], their taus into tk[a] (na = kQbGroup or kQbPanel)
  auto stage = [&](int k, int a0, int na) {
    const double2* V = X + (long long)(kQbPanel * k) * m;
    for (int s = 0; s < na / 2; ++s) {
      const int idx = 512 * a0 + tid + kQbThreads * s;
      const int a = idx >> 9, r = idx & 511;
      vs[idx] = (r < m && r >= kQbPanel * k) ? V[(long long)a * m + r] : double2{0.0, 0.0};
    }
    if (tid < na) tk[a0 + tid] = q.tau[kQbPanel * k + a0 + tid];
    __syncthreads();
  };

  if ((int)blockIdx.x < G) {
    // ------------------------------------------------------------------ panel workgroup
    const int g = blockIdx.x, c0 = kQbPanel * g;
    const int ncol = min(kQbPanel, n - c0);
    const bool mine = wv < ncol;  // this wave holds one of the panel's columns
    double2 x[kQbRows];
#pragma unroll
    for (int i = 0; i < kQbRows; ++i) {
      const int r = lane + 64 * i;
      x[i] = (mine && r < m) ? X[(long long)(c0 + wv) * m + r] : double2{0.0, 0.0};
    }
    for (int k = 0; k < g; ++k) {
      // the panel just before this one is taken a quarter at a time, as its reflectors appear
      const bool by_quarter = k == g - 1;
      const int nq = by_quarter ? kQbQuarters : 1, na = kQbPanel / nq;
      for (int qd = 0; qd < nq; ++qd) {
        if (!wait_flag(by_quarter ? &qflags[kQbQuarters * k + qd] : &flags[k])) {
          if (tid == 0) atomicOr(status, kStatusBarrierTimeout);
          return;
        }
        const int a0 = qd * na;
        stage(k, a0, na);
        const int ilo = (kQbPanel * k) >> 6;  // registers below it hold rows above kQbPanel k
        // H_a^dag x for a = a0 .. a0 + na - 1, one reflector after the other (one pass over V,
        // where the compact-WY form takes two): x -= v_a conj(tau_a) (v_a^dag x)
        if (mine)
          for (int a = a0; a < a0 + na; ++a) {
            double2 v[kQbRows];
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int i = 0; i < kQbRows; ++i) {
              v[i] = i < ilo ? double2{0.0, 0.0} : vs[a * 512 + lane + 64 * i];
              sr = fma(v[i].x, x[i].x, fma(v[i].y, x[i].y, sr));
              si = fma(v[i].x, x[i].y, fma(-v[i].y, x[i].x, si));
            }
            wave_sum2(sr, si);
            const double2 t = tk[a];
            const double2 f = cmul(double2{t.x, -t.y}, double2{sr, si});
#pragma unroll
            for (int i = 0; i < kQbRows; ++i) {
              if (i < ilo) continue;
              const double2 dd = cmul(v[i], f);
              x[i] = double2{x[i].x - dd.x, x[i].y - dd.y};
            }
          }
        __syncthreads();  // vs is staged again
      }
    }

    double2* vb = vs;  // vb[0 .. 511], vb[512 .. 1023]: this step's reflector and the next one
    // reflector of column j = c0 + w from the wave's column: beta = -sign(Re alpha) |x|, tau =
    // (beta - alpha) / beta, v = x / (alpha - beta) below row j; the column becomes v (0 above row
    // j, 1 on it), also written to vb[buf]
    auto form = [&](int w, int buf) {
      const int j = c0 + w, ij = j >> 6;
      double2 al{0.0, 0.0};
      double sq = 0.0, dummy = 0.0;
#pragma unroll
      for (int i = 0; i < kQbRows; ++i) {
        const int r = lane + 64 * i;
        if (r > j) sq = fma(x[i].x, x[i].x, fma(x[i].y, x[i].y, sq));
        if (i == ij) al = x[i];
      }
      wave_sum2(sq, dummy);
      al.x = __shfl(al.x, j & 63);
      al.y = __shfl(al.y, j & 63);
      double2 tv{0.0, 0.0}, sc{0.0, 0.0};
      if (sq > 0.0 || al.y != 0.0) {
        const double xn = sqrt(fma(al.x, al.x, fma(al.y, al.y, sq)));
        const double beta = al.x >= 0.0 ? -xn : xn;
        const double rb = 1.0 / beta;
        tv = double2{(beta - al.x) * rb, -al.y * rb};
        const double2 d{al.x - beta, al.y};
        const double dn = 1.0 / fma(d.x, d.x, d.y * d.y);
        sc = double2{d.x * dn, -d.y * dn};  // 1 / (alpha - beta)
      }
#pragma unroll
      for (int i = 0; i < kQbRows; ++i) {
        const int r = lane + 64 * i;
        x[i] = r < j ? double2{0.0, 0.0} : r == j ? double2{1.0, 0.0} : cmul(x[i], sc);
        vb[buf * 512 + r] = x[i];
        if (r < m) X[(long long)j * m + r] = x[i];  // v_j is final: published at once
      }
      if (lane == 0) tau_s[w] = tv;
    };
    if (wv == 0) form(0, 0);
    __syncthreads();
    for (int jj = 0; jj < ncol; ++jj) {
      const int j = c0 + jj, buf = jj & 1, ilo = j >> 6;
      if (mine && wv > jj) {  // s = v^dag x, x -= v conj(tau) s
        double2 v[kQbRows];
#pragma unroll
        for (int i = 0; i < kQbRows; ++i) v[i] = i < ilo ? double2{0.0, 0.0} : vb[buf * 512 + lane + 64 * i];
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int i = 0; i < kQbRows; ++i) {
          dr = fma(v[i].x, x[i].x, fma(v[i].y, x[i].y, dr));
          di = fma(v[i].x, x[i].y, fma(-v[i].y, x[i].x, di));
        }
        wave_sum2(dr, di);
        const double2 t = tau_s[jj];
        const double2 f = cmul(double2{t.x, -t.y}, double2{dr, di});
#pragma unroll
        for (int i = 0; i < kQbRows; ++i) {
          if (i < ilo) continue;
          const double2 d = cmul(v[i], f);
          x[i] = double2{x[i].x - d.x, x[i].y - d.y};
        }
        if (wv == jj + 1) form(wv, buf ^ 1);
      }
      __syncthreads();
      // reflectors jj + 2 - kQbGroup .. jj + 1 formed (their columns written above): a group for
      // the next panel, which has one only if this panel is full
      if (g + 1 < G && (jj + 2) % kQbGroup == 0 && tid == 0) {
        for (int t = jj + 2 - kQbGroup; t <= jj + 1; ++t) q.tau[kQbPanel * g + t] = tau_s[t];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&qflags[kQbQuarters * g + (jj + 1) / kQbGroup], 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // publish the taus of V_g (its columns are written), then the flag
    if (tid < kQbPanel) q.tau[kQbPanel * g + tid] = tid < ncol ? tau_s[tid] : double2{0.0, 0.0};
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&flags[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }

  // -------------------------------------------------------------------- row workgroup
  const int rb = blockIdx.x - G, row = 16 * rb + wv;
  const bool live = row < m;
  double2 pr[kQbRows];
#pragma unroll
  for (int i = 0; i < kQbRows; ++i) pr[i] = double2{lane + 64 * i == row ? 1.0 : 0.0, 0.0};
  for (int k = 0; k < G; ++k) {
    if (!wait_flag(&flags[k])) {
      if (tid == 0) atomicOr(status, kStatusBarrierTimeout);
      return;
    }
    stage(k, 0, kQbPanel);
    const int ilo = (kQbPanel * k) >> 6;  // registers below it hold columns where V_k is zero
    // P_row B_k = P_row H_0 ... H_15, one reflector after the other: P -= tau_a (P v_a) v_a^dag
    if (live)
      for (int a = 0; a < kQbPanel; ++a) {
        double2 v[kQbRows];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int i = 0; i < kQbRows; ++i) {
          v[i] = i < ilo ? double2{0.0, 0.0} : vs[a * 512 + lane + 64 * i];
          sr = fma(pr[i].x, v[i].x, fma(-pr[i].y, v[i].y, sr));
          si = fma(pr[i].x, v[i].y, fma(pr[i].y, v[i].x, si));
        }
        wave_sum2(sr, si);
        const double2 f = cmul(tk[a], double2{sr, si});
#pragma unroll
        for (int i = 0; i < kQbRows; ++i) {
          if (i < ilo) continue;
          pr[i].x -= fma(f.x, v[i].x, f.y * v[i].y);
          pr[i].y -= fma(f.y, v[i].x, -f.x * v[i].y);
        }
      }
    __syncthreads();  // vs is staged again
  }
  if (!adjoint) {
    if (live)
#pragma unroll
      for (int i = 0; i < kQbRows; ++i) {
        const int c = lane + 64 * i;
        if (c < n) out[(long long)row * n + c] = pr[i];
      }
    return;
  }
  // Q^dag: the 16 rows transposed through LDS (entry (c, w) at c 16 + (w xor (c mod 16)))
#pragma unroll
  for (int i = 0; i < kQbRows; ++i) {
    const int c = lane + 64 * i;
    if (c < n) vs[c * 16 + (wv ^ (c & 15))] = double2{pr[i].x, -pr[i].y};
  }
  __syncthreads();
  const int nrow = min(16, m - 16 * rb);
  for (int idx = tid; idx < 16 * n; idx += kQbThreads) {
    const int c = idx >> 4, w = idx & 15;
    if (w < nrow) out[(long long)c * m + 16 * rb + w] = vs[c * 16 + (w ^ (c & 15))];
  }
}

// Y = R^dag into dst (q.mx = nx rows, q.np columns, column-major, columns from q.nx = min(mx, nx)
// on zero): Y(i, c) = conj(R(c, i)) for c <= i, R(c, i) = X[qperm[i]][c] (p: X's plan, q: the
// Jacobi phase's).
__global__ void svd_rdag_kernel(SvdPlan p, SvdPlan q, SvdWs w, double2* __restrict__ dst) {
  const int n = p.nx, m = p.mx, r = q.nx;
  const long long total = (long long)n * q.np;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n), i = (int)(idx % n);
    double2 v{0.0, 0.0};
    if (c < r && c <= i) {
      const double2 r = w.X[(long long)w.qperm[i] * m + c];
      v = double2{r.x, -r.y};
    }
    dst[idx] = v;
  }
}

template <int RMAX, bool ACC>
const void* jacobi_fn() {
  return reinterpret_cast<const void*>(svd_jacobi_kernel<RMAX, ACC>);
}

const void* jacobi_for(const SvdPlan& p) {
  if (p.acc) return p.rmax == 4 ? jacobi_fn<4, true>() : p.rmax == 8 ? jacobi_fn<8, true>() : jacobi_fn<16, true>();
  return p.rmax == 4 ? jacobi_fn<4, false>() : p.rmax == 8 ? jacobi_fn<8, false>() : jacobi_fn<16, false>();
}

}  // namespace

size_t svd_ws_bound(int maxdim) {
  static std::mutex mu;
  static std::map<int, size_t> memo;
  std::lock_guard<std::mutex> lock(mu);
  auto it = memo.find(maxdim);
  if (it != memo.end()) return it->second;
  size_t best = 0;
  for (int m = 1; m <= maxdim; ++m)
    for (int n = 1; n <= maxdim; ++n)
      for (int dir = 0; dir < 2; ++dir) {
        best = std::max(best, svd_plan(m, n, dir, true).ws);
        if (svd_qr_ok(m, n, dir)) best = std::max(best, svd_plan_qr(m, n, dir).ws);
      }
  memo[maxdim] = best;
  return best;
}

hipError_t svd_configure() {
  const void* fns[] = {jacobi_fn<4, false>(), jacobi_fn<8, false>(), jacobi_fn<16, false>(),
                       jacobi_fn<4, true>(),  jacobi_fn<8, true>(),  jacobi_fn<16, true>()};
  for (const void* f : fns)
    MPOEVO_HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSvdLdsBytes));
  for (const void* f : {reinterpret_cast<const void*>(svd_qrcp_grid_kernel<4>),
                        reinterpret_cast<const void*>(svd_qrcp_grid_kernel<8>)})
    MPOEVO_HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQrLdsBytes));
  MPOEVO_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(qr_blocked_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQrLdsBytes));
  return hipSuccess;
}

void finish_plan(SvdPlan& p, size_t lds_cap);

SvdPlan svd_plan(int m, int n, int direction, bool want_basis, size_t lds_cap) {
  SvdPlan p{};
  p.m = m;
  p.n = n;
  p.direction = direction;
  if (m == n) {
    p.xconj = direction;
    p.acc = 0;
  } else if (m > n) {
    p.xconj = 0;
    p.acc = (direction == 1 || want_basis) ? 1 : 0;
  } else {
    p.xconj = 1;
    p.acc = (direction == 0 || want_basis) ? 1 : 0;
  }
  p.mx = p.xconj == 0 ? m : n;
  p.nx = p.xconj == 0 ? n : m;
  p.frows = p.mx;
  p.rank_max = std::min(m, n);
  finish_plan(p, lds_cap);
  return p;
}

// Block layout of the Jacobi kernel for the plan's mx, nx, acc.
void finish_plan(SvdPlan& p, size_t lds_cap) {
  p.rmax = p.mx <= 256 ? 4 : (p.mx <= 512 ? 8 : 16);
  // Block width: small blocks spread a sweep over more workgroups (compute units) at the price
  // of more grid barriers per sweep; 8 columns (16 workgroups for 256 columns) balances the two
  // (16 columns in 1024-thread workgroups, half the barriers, measured 15 % slower: four waves
  // per SIMD then contend for issue).
  const int bmax = p.rmax <= 8 ? 8 : 4;
  const size_t col_bytes = sizeof(double2) * ((size_t)p.mx + (p.acc ? (size_t)p.nx : 0));
  const size_t col_cap = lds_cap / col_bytes;  // columns that fit in LDS
  int b = std::min<int>((p.nx + 1) / 2, bmax);   // one pair per wave
  b = std::max(1, std::min<int>(b, (int)(col_cap / 2)));
  int nb = (p.nx + b - 1) / b;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  p.b = b;
  p.nb = nb;
  p.np = nb * b;
  p.threads = b * 64;
  p.lds = col_bytes * (size_t)2 * p.b;
  p.np_alloc = p.np;
  p.aux_elems = 0;
  p.ws = ws_bytes(p.mx, p.nx, p.np, p.acc != 0, false, p.np_alloc, 0);
  p.split_ok = 1;
}

bool svd_qr_ok(int m, int n, int direction) {
  (void)direction;
  return std::max(m, n) <= kQrMaxDim;
}

// The plan of the Jacobi phase of a pivoted-QR plan: R^dag is nx x min(mx, nx).
static SvdPlan rdag_plan(const SvdPlan& p) {
  SvdPlan q = p;
  q.mx = p.nx;
  q.nx = std::min(p.mx, p.nx);
  finish_plan(q, kSvdLdsBytes);
  q.frows = p.frows;
  q.qr = 1;
  q.np_alloc = std::max(p.np, q.np);
  q.aux_elems = p.aux_elems;
  return q;
}

SvdPlan svd_plan_qr(int m, int n, int direction, size_t lds_cap) {
  // the factor to keep is X's right singular vectors: U of Theta from X = Theta^dag (direction 0),
  // V of Theta from X = Theta (direction 1)
  SvdPlan p{};
  p.m = m;
  p.n = n;
  p.direction = direction;
  p.xconj = direction == 0 ? 1 : 0;
  p.acc = 0;
  p.qr = 1;
  p.mx = p.xconj == 0 ? m : n;
  p.nx = p.xconj == 0 ? n : m;
  p.frows = std::max(p.mx, p.nx);
  p.rank_max = std::min(m, n);
  finish_plan(p, lds_cap);
  const SvdPlan q = rdag_plan(p);
  p.np_alloc = std::max(p.np, q.np);
  p.aux_elems = std::max((size_t)p.mx * p.np, (size_t)q.mx * q.np);
  p.ws = ws_bytes(p.mx, p.nx, p.np, false, true, p.np_alloc, p.aux_elems);
  p.split_ok = 1;
  return p;
}

SvdPlan svd_jacobi_plan(const SvdPlan& p) { return p.qr ? rdag_plan(p) : p; }

SvdPlan svd_plan_unsplit(SvdPlan p) {
  if (p.split_ok) {
    p.split_ok = 0;
    p.ws -= kGemmScratchBytes;
  }
  return p;
}

const void* svd_jacobi_kernel_ptr(const SvdPlan& p) { return jacobi_for(svd_jacobi_plan(p)); }

double svd_sweep_flop(const SvdPlan& p, int nb) {
  // one full round (every pair inside a block pair) and nb - 2 cross rounds (b x b pairs)
  if (nb <= 0) nb = p.nb;
  const double pair_visits =
      (double)(nb / 2) * (p.b * (2.0 * p.b - 1) + (double)(nb - 2) * p.b * p.b);
  return pair_visits * (36.0 * p.mx + (p.acc ? 20.0 * p.nx : 0.0));
}

hipError_t svd_truncate(const SvdPlan& p, const double2* theta, int Dmax, double cutoff,
                        double2* A_out, double2* B_out, int* k_dev, double* disc_dev,
                        double* norm_dev, double* sigma_dev, void* ws, int* status,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, int* sweeps_dev,
                        const double2* warm, double2* basis_out, bool coop, int* complete_dev,
                        int* blocks_dev) {
  if (p.nb / 2 > kMaxGrid || p.threads != 64 * p.b || (p.acc && p.nx > p.mx) ||
      (p.qr && (p.acc || std::max(p.mx, p.nx) > kQrMaxDim || 2 * p.b > kQrThreads / 64)))
    return hipErrorInvalidConfiguration;
  if (p.qr) warm = nullptr;
  SvdWs w = carve(p, ws);
  const int kcap = std::min(Dmax, std::min(p.m, p.n));
  const bool square = p.m == p.n;
  // A preconditioner needs a complete basis to come back: the columns (square) or Q (rectangular).
  if (!square && !p.acc) warm = nullptr, basis_out = nullptr;
  {
    const long long total = (long long)p.mx * p.np;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(svd_init_kernel, dim3(blocks), dim3(256), 0, st, theta, p, w, warm ? 0 : 1,
                       p.acc ? warm : nullptr);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  if (warm) {  // X = Theta P (xconj 0) or Theta^dag P (xconj 1), column-major
    GemmDesc g{};
    g.batch = 1;
    g.ws = p.split_ok ? w.gemm : nullptr; g.ws_bytes = p.split_ok ? kGemmScratchBytes : 0;
    g.A = theta; g.B = warm; g.C = w.X;
    g.M = p.mx; g.N = p.nx; g.K = p.nx;
    if (p.xconj == 0) { g.sAm = p.n; g.sAk = 1; }
    else { g.sAm = 1; g.sAk = p.n; g.conjA = true; }
    g.sBk = 1; g.sBn = p.nx;
    g.sCm = 1; g.sCn = p.mx;
    MPOEVO_HIP_TRY(gemm_launch(g, true, true, st));
  }
  SvdWs wj = w;  // what Jacobi rotates: X itself, or R^dag of the column-pivoted QR of X
  const SvdPlan pj = p.qr ? rdag_plan(p) : p;  // the plan of the Jacobi phase (R^dag: nx x min(mx, nx))
  if (p.qr) {
    {  // squared column norms of X for the factorisation's stopping test
      const int wpb0 = 4;
      hipLaunchKernelGGL(svd_norms_kernel, dim3((p.nx + wpb0 - 1) / wpb0), dim3(64 * wpb0), 0, st, p, w,
                         status, 1);
      MPOEVO_HIP_TRY(hipGetLastError());
    }
    SvdPlan pp = p;
    SvdWs ww = w;
    int* stp = status;
    void* args[] = {&pp, &ww, &stp};
    const size_t lds = sizeof(double2) * (size_t)(2 * p.b) * p.mx;
    const void* fn = p.mx <= 256 ? reinterpret_cast<const void*>(svd_qrcp_grid_kernel<4>)
                                 : reinterpret_cast<const void*>(svd_qrcp_grid_kernel<8>);
    if (coop)
      MPOEVO_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(p.nb / 2), dim3(kQrThreads), args, (unsigned)lds, st));
    else
      MPOEVO_HIP_TRY(hipLaunchKernel(fn, dim3(p.nb / 2), dim3(kQrThreads), args, lds, st));
    hipLaunchKernelGGL(svd_qrperm_kernel, dim3(1), dim3(1024), 0, st, p, w);
    MPOEVO_HIP_TRY(hipGetLastError());
    const long long total = (long long)pj.mx * pj.np;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(svd_rdag_kernel, dim3(blocks), dim3(256), 0, st, p, pj, w, w.aux);
    MPOEVO_HIP_TRY(hipGetLastError());
    wj.X = w.aux;
  }
  const int wpb = 4;
  hipLaunchKernelGGL(svd_norms_kernel, dim3((pj.nx + wpb - 1) / wpb), dim3(64 * wpb), 0, st, pj, wj,
                     status, 1);
  MPOEVO_HIP_TRY(hipGetLastError());
  {
    // above the rounding floor of a length-mx inner product (|err| <= mx eps |x| |y|)
    const double tol = kEps * std::max(16.0, (double)std::max(p.mx, pj.mx));
    SvdPlan pp = pj;
    SvdWs ww = wj;
    double tt = tol;
    int* stp = status;
    int* swp = sweeps_dev;
    int* bkp = blocks_dev;
    void* args[] = {&pp, &ww, &tt, &stp, &swp, &bkp};
    if (ev0) MPOEVO_HIP_TRY(hipEventRecord(ev0, st));
    if (coop)
      MPOEVO_HIP_TRY(hipLaunchCooperativeKernel(jacobi_for(pj), dim3(pj.nb / 2), dim3(pj.threads), args,
                                                (unsigned)pj.lds, st));
    else
      MPOEVO_HIP_TRY(hipLaunchKernel(jacobi_for(pj), dim3(pj.nb / 2), dim3(pj.threads), args, pj.lds, st));
    if (ev1) MPOEVO_HIP_TRY(hipEventRecord(ev1, st));
  }
  hipLaunchKernelGGL(svd_norms_kernel, dim3((pj.nx + wpb - 1) / wpb), dim3(64 * wpb), 0, st, pj, wj,
                     status, 0);
  MPOEVO_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(svd_select_kernel, dim3(1), dim3(1024), 0, st, pj, wj, kcap, cutoff, k_dev,
                     disc_dev, norm_dev, sigma_dev, complete_dev);
  MPOEVO_HIP_TRY(hipGetLastError());
  // the kept factor comes from the columns when it lies on X's column side, else from Q (with
  // the pivoted QR it is always the columns, i.e. X's right singular vectors)
  const bool from_q = !p.qr && ((p.direction == 0) != (p.xconj == 0));
  double2* iso = p.direction == 0 ? A_out : B_out;
  {
    const long long total = (long long)(p.direction == 0 ? p.m : p.n) * kcap;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(svd_isometry_kernel, dim3(blocks), dim3(256), 0, st, pj, wj, kcap, iso,
                       from_q ? 1 : 0);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  if (basis_out) {
    if (square) {
      const long long total = (long long)p.mx * p.nx;
      const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
      hipLaunchKernelGGL(svd_basis_kernel, dim3(blocks), dim3(256), 0, st, pj, wj, basis_out);
      MPOEVO_HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(svd_complete_kernel, dim3(1), dim3(kCompleteThreads), 0, st, pj, wj, basis_out);
      MPOEVO_HIP_TRY(hipGetLastError());
    } else {  // the accumulated P Q (its first nx columns are contiguous)
      MPOEVO_HIP_TRY(hipMemcpyAsync(basis_out, w.Q, sizeof(double2) * (size_t)p.nx * p.nx,
                                    hipMemcpyDeviceToDevice, st));
    }
  }
  GemmDesc g{};
  g.batch = 1;
  g.ws = p.split_ok ? w.gemm : nullptr; g.ws_bytes = p.split_ok ? kGemmScratchBytes : 0;
  if (p.direction == 0) {  // B_out = U_k^dag Theta  (kcap x n)
    g.A = A_out; g.B = theta; g.C = B_out;
    g.M = kcap; g.N = p.n; g.K = p.m;
    g.sAm = 1; g.sAk = kcap; g.conjA = true;
    g.sBk = p.n; g.sBn = 1; g.sCm = p.n; g.sCn = 1;
  } else {  // A_out = Theta V_k  (m x kcap), V_k = B_out^dag
    g.A = theta; g.B = B_out; g.C = A_out;
    g.M = p.m; g.N = kcap; g.K = p.n;
    g.sAm = p.n; g.sAk = 1;
    g.sBk = 1; g.sBn = p.n; g.conjB = true;
    g.sCm = kcap; g.sCn = 1;
  }
  return gemm_launch(g, true, true, st);
}

hipError_t qr_isometry(const SvdPlan& p, const double2* theta, double2* out, bool adjoint, void* ws,
                       int* status, hipStream_t st, bool coop) {
  const int G = (p.nx + kQbPanel - 1) / kQbPanel;
  if (!p.qr || p.acc || p.mx < p.nx || p.mx > kQrMaxDim || G > kMaxGrid || qb_bytes(p.mx, G) > p.ws)
    return hipErrorInvalidConfiguration;
  const QbWs q = qb_carve(p.mx, G, ws);
  {
    const long long total = (long long)p.mx * kQbPanel * G;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(qb_init_kernel, dim3(blocks), dim3(256), 0, st, theta, p, q, G);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  SvdPlan pp = p;
  QbWs qq = q;
  double2* o = out;
  int adj = adjoint ? 1 : 0;
  int* stp = status;
  void* args[] = {&pp, &qq, &o, &adj, &stp};
  const size_t lds = kQrLdsBytes;  // vs: 16 x 512 complex
  const int wgs = G + (p.mx + 15) / 16;  // the panels, then the row blocks of Q
  const void* fn = reinterpret_cast<const void*>(qr_blocked_kernel);
  if (coop)
    MPOEVO_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(wgs), dim3(kQbThreads), args, (unsigned)lds, st));
  else
    MPOEVO_HIP_TRY(hipLaunchKernel(fn, dim3(wgs), dim3(kQbThreads), args, lds, st));
  last_launch() = LaunchRecord{fn, false};
  return hipSuccess;
}

}  // namespace mpoevo
