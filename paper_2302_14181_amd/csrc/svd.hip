// FP64 SVD of the projected two-site tensor by one-sided (Hestenes) Jacobi, and the truncation
// of the two-site update (keep k <= Dmax singular values, split as U | S V^dag or U S | V^dag).
//
// Orientation follows the sweep direction: left-to-right keeps U, so Jacobi orthogonalises the
// columns of X = Theta (U_j = X_j / |X_j| after convergence) and the other factor is the exact
// projection S V^dag = U^dag Theta; right-to-left keeps V, so X = Theta^dag (V_j = X_j / |X_j|)
// and U S = Theta V. The two products run on the FP64 matrix cores.
//
// Numerically zero columns: a column whose norm is at the rounding level of the matrix,
// floor = 8 eps sqrt(mx) ||Theta||_F, only carries cancellation noise; rotating it against a
// large column regenerates noise of its own size, so pairs with such a column are not rotated
// and those singular values are treated as zero (never kept). Every other pair is rotated until
// |x^dag y| <= tol |x| |y|, so the normalised kept columns are orthonormal to tol.
//
// Parallel schedule: the np columns are cut into nb blocks of b columns; a round pairs the
// blocks (round-robin), one workgroup per block pair holds its 2b columns in LDS and performs one
// cyclic sweep over all their column pairs, one wave per pair with both columns in registers.
// Rounds are separated by a grid barrier of the cooperative launch; a sweep whose largest
// relative inner product is below tol (or below kAccept) ends the iteration.

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "dev_common.h"
#include "svd.h"

namespace mpoevo {
namespace {

constexpr int kMaxSweeps = 60;
constexpr double kAccept = 1e-13;  // columns this orthogonal need no further sweep
constexpr double kEps = 2.220446049250313e-16;
constexpr unsigned long long kBarrierTimeoutTicks = 300000000ull;  // 3 s of the 100 MHz clock

struct SvdWs {  // carved from the caller's workspace
  double2* X;           // [np][mx] column-major
  double* sigma;        // [np]
  int* perm;            // [np]
  unsigned* bar;        // [0] arrival count, [1] generation, [2] timeout flag
  unsigned* sweep_max;  // [kMaxSweeps] bits of the largest |x^dag y| / (|x| |y|) of a sweep
  int* k_shared;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

SvdWs carve(const SvdPlan& p, void* ws) {
  unsigned char* base = static_cast<unsigned char*>(ws);
  SvdWs w;
  size_t off = 0;
  w.X = reinterpret_cast<double2*>(base + off);
  off += align256(sizeof(double2) * (size_t)p.mx * p.np);
  w.sigma = reinterpret_cast<double*>(base + off);
  off += align256(sizeof(double) * p.np);
  w.perm = reinterpret_cast<int*>(base + off);
  off += align256(sizeof(int) * p.np);
  w.bar = reinterpret_cast<unsigned*>(base + off);
  off += 256;
  w.sweep_max = reinterpret_cast<unsigned*>(base + off);
  off += align256(sizeof(unsigned) * kMaxSweeps);
  w.k_shared = reinterpret_cast<int*>(base + off);
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
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Sum over the 64 lanes, identical in every lane (each step adds the same two numbers in both
// partner lanes): pair lanes within quads, then halves of 8, rows of 16, then across rows.
__device__ inline void wave_sum4(double& a, double& b, double& c, double& d) {
  a += dpp_move<0xB1>(a); b += dpp_move<0xB1>(b); c += dpp_move<0xB1>(c); d += dpp_move<0xB1>(d);
  a += dpp_move<0x4E>(a); b += dpp_move<0x4E>(b); c += dpp_move<0x4E>(c); d += dpp_move<0x4E>(d);
  a += dpp_move<0x141>(a); b += dpp_move<0x141>(b); c += dpp_move<0x141>(c); d += dpp_move<0x141>(d);
  a += dpp_move<0x140>(a); b += dpp_move<0x140>(b); c += dpp_move<0x140>(c); d += dpp_move<0x140>(d);
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
    c += __shfl_xor(c, off, 64);
    d += __shfl_xor(d, off, 64);
  }
}

// 1/sqrt(x) and 1/x to full double precision: hardware estimate plus Newton steps.
__device__ inline double rsqrt_d(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r;
}
__device__ inline double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}

// Round-robin pairing of n (even) items: round r in 0..n-2, pair index k in 0..n/2-1.
__device__ inline void rr_pair(int r, int k, int n, int& x, int& y) {
  x = (r + k) % (n - 1);
  y = (k == 0) ? (n - 1) : (r - k + n - 1) % (n - 1);
}

// X = Theta (direction 0) or Theta^dag (direction 1), zero padding columns; clear the state.
__global__ void svd_init_kernel(const double2* __restrict__ theta, SvdPlan p, SvdWs w) {
  const long long total = (long long)p.mx * p.np;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / p.mx), row = (int)(idx % p.mx);
    double2 v{0.0, 0.0};
    if (j < p.nx) {
      if (p.direction == 0) v = theta[(long long)row * p.n + j];
      else {
        const double2 t = theta[(long long)j * p.n + row];
        v = double2{t.x, -t.y};
      }
    }
    w.X[idx] = v;
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x < 3) w.bar[threadIdx.x] = 0u;
    for (int i = threadIdx.x; i < kMaxSweeps; i += blockDim.x) w.sweep_max[i] = 0u;
  }
}

__device__ bool grid_barrier(unsigned* bar, unsigned nblocks) {
  __shared__ int timed_out;
  __syncthreads();
  if (threadIdx.x == 0) {
    timed_out = 0;
    __threadfence();
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived =
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > kBarrierTimeoutTicks) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          timed_out = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();
  }
  __syncthreads();
  return timed_out == 0;
}

// One-sided Jacobi sweeps. RMAX = rows per lane (mx <= 64 RMAX). Launched cooperatively with
// nb / 2 workgroups; dynamic LDS holds 2b columns of mx rows.
template <int RMAX>
__global__ __launch_bounds__(RMAX <= 8 ? 1024 : 512) void svd_jacobi_kernel(SvdPlan p, SvdWs w,
                                                                          double tol, int* status,
                                                                          int* sweeps_out) {
  extern __shared__ double2 cols[];  // [2b][mx]
  __shared__ unsigned wg_max;        // bits of a non-negative float: integer order = value order
  __shared__ double floor2_sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const int two_b = 2 * p.b, mx = p.mx;
  if (tid == 0) {  // squared rounding floor from the initial column norms (fixed order)
    double fro2 = 0.0;
    for (int j = 0; j < p.nx; ++j) fro2 += w.sigma[j];
    const double fl = 8.0 * kEps * sqrt((double)mx);
    floor2_sh = fl * fl * fro2;
  }
  __syncthreads();
  const double floor2 = floor2_sh;
  const double tol2 = tol * tol;
  const unsigned nblk = gridDim.x;
  bool ok = true;
  int sweep = 0;
  for (; sweep < kMaxSweeps && ok; ++sweep) {
    for (int r = 0; r < p.nb - 1 && ok; ++r) {
      int bp, bq;
      rr_pair(r, blockIdx.x, p.nb, bp, bq);
      for (int idx = tid; idx < two_b * mx; idx += blockDim.x) {
        const int c = idx / mx, row = idx - c * mx;
        const int g = (c < p.b) ? bp * p.b + c : bq * p.b + (c - p.b);
        cols[idx] = w.X[(long long)g * mx + row];
      }
      if (tid == 0) wg_max = 0u;
      __syncthreads();
      for (int ir = 0; ir < two_b - 1; ++ir) {
        for (int pk = wave; pk < p.b; pk += nwaves) {
          int x, y;
          rr_pair(ir, pk, two_b, x, y);
          double2* cx = cols + x * mx;
          double2* cy = cols + y * mx;
          double2 u[RMAX], v[RMAX];
          double a = 0.0, bb = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
          for (int t = 0; t < RMAX; ++t) {
            const int row = lane + 64 * t;
            if (row < mx) {
              u[t] = cx[row];
              v[t] = cy[row];
            } else {
              u[t] = double2{0.0, 0.0};
              v[t] = double2{0.0, 0.0};
            }
            a = fma(u[t].x, u[t].x, fma(u[t].y, u[t].y, a));
            bb = fma(v[t].x, v[t].x, fma(v[t].y, v[t].y, bb));
            gr = fma(u[t].x, v[t].x, fma(u[t].y, v[t].y, gr));
            gi = fma(u[t].x, v[t].y, fma(-u[t].y, v[t].x, gi));
          }
          wave_sum4(a, bb, gr, gi);
          // Rotation parameters without divisions or square roots: |gamma|^2 = g2,
          // r = 1/|gamma|, phase e = conj(gamma) r, zeta = (|y|^2 - |x|^2) / (2 |gamma|),
          // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = t c. Only c, s
          // and e must be exact (a unitary rotation); t may carry rounding, which only leaves a
          // slightly larger remainder for the next sweep.
          const double g2 = fma(gr, gr, gi * gi);
          const double ab = a * bb;
          const bool live = fmin(a, bb) > floor2;
          if (live && lane == 0 && ab > 0.0)
            atomicMax(&wg_max, __float_as_uint(sqrtf((float)fmin(g2 * rcp_d(ab), 1.0))));
          if (live && g2 > tol2 * ab) {
            const double r = rsqrt_d(g2);
            const double zeta = 0.5 * (bb - a) * r;
            const double q = (zeta * zeta < 1e300) ? (1.0 + zeta * zeta) * rsqrt_d(1.0 + zeta * zeta) : fabs(zeta);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_d(fabs(zeta) + q);
            const double c = rsqrt_d(1.0 + t * t), s = t * c;
            const double er = gr * r, ei = -gi * r;  // conj(gamma) / |gamma|
#pragma unroll
            for (int tt = 0; tt < RMAX; ++tt) {
              const int row = lane + 64 * tt;
              if (row < mx) {
                const double evx = er * v[tt].x - ei * v[tt].y, evy = er * v[tt].y + ei * v[tt].x;
                cx[row] = double2{c * u[tt].x - s * evx, c * u[tt].y - s * evy};
                cy[row] = double2{s * u[tt].x + c * evx, s * u[tt].y + c * evy};
              }
            }
          }
        }
        __syncthreads();
      }
      for (int idx = tid; idx < two_b * mx; idx += blockDim.x) {
        const int c = idx / mx, row = idx - c * mx;
        const int g = (c < p.b) ? bp * p.b + c : bq * p.b + (c - p.b);
        w.X[(long long)g * mx + row] = cols[idx];
      }
      if (tid == 0 && wg_max) atomicMax(&w.sweep_max[sweep], wg_max);
      ok = grid_barrier(w.bar, nblk);
    }
    if (!ok) break;
    const float mxr = __uint_as_float(
        __hip_atomic_load(&w.sweep_max[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
    if ((double)mxr <= tol || (double)mxr <= kAccept) break;
  }
  if (blockIdx.x == 0 && tid == 0) {
    atomicMax(&status[1], sweep + 1);
    if (sweeps_out) *sweeps_out = sweep + 1;
    if (!ok) atomicOr(status, kStatusBarrierTimeout);
    else if (sweep >= kMaxSweeps) {
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
                                                          double* sigma_dev) {
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
  const double floor_abs = 8.0 * kEps * sqrt((double)p.mx) * sqrt(fro2);
  const double thr = fmax(cutoff * smax, floor_abs);
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
    *w.k_shared = k;
    if (k_dev) *k_dev = k;
    if (disc_dev) *disc_dev = tot > 0.0 ? fmax(0.0, (tot - kept) / tot) : 0.0;
    if (norm_dev) *norm_dev = sqrt(kept);
  }
}

// The kept isometry: direction 0 -> A_out[i][r] = X[i][perm r] / sigma (m x kcap);
// direction 1 -> B_out[r][c] = conj(X[c][perm r]) / sigma (kcap x n). Zero beyond k.
__global__ void svd_isometry_kernel(SvdPlan p, SvdWs w, int kcap, double2* out) {
  const int k = *w.k_shared;
  const long long total = (long long)p.mx * kcap;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int i, rr;
    if (p.direction == 0) { i = (int)(idx / kcap); rr = (int)(idx % kcap); }
    else { rr = (int)(idx / p.mx); i = (int)(idx % p.mx); }
    double2 v{0.0, 0.0};
    if (rr < k) {
      const int j = w.perm[rr];
      const double s = w.sigma[j];
      const double2 x = w.X[(long long)j * p.mx + i];
      if (s > 0.0) v = double2{x.x / s, (p.direction == 0 ? x.y : -x.y) / s};
    }
    out[idx] = v;
  }
}

}  // namespace

size_t svd_ws_bound(int maxdim) {
  static std::mutex mu;
  static std::map<int, size_t> memo;
  std::lock_guard<std::mutex> lock(mu);
  auto it = memo.find(maxdim);
  if (it != memo.end()) return it->second;
  size_t best = 0;
  for (int mx = 1; mx <= maxdim; ++mx)
    for (int nx = 1; nx <= maxdim; ++nx) best = std::max(best, svd_plan(mx, nx, 0).ws);
  memo[maxdim] = best;
  return best;
}

hipError_t svd_configure() {
  MPOEVO_HIP_TRY(hipFuncSetAttribute((const void*)svd_jacobi_kernel<4>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSvdLdsBytes));
  MPOEVO_HIP_TRY(hipFuncSetAttribute((const void*)svd_jacobi_kernel<8>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSvdLdsBytes));
  return hipFuncSetAttribute((const void*)svd_jacobi_kernel<16>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSvdLdsBytes);
}

SvdPlan svd_plan(int m, int n, int direction, size_t lds_cap) {
  SvdPlan p;
  p.m = m;
  p.n = n;
  p.direction = direction;
  p.mx = direction == 0 ? m : n;
  p.nx = direction == 0 ? n : m;
  p.rank_max = std::min(m, n);
  p.rmax = p.mx <= 256 ? 4 : (p.mx <= 512 ? 8 : 16);
  const int waves = p.rmax <= 8 ? 16 : 8;
  const size_t col_cap = lds_cap / (sizeof(double2) * (size_t)p.mx);  // columns that fit in LDS
  int b = std::min<int>((p.nx + 1) / 2, waves);                       // one pair per wave
  b = std::max(1, std::min<int>(b, (int)(col_cap / 2)));
  int nb = (p.nx + b - 1) / b;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  p.b = b;
  p.nb = nb;
  p.np = nb * b;
  p.threads = waves * 64;
  p.lds = sizeof(double2) * (size_t)2 * p.b * p.mx;
  p.ws = align256(sizeof(double2) * (size_t)p.mx * p.np) + align256(sizeof(double) * p.np) +
         align256(sizeof(int) * p.np) + 256 + align256(sizeof(unsigned) * kMaxSweeps) + 256;
  return p;
}

double svd_sweep_flop(const SvdPlan& p) {
  const double pair_visits = (double)(p.nb - 1) * (p.nb / 2) * p.b * (2 * p.b - 1);
  return pair_visits * 36.0 * p.mx;
}

hipError_t svd_truncate(const SvdPlan& p, const double2* theta, int Dmax, double cutoff,
                        double2* A_out, double2* B_out, int* k_dev, double* disc_dev,
                        double* norm_dev, double* sigma_dev, void* ws, int* status,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, int* sweeps_dev) {
  SvdWs w = carve(p, ws);
  const int kcap = std::min(Dmax, std::min(p.m, p.n));
  {
    const long long total = (long long)p.mx * p.np;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(svd_init_kernel, dim3(blocks), dim3(256), 0, st, theta, p, w);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  const int wpb = 4;
  hipLaunchKernelGGL(svd_norms_kernel, dim3((p.nx + wpb - 1) / wpb), dim3(64 * wpb), 0, st, p, w,
                     status, 1);
  MPOEVO_HIP_TRY(hipGetLastError());
  {
    // above the rounding floor of a length-mx inner product (|err| <= mx eps |x| |y|)
    const double tol = kEps * std::max(16.0, (double)p.mx);
    SvdPlan pp = p;
    SvdWs ww = w;
    double tt = tol;
    int* stp = status;
    int* swp = sweeps_dev;
    void* args[] = {&pp, &ww, &tt, &stp, &swp};
    const void* fn = p.rmax == 4 ? (const void*)svd_jacobi_kernel<4>
                     : p.rmax == 8 ? (const void*)svd_jacobi_kernel<8>
                                   : (const void*)svd_jacobi_kernel<16>;
    if (ev0) MPOEVO_HIP_TRY(hipEventRecord(ev0, st));
    MPOEVO_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(p.nb / 2), dim3(p.threads), args,
                                              (unsigned)p.lds, st));
    if (ev1) MPOEVO_HIP_TRY(hipEventRecord(ev1, st));
  }
  hipLaunchKernelGGL(svd_norms_kernel, dim3((p.nx + wpb - 1) / wpb), dim3(64 * wpb), 0, st, p, w,
                     status, 0);
  MPOEVO_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(svd_select_kernel, dim3(1), dim3(1024), 0, st, p, w, kcap, cutoff, k_dev,
                     disc_dev, norm_dev, sigma_dev);
  MPOEVO_HIP_TRY(hipGetLastError());
  double2* iso = p.direction == 0 ? A_out : B_out;
  {
    const long long total = (long long)p.mx * kcap;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(svd_isometry_kernel, dim3(blocks), dim3(256), 0, st, p, w, kcap, iso);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  GemmDesc g{};
  g.batch = 1;
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

}  // namespace mpoevo
