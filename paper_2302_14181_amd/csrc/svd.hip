// FP64 SVD of the projected two-site tensor by one-sided (Hestenes) Jacobi, and the truncation
// of the two-site update (keep k <= Dmax singular values, split as U | S V^dag or U S | V^dag).
//
// Jacobi runs on the columns of X = Theta (if n < m) or X = Theta^dag (if m < n), so the number
// of columns is min(m, n); a square Theta is taken in the orientation whose accumulated factor
// is the isometry the sweep direction keeps (U for left-to-right, V for right-to-left). Each
// column of the work buffer holds X[:, j] (mx rows) followed by the j-th column of the
// accumulated unitary (np rows, starting as the identity): every plane rotation is applied to
// the whole stacked column, so the accumulated factor is unitary to rounding.
//
// Numerically zero columns: a column whose norm is at the rounding level of the matrix,
// floor = 8 eps sqrt(mx) ||Theta||_F, only carries cancellation noise; rotating it against a
// large column regenerates noise of its own size, so pairs with such a column are not rotated
// and those singular values are treated as zero (never kept). All other pairs are rotated
// until |x^dag y| <= tol |x| |y| (relative orthogonality to working precision), so the
// normalised columns of X that are kept are orthonormal to tol.
//
// Parallel schedule: the np columns are cut into nb blocks of b columns; a round pairs the
// blocks (round-robin), one workgroup per block pair loads its 2b stacked columns into LDS and
// performs one cyclic sweep over all of their column pairs (b disjoint pairs per inner round,
// one wave per pair). Rounds are separated by a grid barrier of the cooperative launch. A sweep
// with no rotation above tol * sqrt(|x|^2 |y|^2) ends the iteration.

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "dev_common.h"
#include "svd.h"

namespace mpoevo {
namespace {

constexpr int kJacThreads = 256;
constexpr int kMaxSweeps = 60;
constexpr double kAcceptOrthogonality = 1e-13;  // columns this orthogonal need no further sweep
constexpr unsigned long long kBarrierTimeoutTicks = 300000000ull;  // 3 s of the 100 MHz clock

struct SvdWs {  // carved from the caller's workspace
  double2* Y;
  double* sigma;
  int* perm;
  unsigned* bar;      // [0] arrival count, [1] generation, [2] timeout flag
  unsigned* sweep_max;  // [kMaxSweeps] bits of the largest |x^dag y| / (|x| |y|) seen in a sweep
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

SvdWs carve(const SvdPlan& p, void* ws) {
  unsigned char* base = static_cast<unsigned char*>(ws);
  SvdWs w;
  size_t off = 0;
  w.Y = reinterpret_cast<double2*>(base + off);
  off += align256(sizeof(double2) * (size_t)p.H * p.np);
  w.sigma = reinterpret_cast<double*>(base + off);
  off += align256(sizeof(double) * p.np);
  w.perm = reinterpret_cast<int*>(base + off);
  off += align256(sizeof(int) * p.np);
  w.bar = reinterpret_cast<unsigned*>(base + off);
  off += 256;
  w.sweep_max = reinterpret_cast<unsigned*>(base + off);
  return w;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Round-robin pairing of n (even) items: round r in 0..n-2, pair index k in 0..n/2-1.
__device__ inline void rr_pair(int r, int k, int n, int& x, int& y) {
  x = (r + k) % (n - 1);
  y = (k == 0) ? (n - 1) : (r - k + n - 1) % (n - 1);
}

// Build the stacked work matrix and clear the iteration state.
__global__ void svd_init_kernel(const double2* __restrict__ theta, SvdPlan p, SvdWs w) {
  const long long total = (long long)p.H * p.np;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / p.H), row = (int)(idx % p.H);
    double2 v{0.0, 0.0};
    if (row < p.mx) {
      if (j < p.nx) {
        if (p.on_theta) v = theta[(long long)row * p.n + j];  // X = Theta, column j
        else {
          const double2 t = theta[(long long)j * p.n + row];  // X = Theta^dag, column j
          v = double2{t.x, -t.y};
        }
      }
    } else {
      v.x = (row - p.mx == j) ? 1.0 : 0.0;
    }
    w.Y[idx] = v;
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
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();
  }
  __syncthreads();
  return timed_out == 0;
}

__global__ __launch_bounds__(kJacThreads) void svd_jacobi_kernel(SvdPlan p, SvdWs w, double tol,
                                                                 double accept, int* status) {
  extern __shared__ double2 cols[];  // [2b][H]
  __shared__ unsigned wg_max;  // bits of a non-negative float: integer order = value order
  __shared__ double floor2_sh;
  if (threadIdx.x == 0) {  // squared rounding floor from the initial column norms (fixed order)
    double fro2 = 0.0;
    for (int j = 0; j < p.nx; ++j) fro2 += w.sigma[j];
    const double fl = 8.0 * 2.220446049250313e-16 * sqrt((double)p.mx);
    floor2_sh = fl * fl * fro2;
  }
  __syncthreads();
  const double floor2 = floor2_sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = kJacThreads / 64;
  const int two_b = 2 * p.b, H = p.H;
  const unsigned nblk = gridDim.x;
  bool ok = true;
  int sweep = 0;
  for (; sweep < kMaxSweeps && ok; ++sweep) {
    for (int r = 0; r < p.nb - 1 && ok; ++r) {
      int bp, bq;
      rr_pair(r, blockIdx.x, p.nb, bp, bq);
      for (int idx = tid; idx < two_b * H; idx += kJacThreads) {
        const int c = idx / H, row = idx % H;
        const int g = (c < p.b) ? bp * p.b + c : bq * p.b + (c - p.b);
        cols[idx] = w.Y[(long long)g * H + row];
      }
      if (tid == 0) wg_max = 0u;
      __syncthreads();
      for (int ir = 0; ir < two_b - 1; ++ir) {
        for (int pk = wave; pk < p.b; pk += nwaves) {
          int x, y;
          rr_pair(ir, pk, two_b, x, y);
          double2* cx = cols + x * H;
          double2* cy = cols + y * H;
          double a = 0.0, bb = 0.0, gr = 0.0, gi = 0.0;
          for (int row = lane; row < p.mx; row += 64) {
            const double2 u = cx[row], v = cy[row];
            a = fma(u.x, u.x, fma(u.y, u.y, a));
            bb = fma(v.x, v.x, fma(v.y, v.y, bb));
            gr = fma(u.x, v.x, fma(u.y, v.y, gr));
            gi = fma(u.x, v.y, fma(-u.y, v.x, gi));
          }
          a = wave_sum(a);
          bb = wave_sum(bb);
          gr = wave_sum(gr);
          gi = wave_sum(gi);
          const double g = hypot(gr, gi);
          const double nrm = sqrt(a) * sqrt(bb);
          const bool live = fmin(a, bb) > floor2;  // both columns above the rounding floor
          if (live && lane == 0) atomicMax(&wg_max, __float_as_uint((float)fmin(g / nrm, 1.0)));
          if (live && g > tol * nrm) {
            const double zeta = (bb - a) / (2.0 * g);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            const double er = gr / g, ei = -gi / g;  // conj(gamma) / |gamma|
            for (int row = lane; row < H; row += 64) {
              const double2 u = cx[row], v = cy[row];
              const double evx = er * v.x - ei * v.y, evy = er * v.y + ei * v.x;
              cx[row] = double2{c * u.x - s * evx, c * u.y - s * evy};
              cy[row] = double2{s * u.x + c * evx, s * u.y + c * evy};
            }
          }
        }
        __syncthreads();
      }
      for (int idx = tid; idx < two_b * H; idx += kJacThreads) {
        const int c = idx / H, row = idx % H;
        const int g = (c < p.b) ? bp * p.b + c : bq * p.b + (c - p.b);
        w.Y[(long long)g * H + row] = cols[idx];
      }
      if (tid == 0 && wg_max) atomicMax(&w.sweep_max[sweep], wg_max);
      ok = grid_barrier(w.bar, nblk);
    }
    if (!ok) break;
    // stop when no pair needed a rotation, or every pair was already orthogonal to `accept`
    // (plane rotations at the rounding floor of the inner products can otherwise repeat forever)
    const float mx = __uint_as_float(
        __hip_atomic_load(&w.sweep_max[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
    if ((double)mx <= tol || (double)mx <= accept) break;
  }
  if (blockIdx.x == 0 && tid == 0) {
    atomicMax(&status[1], sweep + 1);
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
  const double2* c = w.Y + (long long)j * p.H;
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
                                                          double* sigma_dev, int* k_shared) {
  __shared__ double sig[1024];
  __shared__ int rank_of[1024];
  __shared__ double red[1024];
  __shared__ int cnt[1024];
  const int t = threadIdx.x;
  const int r = p.nx;
  sig[t] = (t < r) ? w.sigma[t] : -1.0;
  __syncthreads();
  int rk = 0;
  if (t < r) {
    const double s = sig[t];
    for (int i = 0; i < r; ++i) rk += (sig[i] > s || (sig[i] == s && i < t)) ? 1 : 0;
    rank_of[t] = rk;
    w.perm[rk] = t;
    if (sigma_dev) sigma_dev[rk] = s;
  }
  __syncthreads();
  // sigma_max and the count above the cutoff
  double smax = 0.0, fro2 = 0.0;
  for (int i = 0; i < r; ++i) {
    smax = fmax(smax, sig[i]);
    fro2 += sig[i] * sig[i];
  }
  const double floor_abs = 8.0 * 2.220446049250313e-16 * sqrt((double)p.mx) * sqrt(fro2);
  const double thr = fmax(cutoff * smax, floor_abs);
  cnt[t] = (t < r && sig[t] > 0.0 && sig[t] > thr) ? 1 : 0;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) cnt[t] += cnt[t + off];
    __syncthreads();
  }
  int k = cnt[0];
  k = k < 1 ? 1 : (k > kcap ? kcap : k);
  // total weight and kept weight (fixed-order tree sums over rank order)
  __syncthreads();
  red[t] = 0.0;
  if (t < r) red[rank_of[t]] = sig[t] * sig[t];
  __syncthreads();
  __shared__ double kept_part[1024];
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
    *k_shared = k;
    if (k_dev) *k_dev = k;
    if (disc_dev) *disc_dev = tot > 0.0 ? fmax(0.0, (tot - kept) / tot) : 0.0;
    if (norm_dev) *norm_dev = sqrt(kept);
  }
}

// A_out (m x kcap) and B_out (kcap x n); entries at rank >= k are zero.
__global__ void svd_output_kernel(SvdPlan p, SvdWs w, int kcap, int direction,
                                  const int* k_shared, double2* A_out, double2* B_out) {
  const int k = *k_shared;
  const long long na = (long long)p.m * kcap, nbt = (long long)kcap * p.n;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < na + nbt;
       idx += (long long)gridDim.x * blockDim.x) {
    double2 out{0.0, 0.0};
    if (idx < na) {
      const int i = (int)(idx / kcap), rr = (int)(idx % kcap);
      if (rr < k) {
        const int j = w.perm[rr];
        const double s = w.sigma[j];
        const double2* col = w.Y + (long long)j * p.H;
        double2 u;  // U[i][j]
        if (p.on_theta) {
          u = col[i];  // sigma_j U[i][j]
          if (direction == 0) u = (s > 0.0) ? double2{u.x / s, u.y / s} : double2{0.0, 0.0};
        } else {
          u = col[p.mx + i];  // accumulated factor = U
          if (direction == 1) u = double2{u.x * s, u.y * s};
        }
        out = u;
      }
      A_out[idx] = out;
    } else {
      const long long jdx = idx - na;
      const int rr = (int)(jdx / p.n), c = (int)(jdx % p.n);
      if (rr < k) {
        const int j = w.perm[rr];
        const double s = w.sigma[j];
        const double2* col = w.Y + (long long)j * p.H;
        double2 v;  // conj(V[c][j]) scaled: LEFT -> sigma conj(V), RIGHT -> conj(V)
        if (p.on_theta) {
          v = col[p.mx + c];  // accumulated factor = V
          v = double2{v.x, -v.y};
          if (direction == 0) v = double2{v.x * s, v.y * s};
        } else {
          v = col[c];  // sigma_j V[c][j]
          v = double2{v.x, -v.y};
          if (direction == 1) v = (s > 0.0) ? double2{v.x / s, v.y / s} : double2{0.0, 0.0};
        }
        out = v;
      }
      B_out[jdx] = out;
    }
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
    for (int nx = 1; nx <= mx; ++nx) best = std::max(best, svd_plan(mx, nx).ws);
  memo[maxdim] = best;
  return best;
}

hipError_t svd_configure() {
  return hipFuncSetAttribute((const void*)svd_jacobi_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSvdLdsBytes);
}

SvdPlan svd_plan(int m, int n, size_t lds_cap) {
  SvdPlan p;
  p.m = m;
  p.n = n;
  p.on_theta = (n <= m);
  p.mx = p.on_theta ? m : n;
  p.nx = p.on_theta ? n : m;
  // largest b with 2b stacked columns in LDS; the stack height depends on np = nb * b
  const size_t col_cap = lds_cap / sizeof(double2);
  int b = (p.nx + 1) / 2;
  for (;;) {
    int nb = (p.nx + b - 1) / b;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const int np = nb * b;
    const int H = p.mx + np;
    if ((size_t)2 * b * H <= col_cap || b == 1) {
      p.b = b;
      p.nb = nb;
      p.np = np;
      p.H = H;
      break;
    }
    b = (b + 1) / 2 == b ? b - 1 : (b + 1) / 2;
  }
  p.lds = sizeof(double2) * (size_t)2 * p.b * p.H;
  p.ws = align256(sizeof(double2) * (size_t)p.H * p.np) + align256(sizeof(double) * p.np) +
         align256(sizeof(int) * p.np) + 256 + align256(sizeof(int) * kMaxSweeps) + 256;
  return p;
}

hipError_t svd_truncate(const SvdPlan& p, const double2* theta, int Dmax, double cutoff,
                        int direction, double2* A_out, double2* B_out, int* k_dev,
                        double* disc_dev, double* norm_dev, double* sigma_dev, void* ws,
                        int* status, hipStream_t st) {
  if (p.m == p.n && p.on_theta != (direction == 1)) {  // square: keep the isometry exact
    SvdPlan q = p;
    q.on_theta = (direction == 1);
    return svd_truncate(q, theta, Dmax, cutoff, direction, A_out, B_out, k_dev, disc_dev, norm_dev,
                        sigma_dev, ws, status, st);
  }
  SvdWs w = carve(p, ws);
  int* k_shared = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(w.sweep_max) +
                                         align256(sizeof(int) * kMaxSweeps));
  const int kcap = std::min(Dmax, std::min(p.m, p.n));
  {
    const long long total = (long long)p.H * p.np;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(svd_init_kernel, dim3(blocks), dim3(256), 0, st, theta, p, w);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  const int wpb = 4;
  hipLaunchKernelGGL(svd_norms_kernel, dim3((p.nx + wpb - 1) / wpb), dim3(64 * wpb), 0, st, p, w,
                     status, 1);
  MPOEVO_HIP_TRY(hipGetLastError());
  {
    // Above the rounding floor of a length-mx inner product (|err| <= mx eps |x| |y|), so the
    // sweep stops once every pair is orthogonal to working precision.
    const double tol = 2.220446049250313e-16 * std::max(16.0, (double)p.mx);
    const int nblk = p.nb / 2;
    SvdPlan pp = p;
    SvdWs ww = w;
    double tt = tol, acc = kAcceptOrthogonality;
    int* stp = status;
    void* args[] = {&pp, &ww, &tt, &acc, &stp};
    MPOEVO_HIP_TRY(hipLaunchCooperativeKernel((const void*)svd_jacobi_kernel, dim3(nblk),
                                              dim3(kJacThreads), args, (unsigned)p.lds, st));
  }
  hipLaunchKernelGGL(svd_norms_kernel, dim3((p.nx + wpb - 1) / wpb), dim3(64 * wpb), 0, st, p, w,
                     status, 0);
  MPOEVO_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(svd_select_kernel, dim3(1), dim3(1024), 0, st, p, w, kcap, cutoff, k_dev,
                     disc_dev, norm_dev, sigma_dev, k_shared);
  MPOEVO_HIP_TRY(hipGetLastError());
  {
    const long long total = (long long)p.m * kcap + (long long)kcap * p.n;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(svd_output_kernel, dim3(blocks), dim3(256), 0, st, p, w, kcap, direction,
                       k_shared, A_out, B_out);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace mpoevo
