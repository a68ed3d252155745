// Contractions with the MPO tensor W over its short legs (K = w d terms per output). These are
// memory-bound: every thread keeps the K input values of one output column in registers and
// produces a group of kIlp of its w d outputs (one group per workgroup along the grid's z
// dimension), with W staged once per workgroup in LDS.
//
//   left : LB[a'][s'][beta][b]  = sum_{alpha, s} T[a'][alpha][s][b]  W[alpha][s'][s][beta]
//   right: RB[beta][b][t'][c']  = sum_{t, gamma} W[beta][t'][t][gamma] U[b][t][c'][gamma]
//
// T = E_left . ket (first product of the left environment update), U = ket . E_right^T.

#include "dev_common.h"
#include "wmix.h"

namespace mpoevo {
namespace {

template <typename T>
__device__ inline cx_t<T> cmul_add(cx_t<T> acc, cx_t<T> a, cx_t<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}

constexpr int kThreads = 256;
constexpr int kIlp = 8;  // outputs per thread computed together

// Output groups per workgroup: NG groups of kThreads threads take consecutive output groups of
// the same input columns, so that an input's second read comes from the compute unit's cache.
template <int KMAX>
constexpr int groups_per_wg() { return KMAX <= 16 ? 2 : 1; }

// grid: (ceil(Q / 256), P, ceil(d wr / (NG kIlp))), NG kThreads threads. KMAX >= wl * d.
template <typename T, int KMAX, int NG = groups_per_wg<KMAX>()>
__global__ __launch_bounds__(kThreads * NG) void wmix_left_kernel(
    const cx_t<T>* __restrict__ Tin, const cx_t<T>* __restrict__ W, cx_t<T>* __restrict__ out,
    int Q, int wl, int d, int wr) {
  using C2 = cx_t<T>;
  extern __shared__ unsigned char smem_raw[];
  C2* Ws = reinterpret_cast<C2*>(smem_raw);
  const int b = blockIdx.x * kThreads + threadIdx.x % kThreads;
  const int ap = blockIdx.y;
  const int K = wl * d;
  // the input loads are issued before W is staged, so that the two latencies overlap
  const C2* src = Tin + (long long)ap * K * Q + min(b, Q - 1);
  C2 in[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) in[k] = (k < K && b < Q) ? src[(long long)k * Q] : C2{T(0), T(0)};
  const int nW = wl * d * d * wr;
  for (int i = threadIdx.x; i < nW; i += kThreads * NG) Ws[i] = W[i];
  __syncthreads();
  if (b >= Q) return;
  C2* dst = out + (long long)ap * d * wr * Q + b;
  // outputs o = s' wr + beta: thread group h = z NG + threadIdx.x / kThreads computes the output
  // group [h kIlp, h kIlp + kIlp) with independent accumulators (more waves and independent
  // multiply-add chains to cover latency; the inputs are read once per group, mostly from cache)
  const int nout = d * wr;
  {
    const int o0 = (blockIdx.z * NG + threadIdx.x / kThreads) * kIlp;
    C2 acc[kIlp];
    int wo[kIlp];  // offset of (s', beta) in W[alpha][s'][s][beta]
#pragma unroll
    for (int j = 0; j < kIlp; ++j) {
      acc[j] = C2{T(0), T(0)};
      const int o = min(o0 + j, nout - 1), sp = o / wr, be = o % wr;
      wo[j] = sp * d * wr + be;
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < K) {
        const int al = k / d, s = k % d;  // k = alpha * d + s
        const int base = (al * d * d + s) * wr;
#pragma unroll
        for (int j = 0; j < kIlp; ++j) acc[j] = cmul_add<T>(acc[j], in[k], Ws[base + wo[j]]);
      }
    }
#pragma unroll
    for (int j = 0; j < kIlp; ++j)
      if (o0 + j < nout) dst[(long long)(o0 + j) * Q] = acc[j];
  }
}

// grid: (ceil(Pr / 256), Q, ceil(wl d / (NG kIlp))), NG kThreads threads. U[b][t][c'][gamma] with c' < Pr; out RB[beta][b][t'][c'].
template <typename T, int KMAX, int NG = groups_per_wg<KMAX>()>
__global__ __launch_bounds__(kThreads * NG) void wmix_right_kernel(
    const cx_t<T>* __restrict__ U, const cx_t<T>* __restrict__ W, cx_t<T>* __restrict__ out,
    int Q, int Pr, int wl, int d, int wr) {
  using C2 = cx_t<T>;
  extern __shared__ unsigned char smem_raw[];
  C2* Ws = reinterpret_cast<C2*>(smem_raw);
  const int cp = blockIdx.x * kThreads + threadIdx.x % kThreads;
  const int b = blockIdx.y;
  const int K = d * wr;
  C2 in[KMAX];  // loaded before W is staged (the two latencies overlap)
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    C2 v{T(0), T(0)};
    if (k < K && cp < Pr) {
      const int t = k / wr, ga = k % wr;  // k = t * wr + gamma
      v = U[(((long long)b * d + t) * Pr + cp) * wr + ga];
    }
    in[k] = v;
  }
  const int nW = wl * d * d * wr;
  for (int i = threadIdx.x; i < nW; i += kThreads * NG) Ws[i] = W[i];
  __syncthreads();
  if (cp >= Pr) return;
  // outputs o = beta d + t' (W row o: W[beta][t'][t][gamma], (t, gamma) = k): thread group
  // h = z NG + threadIdx.x / kThreads computes the output group [h kIlp, h kIlp + kIlp)
  const int nout = wl * d;
  {
    const int o0 = (blockIdx.z * NG + threadIdx.x / kThreads) * kIlp;
    C2 acc[kIlp];
#pragma unroll
    for (int j = 0; j < kIlp; ++j) acc[j] = C2{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < K) {
#pragma unroll
        for (int j = 0; j < kIlp; ++j) acc[j] = cmul_add<T>(acc[j], Ws[min(o0 + j, nout - 1) * K + k], in[k]);
      }
    }
#pragma unroll
    for (int j = 0; j < kIlp; ++j) {
      const int o = o0 + j;
      if (o < nout) out[(((long long)(o / d) * Q + b) * d + o % d) * Pr + cp] = acc[j];
    }
  }
}

template <typename T, int KMAX>
hipError_t launch_left(const void* Tin, const void* W, void* out, int P, int Q, int wl, int d,
                       int wr, hipStream_t st) {
  const size_t sh = sizeof(cx_t<T>) * (size_t)wl * d * d * wr;
  constexpr int NG = groups_per_wg<KMAX>();
  dim3 grid((Q + kThreads - 1) / kThreads, P, (d * wr + NG * kIlp - 1) / (NG * kIlp));
  hipLaunchKernelGGL((wmix_left_kernel<T, KMAX>), grid, dim3(kThreads * NG), sh, st,
                     (const cx_t<T>*)Tin, (const cx_t<T>*)W, (cx_t<T>*)out, Q, wl, d, wr);
  last_launch() = LaunchRecord{reinterpret_cast<const void*>(wmix_left_kernel<T, KMAX>), false};
  return hipGetLastError();
}

template <typename T, int KMAX>
hipError_t launch_right(const void* U, const void* W, void* out, int Q, int Pr, int wl, int d,
                        int wr, hipStream_t st) {
  const size_t sh = sizeof(cx_t<T>) * (size_t)wl * d * d * wr;
  constexpr int NG = groups_per_wg<KMAX>();
  dim3 grid((Pr + kThreads - 1) / kThreads, Q, (wl * d + NG * kIlp - 1) / (NG * kIlp));
  hipLaunchKernelGGL((wmix_right_kernel<T, KMAX>), grid, dim3(kThreads * NG), sh, st,
                     (const cx_t<T>*)U, (const cx_t<T>*)W, (cx_t<T>*)out, Q, Pr, wl, d, wr);
  last_launch() = LaunchRecord{reinterpret_cast<const void*>(wmix_right_kernel<T, KMAX>), false};
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_left(const void* Tin, const void* W, void* out, int P, int Q, int wl, int d,
                         int wr, hipStream_t st) {
  const int K = wl * d;
  if (K <= 4) return launch_left<T, 4>(Tin, W, out, P, Q, wl, d, wr, st);
  if (K <= 8) return launch_left<T, 8>(Tin, W, out, P, Q, wl, d, wr, st);
  if (K <= 16) return launch_left<T, 16>(Tin, W, out, P, Q, wl, d, wr, st);
  if (K <= 32) return launch_left<T, 32>(Tin, W, out, P, Q, wl, d, wr, st);
  return launch_left<T, 64>(Tin, W, out, P, Q, wl, d, wr, st);
}

template <typename T>
hipError_t dispatch_right(const void* U, const void* W, void* out, int Q, int Pr, int wl, int d,
                          int wr, hipStream_t st) {
  const int K = wr * d;
  if (K <= 4) return launch_right<T, 4>(U, W, out, Q, Pr, wl, d, wr, st);
  if (K <= 8) return launch_right<T, 8>(U, W, out, Q, Pr, wl, d, wr, st);
  if (K <= 16) return launch_right<T, 16>(U, W, out, Q, Pr, wl, d, wr, st);
  if (K <= 32) return launch_right<T, 32>(U, W, out, Q, Pr, wl, d, wr, st);
  return launch_right<T, 64>(U, W, out, Q, Pr, wl, d, wr, st);
}

}  // namespace

bool wmix_supported(int wl, int d, int wr) {
  return wl * d <= kWmixMaxK && wr * d <= kWmixMaxK &&
         (size_t)wl * d * d * wr * sizeof(double2) <= 64 * 1024;
}

hipError_t wmix_left(bool fp64, const void* Tin, const void* W, void* out, int P, int Q, int wl,
                     int d, int wr, hipStream_t st) {
  if (fp64) return dispatch_left<double>(Tin, W, out, P, Q, wl, d, wr, st);
  return dispatch_left<float>(Tin, W, out, P, Q, wl, d, wr, st);
}

hipError_t wmix_right(bool fp64, const void* U, const void* W, void* out, int Q, int Pr, int wl,
                      int d, int wr, hipStream_t st) {
  if (fp64) return dispatch_right<double>(U, W, out, Q, Pr, wl, d, wr, st);
  return dispatch_right<float>(U, W, out, Q, Pr, wl, d, wr, st);
}

}  // namespace mpoevo
