// Device layer of the C ABI: environment updates, the projected two-site tensor, the FP64
// truncation and one full time step of the variational fit (Sec. 2.2; Sec. 8.2).
//
// Data flow of a time step (i = site index, bond i is the left bond of site i):
//   psi  (ket, caller's buffers, bonds Q_i)  and  phi (bra, the new state, bonds P_i).
//   T_i  = Lenv_i . M_i                    (matrix product, K = Q_i)
//   LB_i = T_i . W_i   [a'][s'][beta][b]   (short-leg contraction with the MPO)
//   U_i  = M_i . Renv_{i+1}^T              (matrix product, K = Q_{i+1})
//   RB_i = W_i . U_i   [beta][b][t'][c']
//   Theta(i,i+1) = LB_i . RB_{i+1}         (matrix product, K = w Q_{i+1})
//   Lenv_{i+1} = phi_i^dag . LB_i,  Renv_i = conj(phi_i) . RB_i^T
// LB_i depends only on the sites left of i and RB_{i+1} only on the sites right of i+1, so the
// left-to-right pass computes LB_i once per visit and reuses the RB_{i+1} of the previous
// right-to-left pass (and vice versa): every visit costs one left (or right) block, one
// environment product and the Theta product. All LB_i / RB_i of the chain stay resident in HBM.
//
// Bond dimensions of phi are static upper bounds min(Dmax, m, n) during a step (the kept rank
// is decided on the device, discarded directions are exact zeros), so no visit waits for the
// host; the host reads the kept ranks once at the end of the step and compacts the result.

#include <cxxabi.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "dev_common.h"
#include "internal.h"
#include "svd.h"
#include "wmix.h"

namespace mpoevo {

LaunchRecord& last_launch() {
  static thread_local LaunchRecord r;
  return r;
}

// A step's device work captured into a HIP graph, with the plan it was captured for and the host
// state the work leaves behind (restored whenever the graph replays it).
struct GraphEntry {
  std::vector<long long> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> P, bond_of_visit, k_slot_of_bond, warm_dim;
  std::vector<char> visit_kind, frozen;
  int last_visit_k_slot = 0, updates = 0;
  double gflop = 0.0;
  bool one_site = false, mixed = false;
};
constexpr size_t kMaxGraphs = 8;

struct DeviceState {
  int* status = nullptr;  // sticky status words (device ints)
  int lds_max = 0;
  std::vector<hipEvent_t> events;  // reused by profiled steps
  std::vector<GraphEntry> graphs;  // captured steps, oldest first
  std::vector<std::vector<long long>> seen;  // plans run once, uncaptured
  hipStream_t capture_stream = nullptr;
  int cus = 0;  // compute units
  // U(1) truncations: the charge blocks' SVDs fork from the step's stream to worker streams
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  std::vector<hipStream_t> block_streams;
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
size_t csize(int prec) { return prec == MPOEVO_FP64 ? sizeof(double2) : sizeof(float2); }

int hip_fail(Context& ctx, hipError_t e, const char* what) {
  ctx.err = std::string(what) + ": " + hipGetErrorString(e);
  return MPOEVO_EHIP;
}

// Optional per-kernel-class timing of a step with HIP events on its stream.
struct Prof {
  enum Kind { kJacobi = 0, kGemm = 1, kWmix = 2, kQr = 3 };
  DeviceState* ds = nullptr;
  hipStream_t st = nullptr;
  bool all = true;  // time the products and W contractions too (else the Jacobi kernel only)
  struct Rec { int kind; size_t e0; double work; LaunchRecord launch; };
  std::vector<Rec> recs;
  size_t next = 0;
  hipError_t event(size_t i, hipEvent_t* out) {
    while (ds->events.size() <= i) {
      hipEvent_t e;
      MPOEVO_HIP_TRY(hipEventCreate(&e));
      ds->events.push_back(e);
    }
    *out = ds->events[i];
    return hipSuccess;
  }
  // two fresh events; the caller records them around its launch
  hipError_t pair(hipEvent_t* a, hipEvent_t* b, size_t* first) {
    *first = next;
    MPOEVO_HIP_TRY(event(next++, a));
    return event(next++, b);
  }
  hipError_t begin(size_t* first) {
    hipEvent_t a, b;
    MPOEVO_HIP_TRY(pair(&a, &b, first));
    return hipEventRecord(a, st);
  }
  hipError_t end(int kind, size_t first, double work) {
    MPOEVO_HIP_TRY(hipEventRecord(ds->events[first + 1], st));
    recs.push_back({kind, first, work, last_launch()});
    return hipSuccess;
  }
};

#define PROF_BEGIN(pr, tok) size_t tok = 0; if (pr && (pr)->all) MPOEVO_HIP_TRY((pr)->begin(&tok))
#define PROF_END(pr, tok, kind, work) if (pr && (pr)->all) MPOEVO_HIP_TRY((pr)->end(kind, tok, work))

// ----------------------------------------------------------------------------- small kernels
__global__ void cast_c128_c64(const double2* __restrict__ in, float2* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = float2{(float)in[i].x, (float)in[i].y};
}

template <typename C2>
__global__ void boundary_env(C2* E, int w) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i < w) E[i] = C2{i == 0 ? 1 : 0, 0};
}

// Wt[(s' wr + beta)][(alpha d + s)] = W[alpha][s'][s][beta]: W as the left factor of the
// short-leg contraction done as a product (large MPO bonds).
template <typename C2>
__global__ void permute_w_left(const C2* __restrict__ W, C2* __restrict__ Wt, int wl, int d, int wr) {
  const long long n = (long long)wl * d * d * wr;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int beta = (int)(i % wr);
    long long r = i / wr;
    const int s = (int)(r % d);
    r /= d;
    const int sp = (int)(r % d);
    const int alpha = (int)(r / d);
    Wt[((long long)sp * wr + beta) * (wl * d) + alpha * d + s] = W[i];
  }
}

// The statistics slots of a visit that takes the one-site update: bond k kept, nothing discarded,
// no Jacobi sweeps, a complete basis.
__global__ void one_site_visit_slots(int* kbuf, double* dbuf, double* nbuf, int* sweeps, int* cplt, int* blocks,
                                     int k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *kbuf = k;
    *dbuf = 0.0;
    *nbuf = 0.0;
    *sweeps = 0;
    *cplt = 1;
    *blocks = 0;
  }
}

// E (1 x w x 1) = e_level.
__global__ void boundary_level(double2* E, int w, int level) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i < w) E[i] = double2{i == level ? 1.0 : 0.0, 0.0};
}

__global__ void copy_entry(const double2* __restrict__ src, double2* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

// out (n x n) = identity.
__global__ void fill_identity(double2* out, int n) {
  const long long total = (long long)n * n;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x)
    out[idx] = double2{(idx / n == idx % n) ? 1.0 : 0.0, 0.0};
}

__global__ void scale_by_inverse_norm(double2* x, long long n, const double* norm) {
  const double s = *norm;
  const double f = (s > 0.0 && isfinite(s)) ? 1.0 / s : 1.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = double2{x[i].x * f, x[i].y * f};
}

// dst[a][s][b] (Pa x d x Pb) <- src[a][s][b] with src row pitch (d, Pbs), a < Pa, b < Pb.
__global__ void compact_site(const double2* __restrict__ src, double2* __restrict__ dst, int Pa,
                             int d, int Pb, int Pbs) {
  const long long n = (long long)Pa * d * Pb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(i % Pb);
    const long long as = i / Pb;
    dst[i] = src[as * Pbs + b];
  }
}

// E[c][r] = A[r][c] for an m x k matrix A (the zip-up's carry (U S)^T).
__global__ void transpose_c128(const double2* __restrict__ A, double2* __restrict__ E, int m, int k) {
  const long long n = (long long)m * k;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i % m);
    const long long c = i / m;
    E[i] = A[(long long)r * k + c];
  }
}

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096)); }

hipError_t cast_to_c64(const void* in, void* out, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cast_c128_c64, dim3(grid_for(n)), dim3(256), 0, st, (const double2*)in, (float2*)out, n);
  return hipGetLastError();
}

hipError_t set_boundary(void* E, int w, bool fp64, hipStream_t st) {
  if (fp64) hipLaunchKernelGGL(boundary_env<double2>, dim3((w + 255) / 256), dim3(256), 0, st, (double2*)E, w);
  else hipLaunchKernelGGL(boundary_env<float2>, dim3((w + 255) / 256), dim3(256), 0, st, (float2*)E, w);
  return hipGetLastError();
}

// ------------------------------------------------------------------ contraction building blocks
// LB[a'][s'][beta][b] = sum E[a'][alpha][a] ket[a][s][b] W[alpha][s'][s][beta]
// E: (P, wl, Qa), ket: (Qa, d, Qb), W: (wl, d, d, wr). tmp holds P*wl*d*Qb complex.
double gemm_flop(const GemmDesc& g) { return 8.0 * g.M * g.N * (double)g.K * g.batch; }

// Arithmetic of the contraction products: FP64, FP32, or FP32 operands multiplied as split-BF16x3.
struct Arith {
  bool fp64;
  bool bf16x3;
};
Arith arith_of(int prec) { return Arith{prec == MPOEVO_FP64, prec == MPOEVO_BF16X3}; }

hipError_t gemm_timed(const GemmDesc& g, Arith ar, bool out_fp64, hipStream_t st, Prof* pr) {
  GemmDesc h = g;
  h.bf16x3 = ar.bf16x3 && !ar.fp64;
  // rows that would leave the tile's last row block mostly empty (an MPO bond of 271 on 128-row
  // tiles) go to a second product on a tile of 32 or 64 rows
  const int tail = gemm_row_tail(h, ar.fp64);
  GemmDesc t = h;
  if (tail > 0) {
    h.M -= tail;
    t.M = tail;
    t.row_tail = true;
    t.A = static_cast<const unsigned char*>(g.A) + sizeof(float2) * (size_t)h.M * g.sAm;
    t.C = static_cast<unsigned char*>(g.C) + (out_fp64 ? sizeof(double2) : sizeof(float2)) * (size_t)h.M * g.sCm;
  }
  // tiles that would run as a last, mostly empty round of workgroups go to a launch of their own
  // (which then takes a smaller tile or splits K)
  int cut = 0;
  long long at = 0;
  if (tail == 0) gemm_round_tail(h, ar.fp64, cut, at);
  if (cut != 0) {
    const size_t ci = sizeof(float2), co = out_fp64 ? sizeof(double2) : sizeof(float2);
    GemmDesc u = h;
    if (cut == 1) {
      h.M = (int)at;
      u.M -= (int)at;
      u.A = static_cast<const unsigned char*>(g.A) + ci * (size_t)(at * g.sAm);
      u.C = static_cast<unsigned char*>(g.C) + co * (size_t)(at * g.sCm);
    } else if (cut == 2) {
      h.N = (int)at;
      u.N -= (int)at;
      u.B = static_cast<const unsigned char*>(g.B) + ci * (size_t)(at * g.sBn);
      u.C = static_cast<unsigned char*>(g.C) + co * (size_t)(at * g.sCn);
    } else {
      h.batch = (int)at;
      u.batch -= (int)at;
      u.A = static_cast<const unsigned char*>(g.A) + ci * (size_t)(at * g.bA);
      u.B = static_cast<const unsigned char*>(g.B) + ci * (size_t)(at * g.bB);
      u.C = static_cast<unsigned char*>(g.C) + co * (size_t)(at * g.bC);
    }
    PROF_BEGIN(pr, tok);
    MPOEVO_HIP_TRY(gemm_launch(h, ar.fp64, out_fp64, st));
    PROF_END(pr, tok, Prof::kGemm, gemm_flop(h));
    PROF_BEGIN(pr, tok3);
    MPOEVO_HIP_TRY(gemm_launch(u, ar.fp64, out_fp64, st));
    PROF_END(pr, tok3, Prof::kGemm, gemm_flop(u));
    return hipSuccess;
  }
  PROF_BEGIN(pr, tok);
  MPOEVO_HIP_TRY(gemm_launch(h, ar.fp64, out_fp64, st));
  PROF_END(pr, tok, Prof::kGemm, gemm_flop(h));
  if (tail > 0) {
    PROF_BEGIN(pr, tok2);
    MPOEVO_HIP_TRY(gemm_launch(t, ar.fp64, out_fp64, st));
    PROF_END(pr, tok2, Prof::kGemm, gemm_flop(t));
  }
  return hipSuccess;
}

hipError_t left_block(Arith ar, const void* E, const void* ket, const void* W, void* tmp,
                      void* LB, int P, int wl, int Qa, int d, int Qb, int wr, hipStream_t st,
                      Prof* pr = nullptr, void* gws = nullptr, void* xws = nullptr,
                      size_t gws_bytes = kGemmScratchBytes) {
  const bool fp64 = ar.fp64;
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? gws_bytes : 0;
  g.A = E; g.B = ket; g.C = tmp;
  g.M = P * wl; g.N = d * Qb; g.K = Qa; g.batch = 1;
  g.sAm = Qa; g.sAk = 1; g.sBk = (long long)d * Qb; g.sBn = 1; g.sCm = (long long)d * Qb; g.sCn = 1;
  MPOEVO_HIP_TRY(gemm_timed(g, ar, false, st, pr));
  if (wmix_supported(wl, d, wr)) {
    PROF_BEGIN(pr, tok);
    MPOEVO_HIP_TRY(wmix_left(fp64, tmp, W, LB, P, Qb, wl, d, wr, st));
    const double cs = fp64 ? 16.0 : 8.0;
    PROF_END(pr, tok, Prof::kWmix, cs * ((double)P * wl * d * Qb + (double)P * d * wr * Qb + wl * d * d * wr));
    return hipSuccess;
  }
  // large MPO bond: LB_a'[(s', beta)][b] = sum Wt[(s', beta)][(alpha, s)] T_a'[(alpha, s)][b]
  if (!xws) return hipErrorInvalidValue;
  const long long nW = (long long)wl * d * d * wr;
  if (fp64) hipLaunchKernelGGL(permute_w_left<double2>, dim3(grid_for(nW)), dim3(256), 0, st,
                               (const double2*)W, (double2*)xws, wl, d, wr);
  else hipLaunchKernelGGL(permute_w_left<float2>, dim3(grid_for(nW)), dim3(256), 0, st,
                          (const float2*)W, (float2*)xws, wl, d, wr);
  MPOEVO_HIP_TRY(hipGetLastError());
  GemmDesc h{};
  h.ws = gws;
  h.ws_bytes = gws ? gws_bytes : 0;
  h.A = xws; h.B = tmp; h.C = LB;
  h.M = d * wr; h.N = Qb; h.K = wl * d; h.batch = P;
  h.sAm = (long long)wl * d; h.sAk = 1; h.bA = 0;
  h.sBk = Qb; h.sBn = 1; h.bB = (long long)wl * d * Qb;
  h.sCm = Qb; h.sCn = 1; h.bC = (long long)d * wr * Qb;
  return gemm_timed(h, ar, false, st, pr);
}

// RB[beta][b][t'][c'] = sum W[beta][t'][t][gamma] ket[b][t][c] E[c'][gamma][c]
// ket: (Qa, d, Qb), E: (Pr, wr, Qb), W: (wl, d, d, wr). tmp holds Qa*d*Pr*wr complex.
hipError_t right_block(Arith ar, const void* ket, const void* E, const void* W, void* tmp,
                       void* RB, int Qa, int d, int Qb, int Pr, int wl, int wr, hipStream_t st,
                       Prof* pr = nullptr, void* gws = nullptr, void* /*xws*/ = nullptr,
                       size_t gws_bytes = kGemmScratchBytes) {
  const bool fp64 = ar.fp64;
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? gws_bytes : 0;
  g.A = ket; g.B = E; g.C = tmp;
  g.M = Qa * d; g.K = Qb;
  g.sAm = Qb; g.sAk = 1; g.sBk = 1; g.sCn = 1;
  if (wmix_supported(wl, d, wr)) {
    // U[b][t][c'][gamma] = sum_c ket[b][t][c] E[c'][gamma][c]: one product over the rows (c', gamma)
    g.N = Pr * wr; g.batch = 1;
    g.sBn = Qb; g.sCm = (long long)Pr * wr;
    MPOEVO_HIP_TRY(gemm_timed(g, ar, false, st, pr));
    PROF_BEGIN(pr, tok);
    MPOEVO_HIP_TRY(wmix_right(fp64, tmp, W, RB, Qa, Pr, wl, d, wr, st));
    const double cs = fp64 ? 16.0 : 8.0;
    PROF_END(pr, tok, Prof::kWmix, cs * ((double)Qa * d * Pr * wr + (double)wl * Qa * d * Pr + wl * d * d * wr));
    return hipSuccess;
  }
  // large MPO bond: the same contraction batched over gamma, written as Up[b][t][gamma][c'] (batch
  // gamma reads rows c' of E at stride wr Qb from offset gamma Qb), so that for each t'
  // RB[beta][b][t'][c'] = sum_{(t, gamma)} W[beta][t'][t][gamma] Up_b[(t, gamma)][c'] reads its
  // operand at one stride per index
  g.N = Pr; g.batch = wr;
  g.sBn = (long long)wr * Qb; g.bA = 0; g.bB = Qb;
  g.sCm = (long long)wr * Pr; g.bC = Pr;
  MPOEVO_HIP_TRY(gemm_timed(g, ar, false, st, pr));
  const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
  for (int tp = 0; tp < d; ++tp) {
    GemmDesc h{};
    h.ws = gws;
    h.ws_bytes = gws ? gws_bytes : 0;
    h.A = static_cast<const unsigned char*>(W) + cs * (size_t)tp * d * wr;
    h.B = tmp;
    h.C = static_cast<unsigned char*>(RB) + cs * (size_t)tp * Pr;
    h.M = wl; h.N = Pr; h.K = d * wr; h.batch = Qa;
    h.sAm = (long long)d * d * wr; h.sAk = 1; h.bA = 0;
    h.sBk = Pr; h.sBn = 1; h.bB = (long long)d * wr * Pr;
    h.sCm = (long long)Qa * d * Pr; h.sCn = 1; h.bC = (long long)d * Pr;
    MPOEVO_HIP_TRY(gemm_timed(h, ar, false, st, pr));
  }
  return hipSuccess;
}

// Lnew[b'][beta][b] = sum conj(bra[a'][s'][b']) LB[a'][s'][beta][b]; bra: (Pa, d, Pb).
hipError_t left_env_from_block(Arith ar, const void* bra, const void* LB, void* Lnew, int Pa,
                               int d, int Pb, int wr, int Qb, hipStream_t st,
                         Prof* pr = nullptr, void* gws = nullptr,
                         size_t gws_bytes = kGemmScratchBytes) {
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? gws_bytes : 0;
  g.A = bra; g.B = LB; g.C = Lnew;
  g.M = Pb; g.N = wr * Qb; g.K = Pa * d; g.batch = 1;
  g.sAm = 1; g.sAk = Pb; g.conjA = true;
  g.sBk = (long long)wr * Qb; g.sBn = 1; g.sCm = (long long)wr * Qb; g.sCn = 1;
  return gemm_timed(g, ar, false, st, pr);
}

// Rnew[a'][alpha][a] = sum conj(bra[a'][t'][c']) RB[alpha][a][t'][c']; bra: (Pa, d, Pb).
hipError_t right_env_from_block(Arith ar, const void* bra, const void* RB, void* Rnew, int Pa,
                                int d, int Pb, int wl, int Qa, hipStream_t st,
                         Prof* pr = nullptr, void* gws = nullptr,
                         size_t gws_bytes = kGemmScratchBytes) {
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? gws_bytes : 0;
  g.A = bra; g.B = RB; g.C = Rnew;
  g.M = Pa; g.N = wl * Qa; g.K = d * Pb; g.batch = 1;
  g.sAm = (long long)d * Pb; g.sAk = 1; g.conjA = true;
  g.sBk = 1; g.sBn = (long long)d * Pb; g.sCm = (long long)wl * Qa; g.sCn = 1;
  return gemm_timed(g, ar, false, st, pr);
}

// Theta[(a',s')][(t',c')] = sum LB[(a',s')][(beta,b)] RB[(beta,b)][(t',c')], complex128 out.
hipError_t theta_product(Arith ar, const void* LB, const void* RB, void* theta, int Pa, int d,
                         int wm, int Qm, int Pc, hipStream_t st,
                         Prof* pr = nullptr, void* gws = nullptr) {
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? kGemmScratchBytes : 0;
  g.A = LB; g.B = RB; g.C = theta;
  g.M = Pa * d; g.N = d * Pc; g.K = wm * Qm; g.batch = 1;
  g.sAm = (long long)wm * Qm; g.sAk = 1; g.sBk = (long long)d * Pc; g.sBn = 1;
  g.sCm = (long long)d * Pc; g.sCn = 1;
  return gemm_timed(g, ar, true, st, pr);
}

// One row of the per-kernel statistics of a profiled step: the kernel's name as the runtime
// reports it (demangled) and its summed launches, time and work.
void fill_kernel_stat(mpoevo_kernel_stat& o, const void* kernel, int kind, bool split, int n, double ms,
                      double work, hipStream_t st) {
  std::memset(&o, 0, sizeof(o));
  const char* raw = kernel ? hipKernelNameRefByPtr(kernel, st) : nullptr;
  std::string name = raw ? raw : "unknown kernel";
  int dst = 0;
  char* dem = raw ? abi::__cxa_demangle(raw, nullptr, nullptr, &dst) : nullptr;
  if (dem && dst == 0) name = dem;
  std::free(dem);
  std::strncpy(o.name, name.c_str(), sizeof(o.name) - 1);
  o.kind = kind;
  o.split_k = split ? 1 : 0;
  o.launches = n;
  o.ms = ms;
  o.work = work;
}

// dst = src / ||src|| and *norm_out = ||src|| (one workgroup, fixed summation order).
__global__ __launch_bounds__(256) void norm_scale_kernel(const double2* __restrict__ src,
                                                         double2* __restrict__ dst, long long n,
                                                         double* __restrict__ norm_out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) acc = fma(src[i].x, src[i].x, fma(src[i].y, src[i].y, acc));
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  const double nr = sqrt(part[0]);
  if (threadIdx.x == 0) *norm_out = nr;
  const double f = (nr > 0.0 && isfinite(nr)) ? 1.0 / nr : 1.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) dst[i] = double2{src[i].x * f, src[i].y * f};
}

// One-site projected tensor from the left block (left-to-right pass):
// M[(a',s')][b'] = sum_{(beta,b)} LB[(a',s')][(beta,b)] R[b'][(beta,b)], complex128 out.
hipError_t local_left(Arith ar, const void* LB, const void* R, double2* M, int Pa, int d, int wr,
                      int Qb, int Pb, hipStream_t st, Prof* pr, void* gws) {
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? kGemmScratchBytes : 0;
  g.A = LB; g.B = R; g.C = M;
  g.M = Pa * d; g.N = Pb; g.K = wr * Qb; g.batch = 1;
  g.sAm = (long long)wr * Qb; g.sAk = 1; g.sBk = 1; g.sBn = (long long)wr * Qb;
  g.sCm = Pb; g.sCn = 1;
  return gemm_timed(g, ar, true, st, pr);
}

// One-site projected tensor from the right block (right-to-left pass):
// M[a'][(s',b')] = sum_{(alpha,a)} L[a'][(alpha,a)] RB[(alpha,a)][(s',b')], complex128 out.
hipError_t local_right(Arith ar, const void* L, const void* RB, double2* M, int Pa, int wl, int Qa,
                       int d, int Pb, hipStream_t st, Prof* pr, void* gws) {
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? kGemmScratchBytes : 0;
  g.A = L; g.B = RB; g.C = M;
  g.M = Pa; g.N = d * Pb; g.K = wl * Qa; g.batch = 1;
  g.sAm = (long long)wl * Qa; g.sAk = 1; g.sBk = (long long)d * Pb; g.sBn = 1;
  g.sCm = (long long)d * Pb; g.sCn = 1;
  return gemm_timed(g, ar, true, st, pr);
}

// Algorithmic flops of a Householder QR of an m x n complex matrix (m >= n) with the thin Q formed.
double qr_flop(int m, int n) {
  const double mm = m, nn = n;
  return 2.0 * (8.0 * mm * nn * nn - 8.0 / 3.0 * nn * nn * nn);
}

// ------------------------------------------------------------- U(1): truncation per charge block
// out (mq x nq, row-major) = X[rows[i]][cols[j]] (X row pitch n).
__global__ void gather_block(const double2* __restrict__ X, int n, const int* __restrict__ rows, int mq,
                             const int* __restrict__ cols, int nq, double2* __restrict__ out) {
  const long long total = (long long)mq * nq;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / nq), j = (int)(idx % nq);
    out[idx] = X[(long long)rows[i] * n + cols[j]];
  }
}

// A[rows[i]][off + j] = AQ[i][j], i < mq, j < kq (AQ row pitch pa, A row pitch lda).
__global__ void scatter_block_cols(const double2* __restrict__ AQ, int pa, int mq, int kq,
                                   const int* __restrict__ rows, double2* __restrict__ A, int lda, int off) {
  const long long total = (long long)mq * kq;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / kq), j = (int)(idx % kq);
    A[(long long)rows[i] * lda + off + j] = AQ[(long long)i * pa + j];
  }
}

// B[off + j][cols[c]] = BQ[j][c], j < kq, c < nq (BQ row pitch nq, B row pitch ldb).
__global__ void scatter_block_rows(const double2* __restrict__ BQ, int nq, int kq,
                                   const int* __restrict__ cols, double2* __restrict__ B, int ldb, int off) {
  const long long total = (long long)kq * nq;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nq), c = (int)(idx % nq);
    B[(long long)(off + j) * ldb + cols[c]] = BQ[idx];
  }
}

__global__ void fill_zero_c128(double2* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = double2{0.0, 0.0};
}

// Scratch of a blocked truncation of an m x n matrix with m, n <= dim.
size_t blocked_scratch_bytes(int dim) {
  const size_t mn = (size_t)dim * dim;
  return 3 * a256(sizeof(double2) * mn) + a256(sizeof(int) * 2 * (size_t)dim) + a256(sizeof(double) * dim) +
         a256((sizeof(int) + 2 * sizeof(double)) * (size_t)dim);
}

struct BlockedResult {
  int k = 0;
  double disc = 0.0, norm = 0.0;
  std::vector<int> charges;  // of the kept indices, nondecreasing
};

// X (m x n, row-major, complex128) vanishes unless rq[r] == cq[c]: block diagonal by charge. Each
// charge block gets its own FP64 SVD (the truncation kernels, keeping everything above the
// rounding floor); the Dmax largest singular values over all blocks are kept (k = min(Dmax,
// #{sigma > cutoff sigma_max}) >= 1, ties to the lower charge, then the earlier value), and the
// factors are written densely with the kept indices in charge order: direction LEFT A = U
// (m x k), B = S V^dag (k x n); RIGHT A = U S, B = V^dag. One stream synchronisation (the host
// selects the kept values). The blocks' SVDs run side by side on up to four worker streams
// (forked from st and joined back) when their workspaces (without split-K scratch) fit next to
// each other in svdws (svd_bytes) and their grids fit on three quarters of the compute units
// together (ordinary launches: the device must hold every running grid at once) and the step has
// the device to itself; otherwise one after the other on st.
hipError_t blocked_truncate(Context& ctx, const double2* X, int m, int n, const std::vector<int>& rq,
                            const std::vector<int>& cq, int Dmax, double cutoff, int direction,
                            double2* A, double2* B, unsigned char* scratch, int dim, void* svdws,
                            size_t svd_bytes, hipStream_t st, BlockedResult& res) {
  std::map<int, std::vector<int>> rows, cols;
  for (int r = 0; r < m; ++r) rows[rq[r]].push_back(r);
  for (int c = 0; c < n; ++c) cols[cq[c]].push_back(c);
  struct Blk { int q, mq, nq, kcap; size_t xo, ao, bo, so, io; int kq = 0, off = 0; };
  std::vector<Blk> blks;
  std::vector<int> idx;
  size_t xo = 0, ao = 0, bo = 0, so = 0;
  for (const auto& kv : rows) {
    auto it = cols.find(kv.first);
    if (it == cols.end()) continue;
    Blk b{kv.first, (int)kv.second.size(), (int)it->second.size(), 0, xo, ao, bo, so, idx.size()};
    b.kcap = std::min(b.mq, b.nq);
    idx.insert(idx.end(), kv.second.begin(), kv.second.end());
    idx.insert(idx.end(), it->second.begin(), it->second.end());
    xo += (size_t)b.mq * b.nq;
    ao += (size_t)b.mq * b.kcap;
    bo += (size_t)b.kcap * b.nq;
    so += b.kcap;
    blks.push_back(b);
  }
  if (blks.empty()) return hipErrorInvalidValue;
  const size_t mn = (size_t)dim * dim;
  double2* xq = reinterpret_cast<double2*>(scratch);
  double2* aq = reinterpret_cast<double2*>(scratch + a256(sizeof(double2) * mn));
  double2* bq = reinterpret_cast<double2*>(scratch + 2 * a256(sizeof(double2) * mn));
  unsigned char* rest = scratch + 3 * a256(sizeof(double2) * mn);
  int* idx_dev = reinterpret_cast<int*>(rest);
  double* sig = reinterpret_cast<double*>(rest + a256(sizeof(int) * 2 * (size_t)dim));
  unsigned char* tail = rest + a256(sizeof(int) * 2 * (size_t)dim) + a256(sizeof(double) * dim);
  int* kd = reinterpret_cast<int*>(tail);
  double* dd = reinterpret_cast<double*>(tail + a256(sizeof(int) * (size_t)dim));
  double* nd = dd + dim;
  MPOEVO_HIP_TRY(hipMemcpyAsync(idx_dev, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, st));
  std::vector<SvdPlan> plans;
  size_t wsmax = 0;
  int gmax = 1;
  for (const Blk& b : blks) {
    plans.push_back(svd_plan_unsplit(svd_qr_ok(b.mq, b.nq, direction) ? svd_plan_qr(b.mq, b.nq, direction)
                                                                      : svd_plan(b.mq, b.nq, direction)));
    wsmax = std::max(wsmax, a256(plans.back().ws));
    gmax = std::max(gmax, svd_grid(plans.back()));
  }
  DeviceState& ds = *ctx.dev;
  const int nstreams = (int)std::min<size_t>({size_t(4), blks.size(), svd_bytes / std::max<size_t>(wsmax, 1),
                                              size_t(std::max(1, (3 * ds.cus / 4) / gmax))});
  // (only where this step has the device to itself: not for the chains of step_batched, whose
  // streams already share it)
  const bool par = nstreams > 1 && ctx.coop_jacobi;
  if (par) {
    while ((int)ds.block_streams.size() < nstreams) {
      hipStream_t bs = nullptr;
      MPOEVO_HIP_TRY(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
      ds.block_streams.push_back(bs);
      hipEvent_t ev = nullptr;
      MPOEVO_HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      ds.joins.push_back(ev);
    }
    if (!ds.fork) MPOEVO_HIP_TRY(hipEventCreateWithFlags(&ds.fork, hipEventDisableTiming));
    MPOEVO_HIP_TRY(hipEventRecord(ds.fork, st));
    for (int s_ = 0; s_ < nstreams; ++s_) MPOEVO_HIP_TRY(hipStreamWaitEvent(ds.block_streams[s_], ds.fork, 0));
  }
  for (size_t t = 0; t < blks.size(); ++t) {
    const Blk& b = blks[t];
    const int lane = (int)(t % (size_t)nstreams);
    hipStream_t bst = par ? ds.block_streams[lane] : st;
    void* bws = par ? static_cast<unsigned char*>(svdws) + wsmax * lane : svdws;
    const int* r_dev = idx_dev + b.io;
    const int* c_dev = r_dev + b.mq;
    hipLaunchKernelGGL(gather_block, dim3(grid_for((long long)b.mq * b.nq)), dim3(256), 0, bst, X, n, r_dev, b.mq,
                       c_dev, b.nq, xq + b.xo);
    MPOEVO_HIP_TRY(hipGetLastError());
    MPOEVO_HIP_TRY(svd_truncate(plans[t], xq + b.xo, b.kcap, 0.0, aq + b.ao, bq + b.bo, kd + t, dd + t, nd + t,
                                sig + b.so, bws, ctx.dev->status, bst, nullptr, nullptr, nullptr, nullptr,
                                nullptr, par ? false : ctx.coop_jacobi));
  }
  if (par) {
    for (int s_ = 0; s_ < nstreams; ++s_) {
      MPOEVO_HIP_TRY(hipEventRecord(ds.joins[s_], ds.block_streams[s_]));
      MPOEVO_HIP_TRY(hipStreamWaitEvent(st, ds.joins[s_], 0));
    }
  }
  std::vector<double> sh(so);
  MPOEVO_HIP_TRY(hipMemcpyAsync(sh.data(), sig, sizeof(double) * so, hipMemcpyDeviceToHost, st));
  MPOEVO_HIP_TRY(hipStreamSynchronize(st));
  struct Cand { double s; int t, j; };
  std::vector<Cand> cand;
  double tot = 0.0;
  for (size_t t = 0; t < blks.size(); ++t)
    for (int j = 0; j < blks[t].kcap; ++j) {
      cand.push_back({sh[blks[t].so + j], (int)t, j});
      tot += sh[blks[t].so + j] * sh[blks[t].so + j];
    }
  std::stable_sort(cand.begin(), cand.end(), [&](const Cand& a, const Cand& b) {
    if (a.s != b.s) return a.s > b.s;
    if (blks[a.t].q != blks[b.t].q) return blks[a.t].q < blks[b.t].q;
    return a.j < b.j;
  });
  const double smax = cand.empty() ? 0.0 : cand[0].s;
  int above = 0;
  for (const Cand& c : cand) above += c.s > cutoff * smax ? 1 : 0;
  const int k = std::max(1, std::min<int>({Dmax, (int)cand.size(), std::max(above, 1)}));
  double kept2 = 0.0;
  for (int i = 0; i < k; ++i) {
    blks[cand[i].t].kq += 1;
    kept2 += cand[i].s * cand[i].s;
  }
  res.k = k;
  res.norm = std::sqrt(kept2);
  res.disc = tot > 0.0 ? std::max(0.0, tot - kept2) / tot : 0.0;
  res.charges.clear();
  int off = 0;
  for (Blk& b : blks) {  // blocks come in ascending charge (std::map order)
    b.off = off;
    off += b.kq;
    res.charges.insert(res.charges.end(), b.kq, b.q);
  }
  hipLaunchKernelGGL(fill_zero_c128, dim3(grid_for((long long)m * k)), dim3(256), 0, st, A, (long long)m * k);
  MPOEVO_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(fill_zero_c128, dim3(grid_for((long long)k * n)), dim3(256), 0, st, B, (long long)k * n);
  MPOEVO_HIP_TRY(hipGetLastError());
  for (const Blk& b : blks) {
    if (b.kq == 0) continue;
    const int* r_dev = idx_dev + b.io;
    const int* c_dev = r_dev + b.mq;
    hipLaunchKernelGGL(scatter_block_cols, dim3(grid_for((long long)b.mq * b.kq)), dim3(256), 0, st, aq + b.ao,
                       b.kcap, b.mq, b.kq, r_dev, A, k, b.off);
    MPOEVO_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(scatter_block_rows, dim3(grid_for((long long)b.kq * b.nq)), dim3(256), 0, st, bq + b.bo,
                       b.nq, b.kq, c_dev, B, n, b.off);
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

// Site product site[a][s][b] <- sum_c site_in[a][s][c] R[c][b] (complex128), used to absorb
// the U S factor of the right-canonicalisation into the site on the left.
hipError_t absorb_right(const void* site_in, const void* R, void* site_out, int Pa, int d, int Pc,
                        int Pb, hipStream_t st, void* gws = nullptr) {
  GemmDesc g{};
  g.ws = gws;
  g.ws_bytes = gws ? kGemmScratchBytes : 0;
  g.A = site_in; g.B = R; g.C = site_out;
  g.M = Pa * d; g.N = Pb; g.K = Pc; g.batch = 1;
  g.sAm = Pc; g.sAk = 1; g.sBk = Pb; g.sBn = 1; g.sCm = Pb; g.sCn = 1;
  return gemm_launch(g, true, true, st);
}

// Scratch of the short-leg contraction done as a product (MPO bonds beyond the register kernels):
// W permuted for the left side (the right side needs none).
size_t wcontract_xws(int d, int wl, int wr, size_t cs) {
  if (wmix_supported(wl, d, wr)) return 0;
  return a256(cs * (size_t)d * wr * wl * d);
}

// ------------------------------------------------------------------------- step workspace map
struct StepLayout {
  size_t sitecap, lbcap, envcap, tmpcap, wcap, thetacap;
  size_t off_u1, off_blk, off_token_front, off_phi, off_ketc, off_brac, off_wc, off_lb, off_rb, off_env0, off_env1, off_tmp,
      off_theta, off_svd, off_kbuf, off_dbuf, off_nbuf, off_site_tmp, off_site_tmp2, off_sweeps,
      off_cplt, off_blocks, off_basis, basiscap, off_token, off_gemm, off_xws, total;
};

StepLayout step_layout(int L, int d, int Dmax, int wmax, int prec) {
  StepLayout s{};
  const size_t cs = csize(prec);
  const bool f32 = prec != MPOEVO_FP64;  // complex64 copies of the operands
  s.sitecap = (size_t)Dmax * d * Dmax;
  s.lbcap = (size_t)Dmax * d * wmax * Dmax;
  s.envcap = (size_t)Dmax * wmax * Dmax;
  s.tmpcap = (size_t)Dmax * wmax * d * Dmax;
  s.wcap = (size_t)wmax * d * d * wmax;
  s.thetacap = (size_t)d * Dmax * d * Dmax;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += a256(bytes); return at; };
  // the step token is kept at both ends of the region it guards (an allocation that reused the
  // front of a freed workspace overwrites the first, one that reused its tail the second)
  s.off_token_front = take(sizeof(unsigned long long));
  s.off_phi = take(sizeof(double2) * s.sitecap * L);
  s.off_ketc = take(f32 ? sizeof(float2) * s.sitecap * L : 0);
  s.off_brac = take(f32 ? sizeof(float2) * s.sitecap * L : 0);
  s.off_wc = take(f32 ? sizeof(float2) * s.wcap * L : 0);
  s.off_lb = take(cs * s.lbcap * L);
  s.off_rb = take(cs * s.lbcap * L);
  s.off_env0 = take(cs * s.envcap);
  s.off_env1 = take(cs * s.envcap);
  s.off_tmp = take(cs * s.tmpcap);
  s.off_theta = take(sizeof(double2) * s.thetacap);
  s.off_svd = take(svd_ws_bound(d * Dmax));
  s.off_kbuf = take(sizeof(int) * (size_t)8 * L);
  s.off_dbuf = take(sizeof(double) * (size_t)8 * L);
  s.off_nbuf = take(sizeof(double) * (size_t)8 * L);
  s.off_site_tmp = take(sizeof(double2) * s.sitecap);
  s.off_site_tmp2 = take(sizeof(double2) * s.sitecap);
  s.off_blk = take(cs * s.lbcap);  // one-site updates: the block of the current site
  s.off_u1 = take(blocked_scratch_bytes(d * Dmax));  // U(1) chains: per-charge truncations
  s.off_sweeps = take(sizeof(int) * (size_t)8 * L);
  s.off_cplt = take(sizeof(int) * (size_t)8 * L);  // per visit: the bond matrix had full rank
  s.off_blocks = take(sizeof(int) * (size_t)8 * L);  // per visit: column blocks of the Jacobi rounds
  // one unitary per bond (the Jacobi preconditioner carried between visits and steps)
  s.basiscap = (size_t)d * Dmax * d * Dmax;
  s.off_basis = take(sizeof(double2) * s.basiscap * (size_t)std::max(L - 1, 1));
  s.off_token = take(sizeof(unsigned long long));  // which step last wrote the unitaries
  s.off_gemm = take(kGemmScratchBytes);             // split-K partial products
  s.off_xws = take(wcontract_xws(d, wmax, wmax, cs));  // large MPO bonds
  s.total = o;
  return s;
}

}  // namespace

// ------------------------------------------------------------------------------ init / sizes
namespace {
int noalloc_scratch_init(Context& ctx);
}  // namespace

int device_init(Context& ctx) {
  hipError_t e = hipSetDevice(ctx.device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  int lds = 0, coop = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx.device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceGetAttribute(shared memory)");
  e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, ctx.device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceGetAttribute(cooperative launch)");
  if (!coop) { ctx.err = "device does not support cooperative launches"; return MPOEVO_EUNSUPPORTED; }
  const size_t lds_need = std::max(kSvdLdsBytes, kQrLdsBytes + 1024);
  if ((size_t)lds < lds_need) {
    ctx.err = "device provides " + std::to_string(lds) + " bytes of LDS per workgroup; the SVD needs " +
              std::to_string(lds_need);
    return MPOEVO_EUNSUPPORTED;
  }
  e = svd_configure();
  if (e != hipSuccess) return hip_fail(ctx, e, "svd_configure");
  auto* ds = new DeviceState();
  ds->lds_max = lds;
  e = hipDeviceGetAttribute(&ds->cus, hipDeviceAttributeMultiprocessorCount, ctx.device);
  if (e != hipSuccess) { delete ds; return hip_fail(ctx, e, "hipDeviceGetAttribute(compute units)"); }
  e = hipMalloc(&ds->status, 4 * sizeof(int));
  if (e != hipSuccess) { delete ds; return hip_fail(ctx, e, "hipMalloc(status)"); }
  e = hipMemset(ds->status, 0, 4 * sizeof(int));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) { (void)hipFree(ds->status); delete ds; return hip_fail(ctx, e, "status init"); }
  if (!ctx.tuner) {
    ctx.tuner = gemm_tuner_new();
    if (!ctx.tuner) {
      (void)hipFree(ds->status);
      delete ds;
      ctx.err = "out of host memory (tuner)";
      return MPOEVO_ENOMEM;
    }
    ctx.owns_tuner = true;
  }
  ctx.dev = ds;
  const int rc = noalloc_scratch_init(ctx);
  if (rc != MPOEVO_OK) {
    device_fini(ctx);
    return rc;
  }
  return MPOEVO_OK;
}

void device_fini(Context& ctx) {
  for (auto& c : ctx.chains) device_fini(*c);
  ctx.chains.clear();
  if (ctx.owns_tuner) gemm_tuner_free(ctx.tuner);
  ctx.tuner = nullptr;
  ctx.owns_tuner = false;
  if (!ctx.dev) return;
  (void)hipSetDevice(ctx.device);
  for (void* s : ctx.streams) (void)hipStreamDestroy(static_cast<hipStream_t>(s));
  ctx.streams.clear();
  for (hipEvent_t ev : ctx.dev->events) (void)hipEventDestroy(ev);
  for (GraphEntry& g : ctx.dev->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (ctx.dev->capture_stream) (void)hipStreamDestroy(ctx.dev->capture_stream);
  if (ctx.dev->fork) (void)hipEventDestroy(ctx.dev->fork);
  for (hipEvent_t ev : ctx.dev->joins) (void)hipEventDestroy(ev);
  for (hipStream_t bs : ctx.dev->block_streams) (void)hipStreamDestroy(bs);
  (void)hipFree(ctx.dev->status);
  delete ctx.dev;
  ctx.dev = nullptr;
}

size_t env_update_core(const int* dims, int prec) {
  const size_t Dbl = dims[0], Dkl = dims[1], Dbr = dims[2], Dkr = dims[3], d = dims[4],
               wl = dims[5], wr = dims[6];
  const size_t cs = csize(prec);
  const size_t left = a256(cs * Dbl * wl * d * Dkr) + a256(cs * Dbl * d * wr * Dkr);
  const size_t right = a256(cs * Dkl * d * Dbr * wr) + a256(cs * wl * Dkl * d * Dbr);
  return std::max(left, right);
}

size_t env_update_xws(const int* dims, int prec) {
  return wcontract_xws(dims[4], dims[5], dims[6], csize(prec));
}

size_t env_update_ws(const int* dims, int prec) {
  return env_update_core(dims, prec) + env_update_xws(dims, prec) + kGemmScratchBytes;
}

size_t local_apply_core(const int* dims, int prec) {
  const size_t Dbl = dims[0], Dkm = dims[2], Dbr = dims[4], d = dims[5], wl = dims[6],
               wm = dims[7], wr = dims[8];
  const size_t cs = csize(prec);
  const size_t tmp = std::max(cs * Dbl * wl * d * Dkm, cs * Dkm * d * Dbr * wr);
  return a256(tmp) + a256(cs * Dbl * d * wm * Dkm) + a256(cs * wm * Dkm * d * Dbr);
}

size_t local_apply_xws(const int* dims, int prec) {
  const size_t cs = csize(prec);
  return std::max(wcontract_xws(dims[5], dims[6], dims[7], cs), wcontract_xws(dims[5], dims[7], dims[8], cs));
}

size_t local_apply_ws(const int* dims, int prec) {
  return local_apply_core(dims, prec) + local_apply_xws(dims, prec) + kGemmScratchBytes;
}

// One-site local tensor: dims = {Dbra_l, Dket_l, Dket_r, Dbra_r, d, w_l, w_r}; the left block's
// temporary and the block itself, the large-bond contraction scratch, split-K scratch.
size_t local_apply1_ws(const int* dims, int prec) {
  const size_t Dbl = dims[0], Dkr = dims[2], d = dims[4], wl = dims[5], wr = dims[6];
  const size_t cs = csize(prec);
  return a256(cs * Dbl * wl * d * Dkr) + a256(cs * Dbl * d * wr * Dkr) +
         wcontract_xws(dims[4], dims[5], dims[6], cs) + kGemmScratchBytes;
}

size_t truncate_ws(int m, int n) {
  size_t ws = 0;
  for (int dir : {MPOEVO_LEFT, MPOEVO_RIGHT})
    ws = std::max(ws, svd_qr_ok(m, n, dir) ? svd_plan_qr(m, n, dir).ws : svd_plan(m, n, dir).ws);
  return ws;
}

size_t step_ws(int L, int d, int Dmax, int wmax, int prec) {
  return step_layout(L, d, Dmax, wmax, prec).total;
}

int check_solver_dev(Context& ctx, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  // on the given stream (a step's: no dependence on the legacy stream, which another thread's graph
  // capture would forbid), else on the legacy stream
  const hipStream_t sq = static_cast<hipStream_t>(stream);
  int stv[4] = {0, 0, 0, 0};
  hipError_t e = sq ? hipMemcpyAsync(stv, ctx.dev->status, sizeof(stv), hipMemcpyDeviceToHost, sq)
                    : hipMemcpy(stv, ctx.dev->status, sizeof(stv), hipMemcpyDeviceToHost);
  if (e == hipSuccess && sq) e = hipStreamSynchronize(sq);
  if (e != hipSuccess) return hip_fail(ctx, e, "reading the solver status");
  ctx.max_sweeps = std::max(ctx.max_sweeps, stv[1]);
  const int st = stv[0];
  if (st || stv[1] || stv[2]) {
    e = sq ? hipMemsetAsync(ctx.dev->status, 0, sizeof(stv), sq) : hipMemset(ctx.dev->status, 0, sizeof(stv));
    if (e == hipSuccess && sq) e = hipStreamSynchronize(sq);
    if (e != hipSuccess) return hip_fail(ctx, e, "clearing the solver status");
  }
  if (st) {
    if (st & kStatusNonFinite) { ctx.err = "truncate: non-finite singular values"; return MPOEVO_ENONFINITE; }
    if (st & kStatusBarrierTimeout) { ctx.err = "truncate: grid barrier timed out"; return MPOEVO_ESOLVER; }
    float rel;
    std::memcpy(&rel, &stv[2], sizeof(float));
    ctx.err = "truncate: Jacobi SVD did not converge within its sweep limit (last sweep's largest "
              "relative inner product " + std::to_string(rel) + ")";
    return MPOEVO_ESOLVER;
  }
  return MPOEVO_OK;
}

// ------------------------------------------------------------------------------- ABI calls
namespace {
// The environment update on a scratch region: base holds the intermediate and the block
// (env_update_core bytes), then the large-bond W scratch (env_update_xws bytes); gws / gws_bytes
// is the split-K scratch of the products.
hipError_t env_update_run(int side, int prec, const void* E_in, const void* bra, const void* W,
                          const void* ket, void* E_out, const int* dims, unsigned char* base,
                          void* gws, size_t gws_bytes, hipStream_t st) {
  const int Dbl = dims[0], Dkl = dims[1], Dbr = dims[2], Dkr = dims[3], d = dims[4], wl = dims[5],
            wr = dims[6];
  const Arith ar = arith_of(prec);
  const size_t cs = csize(prec);
  void* xws = base + env_update_core(dims, prec);
  if (side == MPOEVO_LEFT) {
    void* tmp = base;
    void* LB = base + a256(cs * (size_t)Dbl * wl * d * Dkr);
    MPOEVO_HIP_TRY(left_block(ar, E_in, ket, W, tmp, LB, Dbl, wl, Dkl, d, Dkr, wr, st, nullptr, gws, xws,
                              gws_bytes));
    return left_env_from_block(ar, bra, LB, E_out, Dbl, d, Dbr, wr, Dkr, st, nullptr, gws, gws_bytes);
  }
  void* tmp = base;
  void* RB = base + a256(cs * (size_t)Dkl * d * Dbr * wr);
  MPOEVO_HIP_TRY(right_block(ar, ket, E_in, W, tmp, RB, Dkl, d, Dkr, Dbr, wl, wr, st, nullptr, gws, xws,
                             gws_bytes));
  return right_env_from_block(ar, bra, RB, E_out, Dbl, d, Dbr, wl, Dkl, st, nullptr, gws, gws_bytes);
}

// Scratch of env_update_noalloc: one copy per device, held from the library's load until the
// process ends. Host code never passes the array's own name to a kernel (that is a host-side
// stand-in): its device address on each device comes from hipGetSymbolAddress, taken once per
// device at handle creation with that device current.
__device__ __align__(256) unsigned char scratch[MPOEVO_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch_init(Context& ctx) {
  if (ctx.device < 0 || ctx.device >= kMaxDevices) {
    ctx.err = "device index beyond the library's table of per-device scratch addresses";
    return MPOEVO_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[ctx.device]) return MPOEVO_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[ctx.device] = ptr;
  return MPOEVO_OK;
}
}  // namespace

int env_update_dev(Context& ctx, int side, int prec, const void* E_in, const void* bra,
                   const void* W, const void* ket, void* E_out, const int* dims, void* ws,
                   size_t, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  TunerScope tuner_scope(ctx.tuner, ctx.owns_tuner);
  unsigned char* base = static_cast<unsigned char*>(ws);
  void* gws = base + env_update_core(dims, prec) + env_update_xws(dims, prec);
  const hipError_t e = env_update_run(side, prec, E_in, bra, W, ket, E_out, dims, base, gws,
                                      kGemmScratchBytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "env_update");
}

size_t env_update_noalloc_need(const int* dims, int prec) {
  return env_update_core(dims, prec) + env_update_xws(dims, prec);
}

int env_update_noalloc_dev(Context& ctx, int side, int prec, const void* E_in, const void* bra,
                           const void* W, const void* ket, void* E_out, const int* dims, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  TunerScope tuner_scope(ctx.tuner, false);  // tuning would synchronise the stream
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ptr = (ctx.device >= 0 && ctx.device < kMaxDevices) ? g_scratch_ptr[ctx.device] : nullptr;
  }
  if (!ptr) { ctx.err = "env_update_noalloc: no scratch address for this device"; return MPOEVO_EUNSUPPORTED; }
  const size_t need = env_update_noalloc_need(dims, prec);
  if (need > MPOEVO_NOALLOC_SCRATCH_BYTES) {
    ctx.err = "env_update_noalloc: these dimensions need " + std::to_string(need) +
              " bytes of scratch, more than the library's " +
              std::to_string((size_t)MPOEVO_NOALLOC_SCRATCH_BYTES) + " (use env_update with a workspace)";
    return MPOEVO_ENOMEM;
  }
  unsigned char* base = static_cast<unsigned char*>(ptr);
  // what the intermediates leave over serves as the products' split-K scratch (a planner given
  // less scratch splits K fewer ways)
  const size_t gws_bytes = MPOEVO_NOALLOC_SCRATCH_BYTES - need;
  void* gws = gws_bytes > 0 ? base + need : nullptr;
  const hipError_t e = env_update_run(side, prec, E_in, bra, W, ket, E_out, dims, base, gws, gws_bytes,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "env_update_noalloc");
}

int local_apply_dev(Context& ctx, int prec, const void* L, const void* W1, const void* W2,
                    const void* M1, const void* M2, const void* R, void* Theta, const int* dims,
                    void* ws, size_t, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  TunerScope tuner_scope(ctx.tuner, ctx.owns_tuner);
  const int Dbl = dims[0], Dkl = dims[1], Dkm = dims[2], Dkr = dims[3], Dbr = dims[4], d = dims[5],
            wl = dims[6], wm = dims[7], wr = dims[8];
  const Arith ar = arith_of(prec);
  const size_t cs = csize(prec);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* base = static_cast<unsigned char*>(ws);
  const size_t tmpb = a256(std::max(cs * Dbl * wl * d * Dkm, cs * Dkm * d * Dbr * wr));
  void* tmp = base;
  void* LB = base + tmpb;
  void* RB = base + tmpb + a256(cs * (size_t)Dbl * d * wm * Dkm);
  void* xws = base + local_apply_core(dims, prec);
  void* gws = static_cast<unsigned char*>(xws) + local_apply_xws(dims, prec);
  hipError_t e = left_block(ar, L, M1, W1, tmp, LB, Dbl, wl, Dkl, d, Dkm, wm, st, nullptr, gws, xws);
  if (e == hipSuccess)
    e = right_block(ar, M2, R, W2, tmp, RB, Dkm, d, Dkr, Dbr, wm, wr, st, nullptr, gws, xws);
  if (e == hipSuccess) e = theta_product(ar, LB, RB, Theta, Dbl, d, wm, Dkm, Dbr, st, nullptr, gws);
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "local_apply");
}

// Theta[a'][s'][b'] = sum L[a'][alpha][a] M[a][s][b] W[alpha][s'][s][beta] R[b'][beta][b]: the left
// block LB = L M W (as in a left-to-right one-site update), then LB R.
int local_apply1_dev(Context& ctx, int prec, const void* L, const void* W, const void* M, const void* R,
                     void* Theta, const int* dims, void* ws, size_t, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  TunerScope tuner_scope(ctx.tuner, ctx.owns_tuner);
  const int Dbl = dims[0], Dkl = dims[1], Dkr = dims[2], Dbr = dims[3], d = dims[4], wl = dims[5], wr = dims[6];
  const Arith ar = arith_of(prec);
  const size_t cs = csize(prec);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* base = static_cast<unsigned char*>(ws);
  void* tmp = base;
  void* LB = base + a256(cs * (size_t)Dbl * wl * d * Dkr);
  void* xws = static_cast<unsigned char*>(LB) + a256(cs * (size_t)Dbl * d * wr * Dkr);
  void* gws = static_cast<unsigned char*>(xws) + wcontract_xws(d, wl, wr, cs);
  hipError_t e = left_block(ar, L, M, W, tmp, LB, Dbl, wl, Dkl, d, Dkr, wr, st, nullptr, gws, xws);
  if (e == hipSuccess) e = local_left(ar, LB, R, static_cast<double2*>(Theta), Dbl, d, wr, Dkr, Dbr, st, nullptr, gws);
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "local_apply");
}

int truncate_dev(Context& ctx, const void* Theta, int m, int n, int Dmax, double cutoff,
                 int direction, void* A_out, void* B_out, int* k_dev, double* discarded_dev,
                 double* norm_dev, double* sigma_dev, void* ws, size_t, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  TunerScope tuner_scope(ctx.tuner, ctx.owns_tuner);
  // up to 512: Jacobi on R^dag of the column-pivoted QR (a cold start needs few sweeps that way)
  const SvdPlan p = svd_qr_ok(m, n, direction) ? svd_plan_qr(m, n, direction) : svd_plan(m, n, direction);
  hipError_t e = svd_truncate(p, static_cast<const double2*>(Theta), Dmax, cutoff,
                              static_cast<double2*>(A_out), static_cast<double2*>(B_out), k_dev,
                              discarded_dev, norm_dev, sigma_dev, ws, ctx.dev->status,
                              static_cast<hipStream_t>(stream));
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "truncate");
}

// --------------------------------------------------------------------------- expectation
size_t expectation_ws(int L, int d, int Dmax, int wmax) {
  (void)L;
  const size_t env = a256(sizeof(double2) * (size_t)Dmax * wmax * Dmax);
  const size_t blk = a256(sizeof(double2) * (size_t)Dmax * wmax * d * Dmax);
  return 2 * env + 2 * blk + wcontract_xws(d, wmax, wmax, sizeof(double2)) + kGemmScratchBytes;
}

// E <- E . ket_i . O_i . conj(bra_i), i = 0 .. L-1, from E = e_left; out = E[right] = <bra| O |ket>.
int overlap_dev(Context& ctx, const mpoevo_mps* bra, const mpoevo_mpo* mpo, const mpoevo_mps* ket, int left,
                int right, void* out, void* ws, size_t, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  TunerScope tuner_scope(ctx.tuner, ctx.owns_tuner);
  const int L = ket->L, d = ket->d, Dmax = std::max(bra->Dmax, ket->Dmax);
  int wmax = 0;
  for (int i = 0; i <= L; ++i) wmax = std::max(wmax, mpo->w[i]);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* base = static_cast<unsigned char*>(ws);
  const size_t env = a256(sizeof(double2) * (size_t)Dmax * wmax * Dmax);
  const size_t blk = a256(sizeof(double2) * (size_t)Dmax * wmax * d * Dmax);
  double2* E[2] = {reinterpret_cast<double2*>(base), reinterpret_cast<double2*>(base + env)};
  void* tmp = base + 2 * env;
  void* LB = base + 2 * env + blk;
  void* xws = base + 2 * env + 2 * blk;
  void* gws = static_cast<unsigned char*>(xws) + wcontract_xws(d, wmax, wmax, sizeof(double2));
  const int* P = bra->bond_dim;
  const int* Q = ket->bond_dim;
  const int* w = mpo->w;
  hipLaunchKernelGGL(boundary_level, dim3((w[0] + 255) / 256), dim3(256), 0, st, E[0], w[0], left);
  hipError_t e = hipGetLastError();
  int cur = 0;
  for (int i = 0; i < L && e == hipSuccess; ++i) {
    e = left_block(Arith{true, false}, E[cur], ket->site[i], mpo->site[i], tmp, LB, P[i], w[i], Q[i], d, Q[i + 1],
                   w[i + 1], st, nullptr, gws, xws);
    if (e == hipSuccess)
      e = left_env_from_block(Arith{true, false}, bra->site[i], LB, E[cur ^ 1], P[i], d, P[i + 1], w[i + 1],
                              Q[i + 1], st, nullptr, gws);
    cur ^= 1;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(copy_entry, dim3(1), dim3(64), 0, st, E[cur] + right, static_cast<double2*>(out));
    e = hipGetLastError();
  }
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "overlap");
}

int expectation_dev(Context& ctx, const mpoevo_mps* mps, const mpoevo_mpo* mpo, int left, int right,
                    void* out, void* ws, size_t bytes, void* stream) {
  return overlap_dev(ctx, mps, mpo, mps, left, right, out, ws, bytes, stream);
}

// ---------------------------------------------------------------------------------- the step
// The zip-up guess: bond bounds K (K[i] = min(Dmax, rows, columns) of the SVD at site i, the
// carry's bond) and its buffers inside the region of the environment blocks (free until the
// sweeps build them): X and the contraction's temporaries, all FP64, U S and two carries.
struct ZipPlan {
  bool ok = false;
  std::vector<int> K;
  size_t offX = 0, offT = 0, offXws = 0, offA = 0, offE0 = 0, offE1 = 0;
};

ZipPlan zip_plan(int L, int d, int Dmax, const std::vector<int>& Q, const int* w, size_t region) {
  ZipPlan z;
  z.K.assign(L + 1, 1);
  const size_t c16 = sizeof(double2);
  size_t xb = 0, tb = 0, xwb = 0, ab = 0, eb = c16 * (size_t)w[L];
  for (int i = L - 1; i >= 0; --i) {
    const long long m = (long long)w[i] * Q[i], n = (long long)d * z.K[i + 1];
    xb = std::max(xb, c16 * (size_t)(m * n));
    tb = std::max(tb, c16 * (size_t)Q[i] * d * z.K[i + 1] * w[i + 1]);
    xwb = std::max(xwb, wcontract_xws(d, w[i], w[i + 1], c16));
    if (i == 0) break;
    if (m > (long long)d * Dmax) return z;  // beyond the SVD's workspace
    z.K[i] = (int)std::min<long long>(Dmax, std::min(m, n));
    ab = std::max(ab, c16 * (size_t)(m * z.K[i]));
    eb = std::max(eb, c16 * (size_t)(m * z.K[i]));
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += a256(bytes); return at; };
  z.offX = take(xb);
  z.offT = take(tb);
  z.offXws = take(xwb);
  z.offA = take(ab);
  z.offE0 = take(eb);
  z.offE1 = take(eb);
  z.ok = o <= region;
  return z;
}

// Host state the device work of a step leaves behind.
struct StepPost {
  std::vector<int>* P;
  std::vector<int>* bond_of_visit;
  std::vector<int>* k_slot_of_bond;
  int* last_visit_k_slot;
  double* gflop;
  bool* one_site;
  int* updates;
  int* graph_use;  // 0 issued, 1 captured, 2 replayed
  std::vector<char>* visit_kind;  // per visit: 1 one-site, 2 two-site update
  std::vector<char>* frozen;      // per bond: at its largest value when the step started
  bool* mixed;
};

// Issues the device work of a step (body). With opts->use_graph (and neither profiling nor U(1)
// charges, whose truncations wait for the device) the work is captured into a HIP graph the second
// time a step with the same plan runs on the handle -- the plan being everything the launches
// depend on: shapes, options, the buffers, the truncations' preconditioner state and the tile
// tuner's state -- and every later step with that plan replays the graph instead of issuing its
// launches.
// Inside a graph the Jacobi and QR kernels are ordinary launches (the graph runs its nodes one at
// a time, so their workgroups are resident together), not cooperative ones; the arithmetic is
// the same, so replays reproduce the uncaptured step bit for bit.
template <class Body>
int run_step_body(Context& ctx, const mpoevo_step_opts* opts, const mpoevo_mps* mps, const mpoevo_mpo* mpo,
                  const void* ws, const std::vector<int>& Q, bool profiling, bool u1, bool warm_on,
                  hipStream_t& st, Body& body, StepPost post, bool two_site_only) {
  *post.graph_use = 0;
  if (!opts->use_graph || profiling || u1) return body();
  const int L = mps->L;
  std::vector<long long> key = {L, mps->d, mps->Dmax, opts->prec, opts->nsweeps, opts->nsites, opts->guess,
                                two_site_only ? 1 : 0,
                                opts->input_right_canonical, opts->svd_cold_start, warm_on ? 1 : 0,
                                (long long)(uintptr_t)ws, ctx.tuner ? gemm_tuner_mode(ctx.tuner, -1) : -1,
                                ctx.tuner ? (long long)gemm_tuner_generation(ctx.tuner) : -1};
  long long cut = 0;
  std::memcpy(&cut, &opts->cutoff, sizeof(cut));
  key.push_back(cut);
  for (int i = 0; i < L; ++i) {
    key.push_back((long long)(uintptr_t)mps->site[i]);
    key.push_back((long long)(uintptr_t)mpo->site[i]);
  }
  for (int i = 0; i <= L; ++i) {
    key.push_back(Q[i]);
    key.push_back(mpo->w[i]);
  }
  for (size_t i = 0; i < ctx.warm_dim.size(); ++i) {
    key.push_back(ctx.warm_dim[i]);
    key.push_back(ctx.warm_deficient[i]);
  }
  DeviceState& ds = *ctx.dev;
  // a plan is captured the second time it is seen: the first step with it runs uncaptured, which
  // lets the tile tuner time the products it has not seen (it cannot while a stream is captured)
  if (std::find(ds.seen.begin(), ds.seen.end(), key) == ds.seen.end()) {
    bool cached = false;
    for (const GraphEntry& g : ds.graphs) cached = cached || g.key == key;
    if (!cached) {
      if (ds.seen.size() >= 2 * kMaxGraphs) ds.seen.erase(ds.seen.begin());
      ds.seen.push_back(key);
      return body();
    }
  }
  for (GraphEntry& g : ds.graphs) {
    if (g.key != key) continue;
    const hipError_t e = hipGraphLaunch(g.exec, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "step: replaying the captured graph");
    *post.P = g.P;
    *post.bond_of_visit = g.bond_of_visit;
    *post.k_slot_of_bond = g.k_slot_of_bond;
    *post.last_visit_k_slot = g.last_visit_k_slot;
    *post.gflop = g.gflop;
    *post.one_site = g.one_site;
    *post.updates = g.updates;
    *post.visit_kind = g.visit_kind;
    *post.frozen = g.frozen;
    *post.mixed = g.mixed;
    *post.graph_use = 2;
    ctx.warm_dim = g.warm_dim;
    return MPOEVO_OK;
  }
  if (!ds.capture_stream) {
    const hipError_t e = hipStreamCreateWithFlags(&ds.capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(ctx, e, "step: creating the capture stream");
  }
  const hipStream_t orig = st;
  st = ds.capture_stream;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    st = orig;
    return hip_fail(ctx, e, "step: beginning the graph capture");
  }
  const bool coop = ctx.coop_jacobi;
  ctx.coop_jacobi = false;
  const int rc = body();
  ctx.coop_jacobi = coop;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(st, &graph);
  st = orig;
  if (rc != MPOEVO_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "step: ending the graph capture");
  GraphEntry g;
  g.key = std::move(key);
  g.graph = graph;
  e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(ctx, e, "step: instantiating the captured graph");
  }
  g.P = *post.P;
  g.bond_of_visit = *post.bond_of_visit;
  g.k_slot_of_bond = *post.k_slot_of_bond;
  g.last_visit_k_slot = *post.last_visit_k_slot;
  g.gflop = *post.gflop;
  g.one_site = *post.one_site;
  g.updates = *post.updates;
  g.visit_kind = *post.visit_kind;
  g.frozen = *post.frozen;
  g.mixed = *post.mixed;
  g.warm_dim = ctx.warm_dim;
  if (ds.graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(ds.graphs.front().exec);
    (void)hipGraphDestroy(ds.graphs.front().graph);
    ds.graphs.erase(ds.graphs.begin());
  }
  ds.graphs.push_back(std::move(g));
  *post.graph_use = 1;
  e = hipGraphLaunch(ds.graphs.back().exec, st);
  return e == hipSuccess ? MPOEVO_OK : hip_fail(ctx, e, "step: launching the captured graph");
}

// The calling thread's stream-capture mode set to relaxed while it lives. A thread's own mode
// decides whether its synchronous calls (the read-back of a step, the solver check) are refused
// while another thread captures a graph, and the runtime counts every thread's capture there
// (step_batched's workers capture and synchronise side by side); relaxed lets both proceed.
struct RelaxedCaptureMode {
  hipStreamCaptureMode prev = hipStreamCaptureModeRelaxed;
  RelaxedCaptureMode() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
  ~RelaxedCaptureMode() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
  RelaxedCaptureMode(const RelaxedCaptureMode&) = delete;
  RelaxedCaptureMode& operator=(const RelaxedCaptureMode&) = delete;
};

int step_dev(Context& ctx, mpoevo_mps* mps, const mpoevo_mpo* mpo, const mpoevo_step_opts* opts,
             mpoevo_step_stats* stats, void* ws, size_t, void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  const RelaxedCaptureMode capture_mode;
  TunerScope tuner_scope(ctx.tuner, ctx.owns_tuner);
  const int L = mps->L, d = mps->d, Dmax = mps->Dmax, prec = opts->prec;
  const bool fp64 = prec == MPOEVO_FP64;
  const Arith ar = arith_of(prec);
  int wmax = 0;
  for (int i = 0; i <= L; ++i) wmax = std::max(wmax, mpo->w[i]);
  const StepLayout lay = step_layout(L, d, Dmax, wmax, prec);
  const size_t cs = csize(prec);
  unsigned char* base = static_cast<unsigned char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto phi = [&](int i) { return reinterpret_cast<double2*>(base + lay.off_phi) + lay.sitecap * i; };
  auto ket = [&](int i) -> const void* {
    if (fp64) return mps->site[i];
    return reinterpret_cast<float2*>(base + lay.off_ketc) + lay.sitecap * i;
  };
  auto bra = [&](int i) -> const void* {
    if (fp64) return phi(i);
    return reinterpret_cast<float2*>(base + lay.off_brac) + lay.sitecap * i;
  };
  auto wsite = [&](int i) -> const void* {
    if (fp64) return mpo->site[i];
    return reinterpret_cast<float2*>(base + lay.off_wc) + lay.wcap * i;
  };
  auto LB = [&](int i) { return base + lay.off_lb + cs * lay.lbcap * i; };
  auto RB = [&](int i) { return base + lay.off_rb + cs * lay.lbcap * i; };
  void* env0 = base + lay.off_env0;
  void* env1 = base + lay.off_env1;
  void* tmp = base + lay.off_tmp;
  double2* theta = reinterpret_cast<double2*>(base + lay.off_theta);
  void* svdws = base + lay.off_svd;
  int* kbuf = reinterpret_cast<int*>(base + lay.off_kbuf);
  double* dbuf = reinterpret_cast<double*>(base + lay.off_dbuf);
  double* nbuf = reinterpret_cast<double*>(base + lay.off_nbuf);
  double2* site_tmp = reinterpret_cast<double2*>(base + lay.off_site_tmp);
  double2* site_tmp2 = reinterpret_cast<double2*>(base + lay.off_site_tmp2);
  const int* w = mpo->w;
  auto basis = [&](int i) { return reinterpret_cast<double2*>(base + lay.off_basis) + lay.basiscap * i; };
  void* gws = base + lay.off_gemm;
  void* xws = base + lay.off_xws;

  // Jacobi preconditioners: kept in the workspace between steps of the same handle, valid while
  // the workspace and the chain's shape stay the same; otherwise every bond restarts from the
  // identity. warm_dim[i] is the order of the unitary stored for bond i (0: none).
  // U(1) chains: host copies of the charges of the bra bonds (the ket's are fixed during the step)
  const bool u1 = mps->sector_table != nullptr;
  std::vector<std::vector<int>> qch(L + 1);
  std::vector<int> qp(u1 ? d : 0);
  if (u1) {
    for (int s_ = 0; s_ < d; ++s_) qp[s_] = mps->phys_charge[s_];
    for (int b = 0; b <= L; ++b)
      qch[b].assign(mps->sector_table + (size_t)b * Dmax, mps->sector_table + (size_t)b * Dmax + mps->bond_dim[b]);
  }
  unsigned char* u1ws = base + lay.off_u1;
  const bool warm_on = opts->svd_cold_start == 0 && !u1;
  const int sig[5] = {L, d, Dmax, wmax, prec};
  unsigned long long* token_dev = reinterpret_cast<unsigned long long*>(base + lay.off_token);
  unsigned long long* token_front = reinterpret_cast<unsigned long long*>(base + lay.off_token_front);
  bool reuse = warm_on && ctx.warm_ws == ws && std::equal(sig, sig + 5, ctx.warm_sig) &&
               (int)ctx.warm_dim.size() == L - 1 && (int)ctx.warm_deficient.size() == L - 1;
  if (reuse) {  // the workspace must still hold what this handle's last step left there
    unsigned long long tok[2] = {0, 0};
    hipError_t et = hipMemcpyAsync(&tok[0], token_front, sizeof(tok[0]), hipMemcpyDeviceToHost, st);
    if (et == hipSuccess) et = hipMemcpyAsync(&tok[1], token_dev, sizeof(tok[1]), hipMemcpyDeviceToHost, st);
    if (et == hipSuccess) et = hipStreamSynchronize(st);
    if (et != hipSuccess) return hip_fail(ctx, et, "step: reading the workspace token");
    reuse = tok[0] == ctx.warm_token && tok[1] == ctx.warm_token;
  }
  if (!reuse) {
    ctx.warm_dim.assign(std::max(L - 1, 0), 0);
    ctx.warm_deficient.assign(std::max(L - 1, 0), 0);
  }
  ctx.warm_ws = nullptr;  // re-armed when this step completes
  // The unitary kept for bond i has the order of X's column count, min(m, n); a change of shape
  // restarts it from the identity.
  auto warm_for = [&](int i, int m, int n) -> double2* {
    if (!warm_on) return nullptr;
    const int nx = std::min(m, n);
    if (ctx.warm_dim[i] != nx) {
      hipLaunchKernelGGL(fill_identity, dim3(grid_for((long long)nx * nx)), dim3(256), 0, st, basis(i), nx);
      if (hipGetLastError() != hipSuccess) return nullptr;
      ctx.warm_dim[i] = nx;
    }
    return basis(i);
  };
  // the slot a truncation that starts without a preconditioner writes its unitary to
  auto basis_slot = [&](int i, int nx) -> double2* {
    ctx.warm_dim[i] = nx;
    return basis(i);
  };

  ctx.max_sweeps = 0;
  std::vector<int> Q(mps->bond_dim, mps->bond_dim + L + 1);  // ket bonds
  // bonds the last step kept at Dmax: below it the spectrum fell under the cutoff, the bond
  // matrices are numerically rank-deficient and their truncations take the pivoted QR
  std::vector<char> saturated(L + 1);
  for (int b = 0; b <= L; ++b) saturated[b] = Q[b] >= Dmax;
  std::vector<int> P(Q);                                       // bra bonds (upper bounds)
  hipError_t e = hipSuccess;
  Prof prof_obj;
  Prof* prof = nullptr;
  if (opts->profile) {
    prof_obj.ds = ctx.dev;
    prof_obj.st = st;
    prof_obj.all = opts->profile != 2;
    prof = &prof_obj;
  }
  int* sweeps_buf = reinterpret_cast<int*>(base + lay.off_sweeps);
  int* cplt_buf = reinterpret_cast<int*>(base + lay.off_cplt);
  int* blocks_buf = reinterpret_cast<int*>(base + lay.off_blocks);
  struct JacRec { size_t ev; SvdPlan plan; int slot; const void* kernel; };
  std::vector<JacRec> jac_recs;
  double gflop = 0.0;
  auto flop_gemm = [&](double M, double N, double K) { gflop += 8.0 * M * N * K * 1e-9; };
  auto bra_refresh = [&](int i) -> hipError_t {  // fp32 copy of phi_i
    if (fp64) return hipSuccess;
    return cast_to_c64(phi(i), (void*)bra(i), (long long)P[i] * d * P[i + 1], st);
  };
#define STEP_TRY(x)                              \
  do {                                           \
    e = (x);                                     \
    if (e != hipSuccess) return hip_fail(ctx, e, "step"); \
  } while (0)

  // the guess: psi, or the zip-up of W psi (bonds up to Dmax at once)
  auto cap_of = [&](int b) {
    long long c = 1;
    for (int k = 0; k < std::min(b, L - b) && c < Dmax; ++k) c *= d;
    return (int)std::min<long long>(c, Dmax);
  };
  const ZipPlan zp = zip_plan(L, d, Dmax, Q, w, lay.off_env0 - lay.off_lb);
  bool zip = false;
  if (opts->guess == MPOEVO_GUESS_ZIPUP) {
    if (!zp.ok) {
      ctx.err = "step: the zip-up guess needs bond[i] w[i] <= d Dmax at every site i >= 1";
      return MPOEVO_EUNSUPPORTED;
    }
    zip = true;
  } else if (opts->guess == MPOEVO_GUESS_AUTO && !u1 && zp.ok && opts->nsites != 1) {
    for (int b = 1; b < L && !zip; ++b) zip = Q[b] < cap_of(b);
  }

  // ---------------------------------------------------------------- the step's device work
  // Everything from here to the final normalisation is issued without waiting for the device, so
  // that it can be captured into a HIP graph once and replayed by later steps with the same plan.
  int visit = 0;
  const int nvis = opts->nsweeps * 2 * (L - 1);
  int last_visit_k_slot = 0;
  std::vector<int> k_slot_of_bond(L, -1);
  std::vector<int> bond_of_visit(nvis, 0);
  bool one_site = false;
  int updates = 0;
  // automatic mode with bonds still growing: the bonds at their largest value when the step starts
  // are frozen, and a position whose site has both bonds frozen takes that site's one-site update
  std::vector<char> frozen(L + 1, 1), visit_kind(nvis, 2);
  bool mixed = false, two_site_only = false;
  std::vector<int> u1_k(u1 ? nvis : 0);
  std::vector<double> u1_d(u1 ? nvis : 0), u1_n(u1 ? nvis : 0);
  std::vector<int> u1_zero(u1 ? nvis : 0, 0), u1_one(u1 ? nvis : 0, 1);
  const std::vector<int> P0(P);
  std::vector<int> P_guess;  // the guess's bonds (the one-site visits keep them)
  auto body = [&]() -> int {
  P = P0;
  visit = 0;
  last_visit_k_slot = 0;
  std::fill(k_slot_of_bond.begin(), k_slot_of_bond.end(), -1);
  std::fill(visit_kind.begin(), visit_kind.end(), 2);
  gflop = 0.0;
  jac_recs.clear();
  // inputs in contraction precision; phi <- psi
  for (int i = 0; i < L; ++i) {
    const long long ns = (long long)Q[i] * d * Q[i + 1];
    STEP_TRY(hipMemcpyAsync(phi(i), mps->site[i], sizeof(double2) * ns, hipMemcpyDeviceToDevice, st));
    if (!fp64) {
      STEP_TRY(cast_to_c64(mps->site[i], (void*)ket(i), ns, st));
      STEP_TRY(cast_to_c64(mpo->site[i], (void*)wsite(i), (long long)w[i] * d * d * w[i + 1], st));
    }
  }
  // row charges of a bond matrix with rows (a', s') and column charges of one with columns
  // (t', c') (the charge of the bond between them)
  auto row_charges = [&](int bond) {
    std::vector<int> r((size_t)P[bond] * d);
    for (int a = 0; a < P[bond]; ++a)
      for (int s_ = 0; s_ < d; ++s_) r[(size_t)a * d + s_] = qch[bond][a] + qp[s_];
    return r;
  };
  auto col_charges = [&](int bond) {
    std::vector<int> c((size_t)d * P[bond]);
    for (int t = 0; t < d; ++t)
      for (int b = 0; b < P[bond]; ++b) c[(size_t)t * P[bond] + b] = qch[bond][b] - qp[t];
    return c;
  };
  if (zip) {
    // zip-up from the right end in FP64: X_i = W_i psi_i C_{i+1}, rows (alpha, a), columns
    // (s', k); its truncated SVD gives phi_i = V^dag and the next carry C_i = (U S)^T
    const Arith ar64{true, false};
    unsigned char* zb = base + lay.off_lb;
    double2* X = reinterpret_cast<double2*>(zb + zp.offX);
    void* T = zb + zp.offT;
    void* XW = zb + zp.offXws;
    double2* A = reinterpret_cast<double2*>(zb + zp.offA);
    double2* Ec = reinterpret_cast<double2*>(zb + zp.offE0);
    double2* En = reinterpret_cast<double2*>(zb + zp.offE1);
    const std::vector<int>& K = zp.K;
    STEP_TRY(set_boundary(Ec, w[L], true, st));
    for (int i = L - 1; i >= 0; --i) {
      STEP_TRY(right_block(ar64, mps->site[i], Ec, mpo->site[i], T, X, Q[i], d, Q[i + 1], K[i + 1], w[i],
                           w[i + 1], st, prof, gws, XW));
      flop_gemm((double)Q[i] * d, (double)K[i + 1] * w[i + 1], Q[i + 1]);
      flop_gemm((double)w[i] * d * Q[i], K[i + 1], (double)d * w[i + 1]);
      if (i == 0) {  // the left boundary level: the first d K[1] entries of X
        STEP_TRY(hipMemcpyAsync(phi(0), X, sizeof(double2) * (size_t)Q[0] * d * K[1], hipMemcpyDeviceToDevice,
                                st));
        P[0] = Q[0];
        break;
      }
      const int m = w[i] * Q[i], n = d * K[i + 1];
      const SvdPlan sp = svd_qr_ok(m, n, MPOEVO_RIGHT) ? svd_plan_qr(m, n, MPOEVO_RIGHT)
                                                       : svd_plan(m, n, MPOEVO_RIGHT);
      STEP_TRY(svd_truncate(sp, X, Dmax, opts->cutoff, A, phi(i), nullptr, nullptr, nullptr, nullptr, svdws,
                            ctx.dev->status, st, nullptr, nullptr, nullptr, nullptr, nullptr, ctx.coop_jacobi));
      STEP_TRY([&] {
        hipLaunchKernelGGL(transpose_c128, dim3(grid_for((long long)m * K[i])), dim3(256), 0, st, A, En, m, K[i]);
        return hipGetLastError();
      }());
      std::swap(Ec, En);
      P[i] = K[i];
    }
  } else if (!opts->input_right_canonical && u1) {  // right-canonical guess: SVD of each site from the last to the second
    for (int i = L - 1; i >= 1; --i) {  // per charge block: the rows a carry q(a), columns (s, b) q(b) - q(s)
      const int m = P[i], n = d * P[i + 1];
      BlockedResult br;
      STEP_TRY(blocked_truncate(ctx, phi(i), m, n, qch[i], col_charges(i + 1), std::min(m, n), opts->cutoff,
                                MPOEVO_RIGHT, theta, site_tmp, u1ws, d * Dmax, svdws, svd_ws_bound(d * Dmax), st,
                                br));
      STEP_TRY(hipMemcpyAsync(phi(i), site_tmp, sizeof(double2) * (size_t)br.k * n, hipMemcpyDeviceToDevice, st));
      STEP_TRY(absorb_right(phi(i - 1), theta, site_tmp2, P[i - 1], d, m, br.k, st, gws));
      STEP_TRY(hipMemcpyAsync(phi(i - 1), site_tmp2, sizeof(double2) * (size_t)P[i - 1] * d * br.k,
                              hipMemcpyDeviceToDevice, st));
      P[i] = br.k;
      qch[i] = br.charges;
    }
  } else if (!opts->input_right_canonical) {
    for (int i = L - 1; i >= 1; --i) {
      const int m = P[i], n = d * P[i + 1];
      const SvdPlan pl = svd_plan(m, n, MPOEVO_RIGHT);
      const int kcap = std::min(m, n);
      double2* A = theta;  // m x kcap   (U S)
      double2* B = site_tmp;  // kcap x n (V^dag)
      STEP_TRY(svd_truncate(pl, phi(i), kcap, opts->cutoff, A, B, nullptr, nullptr,
                            nullptr, nullptr, svdws, ctx.dev->status, st, nullptr, nullptr,
                            nullptr, nullptr, nullptr, ctx.coop_jacobi));
      STEP_TRY(hipMemcpyAsync(phi(i), B, sizeof(double2) * (size_t)kcap * n, hipMemcpyDeviceToDevice, st));
      // phi_{i-1} <- phi_{i-1} . (U S)
      STEP_TRY(absorb_right(phi(i - 1), A, site_tmp2, P[i - 1], d, m, kcap, st, gws));
      STEP_TRY(hipMemcpyAsync(phi(i - 1), site_tmp2, sizeof(double2) * (size_t)P[i - 1] * d * kcap,
                              hipMemcpyDeviceToDevice, st));
      P[i] = kcap;
    }
  }
  for (int i = 0; i < L; ++i) STEP_TRY(bra_refresh(i));

  // ------------------------------------------------------------------ one-site updates
  // at the bonds of the guess (fixed): each site's projected tensor becomes its FP64 QR factor
  one_site = opts->nsites == 1;
  if (opts->nsites == -1 && !zip) {
    one_site = d * Dmax <= 512 && !u1;
    for (int b = 1; b < L && one_site; ++b) one_site = P[b] == cap_of(b);
  }
  auto qr_visit = [&](int m, int n, bool left_to_right, double2* out) -> hipError_t {
    // left to right: Q of the (D_i d) x D_{i+1} tensor; right to left: Q^dag of the transposed
    const SvdPlan qp = svd_plan_qr(m, n, left_to_right ? MPOEVO_RIGHT : MPOEVO_LEFT);
    PROF_BEGIN(prof, qt);
    MPOEVO_HIP_TRY(qr_isometry(qp, theta, out, !left_to_right, svdws, ctx.dev->status, st, ctx.coop_jacobi));
    PROF_END(prof, qt, Prof::kQr, qr_flop(std::max(m, n), std::min(m, n)));
    return hipSuccess;
  };
  mixed = false;
  P_guess = P;
  std::fill(frozen.begin(), frozen.end(), 1);
  if (opts->nsites == -1 && !zip && !u1 && !one_site && !two_site_only && d * Dmax <= 512) {
    for (int b = 1; b < L; ++b) frozen[b] = P[b] == cap_of(b) ? 1 : 0;
    for (int i = 0; i < L && !mixed; ++i) mixed = frozen[i] && frozen[i + 1];
  }
  // a one-site visit of site i: both its bonds frozen and still at their starting values (a
  // two-site update that shrank one makes the step fall back to two-site updates, see below)
  auto one_site_at = [&](int i) {
    return mixed && frozen[i] && frozen[i + 1] && P[i] == P_guess[i] && P[i + 1] == P_guess[i + 1];
  };
  auto one_site_slots = [&](int v, int k) -> hipError_t {
    hipLaunchKernelGGL(one_site_visit_slots, dim3(1), dim3(64), 0, st, kbuf + v, dbuf + v, nbuf + v,
                       sweeps_buf + v, cplt_buf + v, blocks_buf + v, k);
    return hipGetLastError();
  };
  if (one_site) {
    if (d * Dmax > 512) { ctx.err = "step: one-site updates need d Dmax <= 512"; return MPOEVO_ESHAPE; }
    for (int i = 0; i + 1 < L; ++i)
      if (P[i + 1] > d * P[i]) {
        ctx.err = "step: one-site updates need bond[i+1] <= d bond[i] (bond " + std::to_string(i + 1) + ")";
        return MPOEVO_ESHAPE;
      }
    // Lenv_i (i = 0..L-1) live in the left-block slots, Renv_i (i = 1..L) in the right-block slots
    auto envL = [&](int i) -> void* { return LB(i); };
    auto envR = [&](int i) -> void* { return RB(i - 1); };
    void* blk = base + lay.off_blk;
    STEP_TRY(set_boundary(envR(L), w[L], fp64, st));
    for (int i = L - 1; i >= 1; --i) {
      STEP_TRY(right_block(ar, ket(i), envR(i + 1), wsite(i), tmp, blk, Q[i], d, Q[i + 1], P[i + 1], w[i],
                           w[i + 1], st, prof, gws, xws));
      flop_gemm((double)Q[i] * d, (double)P[i + 1] * w[i + 1], Q[i + 1]);
      flop_gemm((double)w[i] * d * Q[i], P[i + 1], (double)d * w[i + 1]);
      STEP_TRY(right_env_from_block(ar, bra(i), blk, envR(i), P[i], d, P[i + 1], w[i], Q[i], st, prof, gws));
      flop_gemm(P[i], (double)w[i] * Q[i], (double)d * P[i + 1]);
    }
    STEP_TRY(set_boundary(envL(0), w[0], fp64, st));
    updates = 0;
    for (int sw = 0; sw < opts->nsweeps; ++sw) {
      for (int i = 0; i <= L - 2; ++i, ++updates) {
        STEP_TRY(left_block(ar, envL(i), ket(i), wsite(i), tmp, blk, P[i], w[i], Q[i], d, Q[i + 1],
                            w[i + 1], st, prof, gws, xws));
        flop_gemm((double)P[i] * w[i], (double)d * Q[i + 1], Q[i]);
        flop_gemm((double)P[i] * d * w[i + 1], Q[i + 1], (double)w[i] * d);
        STEP_TRY(local_left(ar, blk, envR(i + 1), theta, P[i], d, w[i + 1], Q[i + 1], P[i + 1], st, prof, gws));
        flop_gemm((double)P[i] * d, P[i + 1], (double)w[i + 1] * Q[i + 1]);
        STEP_TRY(qr_visit(P[i] * d, P[i + 1], true, phi(i)));
        STEP_TRY(bra_refresh(i));
        STEP_TRY(left_env_from_block(ar, bra(i), blk, envL(i + 1), P[i], d, P[i + 1], w[i + 1], Q[i + 1], st,
                                     prof, gws));
        flop_gemm(P[i + 1], (double)w[i + 1] * Q[i + 1], (double)P[i] * d);
      }
      for (int i = L - 1; i >= 1; --i, ++updates) {
        STEP_TRY(right_block(ar, ket(i), envR(i + 1), wsite(i), tmp, blk, Q[i], d, Q[i + 1], P[i + 1], w[i],
                             w[i + 1], st, prof, gws, xws));
        flop_gemm((double)Q[i] * d, (double)P[i + 1] * w[i + 1], Q[i + 1]);
        flop_gemm((double)w[i] * d * Q[i], P[i + 1], (double)d * w[i + 1]);
        STEP_TRY(local_right(ar, envL(i), blk, theta, P[i], w[i], Q[i], d, P[i + 1], st, prof, gws));
        flop_gemm(P[i], (double)d * P[i + 1], (double)w[i] * Q[i]);
        STEP_TRY(qr_visit(P[i], d * P[i + 1], false, phi(i)));
        STEP_TRY(bra_refresh(i));
        STEP_TRY(right_env_from_block(ar, bra(i), blk, envR(i), P[i], d, P[i + 1], w[i], Q[i], st, prof, gws));
        flop_gemm(P[i], (double)w[i] * Q[i], (double)d * P[i + 1]);
      }
    }
    // site 0: its projected tensor completes phi; its norm is the fitted norm
    STEP_TRY(right_block(ar, ket(0), envR(1), wsite(0), tmp, blk, Q[0], d, Q[1], P[1], w[0], w[1], st, prof,
                         gws, xws));
    flop_gemm((double)Q[0] * d, (double)P[1] * w[1], Q[1]);
    flop_gemm((double)w[0] * d * Q[0], P[1], (double)d * w[1]);
    STEP_TRY(local_right(ar, envL(0), blk, theta, P[0], w[0], Q[0], d, P[1], st, prof, gws));
    flop_gemm(P[0], (double)d * P[1], (double)w[0] * Q[0]);
    ++updates;
    STEP_TRY([&] {
      hipLaunchKernelGGL(norm_scale_kernel, dim3(1), dim3(256), 0, st, theta, phi(0),
                         (long long)P[0] * d * P[1], nbuf);
      return hipGetLastError();
    }());
    return MPOEVO_OK;
  }

  // right blocks RB_i, i = L-1 .. 1, from the canonical guess
  STEP_TRY(set_boundary(env1, w[L], fp64, st));  // Renv_L
  for (int i = L - 1; i >= 1; --i) {
    STEP_TRY(right_block(ar, ket(i), env1, wsite(i), tmp, RB(i), Q[i], d, Q[i + 1], P[i + 1],
                         w[i], w[i + 1], st, prof, gws, xws));
    flop_gemm((double)Q[i] * d, (double)P[i + 1] * w[i + 1], Q[i + 1]);
    flop_gemm((double)w[i] * d * Q[i], P[i + 1], (double)d * w[i + 1]);  // the W contraction
    if (i > 1) {
      STEP_TRY(right_env_from_block(ar, bra(i), RB(i), env1, P[i], d, P[i + 1], w[i], Q[i], st, prof, gws));
      flop_gemm(P[i], (double)w[i] * Q[i], (double)d * P[i + 1]);
    }
  }

  // U(1): the truncation of a visit per charge block (kept rank, weight and norm known on the host)
  auto u1_visit = [&](int i, int m, int n, int dir, int vis) -> hipError_t {
    BlockedResult br;
    MPOEVO_HIP_TRY(blocked_truncate(ctx, theta, m, n, row_charges(i), col_charges(i + 2), Dmax, opts->cutoff, dir,
                                    phi(i), phi(i + 1), u1ws, d * Dmax, svdws, svd_ws_bound(d * Dmax), st,
                                    br));
    u1_k[vis] = br.k;
    u1_d[vis] = br.disc;
    u1_n[vis] = br.norm;
    qch[i + 1] = br.charges;
    return hipSuccess;
  };
  for (int sw = 0; sw < opts->nsweeps; ++sw) {
    // left to right
    for (int i = 0; i <= L - 2; ++i, ++visit) {
      if (i == 0) STEP_TRY(set_boundary(env0, w[0], fp64, st));
      else {
        STEP_TRY(left_env_from_block(ar, bra(i - 1), LB(i - 1), env0, P[i - 1], d, P[i],
                                     w[i], Q[i], st, prof, gws));
        flop_gemm(P[i], (double)w[i] * Q[i], (double)P[i - 1] * d);
      }
      STEP_TRY(left_block(ar, env0, ket(i), wsite(i), tmp, LB(i), P[i], w[i], Q[i], d, Q[i + 1],
                          w[i + 1], st, prof, gws, xws));
      flop_gemm((double)P[i] * w[i], (double)d * Q[i + 1], Q[i]);
      flop_gemm((double)P[i] * d * w[i + 1], Q[i + 1], (double)w[i] * d);  // the W contraction
      if (one_site_at(i)) {
        // site i's projected tensor against the right environment of bond i + 1 (from the right
        // block of site i + 1), replaced by its QR factor
        STEP_TRY(right_env_from_block(ar, bra(i + 1), RB(i + 1), env1, P[i + 1], d, P[i + 2], w[i + 1], Q[i + 1],
                                      st, prof, gws));
        flop_gemm(P[i + 1], (double)w[i + 1] * Q[i + 1], (double)d * P[i + 2]);
        STEP_TRY(local_left(ar, LB(i), env1, theta, P[i], d, w[i + 1], Q[i + 1], P[i + 1], st, prof, gws));
        flop_gemm((double)P[i] * d, P[i + 1], (double)w[i + 1] * Q[i + 1]);
        STEP_TRY(qr_visit(P[i] * d, P[i + 1], true, phi(i)));
        STEP_TRY(one_site_slots(visit, P[i + 1]));
        visit_kind[visit] = 1;
        bond_of_visit[visit] = i;
        last_visit_k_slot = visit;
        STEP_TRY(bra_refresh(i));
        continue;
      }
      const int m = P[i] * d, n = d * P[i + 2];
      STEP_TRY(theta_product(ar, LB(i), RB(i + 1), theta, P[i], d, w[i + 1], Q[i + 1], P[i + 2], st, prof, gws));
      flop_gemm(m, n, (double)w[i + 1] * Q[i + 1]);
      int kcap = std::min(Dmax, std::min(m, n));
      if (u1) {
        bond_of_visit[visit] = i;
        STEP_TRY(u1_visit(i, m, n, MPOEVO_LEFT, visit));
        kcap = u1_k[visit];
      } else {
        // the first visit of a bond in a step has no fresh preconditioner (Theta moved by a
        // whole time step since the last one), and a bond below Dmax, or one whose matrix the
        // last step found numerically rank-deficient, would need its basis completed: square
        // Theta then goes through the pivoted QR, handing on a basis only where the next visit
        // can use it (rectangular Theta: when no basis of its size is at hand)
        const bool deficient = !saturated[i + 1] || ctx.warm_deficient[i];
        const bool qr = warm_on && svd_qr_ok(m, n, MPOEVO_LEFT) &&
                        (m == n ? (sw == 0 || ctx.warm_dim[i] != m || deficient)
                                : ctx.warm_dim[i] != std::min(m, n));
        SvdPlan sp = qr ? svd_plan_qr(m, n, MPOEVO_LEFT) : svd_plan(m, n, MPOEVO_LEFT, warm_on);
        if (!fp64) sp.accept = kSvdAcceptFp32;
        hipEvent_t j0 = nullptr, j1 = nullptr;
        size_t jf = 0;
        if (prof) STEP_TRY(prof->pair(&j0, &j1, &jf));
        double2* wb = qr ? (m == n && !deficient ? basis_slot(i, m) : nullptr) : warm_for(i, m, n);
        if (qr && !wb) ctx.warm_dim[i] = 0;
        bond_of_visit[visit] = i;
        STEP_TRY(svd_truncate(sp, theta, Dmax, opts->cutoff, phi(i), phi(i + 1), kbuf + visit,
                              dbuf + visit, nbuf + visit, nullptr, svdws, ctx.dev->status, st, j0,
                              j1, sweeps_buf + visit, qr ? nullptr : wb, wb, ctx.coop_jacobi,
                              cplt_buf + visit, blocks_buf + visit));
        if (prof) jac_recs.push_back({jf, sp, visit, svd_jacobi_kernel_ptr(sp)});
      }
      P[i + 1] = kcap;
      k_slot_of_bond[i + 1] = visit;
      last_visit_k_slot = visit;
      STEP_TRY(bra_refresh(i));
      STEP_TRY(bra_refresh(i + 1));
    }
    // right to left
    for (int i = L - 2; i >= 0; --i, ++visit) {
      if (i < L - 2) {
        STEP_TRY(right_env_from_block(ar, bra(i + 2), RB(i + 2), env1, P[i + 2], d, P[i + 3],
                                      w[i + 2], Q[i + 2], st, prof, gws));
        flop_gemm(P[i + 2], (double)w[i + 2] * Q[i + 2], (double)d * P[i + 3]);
        STEP_TRY(right_block(ar, ket(i + 1), env1, wsite(i + 1), tmp, RB(i + 1), Q[i + 1], d,
                             Q[i + 2], P[i + 2], w[i + 1], w[i + 2], st, prof, gws, xws));
        flop_gemm((double)Q[i + 1] * d, (double)P[i + 2] * w[i + 2], Q[i + 2]);
        flop_gemm((double)w[i + 1] * d * Q[i + 1], P[i + 2], (double)d * w[i + 2]);  // the W contraction
      }
      if (one_site_at(i + 1)) {
        // site i + 1's projected tensor against the left environment of bond i + 1 (from the left
        // block of site i), replaced by the adjoint QR factor of its adjoint
        STEP_TRY(left_env_from_block(ar, bra(i), LB(i), env0, P[i], d, P[i + 1], w[i + 1], Q[i + 1], st, prof,
                                     gws));
        flop_gemm(P[i + 1], (double)w[i + 1] * Q[i + 1], (double)P[i] * d);
        STEP_TRY(local_right(ar, env0, RB(i + 1), theta, P[i + 1], w[i + 1], Q[i + 1], d, P[i + 2], st, prof, gws));
        flop_gemm(P[i + 1], (double)d * P[i + 2], (double)w[i + 1] * Q[i + 1]);
        STEP_TRY(qr_visit(P[i + 1], d * P[i + 2], false, phi(i + 1)));
        STEP_TRY(one_site_slots(visit, P[i + 1]));
        visit_kind[visit] = 1;
        bond_of_visit[visit] = i;
        last_visit_k_slot = visit;
        STEP_TRY(bra_refresh(i + 1));
        continue;
      }
      const int m = P[i] * d, n = d * P[i + 2];
      STEP_TRY(theta_product(ar, LB(i), RB(i + 1), theta, P[i], d, w[i + 1], Q[i + 1], P[i + 2], st, prof, gws));
      flop_gemm(m, n, (double)w[i + 1] * Q[i + 1]);
      int kcap = std::min(Dmax, std::min(m, n));
      if (u1) {
        bond_of_visit[visit] = i;
        STEP_TRY(u1_visit(i, m, n, MPOEVO_RIGHT, visit));
        kcap = u1_k[visit];
      } else {
        const bool deficient = !saturated[i + 1] || ctx.warm_deficient[i];
        const bool qr = warm_on && svd_qr_ok(m, n, MPOEVO_RIGHT) &&
                        (m == n ? (ctx.warm_dim[i] != m || deficient)
                                : ctx.warm_dim[i] != std::min(m, n));
        SvdPlan sp = qr ? svd_plan_qr(m, n, MPOEVO_RIGHT) : svd_plan(m, n, MPOEVO_RIGHT, warm_on);
        if (!fp64) sp.accept = kSvdAcceptFp32;
        hipEvent_t j0 = nullptr, j1 = nullptr;
        size_t jf = 0;
        if (prof) STEP_TRY(prof->pair(&j0, &j1, &jf));
        // the last visit of a square bond in the step hands on no basis: the next step's first
        // visit starts from the pivoted QR (a warm start keeps its input unitary in the slot)
        const bool last = sw + 1 == opts->nsweeps && m == n && svd_qr_ok(m, n, MPOEVO_LEFT);
        double2* wb = qr ? (m == n && !deficient && !last ? basis_slot(i, m) : nullptr) : warm_for(i, m, n);
        if (qr && !wb) ctx.warm_dim[i] = 0;
        bond_of_visit[visit] = i;
        STEP_TRY(svd_truncate(sp, theta, Dmax, opts->cutoff, phi(i), phi(i + 1), kbuf + visit,
                              dbuf + visit, nbuf + visit, nullptr, svdws, ctx.dev->status, st, j0,
                              j1, sweeps_buf + visit, qr ? nullptr : wb, last ? nullptr : wb,
                              ctx.coop_jacobi, cplt_buf + visit, blocks_buf + visit));
        if (prof) jac_recs.push_back({jf, sp, visit, svd_jacobi_kernel_ptr(sp)});
      }
      P[i + 1] = kcap;
      k_slot_of_bond[i + 1] = visit;
      last_visit_k_slot = visit;
      STEP_TRY(bra_refresh(i));
      STEP_TRY(bra_refresh(i + 1));
    }
  }
  if (u1) {  // the visit slots the dense truncation fills on the device
    STEP_TRY(hipMemcpyAsync(kbuf, u1_k.data(), sizeof(int) * nvis, hipMemcpyHostToDevice, st));
    STEP_TRY(hipMemcpyAsync(dbuf, u1_d.data(), sizeof(double) * nvis, hipMemcpyHostToDevice, st));
    STEP_TRY(hipMemcpyAsync(nbuf, u1_n.data(), sizeof(double) * nvis, hipMemcpyHostToDevice, st));
    STEP_TRY(hipMemcpyAsync(sweeps_buf, u1_zero.data(), sizeof(int) * nvis, hipMemcpyHostToDevice, st));
    STEP_TRY(hipMemcpyAsync(cplt_buf, u1_one.data(), sizeof(int) * nvis, hipMemcpyHostToDevice, st));
    STEP_TRY(hipMemcpyAsync(blocks_buf, u1_zero.data(), sizeof(int) * nvis, hipMemcpyHostToDevice, st));
  }
  if (mixed && visit_kind[visit - 1] == 1) {
    // the last visit updated site 1: site 0's projected tensor completes phi (its norm is the
    // fitted norm, kept in that visit's slot)
    STEP_TRY(right_env_from_block(ar, bra(1), RB(1), env1, P[1], d, P[2], w[1], Q[1], st, prof, gws));
    flop_gemm(P[1], (double)w[1] * Q[1], (double)d * P[2]);
    STEP_TRY(right_block(ar, ket(0), env1, wsite(0), tmp, LB(0), Q[0], d, Q[1], P[1], w[0], w[1], st, prof, gws,
                         xws));
    flop_gemm((double)Q[0] * d, (double)P[1] * w[1], Q[1]);
    flop_gemm((double)w[0] * d * Q[0], P[1], (double)d * w[1]);
    STEP_TRY(set_boundary(env0, w[0], fp64, st));
    STEP_TRY(local_right(ar, env0, LB(0), theta, P[0], w[0], Q[0], d, P[1], st, prof, gws));
    flop_gemm(P[0], (double)d * P[1], (double)w[0] * Q[0]);
    STEP_TRY([&] {
      hipLaunchKernelGGL(norm_scale_kernel, dim3(1), dim3(256), 0, st, theta, phi(0),
                         (long long)P[0] * d * P[1], nbuf + (visit - 1));
      return hipGetLastError();
    }());
    last_visit_k_slot = visit - 1;
  } else {
    // normalise with the norm of the last visit (phi_0 holds U S)
    STEP_TRY([&] {
      hipLaunchKernelGGL(scale_by_inverse_norm, dim3(grid_for((long long)P[0] * d * P[1])), dim3(256), 0,
                         st, phi(0), (long long)P[0] * d * P[1], nbuf + last_visit_k_slot);
      return hipGetLastError();
    }());
  }
    return MPOEVO_OK;
  };

  int graph_use = 0;
  // a second pass (two-site updates throughout) when the mixed step's check below fails
  for (int pass = 0;; ++pass) {
    if (const int rc = run_step_body(ctx, opts, mps, mpo, ws, Q, prof != nullptr, u1, warm_on, st, body,
                                     StepPost{&P, &bond_of_visit, &k_slot_of_bond, &last_visit_k_slot, &gflop,
                                              &one_site, &updates, &graph_use, &visit_kind, &frozen, &mixed},
                                     two_site_only);
        rc != MPOEVO_OK)
      return rc;

    if (one_site) {
      double norm = 0.0;
      STEP_TRY(hipMemcpyAsync(&norm, nbuf, sizeof(double), hipMemcpyDeviceToHost, st));
      for (int i = 0; i < L; ++i) {  // the bonds are the guess's: copy phi back whole
        STEP_TRY(hipMemcpyAsync(mps->site[i], phi(i), sizeof(double2) * (size_t)P[i] * d * P[i + 1],
                                hipMemcpyDeviceToDevice, st));
      }
      STEP_TRY(hipStreamSynchronize(st));
      const int sres = check_solver_dev(ctx, st);
      if (sres != MPOEVO_OK) return sres;
      int maxb = 1;
      for (int b = 0; b <= L; ++b) {
        mps->bond_dim[b] = P[b];
        maxb = std::max(maxb, P[b]);
      }
      if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->norm = norm;
        stats->visits = updates;
        stats->one_site_visits = updates;
        stats->max_bond = maxb;
        stats->gflop = gflop;
        stats->graph = graph_use;
        if (prof) {
          struct Agg { int kind; int n; double ms, work; };
          std::map<const void*, Agg> per_kernel;
          for (const auto& r : prof->recs) {
            float ms = 0.f;
            STEP_TRY(hipEventElapsedTime(&ms, ctx.dev->events[r.e0], ctx.dev->events[r.e0 + 1]));
            const int kind = r.kind == Prof::kGemm ? 1 : r.kind == Prof::kQr ? 3 : 2;
            if (kind == 1) { stats->t_gemm_ms += ms; stats->gemm_gflop += r.work * 1e-9; stats->n_gemm += 1; }
            if (kind == 2) { stats->t_wmix_ms += ms; stats->wmix_gbyte += r.work * 1e-9; stats->n_wmix += 1; }
            Agg& a = per_kernel[r.launch.kernel];
            a.kind = kind;
            a.n += 1;
            a.ms += ms;
            a.work += r.work * 1e-9;
          }
          std::vector<std::pair<const void*, Agg>> order(per_kernel.begin(), per_kernel.end());
          std::stable_sort(order.begin(), order.end(),
                           [](const auto& a, const auto& b) { return a.second.ms > b.second.ms; });
          for (const auto& kv : order) {
            if (stats->n_kernel_stats >= MPOEVO_MAX_KERNEL_STATS) break;
            fill_kernel_stat(stats->kernel_stats[stats->n_kernel_stats++], kv.first, kv.second.kind, false,
                             kv.second.n, kv.second.ms, kv.second.work, st);
          }
        }
      }
      if (!std::isfinite(norm)) { ctx.err = "step: fitted norm is not finite"; return MPOEVO_ENONFINITE; }
      return MPOEVO_OK;
    }

    // read back the kept ranks and statistics (one synchronisation per step)
    std::vector<int> kh(nvis), swh(nvis), ch(nvis);
    std::vector<double> dh(nvis), nh(nvis);
    STEP_TRY(hipMemcpyAsync(swh.data(), sweeps_buf, sizeof(int) * nvis, hipMemcpyDeviceToHost, st));
    STEP_TRY(hipMemcpyAsync(ch.data(), cplt_buf, sizeof(int) * nvis, hipMemcpyDeviceToHost, st));
    std::vector<int> bh(nvis, 0);
    if (prof) STEP_TRY(hipMemcpyAsync(bh.data(), blocks_buf, sizeof(int) * nvis, hipMemcpyDeviceToHost, st));
    STEP_TRY(hipMemcpyAsync(kh.data(), kbuf, sizeof(int) * nvis, hipMemcpyDeviceToHost, st));
    STEP_TRY(hipMemcpyAsync(dh.data(), dbuf, sizeof(double) * nvis, hipMemcpyDeviceToHost, st));
    STEP_TRY(hipMemcpyAsync(nh.data(), nbuf, sizeof(double) * nvis, hipMemcpyDeviceToHost, st));
    STEP_TRY(hipStreamSynchronize(st));
    const int sres = check_solver_dev(ctx, st);
    if (sres != MPOEVO_OK) return sres;
    if (mixed && pass == 0) {
      // a two-site update that left a frozen bond below its value changed a bond that the one-site
      // updates next to it took as fixed: the step is redone with two-site updates throughout
      bool shrunk = false;
      for (int v = 0; v < nvis && !shrunk; ++v) {
        const int b = bond_of_visit[v] + 1;
        shrunk = visit_kind[v] == 2 && frozen[b] && kh[v] < cap_of(b);
      }
      if (shrunk) {
        two_site_only = true;
        if (prof) {
          prof->recs.clear();
          prof->next = 0;
        }
        continue;
      }
    }
    std::vector<int> Pact(L + 1, 1);
    for (int b = 1; b < L; ++b) Pact[b] = k_slot_of_bond[b] >= 0 ? kh[k_slot_of_bond[b]] : P[b];
    // a bond is taken as rank-deficient when any of its truncations in this step was (near the
    // onset of the rank deficiency the visits of one bond disagree, and a needless QR costs less
    // than a completion)
    std::fill(ctx.warm_deficient.begin(), ctx.warm_deficient.end(), 0);
    for (int v = 0; v < nvis; ++v)
      if (ch[v] == 0) ctx.warm_deficient[bond_of_visit[v]] = 1;
    // compact phi into the caller's site buffers
    for (int i = 0; i < L; ++i) {
      const long long n = (long long)Pact[i] * d * Pact[i + 1];
      // rows beyond Pact[i] are zero; keep a' < Pact[i], b < Pact[i+1] of the padded (P[i], d, P[i+1])
      hipLaunchKernelGGL(compact_site, dim3(grid_for(n)), dim3(256), 0, st, phi(i),
                         static_cast<double2*>(mps->site[i]), Pact[i], d, Pact[i + 1], P[i + 1]);
      STEP_TRY(hipGetLastError());
    }
    STEP_TRY(hipStreamSynchronize(st));
    const double norm = nh[last_visit_k_slot];
    int maxb = 1;
    for (int b = 0; b <= L; ++b) {
      mps->bond_dim[b] = Pact[b];
      maxb = std::max(maxb, Pact[b]);
    }
    if (u1)
      for (int b = 1; b < L; ++b) std::copy(qch[b].begin(), qch[b].end(), mps->sector_table + (size_t)b * Dmax);
    if (stats) {
      stats->norm = norm;
      stats->discarded_max = 0.0;
      stats->discarded_sum = 0.0;
      for (int v = 0; v < nvis; ++v) {
        stats->discarded_max = std::max(stats->discarded_max, dh[v]);
        stats->discarded_sum += dh[v];
      }
      stats->visits = nvis;
      stats->one_site_visits = 0;
      for (int v = 0; v < nvis; ++v) stats->one_site_visits += mixed && visit_kind[v] == 1 ? 1 : 0;
      stats->two_site_redo = two_site_only ? 1 : 0;
      stats->max_bond = maxb;
      stats->gflop = gflop;
      stats->svd_sweeps_max = ctx.max_sweeps;
      stats->svd_sweeps_total = 0;
      for (int& c : stats->svd_sweeps_hist) c = 0;
      for (int v = 0; v < nvis; ++v) {
        stats->svd_sweeps_total += swh[v];
        stats->svd_sweeps_hist[std::min(std::max(swh[v], 0), 31)] += 1;
      }
      stats->t_jacobi_ms = stats->jacobi_gflop = stats->t_gemm_ms = stats->gemm_gflop = 0.0;
      stats->t_wmix_ms = stats->wmix_gbyte = 0.0;
      stats->n_jacobi = stats->n_gemm = stats->n_wmix = 0;
      stats->n_kernel_stats = 0;
      stats->graph = graph_use;
      stats->guess = zip ? 1 : 0;
      if (prof) {
        const std::vector<int>& sw = swh;
        struct Agg { int kind; int split; int n; double ms, work; };
        std::map<std::pair<const void*, int>, Agg> per_kernel;
        auto add = [&](const void* k, int kind, bool split, double ms, double work) {
          Agg& a = per_kernel[{k, split ? 1 : 0}];
          a.kind = kind;
          a.split = split ? 1 : 0;
          a.n += 1;
          a.ms += ms;
          a.work += work;
        };
        for (const auto& r : jac_recs) {
          float ms = 0.f;
          STEP_TRY(hipEventElapsedTime(&ms, ctx.dev->events[r.ev], ctx.dev->events[r.ev + 1]));
          const double gf = sw[r.slot] * svd_sweep_flop(svd_jacobi_plan(r.plan), bh[r.slot]) * 1e-9;
          stats->t_jacobi_ms += ms;
          stats->jacobi_gflop += gf;
          stats->n_jacobi += 1;
          add(r.kernel, 0, false, ms, gf);
        }
        for (const auto& r : prof->recs) {
          float ms = 0.f;
          STEP_TRY(hipEventElapsedTime(&ms, ctx.dev->events[r.e0], ctx.dev->events[r.e0 + 1]));
          if (r.kind == Prof::kGemm) {
            stats->t_gemm_ms += ms;
            stats->gemm_gflop += r.work * 1e-9;
            stats->n_gemm += 1;
            add(r.launch.kernel, 1, r.launch.split, ms, r.work * 1e-9);
          } else if (r.kind == Prof::kQr) {
            add(r.launch.kernel, 3, false, ms, r.work * 1e-9);
          } else {
            stats->t_wmix_ms += ms;
            stats->wmix_gbyte += r.work * 1e-9;
            stats->n_wmix += 1;
            add(r.launch.kernel, 2, false, ms, r.work * 1e-9);
          }
        }
        std::vector<std::pair<std::pair<const void*, int>, Agg>> order(per_kernel.begin(), per_kernel.end());
        std::stable_sort(order.begin(), order.end(),
                         [](const auto& a, const auto& b) { return a.second.ms > b.second.ms; });
        for (const auto& kv : order) {
          if (stats->n_kernel_stats >= MPOEVO_MAX_KERNEL_STATS) break;
          fill_kernel_stat(stats->kernel_stats[stats->n_kernel_stats++], kv.first.first, kv.second.kind,
                           kv.second.split != 0, kv.second.n, kv.second.ms, kv.second.work, st);
        }
      }
    }
    if (!std::isfinite(norm)) { ctx.err = "step: fitted norm is not finite"; return MPOEVO_ENONFINITE; }
    if (warm_on) {
      static std::atomic<unsigned long long> next_token{1};
      ctx.warm_token = next_token.fetch_add(1);
      STEP_TRY(hipMemcpyAsync(token_front, &ctx.warm_token, sizeof(ctx.warm_token), hipMemcpyHostToDevice, st));
      STEP_TRY(hipMemcpyAsync(token_dev, &ctx.warm_token, sizeof(ctx.warm_token), hipMemcpyHostToDevice, st));
      STEP_TRY(hipStreamSynchronize(st));
      ctx.warm_ws = ws;
      std::copy(sig, sig + 5, ctx.warm_sig);
    }
    return MPOEVO_OK;
  }
#undef STEP_TRY
}

// ------------------------------------------------------------------------- batched chains
namespace {
// Worker streams: by default the number of hardware queues a process gets (4); the environment
// variable MPOEVO_BATCH_STREAMS (1..16) overrides it.
int batch_streams() {
  const char* v = std::getenv("MPOEVO_BATCH_STREAMS");
  const int n = v ? std::atoi(v) : 0;
  return (n >= 1 && n <= 16) ? n : 4;
}

size_t chain_ws(const int* dims, int prec) {  // dims = {L, d, Dmax, wmax}
  return a256(step_ws(dims[0], dims[1], dims[2], dims[3], prec));
}
}  // namespace

size_t step_batched_ws(int n, const int* dims, int prec) {
  size_t total = 0;
  for (int c = 0; c < n; ++c) total += chain_ws(dims + 4 * c, prec);
  return total;
}

// Independent chains share nothing but the device: each chain runs the single-chain step on
// one of a few worker streams (host thread per stream, chains taken largest first), so the
// latency-bound truncations of different chains overlap. Their Jacobi launches are ordinary
// launches; the number of streams is bounded so that the Jacobi workgroups of all streams fit
// on three quarters of the compute units at once.
int step_batched_dev(Context& ctx, int n, mpoevo_mps* mps, const mpoevo_mpo* mpo,
                     const mpoevo_step_opts* opts, mpoevo_step_stats* stats, void* ws, size_t,
                     void* stream) {
  if (hipError_t e0 = hipSetDevice(ctx.device); e0 != hipSuccess) return hip_fail(ctx, e0, "hipSetDevice");
  // the chains' inputs may have been written on the caller's stream
  if (hipError_t e0 = hipStreamSynchronize(static_cast<hipStream_t>(stream)); e0 != hipSuccess)
    return hip_fail(ctx, e0, "step_batched: stream synchronisation");
  while ((int)ctx.chains.size() < n) {
    auto c = std::make_unique<Context>();
    c->device = ctx.device;
    c->coop_jacobi = false;
    c->tuner = ctx.tuner;  // borrowed: the chains use the handle's tuned plans and tune nothing
    c->owns_tuner = false;
    const int rc = device_init(*c);
    if (rc != MPOEVO_OK) {
      ctx.err = "step_batched: " + c->err;
      return rc;
    }
    ctx.chains.push_back(std::move(c));
  }
  int cus = 0;
  if (hipError_t e0 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx.device);
      e0 != hipSuccess)
    return hip_fail(ctx, e0, "hipDeviceGetAttribute(compute units)");
  std::vector<size_t> off(n + 1, 0);
  std::vector<double> cost(n);
  int maxgrid = 1;
  for (int c = 0; c < n; ++c) {
    int wmax = 0;
    for (int i = 0; i <= mpo[c].L; ++i) wmax = std::max(wmax, mpo[c].w[i]);
    const int dims[4] = {mps[c].L, mps[c].d, mps[c].Dmax, wmax};
    off[c + 1] = off[c] + chain_ws(dims, opts->prec);
    const int side = mps[c].d * mps[c].Dmax;
    maxgrid = std::max(maxgrid, svd_grid(svd_plan(side, side, MPOEVO_LEFT, true)));
    cost[c] = (double)mps[c].L * side * side * side;
  }
  const int nstreams = std::max(1, std::min({batch_streams(), n, (3 * cus / 4) / maxgrid}));
  while ((int)ctx.streams.size() < nstreams) {
    hipStream_t s = nullptr;
    if (hipError_t e0 = hipStreamCreateWithFlags(&s, hipStreamNonBlocking); e0 != hipSuccess)
      return hip_fail(ctx, e0, "hipStreamCreateWithFlags");
    ctx.streams.push_back(s);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::atomic<int> next{0};
  std::vector<int> rc(n, MPOEVO_OK);
  unsigned char* base = static_cast<unsigned char*>(ws);
  auto worker = [&](int t) {
    for (;;) {
      const int j = next.fetch_add(1);
      if (j >= n) break;
      const int c = order[j];
      rc[c] = step_dev(*ctx.chains[c], &mps[c], &mpo[c], opts, stats ? &stats[c] : nullptr,
                       base + off[c], off[c + 1] - off[c], ctx.streams[t]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nstreams; ++t) pool.emplace_back(worker, t);
  worker(0);
  for (auto& th : pool) th.join();
  ctx.max_sweeps = 0;
  for (int c = 0; c < n; ++c) ctx.max_sweeps = std::max(ctx.max_sweeps, ctx.chains[c]->max_sweeps);
  for (int c = 0; c < n; ++c)
    if (rc[c] != MPOEVO_OK) {
      ctx.err = "step_batched: chain " + std::to_string(c) + ": " + ctx.chains[c]->err;
      return rc[c];
    }
  return MPOEVO_OK;
}

}  // namespace mpoevo
