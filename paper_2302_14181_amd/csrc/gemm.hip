// Complex strided-batched matrix products on the gfx950 matrix cores.
//
// FP32 operands: three real products per complex multiply-add (cgemm3m_kernel, below). FP64:
// a complex product C = A B (M x N x K complex multiply-adds) is computed as the real product
// C' = A' B' of size M x 2N x 2K with
//   A'[m][2k + p]          = (re, im)[p] of A[m][k]            (the interleaved storage itself)
//   B'[2k + p][2n + q]     = [[re, im], [-im, re]][p][q] of B[k][n]
//   C'[m][2n + q]          = (re, im)[q] of C[m][n]            (interleaved output)
// which is exactly the four real products of complex arithmetic (8 real flops per complex
// multiply-add) and needs no extra pass over memory: A tiles are stored to LDS planar by real
// k, B tiles are expanded to their real 2x2 form while they are staged.
//
// fp32 (the three-product kernel, on each real operand plane): v_mfma_f32_32x32x2f32 (lane l
//       supplies A[l%32][l/32], B[l/32][l%32]; accumulator r of lane l holds
//       C[(r/4)*8 + (l/32)*4 + r%4][l%32]).
// fp64: v_mfma_f64_16x16x4f64 (lane l supplies A'[l%16][l/16], B'[l/16][l%16]; accumulator r of
//       lane l holds C'[4r + l/16][l%16]).
// A workgroup of 4 waves (2 x 2, each wave WR x WC matrix-instruction tiles) owns a BM x BN
// complex tile, double-buffered in LDS with one barrier per K step of BK complex (8 for the large
// tiles, 16 for the small ones, whose single workgroup per compute unit needs the longer step to
// cover the latency of the next step's global loads, issued before the current step's matrix
// instructions).
//
// split-BF16x3 (fp32 operands): each real value x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
// (round to nearest), and A B ~ hi_A hi_B + hi_A lo_B + lo_A hi_B with fp32 accumulation on
// v_mfma_f32_32x32x16_bf16 (lane l supplies A'[l%32][8(l/32) + j] and B'[8(l/32) + j][l%32],
// j = 0..7; accumulators as for the fp32 instruction). The dropped lo lo term leaves about
// 2^-16 relative error per product. A tiles are staged as bf16 rows [m][k], B tiles as bf16
// columns [n][k] of the real expanded B', so that each lane reads its eight k values with one
// 16-byte LDS load.
//
// Occupancy: the products of a sweep are small (M x N of a few hundred), so a planner picks the
// largest tile that still gives every compute unit a workgroup, and when even the smallest tile
// leaves most of the 256 compute units idle it splits K: each split writes its partial tile to
// scratch and a second kernel sums the splits in a fixed order (results do not depend on
// scheduling).

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dev_common.h"
#include "internal.h"

namespace mpoevo {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// fp32 32 x 32 instructions (the three-product and split-BF16x3 kernels): element type of the
// plans, and the output layout of an accumulator.
struct MfmaF32 {
  using T = float;
  __device__ static int out_row(int l, int r) { return (r >> 2) * 8 + (l >> 5) * 4 + (r & 3); }
  __device__ static int out_col(int l) { return l & 31; }
};

struct MfmaF64 {
  using T = double;
  using acc_t = f64x4;
  static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int out_row(int l, int r) { return 4 * r + (l >> 4); }
  __device__ static int out_col(int l) { return l & 15; }
};

constexpr int kThreads = 256;
constexpr int kKGrain = 8;      // split-K chunks are multiples of this
constexpr int kMinWgs = 256;    // a tile giving at least this many workgroups is used as is
constexpr int kTargetWgs = 256; // split K up to this many workgroups (one per compute unit:
                                // more splits cost more in the reduction than they gain)
constexpr int kMaxSplits = 32;  // (the one-site local tensor at D = 256, w = 271: 128 x 128 tiles, 32 splits)
constexpr int kMinSplitK = 32;  // complex K per split, at least

// LDS staging: A as rows [m][k] and the expanded B as columns [n][k] (real k), each row of
// KR values plus 16 bytes of padding (an odd number of 16-byte units, so the 16-byte reads of
// 16 consecutive rows hit distinct banks). Within each group of G = KT * V real k the values are
// stored in the order the matrix instruction consumes them: a lane with k offset a (0..KT-1)
// uses k = KT q + a in its q-th instruction of the group, so position a V + q holds it and the
// lane fetches the operands of V instructions with one 16-byte read.
template <class Mf, int WR, int WC, int BK_>
struct Tile {
  static constexpr int BK = BK_;                      // complex K per stage
  using T = typename Mf::T;
  static constexpr int BM = 2 * WR * Mf::MT;          // complex rows per workgroup
  static constexpr int BNR = 2 * WC * Mf::NT;         // real columns per workgroup
  static constexpr int BN = BNR / 2;                  // complex columns
  static constexpr int KR = 2 * BK;                   // real k per stage
  static constexpr int V = 16 / (int)sizeof(T);       // values per 16-byte read
  static constexpr int G = Mf::KT * V;                // real k per group (8)
  static constexpr int PITCH = KR + V;                // LDS row length (elements)
  static constexpr int A_ELEMS = BM * BK / kThreads;   // complex loads per thread
  static constexpr int B_ELEMS = BN * BK / kThreads;
  static constexpr int LDS_ELEMS = (BM + BNR) * PITCH;
  static_assert(A_ELEMS >= 1 && B_ELEMS >= 1, "tile too small for the staging scheme");
  static_assert(KR % G == 0 && ((PITCH * (int)sizeof(T) / 16) & 1), "staging layout");
  // position of real k within its row
  __device__ static int kpos(int kr) {
    const int w = kr % G;
    return kr - w + (w % Mf::KT) * V + w / Mf::KT;
  }
};

// splits > 1: the workgroup at blockIdx.z = batch * splits + s covers K in [s kchunk, (s+1)
// kchunk) and writes its partial tile (precision T) to part[s][batch][M][N].
template <class Mf, int WR, int WC, int BK, typename TO, bool AKC, bool BNC>
__global__ __launch_bounds__(kThreads) void cgemm_kernel(GemmDesc g, int splits, int kchunk,
                                                         void* part) {
  using T = typename Mf::T;
  using C2 = cx_t<T>;
  using TT = Tile<Mf, WR, WC, BK>;
  __shared__ __attribute__((aligned(16))) T lds[2 * TT::LDS_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int bz = blockIdx.z / splits;
  const int sk = blockIdx.z - bz * splits;
  const int kbeg = sk * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int m0 = blockIdx.y * TT::BM;
  const int n0 = blockIdx.x * TT::BN;

  const C2* A = reinterpret_cast<const C2*>(g.A) + bz * g.bA;
  const C2* B = reinterpret_cast<const C2*>(g.B) + bz * g.bB;
  const T sgnA = g.conjA ? T(-1) : T(1);
  const T sgnB = g.conjB ? T(-1) : T(1);

  C2 ra[TT::A_ELEMS];
  C2 rb[TT::B_ELEMS];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int i = 0; i < TT::A_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int m, k;
      if (AKC) { m = e / BK; k = e % BK; } else { k = e / TT::BM; m = e % TT::BM; }
      const int gm = m0 + m, gk = k0 + k;
      C2 v{T(0), T(0)};
      if (gm < g.M && gk < kend) v = A[gm * g.sAm + gk * g.sAk];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < TT::B_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int k, n;
      if (BNC) { k = e / TT::BN; n = e % TT::BN; } else { n = e / BK; k = e % BK; }
      const int gk = k0 + k, gn = n0 + n;
      C2 v{T(0), T(0)};
      if (gk < kend && gn < g.N) v = B[gk * g.sBk + gn * g.sBn];
      rb[i] = v;
    }
  };
  // A' = [re, sgnA im] over real k = 2k, 2k+1; B' holds 2 x 2 real blocks per complex entry:
  // column 2n = (re, -im'), column 2n+1 = (im', re) over real k = 2k, 2k+1 (im' = sgnB im).
  auto store_tiles = [&](int buf) {
    T* As = lds + buf * TT::LDS_ELEMS;
    T* Bs = As + TT::BM * TT::PITCH;
#pragma unroll
    for (int i = 0; i < TT::A_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int m, k;
      if (AKC) { m = e / BK; k = e % BK; } else { k = e / TT::BM; m = e % TT::BM; }
      T* row = As + m * TT::PITCH;
      row[TT::kpos(2 * k)] = ra[i].x;
      row[TT::kpos(2 * k + 1)] = sgnA * ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < TT::B_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int k, n;
      if (BNC) { k = e / TT::BN; n = e % TT::BN; } else { n = e / BK; k = e % BK; }
      const T re = rb[i].x, im = sgnB * rb[i].y;
      T* c0 = Bs + (2 * n) * TT::PITCH;
      T* c1 = c0 + TT::PITCH;
      const int p0 = TT::kpos(2 * k), p1 = TT::kpos(2 * k + 1);
      c0[p0] = re;
      c0[p1] = -im;
      c1[p0] = im;
      c1[p1] = re;
    }
  };

  typename Mf::acc_t acc[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < Mf::NACC; ++r) acc[i][j][r] = T(0);

  const int nk = (kend - kbeg + BK - 1) / BK;
  load_tiles(kbeg);
  store_tiles(0);
  __syncthreads();

  const int arow = Mf::a_row(lane), ak = Mf::a_k(lane);
  using VecT = T __attribute__((ext_vector_type(TT::V)));
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles(kbeg + (kt + 1) * BK);
    const T* As = lds + cur * TT::LDS_ELEMS;
    const T* Bs = As + TT::BM * TT::PITCH;
#pragma unroll
    for (int kg = 0; kg < TT::KR; kg += TT::G) {
      VecT af[WR], bf[WC];
#pragma unroll
      for (int i = 0; i < WR; ++i)
        af[i] = *reinterpret_cast<const VecT*>(
            As + (wm * (WR * Mf::MT) + i * Mf::MT + arow) * TT::PITCH + kg + ak * TT::V);
#pragma unroll
      for (int j = 0; j < WC; ++j)
        bf[j] = *reinterpret_cast<const VecT*>(
            Bs + (wn * (WC * Mf::NT) + j * Mf::NT + arow) * TT::PITCH + kg + ak * TT::V);
#pragma unroll
      for (int q = 0; q < TT::V; ++q)
#pragma unroll
        for (int i = 0; i < WR; ++i)
#pragma unroll
          for (int j = 0; j < WC; ++j) acc[i][j] = Mf::mma(af[i][q], bf[j][q], acc[i][j]);
    }
    if (kt + 1 < nk) store_tiles(cur ^ 1);
    __syncthreads();
  }

  if (splits == 1) {
    TO* C = reinterpret_cast<TO*>(g.C);
    const long long cbase = (long long)bz * g.bC;
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < Mf::NACC; ++r) {
          const int row = m0 + wm * (WR * Mf::MT) + i * Mf::MT + Mf::out_row(lane, r);
          const int rcol = wn * (WC * Mf::NT) + j * Mf::NT + Mf::out_col(lane);
          const int col = n0 + (rcol >> 1);
          if (row < g.M && col < g.N)
            C[2 * (cbase + row * g.sCm + col * g.sCn) + (rcol & 1)] = TO(acc[i][j][r]);
        }
  } else {
    T* P = reinterpret_cast<T*>(part);
    const long long pbase = (long long)(sk * g.batch + bz) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < Mf::NACC; ++r) {
          const int row = m0 + wm * (WR * Mf::MT) + i * Mf::MT + Mf::out_row(lane, r);
          const int rcol = wn * (WC * Mf::NT) + j * Mf::NT + Mf::out_col(lane);
          const int col = n0 + (rcol >> 1);
          if (row < g.M && col < g.N)
            P[2 * (pbase + (long long)row * g.N + col) + (rcol & 1)] = acc[i][j][r];
        }
  }
}

// FP32 complex product with three real products per complex multiply-add (Gauss):
//   P1 = Re A Re B,  P2 = Im A Im B,  P3 = (Re A + Im A)(Re B + Im B),
//   Re C = P1 - P2,  Im C = P3 - P1 - P2,
// three v_mfma_f32_32x32x2f32 accumulators per 32 x 32 complex block instead of the four real
// products of the expanded form (the algorithmic count stays 8 flops per complex multiply-add).
// A and B are staged in LDS as two k-contiguous planes each (real and imaginary part; the sum the
// third product takes is formed in registers after the read), rows [m][k] and [n][k], in the
// consumption order of the fp32 instruction (kpos below), so that each lane fetches the operands
// of four instructions with one 16-byte read per plane. A workgroup of KW groups of WGM x 2 waves (each wave WR x WC blocks of
// 32 x 32 complex outputs) owns a BM x BN complex tile, double-buffered with one barrier per K
// step of BK; with KW > 1 the groups take equal slices of every step (two waves per SIMD, so that
// one wave's staging and barrier wait overlap the other's matrix instructions) and their partial
// sums meet in LDS at the end, in group order. Tiles: 128 x 128 (one group of 4 x 2 waves, each
// 32 x 64: half the operand traffic per flop of 128 x 64, for the large products of wide MPO
// bonds; eight waves of 96 accumulator registers leave room for two waves per SIMD, which hide
// each other's staging and barrier waits -- four waves of 64 x 64 held one per SIMD and ran the
// long-range one-site step 5 % slower), 128 x 64 (one group of 4 x 2 waves of 32 x 32, BK = 32,
// for the same reason), 64 x 64 (two groups), 32 x 64 (four groups of 1 x 2 waves, BK = 64: 256
// workgroups for a 256 x 2048 output without splitting K).
// Rounding: the sums carry one more rounding and Im C a difference of products, so its error
// bound is about twice that of the expanded form, normwise.
template <int WR, int WC, int BK_, int KW_, int WGM_>
struct Tile3 {
  static constexpr int BK = BK_;               // complex K per stage
  static constexpr int KW = KW_;               // wave groups along K
  static constexpr int WGM = WGM_;             // wave rows per group (2 wave columns)
  static constexpr int GT = 128 * WGM;         // threads per wave group
  static constexpr int NT = GT * KW;           // threads per workgroup
  static constexpr int BM = WGM * WR * 32;     // complex rows per workgroup
  static constexpr int BN = 2 * WC * 32;       // complex columns per workgroup
  static constexpr int V = 4, KT = 2, G = KT * V;
  static constexpr int KG = BK / KW;           // complex K per wave group and stage
  static constexpr int PITCH = BK + V;         // LDS row length (floats)
  static constexpr int A_ELEMS = BM * BK / NT;
  static constexpr int B_ELEMS = BN * BK / NT;
  static constexpr int PLANE_A = BM * PITCH, PLANE_B = BN * PITCH;
  static constexpr int STAGE = 2 * (PLANE_A + PLANE_B);  // real and imaginary planes
  static_assert(A_ELEMS >= 4 && B_ELEMS >= 4 && A_ELEMS % 4 == 0 && B_ELEMS % 4 == 0,
                "tile too small for the staging scheme");
  static_assert(BK % G == 0 && KG % G == 0 && ((PITCH * 4 / 16) & 1), "staging layout");
  static_assert(KW == 1 || 2 * KW * BM * BN <= 2 * STAGE, "LDS too small for the wave-group sum");
  static_assert(16 % KW == 0, "groups share out the accumulator entries");
  static_assert(NT <= 1024, "workgroup size");
  __device__ static int kpos(int k) {
    const int w = k % G;
    return k - w + (w % KT) * V + w / KT;
  }
};

// Tile of a workgroup when the grid is renumbered for the eight XCDs (each with its own L2), which
// take the workgroups in turn: XCD x runs the x-th contiguous run of tiles (x fastest, then y,
// then z), so the tiles sharing an operand row (or batch) meet in one L2 instead of eight.
__device__ inline void xcd_tile(int& bx, int& by, int& bz) {
  const unsigned gx = gridDim.x, gy = gridDim.y, total = gx * gy * gridDim.z;
  const unsigned id = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const unsigned xcd = id % 8u, k = id / 8u, q = total / 8u, r = total % 8u;
  const unsigned nid = xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
  bx = (int)(nid % gx);
  by = (int)((nid / gx) % gy);
  bz = (int)(nid / (gx * gy));
}

template <int WR, int WC, int BK, int KW, int WGM, typename TO, bool AKC, bool BNC, bool XCD = false>
__global__ __launch_bounds__(128 * WGM * KW) void cgemm3m_kernel(GemmDesc g, int splits,
                                                                 int kchunk, void* part) {
  using TT = Tile3<WR, WC, BK, KW, WGM>;
  using C2 = float2;
  __shared__ __attribute__((aligned(16))) float lds[2 * TT::STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wq = wave % (2 * WGM);  // wave within its group
  const int kw = wave / (2 * WGM);  // wave group: the K slice [kw KG, (kw+1) KG) of every stage
  const int wm = wq >> 1, wn = wq & 1;
  int tx = blockIdx.x, ty = blockIdx.y, tz = blockIdx.z;
  if (XCD) xcd_tile(tx, ty, tz);
  const int bz = tz / splits;
  const int sk = tz - bz * splits;
  const int kbeg = sk * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int m0 = ty * TT::BM;
  const int n0 = tx * TT::BN;

  const C2* A = reinterpret_cast<const C2*>(g.A) + bz * g.bA;
  const C2* B = reinterpret_cast<const C2*>(g.B) + bz * g.bB;
  const float sgnA = g.conjA ? -1.f : 1.f;
  const float sgnB = g.conjB ? -1.f : 1.f;

  // An operand whose LDS rows ([m][k] for A, [n][k] for B) are not contiguous in memory along k
  // (A with unit stride in m, B with unit stride in n) is staged in quads: a thread loads
  // k = kb, kb + 2, kb + 4, kb + 6 of one row (each load
  // coalesced across the lanes, which take consecutive rows) and writes them, adjacent in the
  // instruction order, with one 16-byte LDS store per plane (conflict-free: the row pitch is an
  // odd number of 16-byte units). A k-contiguous operand is staged element by element, the lanes
  // running along k.
  C2 ra[TT::A_ELEMS];
  C2 rb[TT::B_ELEMS];
  auto quad = [](int q, int rows, int& r, int& kb, int& pos) {
    r = q % rows;
    const int kk = q / rows;  // (group of 8 k, parity)
    kb = 8 * (kk >> 1) + (kk & 1);
    pos = 8 * (kk >> 1) + 4 * (kk & 1);
  };
  // Per-thread load addresses, set up once and advanced by one stage (BK k) per load_tiles call;
  // an element is loaded when its row is inside the matrix and its k below kend. Rows past the
  // edge address the last row (never read).
  const C2* pa[TT::A_ELEMS];
  const C2* pb[TT::B_ELEMS];
  int ka[TT::A_ELEMS], kb_[TT::B_ELEMS];
  bool va[TT::A_ELEMS], vb[TT::B_ELEMS];
#pragma unroll
  for (int i = 0; i < TT::A_ELEMS; ++i) {
    int m, k;
    if (AKC) {
      const int e = tid + i * TT::NT;
      m = e / BK; k = e % BK;
    } else {
      int kb, pos;
      quad(tid + (i / 4) * TT::NT, TT::BM, m, kb, pos);
      k = kb + 2 * (i % 4);
    }
    va[i] = m0 + m < g.M;
    ka[i] = k;
    pa[i] = A + (long long)min(m0 + m, g.M - 1) * g.sAm + (long long)(kbeg + k) * g.sAk;
  }
#pragma unroll
  for (int i = 0; i < TT::B_ELEMS; ++i) {
    int n, k;
    if (!BNC) {
      const int e = tid + i * TT::NT;
      n = e / BK; k = e % BK;
    } else {
      int kb, pos;
      quad(tid + (i / 4) * TT::NT, TT::BN, n, kb, pos);
      k = kb + 2 * (i % 4);
    }
    vb[i] = n0 + n < g.N;
    kb_[i] = k;
    pb[i] = B + (long long)(kbeg + k) * g.sBk + (long long)min(n0 + n, g.N - 1) * g.sBn;
  }
  const long long stepA = (long long)BK * g.sAk, stepB = (long long)BK * g.sBk;
  int krem = kend - kbeg;  // k left from the next stage to load on
  auto load_tiles = [&]() {
#pragma unroll
    for (int i = 0; i < TT::A_ELEMS; ++i) {
      C2 v{0.f, 0.f};
      if (va[i] && ka[i] < krem) v = *pa[i];
      ra[i] = v;
      pa[i] += stepA;
    }
#pragma unroll
    for (int i = 0; i < TT::B_ELEMS; ++i) {
      C2 v{0.f, 0.f};
      if (vb[i] && kb_[i] < krem) v = *pb[i];
      rb[i] = v;
      pb[i] += stepB;
    }
    krem -= BK;
  };
  using V4 = float __attribute__((ext_vector_type(4)));
  auto store_tiles = [&](int buf) {
    float* Ar = lds + buf * TT::STAGE;
    float* Ai = Ar + TT::PLANE_A;
    float* Br = Ai + TT::PLANE_A;
    float* Bi = Br + TT::PLANE_B;
    if (AKC) {
#pragma unroll
      for (int i = 0; i < TT::A_ELEMS; ++i) {
        const int e = tid + i * TT::NT;
        const int pp = (e / BK) * TT::PITCH + TT::kpos(e % BK);
        const float re = ra[i].x, im = sgnA * ra[i].y;
        Ar[pp] = re;
        Ai[pp] = im;
      }
    } else {
#pragma unroll
      for (int i = 0; i < TT::A_ELEMS / 4; ++i) {
        int m, kb, pos;
        quad(tid + i * TT::NT, TT::BM, m, kb, pos);
        const int pp = m * TT::PITCH + pos;
        V4 re, im;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          re[j] = ra[4 * i + j].x;
          im[j] = sgnA * ra[4 * i + j].y;
        }
        *reinterpret_cast<V4*>(Ar + pp) = re;
        *reinterpret_cast<V4*>(Ai + pp) = im;
      }
    }
    if (!BNC) {
#pragma unroll
      for (int i = 0; i < TT::B_ELEMS; ++i) {
        const int e = tid + i * TT::NT;
        const int pp = (e / BK) * TT::PITCH + TT::kpos(e % BK);
        const float re = rb[i].x, im = sgnB * rb[i].y;
        Br[pp] = re;
        Bi[pp] = im;
      }
    } else {
#pragma unroll
      for (int i = 0; i < TT::B_ELEMS / 4; ++i) {
        int n, kb, pos;
        quad(tid + i * TT::NT, TT::BN, n, kb, pos);
        const int pp = n * TT::PITCH + pos;
        V4 re, im;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          re[j] = rb[4 * i + j].x;
          im[j] = sgnB * rb[4 * i + j].y;
        }
        *reinterpret_cast<V4*>(Br + pp) = re;
        *reinterpret_cast<V4*>(Bi + pp) = im;
      }
    }
  };

  f32x16 p1[WR][WC], p2[WR][WC], p3[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) p1[i][j][r] = p2[i][j][r] = p3[i][j][r] = 0.f;

  // Software pipeline: the tile of stage kt + 1, loaded into registers during stage kt - 1, is
  // stored to the other LDS buffer at the top of stage kt, then the loads of stage kt + 2 are
  // issued, then stage kt's matrix instructions run; one barrier per stage.
  const int nk = (kend - kbeg + BK - 1) / BK;
  load_tiles();
  store_tiles(0);
  if (nk > 1) load_tiles();
  __syncthreads();

  const int arow = lane & 31, ak = lane >> 5;
  using VecT = float __attribute__((ext_vector_type(4)));
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      store_tiles(cur ^ 1);  // its readers finished at the previous barrier
      if (kt + 2 < nk) load_tiles();
    }
    const float* Ar = lds + cur * TT::STAGE;
    const float* Ai = Ar + TT::PLANE_A;
    const float* Br = Ai + TT::PLANE_A;
    const float* Bi = Br + TT::PLANE_B;
#pragma unroll
    for (int kg = kw * TT::KG; kg < (kw + 1) * TT::KG; kg += TT::G) {
      VecT ar_[WR], ai_[WR], as_[WR], br_[WC], bi_[WC], bs_[WC];
#pragma unroll
      for (int i = 0; i < WR; ++i) {
        const int o = (wm * (WR * 32) + i * 32 + arow) * TT::PITCH + kg + ak * TT::V;
        ar_[i] = *reinterpret_cast<const VecT*>(Ar + o);
        ai_[i] = *reinterpret_cast<const VecT*>(Ai + o);
        as_[i] = ar_[i] + ai_[i];  // the summed operand of the third product, formed in registers
      }
#pragma unroll
      for (int j = 0; j < WC; ++j) {
        const int o = (wn * (WC * 32) + j * 32 + arow) * TT::PITCH + kg + ak * TT::V;
        br_[j] = *reinterpret_cast<const VecT*>(Br + o);
        bi_[j] = *reinterpret_cast<const VecT*>(Bi + o);
        bs_[j] = br_[j] + bi_[j];
      }
      // a wave issuing its matrix instructions goes first (the other wave on the SIMD is then
      // staging or reading fragments): 1 % on the long-range one-site step, 3 % on its
      // environment update
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int q = 0; q < TT::V; ++q)
#pragma unroll
        for (int i = 0; i < WR; ++i)
#pragma unroll
          for (int j = 0; j < WC; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar_[i][q], br_[j][q], p1[i][j], 0, 0, 0);
            p2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai_[i][q], bi_[j][q], p2[i][j], 0, 0, 0);
            p3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(as_[i][q], bs_[j][q], p3[i][j], 0, 0, 0);
          }
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
  }

  // KW > 1: every wave group stores its partial (Re C, Im C) to LDS (the stage buffers are free
  // after the last barrier of the K loop); group h then finishes the accumulator entries
  // r in [h 16 / KW, (h + 1) 16 / KW) of every block, summing the groups' partials in group order,
  // so the global stores are spread over all waves.
  constexpr int NR = WR * WC * 16;  // partial values per lane
  const float2* red = reinterpret_cast<const float2*>(lds);
  const int slot = wq * 64 + lane;
  if (KW > 1) {
    float2* wr = reinterpret_cast<float2*>(lds);
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float a = p1[i][j][r], b = p2[i][j][r];
          wr[(kw * NR + (i * WC + j) * 16 + r) * TT::GT + slot] = float2{a - b, p3[i][j][r] - a - b};
        }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (KW > 1 && r / (16 / KW) != kw) continue;
        const int row = m0 + wm * (WR * 32) + i * 32 + MfmaF32::out_row(lane, r);
        const int col = n0 + wn * (WC * 32) + j * 32 + MfmaF32::out_col(lane);
        if (row >= g.M || col >= g.N) continue;
        float re, im;
        if (KW == 1) {
          const float a = p1[i][j][r], b = p2[i][j][r];
          re = a - b;
          im = p3[i][j][r] - a - b;
        } else {
          const float2 o = red[((i * WC + j) * 16 + r) * TT::GT + slot];
          re = o.x;
          im = o.y;
#pragma unroll
          for (int h = 1; h < KW; ++h) {
            const float2 v = red[(h * NR + (i * WC + j) * 16 + r) * TT::GT + slot];
            re += v.x;
            im += v.y;
          }
        }
        if (splits == 1) {
          TO* C = reinterpret_cast<TO*>(g.C);
          const long long o = (long long)bz * g.bC + (long long)row * g.sCm + (long long)col * g.sCn;
          C[2 * o] = TO(re);
          C[2 * o + 1] = TO(im);
        } else {
          float* P = reinterpret_cast<float*>(part);
          const long long o = (long long)(sk * g.batch + bz) * g.M * g.N + (long long)row * g.N + col;
          P[2 * o] = re;
          P[2 * o + 1] = im;
        }
      }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__device__ inline unsigned pack_bf16(__bf16 a, __bf16 b) {
  return (unsigned)__builtin_bit_cast(unsigned short, a) |
         ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}

template <int WR, int WC, int BK, typename TO, bool AKC, bool BNC>
__global__ __launch_bounds__(kThreads) void cgemm_bf16x3_kernel(GemmDesc g, int splits, int kchunk,
                                                                void* part) {
  using C2 = float2;
  using Mf = MfmaF32;  // output layout of the 32 x 32 instructions
  constexpr int BM = 2 * WR * 32, BNR = 2 * WC * 32, BN = BNR / 2;
  constexpr int KR = 2 * BK;     // real k per stage, a multiple of 16
  constexpr int PITCH = KR + 8;  // bf16 per LDS row: 16-byte aligned rows, shifted banks
  constexpr int A_ELEMS = BM * BK / kThreads, B_ELEMS = BN * BK / kThreads;
  constexpr int A_PLANE = BM * PITCH, B_PLANE = BNR * PITCH;
  constexpr int STAGE = 2 * A_PLANE + 2 * B_PLANE;  // hi and lo planes of A and B
  static_assert(KR % 16 == 0 && A_ELEMS >= 1 && B_ELEMS >= 1, "bf16x3 tile");
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int bz = blockIdx.z / splits;
  const int sk = blockIdx.z - bz * splits;
  const int kbeg = sk * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int m0 = blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;
  const C2* A = reinterpret_cast<const C2*>(g.A) + bz * g.bA;
  const C2* B = reinterpret_cast<const C2*>(g.B) + bz * g.bB;
  const float sgnA = g.conjA ? -1.f : 1.f;
  const float sgnB = g.conjB ? -1.f : 1.f;

  // Staging: a thread takes single elements, or, for an operand whose LDS rows are not
  // contiguous in memory along k (A with unit stride in m, B with unit stride in n) and that gives
  // every thread a multiple of 4 elements, quads of consecutive k of one row (each load coalesced
  // across the lanes, which take consecutive rows), stored with 16-byte LDS writes (the four
  // complex values are 8 adjacent bf16 of a row). Load addresses are set up once and advanced by
  // one stage per load_tiles call; a row past the edge addresses the last row (never read).
  constexpr bool QA = !AKC && A_ELEMS % 4 == 0;
  constexpr bool QB = BNC && B_ELEMS % 4 == 0;
  C2 ra[A_ELEMS];
  C2 rb[B_ELEMS];
  const C2* pa[A_ELEMS];
  const C2* pb[B_ELEMS];
  int ka[A_ELEMS], kbv[B_ELEMS];
  bool va[A_ELEMS], vb[B_ELEMS];
  auto a_pos = [&](int i, int& m, int& k) {  // row and k of A element i of this thread
    if (QA) {
      const int q = tid + (i / 4) * kThreads;
      m = q % BM; k = 4 * (q / BM) + i % 4;
    } else {
      const int e = tid + i * kThreads;
      if (AKC) { m = e / BK; k = e % BK; } else { k = e / BM; m = e % BM; }
    }
  };
  auto b_pos = [&](int i, int& n, int& k) {
    if (QB) {
      const int q = tid + (i / 4) * kThreads;
      n = q % BN; k = 4 * (q / BN) + i % 4;
    } else {
      const int e = tid + i * kThreads;
      if (BNC) { k = e / BN; n = e % BN; } else { n = e / BK; k = e % BK; }
    }
  };
#pragma unroll
  for (int i = 0; i < A_ELEMS; ++i) {
    int m, k;
    a_pos(i, m, k);
    va[i] = m0 + m < g.M;
    ka[i] = k;
    pa[i] = A + (long long)min(m0 + m, g.M - 1) * g.sAm + (long long)(kbeg + k) * g.sAk;
  }
#pragma unroll
  for (int i = 0; i < B_ELEMS; ++i) {
    int n, k;
    b_pos(i, n, k);
    vb[i] = n0 + n < g.N;
    kbv[i] = k;
    pb[i] = B + (long long)(kbeg + k) * g.sBk + (long long)min(n0 + n, g.N - 1) * g.sBn;
  }
  const long long stepA = (long long)BK * g.sAk, stepB = (long long)BK * g.sBk;
  int krem = kend - kbeg;
  auto load_tiles = [&]() {
#pragma unroll
    for (int i = 0; i < A_ELEMS; ++i) {
      C2 v{0.f, 0.f};
      if (va[i] && ka[i] < krem) v = *pa[i];
      ra[i] = v;
      pa[i] += stepA;
    }
#pragma unroll
    for (int i = 0; i < B_ELEMS; ++i) {
      C2 v{0.f, 0.f};
      if (vb[i] && kbv[i] < krem) v = *pb[i];
      rb[i] = v;
      pb[i] += stepB;
    }
    krem -= BK;
  };
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  auto store_tiles = [&](int buf) {
    __bf16* Ah = lds + buf * STAGE;
    __bf16* Al = Ah + A_PLANE;
    __bf16* Bh = Al + A_PLANE;
    __bf16* Bl = Bh + B_PLANE;
    if (QA) {
#pragma unroll
      for (int i = 0; i < A_ELEMS; i += 4) {
        int m, k;
        a_pos(i, m, k);
        u32x4 hv, lv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          __bf16 h0, l0, h1, l1;
          split_bf16(ra[i + j].x, h0, l0);
          split_bf16(sgnA * ra[i + j].y, h1, l1);
          hv[j] = pack_bf16(h0, h1);
          lv[j] = pack_bf16(l0, l1);
        }
        *reinterpret_cast<u32x4*>(Ah + m * PITCH + 2 * k) = hv;
        *reinterpret_cast<u32x4*>(Al + m * PITCH + 2 * k) = lv;
      }
    } else {
#pragma unroll
      for (int i = 0; i < A_ELEMS; ++i) {
        int m, k;
        a_pos(i, m, k);
        __bf16 h0, l0, h1, l1;
        split_bf16(ra[i].x, h0, l0);
        split_bf16(sgnA * ra[i].y, h1, l1);
        *reinterpret_cast<unsigned*>(Ah + m * PITCH + 2 * k) = pack_bf16(h0, h1);
        *reinterpret_cast<unsigned*>(Al + m * PITCH + 2 * k) = pack_bf16(l0, l1);
      }
    }
    // real column 2n: (re, -im) at k' = 2k, 2k+1; real column 2n+1: (im, re)
    if (QB) {
#pragma unroll
      for (int i = 0; i < B_ELEMS; i += 4) {
        int n, k;
        b_pos(i, n, k);
        u32x4 h0v, l0v, h1v, l1v;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          __bf16 hr, lr, hi_, li;
          split_bf16(rb[i + j].x, hr, lr);
          split_bf16(sgnB * rb[i + j].y, hi_, li);
          h0v[j] = pack_bf16(hr, -hi_);
          l0v[j] = pack_bf16(lr, -li);
          h1v[j] = pack_bf16(hi_, hr);
          l1v[j] = pack_bf16(li, lr);
        }
        *reinterpret_cast<u32x4*>(Bh + (2 * n) * PITCH + 2 * k) = h0v;
        *reinterpret_cast<u32x4*>(Bl + (2 * n) * PITCH + 2 * k) = l0v;
        *reinterpret_cast<u32x4*>(Bh + (2 * n + 1) * PITCH + 2 * k) = h1v;
        *reinterpret_cast<u32x4*>(Bl + (2 * n + 1) * PITCH + 2 * k) = l1v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < B_ELEMS; ++i) {
        int n, k;
        b_pos(i, n, k);
        __bf16 hr, lr, hi_, li;
        split_bf16(rb[i].x, hr, lr);
        split_bf16(sgnB * rb[i].y, hi_, li);
        *reinterpret_cast<unsigned*>(Bh + (2 * n) * PITCH + 2 * k) = pack_bf16(hr, -hi_);
        *reinterpret_cast<unsigned*>(Bl + (2 * n) * PITCH + 2 * k) = pack_bf16(lr, -li);
        *reinterpret_cast<unsigned*>(Bh + (2 * n + 1) * PITCH + 2 * k) = pack_bf16(hi_, hr);
        *reinterpret_cast<unsigned*>(Bl + (2 * n + 1) * PITCH + 2 * k) = pack_bf16(li, lr);
      }
    }
  };

  f32x16 acc[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // software pipeline as in the three-product kernel: the tile of stage kt + 1 (in registers
  // since stage kt - 1) is stored at the top of stage kt, then stage kt + 2 is loaded
  const int nk = (kend - kbeg + BK - 1) / BK;
  load_tiles();
  store_tiles(0);
  if (nk > 1) load_tiles();
  __syncthreads();
  const int lrow = lane & 31, lk = 8 * (lane >> 5);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      store_tiles(cur ^ 1);
      if (kt + 2 < nk) load_tiles();
    }
    const __bf16* Ah = lds + cur * STAGE;
    const __bf16* Al = Ah + A_PLANE;
    const __bf16* Bh = Al + A_PLANE;
    const __bf16* Bl = Bh + B_PLANE;
#pragma unroll
    for (int ks = 0; ks < KR; ks += 16) {
      bf16x8 ah[WR], al[WR], bh[WC], bl[WC];
#pragma unroll
      for (int i = 0; i < WR; ++i) {
        const int off = (wm * (WR * 32) + i * 32 + lrow) * PITCH + ks + lk;
        ah[i] = *reinterpret_cast<const bf16x8*>(Ah + off);
        al[i] = *reinterpret_cast<const bf16x8*>(Al + off);
      }
#pragma unroll
      for (int j = 0; j < WC; ++j) {
        const int off = (wn * (WC * 32) + j * 32 + lrow) * PITCH + ks + lk;
        bh[j] = *reinterpret_cast<const bf16x8*>(Bh + off);
        bl[j] = *reinterpret_cast<const bf16x8*>(Bl + off);
      }
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WC; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }

  if (splits == 1) {
    TO* C = reinterpret_cast<TO*>(g.C);
    const long long cbase = (long long)bz * g.bC;
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = m0 + wm * (WR * 32) + i * 32 + Mf::out_row(lane, r);
          const int rcol = wn * (WC * 32) + j * 32 + Mf::out_col(lane);
          const int col = n0 + (rcol >> 1);
          if (row < g.M && col < g.N)
            C[2 * (cbase + row * g.sCm + col * g.sCn) + (rcol & 1)] = TO(acc[i][j][r]);
        }
  } else {
    float* P = reinterpret_cast<float*>(part);
    const long long pbase = (long long)(sk * g.batch + bz) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = m0 + wm * (WR * 32) + i * 32 + Mf::out_row(lane, r);
          const int rcol = wn * (WC * 32) + j * 32 + Mf::out_col(lane);
          const int col = n0 + (rcol >> 1);
          if (row < g.M && col < g.N)
            P[2 * (pbase + (long long)row * g.N + col) + (rcol & 1)] = acc[i][j][r];
        }
  }
}

// C[b][m][n] = sum over s = 0..splits-1 (in that order) of part[s][b][m][n].
template <typename T, typename TO>
__global__ void splitk_reduce(GemmDesc g, int splits, const T* __restrict__ part) {
  using C2 = cx_t<T>;
  using CO = cx_t<TO>;
  const long long mn = (long long)g.M * g.N;
  const long long total = mn * g.batch;
  const C2* pc = reinterpret_cast<const C2*>(part);
  CO* C = reinterpret_cast<CO*>(g.C);
  // a row-major output packed like the partial tiles needs no index arithmetic (no 64-bit
  // divisions, which would set the pace here)
  const bool packed = g.sCn == 1 && g.sCm == g.N && (g.batch == 1 || g.bC == mn);
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    C2 acc{T(0), T(0)};
    for (int s = 0; s < splits; ++s) {  // one complex load per split
      const C2 v = pc[s * total + idx];
      acc.x += v.x;
      acc.y += v.y;
    }
    long long o = idx;
    if (!packed) {
      const long long b = idx / mn, rem = idx - b * mn;
      const long long row = rem / g.N, col = rem - row * g.N;
      o = b * g.bC + row * g.sCm + col * g.sCn;
    }
    C[o] = CO{TO(acc.x), TO(acc.y)};
  }
}

struct Plan {
  int cfg;     // index into the precision's tile table
  int bm, bn;  // complex tile
  int splits, kchunk;
};

template <class Mf>
Plan make_plan(const GemmDesc& g, const int (*cfgs)[2], int ncfg) {
  auto tiles = [&](int c) {
    return (long long)((g.M + cfgs[c][0] - 1) / cfgs[c][0]) * ((g.N + cfgs[c][1] - 1) / cfgs[c][1]) * g.batch;
  };
  Plan p{ncfg - 1, cfgs[ncfg - 1][0], cfgs[ncfg - 1][1], 1, g.K};
  if (g.row_tail) {  // the smallest tile rows that hold M (the table lists tiles by falling rows)
    for (int c = ncfg - 1; c >= 0; --c)
      if (cfgs[c][0] >= g.M) {
        p.cfg = c; p.bm = cfgs[c][0]; p.bn = cfgs[c][1];
        return p;
      }
    return p;
  }
  for (int c = 0; c < ncfg; ++c)
    if (tiles(c) >= kMinWgs && cfgs[c][1] <= std::max(g.N, 64)) {  // no tile twice as wide as C
      p.cfg = c; p.bm = cfgs[c][0]; p.bn = cfgs[c][1];
      return p;
    }
  if (!g.ws || tiles(p.cfg) >= kTargetWgs) return p;
  // split K: the largest tile whose splits (at most kMaxSplits, of at least kMinSplitK each, their
  // partial tiles within the scratch) bring the workgroups to kTargetWgs, else the smallest tile
  // with as many splits as allowed
  const size_t per = sizeof(typename Mf::T) * 2 * (size_t)g.M * g.N * g.batch;
  const int smax = (int)std::min<size_t>({(size_t)kMaxSplits, (size_t)std::max(g.K / kMinSplitK, 1),
                                          per ? g.ws_bytes / per : 0});
  int s = 0;
  for (int c = 0; c < ncfg && s == 0; ++c) {
    if (cfgs[c][1] > std::max(g.N, 64)) continue;
    const long long t = tiles(c);
    const long long need = (kTargetWgs + t - 1) / t;
    if (need <= smax) {
      p.cfg = c; p.bm = cfgs[c][0]; p.bn = cfgs[c][1];
      s = (int)need;
    }
  }
  if (s == 0) s = std::min<int>(smax, (int)((kTargetWgs + tiles(p.cfg) - 1) / tiles(p.cfg)));
  if (s < 2) return p;
  const int kc = ((g.K + s - 1) / s + kKGrain - 1) / kKGrain * kKGrain;
  p.kchunk = kc;
  p.splits = (g.K + kc - 1) / kc;
  return p;
}

constexpr int kF32Cfg[3][2] = {{128, 64}, {64, 64}, {64, 32}};  // split-BF16x3 tiles
constexpr int kF64Cfg[2][2] = {{64, 64}, {32, 32}};

template <class Mf, int WR, int WC, int BK, typename TO>
hipError_t launch_cfg(const GemmDesc& g, const Plan& pl, hipStream_t st) {
  using TT = Tile<Mf, WR, WC, BK>;
  dim3 grid((g.N + TT::BN - 1) / TT::BN, (g.M + TT::BM - 1) / TT::BM, g.batch * pl.splits);
  const bool akc = (g.sAk == 1) || (g.K == 1);
  const bool bnc = (g.sBn == 1) || (g.N == 1);
  void* part = pl.splits > 1 ? g.ws : nullptr;
  if (akc && bnc)
    hipLaunchKernelGGL((cgemm_kernel<Mf, WR, WC, BK, TO, true, true>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  else if (akc)
    hipLaunchKernelGGL((cgemm_kernel<Mf, WR, WC, BK, TO, true, false>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  else if (bnc)
    hipLaunchKernelGGL((cgemm_kernel<Mf, WR, WC, BK, TO, false, true>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  else
    hipLaunchKernelGGL((cgemm_kernel<Mf, WR, WC, BK, TO, false, false>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  {
    const void* k = nullptr;
    if (akc && bnc) k = reinterpret_cast<const void*>(cgemm_kernel<Mf, WR, WC, BK, TO, true, true>);
    else if (akc) k = reinterpret_cast<const void*>(cgemm_kernel<Mf, WR, WC, BK, TO, true, false>);
    else if (bnc) k = reinterpret_cast<const void*>(cgemm_kernel<Mf, WR, WC, BK, TO, false, true>);
    else k = reinterpret_cast<const void*>(cgemm_kernel<Mf, WR, WC, BK, TO, false, false>);
    last_launch() = LaunchRecord{k, pl.splits > 1};
  }
  MPOEVO_HIP_TRY(hipGetLastError());
  if (pl.splits > 1) {
    using T = typename Mf::T;
    const long long total = (long long)g.M * g.N * g.batch;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((splitk_reduce<T, TO>), dim3(blocks), dim3(256), 0, st, g, pl.splits,
                       static_cast<const T*>(g.ws));
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

constexpr int k3mCfg[4][2] = {{128, 128}, {128, 64}, {64, 64}, {32, 64}};

template <int WR, int WC, int BK, int KW, int WGM, typename TO, bool XCD = false>
hipError_t launch_3m_cfg(const GemmDesc& g, const Plan& pl, hipStream_t st) {
  using TT = Tile3<WR, WC, BK, KW, WGM>;
  dim3 grid((g.N + TT::BN - 1) / TT::BN, (g.M + TT::BM - 1) / TT::BM, g.batch * pl.splits);
  const bool akc = (g.sAk == 1) || (g.K == 1);
  const bool bnc = (g.sBn == 1) || (g.N == 1);
  void* part = pl.splits > 1 ? g.ws : nullptr;
  if (akc && bnc)
    hipLaunchKernelGGL((cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, true, true, XCD>), grid, dim3(TT::NT), 0, st, g, pl.splits, pl.kchunk, part);
  else if (akc)
    hipLaunchKernelGGL((cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, true, false, XCD>), grid, dim3(TT::NT), 0, st, g, pl.splits, pl.kchunk, part);
  else if (bnc)
    hipLaunchKernelGGL((cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, false, true, XCD>), grid, dim3(TT::NT), 0, st, g, pl.splits, pl.kchunk, part);
  else
    hipLaunchKernelGGL((cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, false, false, XCD>), grid, dim3(TT::NT), 0, st, g, pl.splits, pl.kchunk, part);
  {
    const void* k = nullptr;
    if (akc && bnc) k = reinterpret_cast<const void*>(cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, true, true, XCD>);
    else if (akc) k = reinterpret_cast<const void*>(cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, true, false, XCD>);
    else if (bnc) k = reinterpret_cast<const void*>(cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, false, true, XCD>);
    else k = reinterpret_cast<const void*>(cgemm3m_kernel<WR, WC, BK, KW, WGM, TO, false, false, XCD>);
    last_launch() = LaunchRecord{k, pl.splits > 1};
  }
  MPOEVO_HIP_TRY(hipGetLastError());
  if (pl.splits > 1) {
    const long long total = (long long)g.M * g.N * g.batch;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((splitk_reduce<float, TO>), dim3(blocks), dim3(256), 0, st, g, pl.splits,
                       static_cast<const float*>(part));
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

template <int WR, int WC, int BK, typename TO>
hipError_t launch_bf16x3_cfg(const GemmDesc& g, const Plan& pl, hipStream_t st) {
  constexpr int BM = 2 * WR * 32, BN = WC * 32;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.batch * pl.splits);
  const bool akc = (g.sAk == 1) || (g.K == 1);
  const bool bnc = (g.sBn == 1) || (g.N == 1);
  void* part = pl.splits > 1 ? g.ws : nullptr;
  if (akc && bnc)
    hipLaunchKernelGGL((cgemm_bf16x3_kernel<WR, WC, BK, TO, true, true>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  else if (akc)
    hipLaunchKernelGGL((cgemm_bf16x3_kernel<WR, WC, BK, TO, true, false>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  else if (bnc)
    hipLaunchKernelGGL((cgemm_bf16x3_kernel<WR, WC, BK, TO, false, true>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  else
    hipLaunchKernelGGL((cgemm_bf16x3_kernel<WR, WC, BK, TO, false, false>), grid, dim3(kThreads), 0, st, g, pl.splits, pl.kchunk, part);
  {
    const void* k = nullptr;
    if (akc && bnc) k = reinterpret_cast<const void*>(cgemm_bf16x3_kernel<WR, WC, BK, TO, true, true>);
    else if (akc) k = reinterpret_cast<const void*>(cgemm_bf16x3_kernel<WR, WC, BK, TO, true, false>);
    else if (bnc) k = reinterpret_cast<const void*>(cgemm_bf16x3_kernel<WR, WC, BK, TO, false, true>);
    else k = reinterpret_cast<const void*>(cgemm_bf16x3_kernel<WR, WC, BK, TO, false, false>);
    last_launch() = LaunchRecord{k, pl.splits > 1};
  }
  MPOEVO_HIP_TRY(hipGetLastError());
  if (pl.splits > 1) {
    const long long total = (long long)g.M * g.N * g.batch;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((splitk_reduce<float, TO>), dim3(blocks), dim3(256), 0, st, g, pl.splits,
                       static_cast<const float*>(g.ws));
    MPOEVO_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

// ------------------------------------------------------------------------------ tile tuner
// The fixed rule above (largest tile with a workgroup per compute unit, else split K) is the
// default. A handle can instead time the candidate plans of each product shape the first time
// it meets it (every tile of the precision's table, unsplit and with the rule's split count) and
// keep the fastest for every later product of that shape.
enum Kind : int { kKind3m = 0, kKindBf16x3 = 1, kKindF64 = 2 };

struct TuneKey {
  int kind, out64, akc, bnc, M, N, K, batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(kind, out64, akc, bnc, M, N, K, batch) <
           std::tie(o.kind, o.out64, o.akc, o.bnc, o.M, o.N, o.K, o.batch);
  }
};

struct Tuner {
  std::mutex mu;
  int mode = MPOEVO_TUNE_OFF;
  std::map<TuneKey, Plan> table;
  unsigned long long generation = 0;  // bumped when the mode changes or the table is cleared
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~Tuner() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

thread_local Tuner* t_tuner = nullptr;
thread_local bool t_tune_allowed = false;

template <class Mf>
std::vector<Plan> candidate_plans(const GemmDesc& g, const int (*cfgs)[2], int ncfg) {
  std::vector<Plan> out;
  for (int c = 0; c < ncfg; ++c) {
    const long long t = (long long)((g.M + cfgs[c][0] - 1) / cfgs[c][0]) *
                        ((g.N + cfgs[c][1] - 1) / cfgs[c][1]) * g.batch;
    out.push_back(Plan{c, cfgs[c][0], cfgs[c][1], 1, g.K});
    if (!g.ws || t >= kTargetWgs) continue;
    int s = (int)std::min<long long>((kTargetWgs + t - 1) / t, kMaxSplits);
    s = std::min(s, g.K / kMinSplitK);
    const size_t per = sizeof(typename Mf::T) * 2 * (size_t)g.M * g.N * g.batch;
    s = (int)std::min<size_t>((size_t)s, per ? g.ws_bytes / per : 0);
    if (s < 2) continue;
    const int kc = ((g.K + s - 1) / s + kKGrain - 1) / kKGrain * kKGrain;
    out.push_back(Plan{c, cfgs[c][0], cfgs[c][1], (g.K + kc - 1) / kc, kc});
  }
  return out;
}

TuneKey key_of(const GemmDesc& g, int kind, bool out64) {
  return TuneKey{kind, out64 ? 1 : 0, (g.sAk == 1 || g.K == 1) ? 1 : 0, (g.sBn == 1 || g.N == 1) ? 1 : 0,
                 g.M, g.N, g.K, g.batch};
}

// The plan a product takes: the tuned one, a freshly tuned one (tuning allowed, stream not being
// captured), or the rule.
template <class Mf, class Run>
hipError_t plan_and_run(const GemmDesc& g, const int (*cfgs)[2], int ncfg, int kind, bool out64,
                        hipStream_t st, Run run) {
  const Plan rule = make_plan<Mf>(g, cfgs, ncfg);
  Tuner* t = t_tuner;
  if (!t) return run(g, rule, st);
  const TuneKey key = key_of(g, kind, out64);
  {
    std::lock_guard<std::mutex> lk(t->mu);
    if (t->mode == MPOEVO_TUNE_OFF) return run(g, rule, st);
    auto it = t->table.find(key);
    if (it != t->table.end()) return run(g, it->second, st);
    if (t->mode != MPOEVO_TUNE_ON || !t_tune_allowed) return run(g, rule, st);
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  MPOEVO_HIP_TRY(hipStreamIsCapturing(st, &cap));
  if (cap != hipStreamCaptureStatusNone) return run(g, rule, st);
  std::lock_guard<std::mutex> lk(t->mu);
  for (hipEvent_t& e : t->ev)
    if (!e) MPOEVO_HIP_TRY(hipEventCreate(&e));
  MPOEVO_HIP_TRY(hipStreamSynchronize(st));
  Plan best = rule;
  float best_ms = 0.f;
  bool have = false;
  for (const Plan& p : candidate_plans<Mf>(g, cfgs, ncfg)) {
    MPOEVO_HIP_TRY(run(g, p, st));  // warm-up (and instruction cache)
    MPOEVO_HIP_TRY(hipEventRecord(t->ev[0], st));
    for (int r = 0; r < 3; ++r) MPOEVO_HIP_TRY(run(g, p, st));
    MPOEVO_HIP_TRY(hipEventRecord(t->ev[1], st));
    MPOEVO_HIP_TRY(hipEventSynchronize(t->ev[1]));
    float ms = 0.f;
    MPOEVO_HIP_TRY(hipEventElapsedTime(&ms, t->ev[0], t->ev[1]));
    if (!have || ms < best_ms) { best = p; best_ms = ms; have = true; }
  }
  t->table[key] = best;
  return run(g, best, st);  // the output of the kept plan
}

template <typename TO>
hipError_t run_3m(const GemmDesc& g, const Plan& pl, hipStream_t st) {
  if (pl.cfg == 0) return launch_3m_cfg<1, 2, 16, 1, 4, TO, true>(g, pl, st);
  if (pl.cfg == 1) return launch_3m_cfg<1, 1, 32, 1, 4, TO>(g, pl, st);
  if (pl.cfg == 2) return launch_3m_cfg<1, 1, 32, 2, 2, TO>(g, pl, st);
  return launch_3m_cfg<1, 1, 64, 4, 1, TO>(g, pl, st);
}

template <typename TO>
hipError_t run_bf16x3(const GemmDesc& g, const Plan& pl, hipStream_t st) {
  switch (pl.cfg) {
    case 0: return launch_bf16x3_cfg<2, 2, 16, TO>(g, pl, st);
    case 1: return launch_bf16x3_cfg<1, 2, 16, TO>(g, pl, st);
    default: return launch_bf16x3_cfg<1, 1, 16, TO>(g, pl, st);
  }
}

hipError_t run_f64(const GemmDesc& g, const Plan& pl, hipStream_t st) {
  if (pl.cfg == 0) return launch_cfg<MfmaF64, 2, 4, 8, double>(g, pl, st);
  return launch_cfg<MfmaF64, 1, 2, 16, double>(g, pl, st);
}

}  // namespace

void* gemm_tuner_new() { return new (std::nothrow) Tuner(); }
void gemm_tuner_free(void* t) { delete static_cast<Tuner*>(t); }

int gemm_tuner_mode(void* t, int set) {
  auto* tu = static_cast<Tuner*>(t);
  std::lock_guard<std::mutex> lk(tu->mu);
  if (set >= 0 && set != tu->mode) {
    tu->mode = set;
    ++tu->generation;
  }
  return tu->mode;
}

unsigned long long gemm_tuner_generation(void* t) {
  auto* tu = static_cast<Tuner*>(t);
  std::lock_guard<std::mutex> lk(tu->mu);
  return tu->generation;
}

size_t gemm_tuner_entries(void* t) {
  auto* tu = static_cast<Tuner*>(t);
  std::lock_guard<std::mutex> lk(tu->mu);
  return tu->table.size();
}

void gemm_tuner_clear(void* t) {
  auto* tu = static_cast<Tuner*>(t);
  std::lock_guard<std::mutex> lk(tu->mu);
  tu->table.clear();
  ++tu->generation;
}

TunerScope::TunerScope(void* t, bool allow) : prev_(t_tuner), prev_allow_(t_tune_allowed) {
  t_tuner = static_cast<Tuner*>(t);
  t_tune_allowed = allow;
}
TunerScope::~TunerScope() {
  t_tuner = static_cast<Tuner*>(prev_);
  t_tune_allowed = prev_allow_;
}

int gemm_plan_query(void* t, int prec, int M, int N, int K, int batch, int* out) {
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.sAk = 1; g.sBn = 1;
  static char sentinel;
  g.ws = &sentinel;  // the split-K scratch of every caller
  g.ws_bytes = kGemmScratchBytes;
  Plan p{};
  int kind = 0;
  if (prec == MPOEVO_FP64) { p = make_plan<MfmaF64>(g, kF64Cfg, 2); kind = kKindF64; }
  else if (prec == MPOEVO_BF16X3) { p = make_plan<MfmaF32>(g, kF32Cfg, 3); kind = kKindBf16x3; }
  else { p = make_plan<MfmaF32>(g, k3mCfg, 4); kind = kKind3m; }
  int tuned = 0;
  if (t) {
    auto* tu = static_cast<Tuner*>(t);
    std::lock_guard<std::mutex> lk(tu->mu);
    for (int o64 = 0; o64 < 2 && !tuned; ++o64) {
      auto it = tu->table.find(key_of(g, kind, o64 != 0));
      if (tu->mode != MPOEVO_TUNE_OFF && it != tu->table.end()) { p = it->second; tuned = 1; }
    }
  }
  out[0] = p.bm; out[1] = p.bn; out[2] = p.splits; out[3] = tuned;
  return 0;
}

int gemm_row_tail(const GemmDesc& g, bool fp64) {
  if (fp64 || g.bf16x3 || g.row_tail || g.M <= 0 || g.N <= 0 || g.batch <= 0) return 0;
  const Plan p = make_plan<MfmaF32>(g, k3mCfg, 4);
  const int rem = g.M % p.bm;
  const int tail_rows = rem <= 32 ? 32 : 64;  // the tile the rows past the whole blocks would take
  return (g.M > p.bm && rem > 0 && 2 * rem <= p.bm && rem <= 64 && tail_rows < p.bm) ? rem : 0;
}

void gemm_round_tail(const GemmDesc& g, bool fp64, int& dim, long long& at) {
  dim = 0;
  at = 0;
  if (fp64 || g.bf16x3 || g.row_tail || g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  const Plan p = make_plan<MfmaF32>(g, k3mCfg, 4);
  if (p.splits != 1) return;
  const long long tm = (g.M + p.bm - 1) / p.bm, tn = (g.N + p.bn - 1) / p.bn;
  const long long t = tm * tn * g.batch, r = t % kMinWgs;
  if (t <= kMinWgs || r == 0 || 2 * r > kMinWgs) return;
  // the cut removes exactly the r tiles of the last round: whole batch entries, else whole
  // column blocks of every entry, else whole row blocks
  if (g.batch > 1 && r % (tm * tn) == 0) {
    dim = 3;
    at = g.batch - r / (tm * tn);
  } else if (r % (tm * g.batch) == 0 && r / (tm * g.batch) < tn) {
    dim = 2;
    at = (tn - r / (tm * g.batch)) * p.bn;
  } else if (r % (tn * g.batch) == 0 && r / (tn * g.batch) < tm) {
    dim = 1;
    at = (tm - r / (tn * g.batch)) * p.bm;
  }
}

hipError_t gemm_launch(const GemmDesc& g, bool fp64, bool out_fp64, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  if (fp64) return plan_and_run<MfmaF64>(g, kF64Cfg, 2, kKindF64, true, st, run_f64);
  if (g.bf16x3)
    return out_fp64 ? plan_and_run<MfmaF32>(g, kF32Cfg, 3, kKindBf16x3, true, st, run_bf16x3<double>)
                    : plan_and_run<MfmaF32>(g, kF32Cfg, 3, kKindBf16x3, false, st, run_bf16x3<float>);
  return out_fp64 ? plan_and_run<MfmaF32>(g, k3mCfg, 4, kKind3m, true, st, run_3m<double>)
                  : plan_and_run<MfmaF32>(g, k3mCfg, 4, kKind3m, false, st, run_3m<float>);
}

}  // namespace mpoevo
