// Complex strided-batched matrix products on the gfx950 matrix cores.
//
// A complex product C = A B (M x N x K complex multiply-adds) is computed as the real product
// C' = A' B' of size M x 2N x 2K with
//   A'[m][2k + p]          = (re, im)[p] of A[m][k]            (the interleaved storage itself)
//   B'[2k + p][2n + q]     = [[re, im], [-im, re]][p][q] of B[k][n]
//   C'[m][2n + q]          = (re, im)[q] of C[m][n]            (interleaved output)
// which is exactly the four real products of complex arithmetic (8 real flops per complex
// multiply-add) and needs no extra pass over memory: A tiles are stored to LDS planar by real
// k, B tiles are expanded to their real 2x2 form while they are staged.
//
// fp32: v_mfma_f32_32x32x2f32 (lane l supplies A'[l%32][l/32], B'[l/32][l%32]; accumulator r of
//       lane l holds C'[(r/4)*8 + (l/32)*4 + r%4][l%32]).
// fp64: v_mfma_f64_16x16x4f64 (lane l supplies A'[l%16][l/16], B'[l/16][l%16]; accumulator r of
//       lane l holds C'[4r + l/16][l%16]).
// A workgroup of 4 waves (2 x 2) owns a BM x BN complex tile, double-buffered in LDS with one
// barrier per K step; global loads of the next K step are issued before the current step's
// matrix instructions.

#include "dev_common.h"

namespace mpoevo {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct MfmaF32 {
  using T = float;
  using acc_t = f32x16;
  static constexpr int MT = 32, NT = 32, KT = 2, NACC = 16;
  static constexpr int WR = 2, WC = 2;  // MFMA tiles per wave (rows, real cols)
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static int a_row(int l) { return l & 31; }
  __device__ static int a_k(int l) { return l >> 5; }
  __device__ static int out_row(int l, int r) { return (r >> 2) * 8 + (l >> 5) * 4 + (r & 3); }
  __device__ static int out_col(int l) { return l & 31; }
};

struct MfmaF64 {
  using T = double;
  using acc_t = f64x4;
  static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4;
  static constexpr int WR = 2, WC = 4;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int out_row(int l, int r) { return 4 * r + (l >> 4); }
  __device__ static int out_col(int l) { return l & 15; }
};

constexpr int kThreads = 256;
constexpr int kBK = 8;  // complex K per stage

template <class Mf>
struct Tile {
  using T = typename Mf::T;
  static constexpr int BM = 2 * Mf::WR * Mf::MT;      // complex rows per workgroup
  static constexpr int BNR = 2 * Mf::WC * Mf::NT;     // real columns per workgroup
  static constexpr int BN = BNR / 2;                  // complex columns
  static constexpr int KR = 2 * kBK;                  // real k per stage
  static constexpr int LDA = BM + 4;                  // padded LDS row lengths (elements)
  static constexpr int LDB = BNR + 4;
  static constexpr int A_ELEMS = BM * kBK / kThreads;  // complex loads per thread
  static constexpr int B_ELEMS = BN * kBK / kThreads;
  static constexpr int LDS_ELEMS = KR * LDA + KR * LDB;
};

template <class Mf, typename TO, bool AKC, bool BNC>
__global__ __launch_bounds__(kThreads) void cgemm_kernel(GemmDesc g) {
  using T = typename Mf::T;
  using C2 = cx_t<T>;
  using TT = Tile<Mf>;
  __shared__ T lds[2 * TT::LDS_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int bz = blockIdx.z;
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
      if (AKC) { m = e / kBK; k = e % kBK; } else { k = e / TT::BM; m = e % TT::BM; }
      const int gm = m0 + m, gk = k0 + k;
      C2 v{T(0), T(0)};
      if (gm < g.M && gk < g.K) v = A[gm * g.sAm + gk * g.sAk];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < TT::B_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int k, n;
      if (BNC) { k = e / TT::BN; n = e % TT::BN; } else { n = e / kBK; k = e % kBK; }
      const int gk = k0 + k, gn = n0 + n;
      C2 v{T(0), T(0)};
      if (gk < g.K && gn < g.N) v = B[gk * g.sBk + gn * g.sBn];
      rb[i] = v;
    }
  };
  auto store_tiles = [&](int buf) {
    T* As = lds + buf * TT::LDS_ELEMS;
    T* Bs = As + TT::KR * TT::LDA;
#pragma unroll
    for (int i = 0; i < TT::A_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int m, k;
      if (AKC) { m = e / kBK; k = e % kBK; } else { k = e / TT::BM; m = e % TT::BM; }
      As[(2 * k) * TT::LDA + m] = ra[i].x;
      As[(2 * k + 1) * TT::LDA + m] = sgnA * ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < TT::B_ELEMS; ++i) {
      const int e = tid + i * kThreads;
      int k, n;
      if (BNC) { k = e / TT::BN; n = e % TT::BN; } else { n = e / kBK; k = e % kBK; }
      const T re = rb[i].x, im = sgnB * rb[i].y;
      T* r0 = Bs + (2 * k) * TT::LDB + 2 * n;
      T* r1 = r0 + TT::LDB;
      r0[0] = re;
      r0[1] = im;
      r1[0] = -im;
      r1[1] = re;
    }
  };

  typename Mf::acc_t acc[Mf::WR][Mf::WC];
#pragma unroll
  for (int i = 0; i < Mf::WR; ++i)
#pragma unroll
    for (int j = 0; j < Mf::WC; ++j)
#pragma unroll
      for (int r = 0; r < Mf::NACC; ++r) acc[i][j][r] = T(0);

  const int nk = (g.K + kBK - 1) / kBK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();

  const int arow = Mf::a_row(lane), ak = Mf::a_k(lane);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * kBK);
    const T* As = lds + cur * TT::LDS_ELEMS;
    const T* Bs = As + TT::KR * TT::LDA;
#pragma unroll
    for (int kr = 0; kr < TT::KR; kr += Mf::KT) {
      T af[Mf::WR], bf[Mf::WC];
#pragma unroll
      for (int i = 0; i < Mf::WR; ++i)
        af[i] = As[(kr + ak) * TT::LDA + wm * (Mf::WR * Mf::MT) + i * Mf::MT + arow];
#pragma unroll
      for (int j = 0; j < Mf::WC; ++j)
        bf[j] = Bs[(kr + ak) * TT::LDB + wn * (Mf::WC * Mf::NT) + j * Mf::NT + arow];
#pragma unroll
      for (int i = 0; i < Mf::WR; ++i)
#pragma unroll
        for (int j = 0; j < Mf::WC; ++j) acc[i][j] = Mf::mma(af[i], bf[j], acc[i][j]);
    }
    if (kt + 1 < nk) store_tiles(cur ^ 1);
    __syncthreads();
  }

  TO* C = reinterpret_cast<TO*>(g.C);
  const long long cbase = (long long)bz * g.bC;
#pragma unroll
  for (int i = 0; i < Mf::WR; ++i)
#pragma unroll
    for (int j = 0; j < Mf::WC; ++j)
#pragma unroll
      for (int r = 0; r < Mf::NACC; ++r) {
        const int row = m0 + wm * (Mf::WR * Mf::MT) + i * Mf::MT + Mf::out_row(lane, r);
        const int rcol = wn * (Mf::WC * Mf::NT) + j * Mf::NT + Mf::out_col(lane);
        const int col = n0 + (rcol >> 1);
        if (row < g.M && col < g.N)
          C[2 * (cbase + row * g.sCm + col * g.sCn) + (rcol & 1)] = TO(acc[i][j][r]);
      }
}

template <class Mf, typename TO, bool AKC, bool BNC>
hipError_t launch_one(const GemmDesc& g, hipStream_t st) {
  using TT = Tile<Mf>;
  dim3 grid((g.N + TT::BN - 1) / TT::BN, (g.M + TT::BM - 1) / TT::BM, g.batch);
  hipLaunchKernelGGL((cgemm_kernel<Mf, TO, AKC, BNC>), grid, dim3(kThreads), 0, st, g);
  return hipGetLastError();
}

template <class Mf, typename TO>
hipError_t launch_layout(const GemmDesc& g, hipStream_t st) {
  const bool akc = (g.sAk == 1) || (g.K == 1);
  const bool bnc = (g.sBn == 1) || (g.N == 1);
  if (akc && bnc) return launch_one<Mf, TO, true, true>(g, st);
  if (akc && !bnc) return launch_one<Mf, TO, true, false>(g, st);
  if (!akc && bnc) return launch_one<Mf, TO, false, true>(g, st);
  return launch_one<Mf, TO, false, false>(g, st);
}

}  // namespace

hipError_t gemm_launch(const GemmDesc& g, bool fp64, bool out_fp64, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  if (fp64) return launch_layout<MfmaF64, double>(g, st);
  if (out_fp64) return launch_layout<MfmaF32, double>(g, st);
  return launch_layout<MfmaF32, float>(g, st);
}

}  // namespace mpoevo
