// Shared device-side definitions for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace mpoevo {

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <typename T> using cx_t = typename Cx<T>::type;

// Arguments of a strided-batched complex product C = op(A) op(B) (complex elements, strides in
// complex elements). A(m, k) at A + batch*bA + m*sAm + k*sAk, B(k, n) at B + batch*bB + k*sBk +
// n*sBn, C(m, n) at C + batch*bC + m*sCm + n*sCn; conjA / conjB conjugate the operand.
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K, batch;
  long long sAm, sAk, sBk, sBn, sCm, sCn;
  long long bA, bB, bC;
  bool conjA, conjB;
  void* ws;         // optional scratch for split-K partial tiles (null: never split)
  size_t ws_bytes;
  bool bf16x3;      // fp32 operands: split-BF16x3 products on the bf16 matrix cores
  bool row_tail;    // the rows past another launch's whole row blocks: the smallest tile that
                    // holds them in one row block, K unsplit
};

// Scratch a caller gives gemm_launch for split-K partial results (the planner never needs more).
constexpr size_t kGemmScratchBytes = size_t(32) << 20;

// Launch a complex product with real fp32 (T = float) or fp64 (T = double) matrix-core
// arithmetic. out_fp64: store C as complex128 even when T = float. Returns a hipError_t.
hipError_t gemm_launch(const GemmDesc& g, bool fp64, bool out_fp64, hipStream_t st);

// Rows to launch apart from a product's whole row blocks: M mod the rule's tile rows when that
// tile's last row block would be at most half filled and a smaller tile (32 or 64 rows) holds
// them, else 0. Only the FP32 three-product path splits.
int gemm_row_tail(const GemmDesc& g, bool fp64);

// Where to cut a product so that its whole rounds of workgroups (kMinWgs tiles each) run in one
// launch and the few tiles of a last, mostly empty round in a second one, which the planner then
// gives a smaller tile or split K: dim 0 no cut, 1 rows [at, M), 2 columns [at, N), 3 batch
// entries [at, batch) go to the second launch. Only the FP32 three-product path on its own tile
// rule (no K split) is cut, when the last round would hold at most half of its tiles.
void gemm_round_tail(const GemmDesc& g, bool fp64, int& dim, long long& at);

// Host function of the kernel this thread launched last among the timed kernel classes (the
// products' main kernel, the W contractions, the Jacobi kernel) and whether a split-K sum
// followed it: a profiled step names each timed launch by it.
struct LaunchRecord {
  const void* kernel = nullptr;
  bool split = false;
};
LaunchRecord& last_launch();

#define MPOEVO_HIP_TRY(expr)                                  \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return e_;                          \
  } while (0)

}  // namespace mpoevo
