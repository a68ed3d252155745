#pragma once

#include <hip/hip_runtime.h>

namespace mpoevo {

constexpr int kWmixMaxK = 64;

// True if the short-leg contractions with W of these dimensions fit the register kernels.
bool wmix_supported(int wl, int d, int wr);

// LB[a'][s'][beta][b] = sum T[a'][alpha][s][b] W[alpha][s'][s][beta]; a' < P, b < Q.
hipError_t wmix_left(bool fp64, const void* Tin, const void* W, void* out, int P, int Q, int wl,
                     int d, int wr, hipStream_t st);
// RB[beta][b][t'][c'] = sum W[beta][t'][t][gamma] U[b][t][c'][gamma]; b < Q, c' < Pr.
hipError_t wmix_right(bool fp64, const void* U, const void* W, void* out, int Q, int Pr, int wl,
                      int d, int wr, hipStream_t st);

}  // namespace mpoevo
