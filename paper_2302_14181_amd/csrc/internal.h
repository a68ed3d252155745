// Internal interface between the C ABI layer (abi.cpp, no HIP headers) and the device code
// (device.hip). Only plain C++ types cross this boundary.
#pragma once

#include <cstddef>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mpoevo.h"

namespace mpoevo {

int build_mpo_host(int d, int chi, const double* A, const double* B, const double* C,
                   const double* D, int order, double tau_re, double tau_im, int variant,
                   const int* inner_charge, const int* phys_charge, int* w_out, double* W_out,
                   size_t W_capacity, int* level_charge_out, std::string& err);

struct DeviceState;  // defined in device.hip

struct Context {
  int device = 0;
  std::string err;
  int max_sweeps = 0;  // largest Jacobi sweep count seen by mpoevo_check_solver / step
  DeviceState* dev = nullptr;
  // Jacobi preconditioners left in a step workspace by the last completed step: the workspace,
  // the chain's shape {L, d, Dmax, wmax, prec} and the order of the unitary stored per bond.
  const void* warm_ws = nullptr;
  int warm_sig[5] = {0, 0, 0, 0, 0};
  unsigned long long warm_token = 0;  // also stored in the workspace by the step that wrote them
  std::vector<int> warm_dim;
  // per bond: a truncation of the last step found the bond matrix numerically rank-deficient
  // (its columns would need completing to hand on a basis)
  std::vector<char> warm_deficient;
  // Jacobi launches: cooperative on a handle; ordinary (overlapping other streams) on the
  // per-chain contexts of step_batched, which bound the workgroups in flight themselves.
  bool coop_jacobi = true;
  // step_batched: one context per chain index (own status words and preconditioner state) and
  // the worker streams (hipStream_t, default priority), created on first use.
  std::vector<std::unique_ptr<Context>> chains;
  std::vector<void*> streams;
  // product tile tuner (owned by the handle; the per-chain contexts of step_batched borrow the
  // handle's and never tune)
  void* tuner = nullptr;
  bool owns_tuner = false;
};

// Product tile tuner (gemm.hip): per-handle table of the plan chosen for each product shape.
void* gemm_tuner_new();
void gemm_tuner_free(void* t);
int gemm_tuner_mode(void* t, int set);  // set < 0: query only; returns the mode
size_t gemm_tuner_entries(void* t);
void gemm_tuner_clear(void* t);
unsigned long long gemm_tuner_generation(void* t);  // changes with the mode and on every clear
// The plan a product of this shape (operands contiguous along k and n) takes with tuner t
// (nullable): out = {tile rows, tile columns, K splits, 1 if tuned else 0}.
int gemm_plan_query(void* t, int prec, int M, int N, int K, int batch, int* out);
// Makes t the tuner of the products launched by this thread while the scope lives; allow:
// new shapes may be tuned (otherwise they take the rule).
class TunerScope {
 public:
  TunerScope(void* t, bool allow);
  ~TunerScope();
  TunerScope(const TunerScope&) = delete;
  TunerScope& operator=(const TunerScope&) = delete;

 private:
  void* prev_;
  bool prev_allow_;
};

int device_init(Context& ctx);
void device_fini(Context& ctx);

size_t env_update_ws(const int* dims, int prec);
size_t local_apply_ws(const int* dims, int prec);
size_t local_apply1_ws(const int* dims, int prec);  // one-site: dims {Dbl, Dkl, Dkr, Dbr, d, wl, wr}
size_t truncate_ws(int m, int n);
size_t step_ws(int L, int d, int Dmax, int wmax, int prec);
size_t expectation_ws(int L, int d, int Dmax, int wmax);

int env_update_dev(Context& ctx, int side, int prec, const void* E_in, const void* bra,
                   const void* W, const void* ket, void* E_out, const int* dims, void* ws,
                   size_t ws_bytes, void* stream);
// env_update on the library's per-device static scratch (no allocation, no workspace argument)
size_t env_update_noalloc_need(const int* dims, int prec);
int env_update_noalloc_dev(Context& ctx, int side, int prec, const void* E_in, const void* bra,
                           const void* W, const void* ket, void* E_out, const int* dims, void* stream);
int local_apply1_dev(Context& ctx, int prec, const void* L, const void* W, const void* M, const void* R,
                     void* Theta, const int* dims, void* ws, size_t ws_bytes, void* stream);
int local_apply_dev(Context& ctx, int prec, const void* L, const void* W1, const void* W2,
                    const void* M1, const void* M2, const void* R, void* Theta, const int* dims,
                    void* ws, size_t ws_bytes, void* stream);
int truncate_dev(Context& ctx, const void* Theta, int m, int n, int Dmax, double cutoff,
                 int direction, void* A_out, void* B_out, int* k_dev, double* discarded_dev,
                 double* norm_dev, double* sigma_dev, void* ws, size_t ws_bytes, void* stream);
int check_solver_dev(Context& ctx, void* stream = nullptr);
int step_dev(Context& ctx, mpoevo_mps* mps, const mpoevo_mpo* mpo, const mpoevo_step_opts* opts,
             mpoevo_step_stats* stats, void* ws, size_t ws_bytes, void* stream);
int overlap_dev(Context& ctx, const mpoevo_mps* bra, const mpoevo_mpo* mpo, const mpoevo_mps* ket, int left,
                int right, void* out, void* ws, size_t ws_bytes, void* stream);
int expectation_dev(Context& ctx, const mpoevo_mps* mps, const mpoevo_mpo* mpo, int left, int right,
                    void* out, void* ws, size_t ws_bytes, void* stream);
size_t step_batched_ws(int n, const int* dims, int prec);  // dims: {L, d, Dmax, wmax} per chain
int step_batched_dev(Context& ctx, int n, mpoevo_mps* mps, const mpoevo_mpo* mpo,
                     const mpoevo_step_opts* opts, mpoevo_step_stats* stats, void* ws,
                     size_t ws_bytes, void* stream);

}  // namespace mpoevo
