// C ABI of libmpoevo.so: argument validation, error text, dispatch to the device layer.
// This translation unit includes no HIP or POSIX headers (the ABI exports a function named
// `truncate`, which must not meet the libc declaration of the same name).

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.h"

namespace {
thread_local std::string g_thread_err;

int fail(mpoevo::Context* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_thread_err = msg;
  return code;
}

bool valid_prec(int prec) { return prec == MPOEVO_FP64 || prec == MPOEVO_FP32 || prec == MPOEVO_BF16X3; }
}  // namespace

extern "C" {

const char* mpoevo_version(void) { return "mpoevo 0.1 (gfx950)"; }

int mpoevo_create(mpoevo_handle* h, int device) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "mpoevo_create: h is NULL");
  *h = nullptr;
  auto* ctx = new (std::nothrow) mpoevo::Context();
  if (!ctx) return fail(nullptr, MPOEVO_ENOMEM, "mpoevo_create: out of host memory");
  ctx->device = device;
  const int rc = mpoevo::device_init(*ctx);
  if (rc != MPOEVO_OK) {
    g_thread_err = ctx->err;
    delete ctx;
    return rc;
  }
  *h = reinterpret_cast<mpoevo_handle>(ctx);
  return MPOEVO_OK;
}

int mpoevo_destroy(mpoevo_handle h) {
  if (!h) return MPOEVO_OK;
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  mpoevo::device_fini(*ctx);
  delete ctx;
  return MPOEVO_OK;
}

const char* mpoevo_last_error(mpoevo_handle h) {
  if (!h) return g_thread_err.c_str();
  return reinterpret_cast<mpoevo::Context*>(h)->err.c_str();
}

int mpo_build(int d, int chi, const double* A, const double* B, const double* C, const double* D,
              int order, double tau_re, double tau_im, int variant, const int* inner_charge,
              const int* phys_charge, int* w_out, double* W_out, size_t W_capacity,
              int* level_charge_out) {
  std::string err;
  const int rc = mpoevo::build_mpo_host(d, chi, A, B, C, D, order, tau_re, tau_im, variant,
                                        inner_charge, phys_charge, w_out, W_out, W_capacity,
                                        level_charge_out, err);
  if (rc != MPOEVO_OK) g_thread_err = err;
  return rc;
}

int mpoevo_set_tuning(mpoevo_handle h, int mode, int clear) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "mpoevo_set_tuning: h is NULL");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (mode != MPOEVO_TUNE_OFF && mode != MPOEVO_TUNE_ON && mode != MPOEVO_TUNE_FROZEN)
    return fail(ctx, MPOEVO_EINVAL, "mpoevo_set_tuning: unknown mode");
  if (clear) mpoevo::gemm_tuner_clear(ctx->tuner);
  mpoevo::gemm_tuner_mode(ctx->tuner, mode);
  return MPOEVO_OK;
}

int mpoevo_product_plan(mpoevo_handle h, int prec, int M, int N, int K, int batch, int* plan,
                        int* entries) {
  if (!h || !plan) return fail(nullptr, MPOEVO_EINVAL, "mpoevo_product_plan: NULL argument");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (!valid_prec(prec)) return fail(ctx, MPOEVO_EINVAL, "mpoevo_product_plan: unknown precision");
  if (M < 1 || N < 1 || K < 1 || batch < 1)
    return fail(ctx, MPOEVO_ESHAPE, "mpoevo_product_plan: non-positive size");
  mpoevo::gemm_plan_query(ctx->tuner, prec, M, N, K, batch, plan);
  if (entries) *entries = (int)mpoevo::gemm_tuner_entries(ctx->tuner);
  return MPOEVO_OK;
}

int mpoevo_workspace_size(int call_id, const int* dims, int prec, size_t* bytes) {
  if (!dims || !bytes) return fail(nullptr, MPOEVO_EINVAL, "mpoevo_workspace_size: NULL argument");
  if (!valid_prec(prec)) return fail(nullptr, MPOEVO_EINVAL, "unknown precision");
  switch (call_id) {
    case MPOEVO_CALL_ENV_UPDATE:
      for (int i = 0; i < 7; ++i) if (dims[i] < 1) return fail(nullptr, MPOEVO_ESHAPE, "non-positive dimension");
      *bytes = mpoevo::env_update_ws(dims, prec);
      return MPOEVO_OK;
    case MPOEVO_CALL_LOCAL_APPLY:
      for (int i = 0; i < 9; ++i) if (dims[i] < 1) return fail(nullptr, MPOEVO_ESHAPE, "non-positive dimension");
      *bytes = mpoevo::local_apply_ws(dims, prec);
      return MPOEVO_OK;
    case MPOEVO_CALL_LOCAL_APPLY1:
      for (int i = 0; i < 7; ++i) if (dims[i] < 1) return fail(nullptr, MPOEVO_ESHAPE, "non-positive dimension");
      *bytes = mpoevo::local_apply1_ws(dims, prec);
      return MPOEVO_OK;
    case MPOEVO_CALL_TRUNCATE:
      if (dims[0] < 1 || dims[1] < 1 || dims[0] > MPOEVO_SVD_MAX_DIM || dims[1] > MPOEVO_SVD_MAX_DIM)
        return fail(nullptr, MPOEVO_ESHAPE, "truncate: m, n must be in 1..MPOEVO_SVD_MAX_DIM");
      *bytes = mpoevo::truncate_ws(dims[0], dims[1]);
      return MPOEVO_OK;
    case MPOEVO_CALL_STEP:
      if (dims[0] < 2 || dims[1] < 1 || dims[2] < 1 || dims[3] < 1)
        return fail(nullptr, MPOEVO_ESHAPE, "step: need L >= 2, d, Dmax, wmax >= 1");
      if ((long)dims[1] * dims[2] > MPOEVO_SVD_MAX_DIM)
        return fail(nullptr, MPOEVO_ESHAPE, "step: d * Dmax exceeds MPOEVO_SVD_MAX_DIM");
      *bytes = mpoevo::step_ws(dims[0], dims[1], dims[2], dims[3], prec);
      return MPOEVO_OK;
    case MPOEVO_CALL_STEP_BATCHED: {
      const int n = dims[0];
      if (n < 1 || n > MPOEVO_MAX_CHAINS) return fail(nullptr, MPOEVO_EINVAL, "step_batched: n must be in 1..MPOEVO_MAX_CHAINS");
      for (int c = 0; c < n; ++c) {
        const int* dc = dims + 1 + 4 * c;
        if (dc[0] < 2 || dc[1] < 1 || dc[2] < 1 || dc[3] < 1)
          return fail(nullptr, MPOEVO_ESHAPE, "step_batched: need L >= 2, d, Dmax, wmax >= 1 per chain");
        if ((long)dc[1] * dc[2] > MPOEVO_SVD_MAX_DIM)
          return fail(nullptr, MPOEVO_ESHAPE, "step_batched: d * Dmax exceeds MPOEVO_SVD_MAX_DIM");
      }
      *bytes = mpoevo::step_batched_ws(n, dims + 1, prec);
      return MPOEVO_OK;
    }
    case MPOEVO_CALL_EXPECTATION:
      if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || dims[3] < 1)
        return fail(nullptr, MPOEVO_ESHAPE, "expectation: need L, d, Dmax, wmax >= 1");
      if (prec != MPOEVO_FP64) return fail(nullptr, MPOEVO_EINVAL, "expectation: FP64 only");
      *bytes = mpoevo::expectation_ws(dims[0], dims[1], dims[2], dims[3]);
      return MPOEVO_OK;
    default:
      return fail(nullptr, MPOEVO_EINVAL, "mpoevo_workspace_size: unknown call id");
  }
}

int env_update(mpoevo_handle h, int side, int prec, const void* E_in, const void* bra,
               const void* W, const void* ket, void* E_out, const int* dims, void* workspace,
               size_t workspace_bytes, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "env_update: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (side != MPOEVO_LEFT && side != MPOEVO_RIGHT) return fail(ctx, MPOEVO_EINVAL, "env_update: unknown side");
  if (!valid_prec(prec)) return fail(ctx, MPOEVO_EINVAL, "env_update: unknown precision");
  if (!E_in || !bra || !W || !ket || !E_out || !dims) return fail(ctx, MPOEVO_EINVAL, "env_update: NULL pointer");
  for (int i = 0; i < 7; ++i) if (dims[i] < 1) return fail(ctx, MPOEVO_ESHAPE, "env_update: non-positive dimension");
  if (workspace_bytes < mpoevo::env_update_ws(dims, prec) || (!workspace && workspace_bytes))
    return fail(ctx, MPOEVO_ENOMEM, "env_update: workspace too small");
  return mpoevo::env_update_dev(*ctx, side, prec, E_in, bra, W, ket, E_out, dims, workspace,
                                workspace_bytes, stream);
}

int env_update_noalloc(mpoevo_handle h, int side, int prec, const void* E_in, const void* bra,
                       const void* W, const void* ket, void* E_out, const int* dims, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "env_update_noalloc: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (side != MPOEVO_LEFT && side != MPOEVO_RIGHT) return fail(ctx, MPOEVO_EINVAL, "env_update_noalloc: unknown side");
  if (!valid_prec(prec)) return fail(ctx, MPOEVO_EINVAL, "env_update_noalloc: unknown precision");
  if (!E_in || !bra || !W || !ket || !E_out || !dims)
    return fail(ctx, MPOEVO_EINVAL, "env_update_noalloc: NULL pointer");
  for (int i = 0; i < 7; ++i)
    if (dims[i] < 1) return fail(ctx, MPOEVO_ESHAPE, "env_update_noalloc: non-positive dimension");
  return mpoevo::env_update_noalloc_dev(*ctx, side, prec, E_in, bra, W, ket, E_out, dims, stream);
}

int local_apply(mpoevo_handle h, int nsites, int prec, const void* L, const void* W1,
                const void* W2, const void* M1, const void* M2, const void* R, void* Theta,
                const int* dims, void* workspace, size_t workspace_bytes, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "local_apply: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (nsites != 1 && nsites != 2) return fail(ctx, MPOEVO_EINVAL, "local_apply: nsites must be 1 or 2");
  if (!valid_prec(prec)) return fail(ctx, MPOEVO_EINVAL, "local_apply: unknown precision");
  if (nsites == 1) {  // L, W1, M1, R; W2 and M2 unused
    if (!L || !W1 || !M1 || !R || !Theta || !dims) return fail(ctx, MPOEVO_EINVAL, "local_apply: NULL pointer");
    for (int i = 0; i < 7; ++i) if (dims[i] < 1) return fail(ctx, MPOEVO_ESHAPE, "local_apply: non-positive dimension");
    if (workspace_bytes < mpoevo::local_apply1_ws(dims, prec) || (!workspace && workspace_bytes))
      return fail(ctx, MPOEVO_ENOMEM, "local_apply: workspace too small");
    return mpoevo::local_apply1_dev(*ctx, prec, L, W1, M1, R, Theta, dims, workspace, workspace_bytes, stream);
  }
  if (!L || !W1 || !W2 || !M1 || !M2 || !R || !Theta || !dims) return fail(ctx, MPOEVO_EINVAL, "local_apply: NULL pointer");
  for (int i = 0; i < 9; ++i) if (dims[i] < 1) return fail(ctx, MPOEVO_ESHAPE, "local_apply: non-positive dimension");
  if (workspace_bytes < mpoevo::local_apply_ws(dims, prec) || (!workspace && workspace_bytes))
    return fail(ctx, MPOEVO_ENOMEM, "local_apply: workspace too small");
  return mpoevo::local_apply_dev(*ctx, prec, L, W1, W2, M1, M2, R, Theta, dims, workspace,
                                 workspace_bytes, stream);
}

int truncate(mpoevo_handle h, const void* Theta, int m, int n, int Dmax, double cutoff,
             int direction, void* A_out, void* B_out, int* k_dev, double* discarded_dev,
             double* norm_dev, double* sigma_dev, void* workspace, size_t workspace_bytes,
             void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "truncate: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (!Theta || !A_out || !B_out) return fail(ctx, MPOEVO_EINVAL, "truncate: NULL pointer");
  if (direction != MPOEVO_LEFT && direction != MPOEVO_RIGHT) return fail(ctx, MPOEVO_EINVAL, "truncate: unknown direction");
  if (m < 1 || n < 1 || m > MPOEVO_SVD_MAX_DIM || n > MPOEVO_SVD_MAX_DIM || Dmax < 1)
    return fail(ctx, MPOEVO_ESHAPE, "truncate: m, n must be in 1..MPOEVO_SVD_MAX_DIM and Dmax >= 1");
  if (!(cutoff >= 0.0) || cutoff >= 1.0) return fail(ctx, MPOEVO_EINVAL, "truncate: cutoff must be in [0, 1)");
  if (workspace_bytes < mpoevo::truncate_ws(m, n) || !workspace)
    return fail(ctx, MPOEVO_ENOMEM, "truncate: workspace too small");
  return mpoevo::truncate_dev(*ctx, Theta, m, n, Dmax, cutoff, direction, A_out, B_out, k_dev,
                              discarded_dev, norm_dev, sigma_dev, workspace, workspace_bytes, stream);
}

int mpoevo_check_solver(mpoevo_handle h, int* max_sweeps) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "mpoevo_check_solver: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  ctx->max_sweeps = 0;
  const int rc = mpoevo::check_solver_dev(*ctx);
  if (max_sweeps) *max_sweeps = ctx->max_sweeps;
  return rc;
}

namespace {
// Checks one chain's arguments of step / step_batched; on success *wmax is its largest MPO bond.
int check_chain(mpoevo::Context* ctx, const std::string& who, const mpoevo_mps* mps,
                const mpoevo_mpo* mpo, int* wmax) {
  if (!mps || !mpo || !mps->bond_dim || !mps->site || !mpo->w || !mpo->site)
    return fail(ctx, MPOEVO_EINVAL, who + ": NULL argument");
  const int L = mps->L, d = mps->d, Dmax = mps->Dmax;
  if (L < 2 || d < 1 || Dmax < 1 || mpo->L != L || mpo->d != d)
    return fail(ctx, MPOEVO_ESHAPE, who + ": need L >= 2 and matching L, d of MPS and MPO");
  if ((long)d * Dmax > MPOEVO_SVD_MAX_DIM) return fail(ctx, MPOEVO_ESHAPE, who + ": d * Dmax exceeds MPOEVO_SVD_MAX_DIM");
  if (mps->bond_dim[0] != 1 || mps->bond_dim[L] != 1) return fail(ctx, MPOEVO_ESHAPE, who + ": boundary bonds must be 1");
  *wmax = 0;
  for (int i = 0; i <= L; ++i) {
    if (i > 0 && i < L && (mps->bond_dim[i] < 1 || mps->bond_dim[i] > Dmax))
      return fail(ctx, MPOEVO_ESHAPE, who + ": MPS bond dimension outside 1..Dmax");
    if (mpo->w[i] < 1) return fail(ctx, MPOEVO_ESHAPE, who + ": MPO bond dimension < 1");
    if (mpo->w[i] > *wmax) *wmax = mpo->w[i];
  }
  for (int i = 0; i < L; ++i)
    if (!mps->site[i] || !mpo->site[i]) return fail(ctx, MPOEVO_EINVAL, who + ": NULL site pointer");
  if ((mps->sector_table == nullptr) != (mps->phys_charge == nullptr))
    return fail(ctx, MPOEVO_EINVAL, who + ": give both sector_table and phys_charge or neither");
  if (mps->sector_table) {
    for (int b = 0; b <= L; ++b)
      for (int j = 1; j < mps->bond_dim[b]; ++j)
        if (mps->sector_table[(size_t)b * Dmax + j] < mps->sector_table[(size_t)b * Dmax + j - 1])
          return fail(ctx, MPOEVO_EINVAL, who + ": sector_table must be nondecreasing within each bond");
  }
  return MPOEVO_OK;
}

int check_opts(mpoevo::Context* ctx, const std::string& who, const mpoevo_step_opts* opts) {
  if (!opts) return fail(ctx, MPOEVO_EINVAL, who + ": NULL argument");
  if (!valid_prec(opts->prec)) return fail(ctx, MPOEVO_EINVAL, who + ": unknown precision");
  if (opts->nsweeps < 1 || opts->nsweeps > 4) return fail(ctx, MPOEVO_EINVAL, who + ": nsweeps must be 1..4");
  if (!(opts->cutoff >= 0.0) || opts->cutoff >= 1.0) return fail(ctx, MPOEVO_EINVAL, who + ": cutoff must be in [0, 1)");
  if (opts->profile < 0 || opts->profile > 2) return fail(ctx, MPOEVO_EINVAL, who + ": profile must be 0, 1 or 2");
  if (opts->nsites < -1 || opts->nsites > 2) return fail(ctx, MPOEVO_EINVAL, who + ": nsites must be -1, 0, 1 or 2");
  if (opts->use_graph < 0 || opts->use_graph > 1) return fail(ctx, MPOEVO_EINVAL, who + ": use_graph must be 0 or 1");
  if (opts->guess < -1 || opts->guess > 1) return fail(ctx, MPOEVO_EINVAL, who + ": guess must be -1, 0 or 1");
  if (opts->guess == MPOEVO_GUESS_ZIPUP && opts->nsites == 1)
    return fail(ctx, MPOEVO_EUNSUPPORTED, who + ": the zip-up guess is followed by two-site updates only");
  return MPOEVO_OK;
}
}  // namespace

int step(mpoevo_handle h, mpoevo_mps* mps, const mpoevo_mpo* mpo, const mpoevo_step_opts* opts,
         mpoevo_step_stats* stats, void* workspace, size_t workspace_bytes, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "step: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  int wmax = 0;
  if (int rc = check_opts(ctx, "step", opts); rc != MPOEVO_OK) return rc;
  if (int rc = check_chain(ctx, "step", mps, mpo, &wmax); rc != MPOEVO_OK) return rc;
  if (workspace_bytes < mpoevo::step_ws(mps->L, mps->d, mps->Dmax, wmax, opts->prec) || !workspace)
    return fail(ctx, MPOEVO_ENOMEM, "step: workspace too small");
  if (mps->sector_table && opts->nsites == 1)
    return fail(ctx, MPOEVO_EUNSUPPORTED, "step: one-site updates of U(1) chains are not built");
  if (mps->sector_table && opts->guess == MPOEVO_GUESS_ZIPUP)
    return fail(ctx, MPOEVO_EUNSUPPORTED, "step: the zip-up guess of U(1) chains is not built");
  return mpoevo::step_dev(*ctx, mps, mpo, opts, stats, workspace, workspace_bytes, stream);
}

int step_batched(mpoevo_handle h, int n, mpoevo_mps* mps, const mpoevo_mpo* mpo,
                 const mpoevo_step_opts* opts, mpoevo_step_stats* stats, void* workspace,
                 size_t workspace_bytes, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "step_batched: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (n < 1 || n > MPOEVO_MAX_CHAINS) return fail(ctx, MPOEVO_EINVAL, "step_batched: n must be in 1..MPOEVO_MAX_CHAINS");
  if (!mps || !mpo) return fail(ctx, MPOEVO_EINVAL, "step_batched: NULL argument");
  if (int rc = check_opts(ctx, "step_batched", opts); rc != MPOEVO_OK) return rc;
  std::vector<int> dims(4 * (size_t)n);
  std::unordered_set<const void*> seen;  // every site buffer and bond array belongs to one chain
  for (int c = 0; c < n; ++c) {
    int wmax = 0;
    const std::string who = "step_batched: chain " + std::to_string(c);
    if (int rc = check_chain(ctx, who, &mps[c], &mpo[c], &wmax); rc != MPOEVO_OK) return rc;
    bool fresh = seen.insert(mps[c].bond_dim).second;
    for (int i = 0; i < mps[c].L; ++i) fresh = seen.insert(mps[c].site[i]).second && fresh;
    if (!fresh) return fail(ctx, MPOEVO_EINVAL, who + ": shares a site buffer or its bond array");
    dims[4 * c] = mps[c].L; dims[4 * c + 1] = mps[c].d; dims[4 * c + 2] = mps[c].Dmax; dims[4 * c + 3] = wmax;
  }
  if (!workspace || workspace_bytes < mpoevo::step_batched_ws(n, dims.data(), opts->prec))
    return fail(ctx, MPOEVO_ENOMEM, "step_batched: workspace too small");
  return mpoevo::step_batched_dev(*ctx, n, mps, mpo, opts, stats, workspace, workspace_bytes, stream);
}

int expectation(mpoevo_handle h, const mpoevo_mps* mps, const mpoevo_mpo* mpo, int left, int right,
                void* out, void* workspace, size_t workspace_bytes, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "expectation: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (!mps || !mpo || !out || !mps->bond_dim || !mps->site || !mpo->w || !mpo->site)
    return fail(ctx, MPOEVO_EINVAL, "expectation: NULL argument");
  const int L = mps->L, d = mps->d, Dmax = mps->Dmax;
  if (L < 1 || d < 1 || Dmax < 1 || mpo->L != L || mpo->d != d)
    return fail(ctx, MPOEVO_ESHAPE, "expectation: need L >= 1 and matching L, d of MPS and MPO");
  if (mps->bond_dim[0] != 1 || mps->bond_dim[L] != 1)
    return fail(ctx, MPOEVO_ESHAPE, "expectation: boundary bonds must be 1");
  int wmax = 0;
  for (int i = 0; i <= L; ++i) {
    if (i > 0 && i < L && (mps->bond_dim[i] < 1 || mps->bond_dim[i] > Dmax))
      return fail(ctx, MPOEVO_ESHAPE, "expectation: MPS bond dimension outside 1..Dmax");
    if (mpo->w[i] < 1) return fail(ctx, MPOEVO_ESHAPE, "expectation: MPO bond dimension < 1");
    if (mpo->w[i] > wmax) wmax = mpo->w[i];
  }
  if (left < 0 || left >= mpo->w[0] || right < 0 || right >= mpo->w[L])
    return fail(ctx, MPOEVO_EINVAL, "expectation: boundary level out of range");
  for (int i = 0; i < L; ++i)
    if (!mps->site[i] || !mpo->site[i]) return fail(ctx, MPOEVO_EINVAL, "expectation: NULL site pointer");
  if (!workspace || workspace_bytes < mpoevo::expectation_ws(L, d, Dmax, wmax))
    return fail(ctx, MPOEVO_ENOMEM, "expectation: workspace too small");
  return mpoevo::expectation_dev(*ctx, mps, mpo, left, right, out, workspace, workspace_bytes, stream);
}

namespace {
int check_measured(mpoevo::Context* ctx, const char* who, const mpoevo_mps* mps, const mpoevo_mpo* mpo,
                   int* wmax) {
  const std::string w_ = who;
  if (!mps || !mpo || !mps->bond_dim || !mps->site || !mpo->w || !mpo->site)
    return fail(ctx, MPOEVO_EINVAL, w_ + ": NULL argument");
  const int L = mps->L, d = mps->d, Dmax = mps->Dmax;
  if (L < 1 || d < 1 || Dmax < 1 || mpo->L != L || mpo->d != d)
    return fail(ctx, MPOEVO_ESHAPE, w_ + ": need L >= 1 and matching L, d of MPS and MPO");
  if (mps->bond_dim[0] != 1 || mps->bond_dim[L] != 1) return fail(ctx, MPOEVO_ESHAPE, w_ + ": boundary bonds must be 1");
  *wmax = 0;
  for (int i = 0; i <= L; ++i) {
    if (i > 0 && i < L && (mps->bond_dim[i] < 1 || mps->bond_dim[i] > Dmax))
      return fail(ctx, MPOEVO_ESHAPE, w_ + ": MPS bond dimension outside 1..Dmax");
    if (mpo->w[i] < 1) return fail(ctx, MPOEVO_ESHAPE, w_ + ": MPO bond dimension < 1");
    if (mpo->w[i] > *wmax) *wmax = mpo->w[i];
  }
  for (int i = 0; i < L; ++i)
    if (!mps->site[i] || !mpo->site[i]) return fail(ctx, MPOEVO_EINVAL, w_ + ": NULL site pointer");
  return MPOEVO_OK;
}
}  // namespace

int overlap(mpoevo_handle h, const mpoevo_mps* bra, const mpoevo_mpo* mpo, const mpoevo_mps* ket, int left,
            int right, void* out, void* workspace, size_t workspace_bytes, void* stream) {
  if (!h) return fail(nullptr, MPOEVO_EINVAL, "overlap: NULL handle");
  auto* ctx = reinterpret_cast<mpoevo::Context*>(h);
  if (!out) return fail(ctx, MPOEVO_EINVAL, "overlap: NULL argument");
  int wb = 0, wk = 0;
  if (int rc = check_measured(ctx, "overlap", bra, mpo, &wb); rc != MPOEVO_OK) return rc;
  if (int rc = check_measured(ctx, "overlap", ket, mpo, &wk); rc != MPOEVO_OK) return rc;
  if (left < 0 || left >= mpo->w[0] || right < 0 || right >= mpo->w[ket->L])
    return fail(ctx, MPOEVO_EINVAL, "overlap: boundary level out of range");
  const int Dmax = std::max(bra->Dmax, ket->Dmax);
  if (!workspace || workspace_bytes < mpoevo::expectation_ws(ket->L, ket->d, Dmax, wk))
    return fail(ctx, MPOEVO_ENOMEM, "overlap: workspace too small");
  return mpoevo::overlap_dev(*ctx, bra, mpo, ket, left, right, out, workspace, workspace_bytes, stream);
}

}  // extern "C"
