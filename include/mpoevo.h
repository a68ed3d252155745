/*
 * mpoevo: higher-order MPO time evolution on MI355X (gfx950).
 *
 * C ABI of the library libmpoevo.so. The method is that of "Efficient higher-order matrix
 * product operators for time evolution" (Van Damme, Haegeman, McCulloch, Vanderstraeten):
 *   - mpo_build   builds the order-N MPO approximation of exp(tau H) from the Jordan blocks of a
 *                 first-degree Hamiltonian MPO (Sec. 2.3, Sec. 3 Alg. 1, Sec. 4 Alg. 2,
 *                 Sec. 5 Alg. 3, Sec. 6 Alg. 4, boundary vectors of Sec. 3);
 *   - env_update, local_apply, truncate are the three device operations of the variational
 *                 fit of W|psi> at fixed maximal bond dimension (Sec. 2.2 and Table 1, the
 *                 sweeping (DMRG-like) scheme used in every benchmark of Sec. 8);
 *   - step        runs one complete time step of that fit (two-site updates, two sweeps).
 *
 * Conventions for every array argument:
 *   - complex numbers are interleaved {re, im}: complex128 = 2 x double, complex64 = 2 x float;
 *   - arrays are row-major, last index fastest;
 *   - MPS site tensor M[a][s][b] (left bond, physical, right bond);
 *   - MPO site tensor W[alpha][s_out][s_in][beta];
 *   - environment E[bra][mpo][ket]; the bra tensor is conjugated inside the contractions.
 * Precision: MPOEVO_FP64 contracts in double (complex128 inputs/outputs); MPOEVO_FP32 contracts
 * in float on the matrix cores with float accumulation (complex64 inputs/outputs);
 * MPOEVO_BF16X3 takes the same complex64 inputs/outputs as MPOEVO_FP32 but multiplies on the
 * bf16 matrix cores: each float operand is split into a bf16 head and a bf16 tail, the three
 * products head*head + head*tail + tail*head are accumulated in float (relative error of each
 * product about 2^-16 against about 2^-24 for FP32, at a higher matrix-core rate). The SVD,
 * the truncation and all norms are FP64 in every mode.
 *
 * Ownership: the caller allocates every input, output and workspace buffer; the library never
 * frees or reallocates them. A handle owns only its own small bookkeeping (error text, device
 * id, a few device flags). Device calls are asynchronous on the given stream (hipStream_t,
 * passed as void*; NULL = the default stream) unless stated otherwise. A handle is not
 * thread-safe: use one per host thread.
 *
 * Errors: every call returns MPOEVO_OK (0) or a negative status; nothing is thrown across the
 * ABI. mpoevo_last_error(h) returns the text of the last error of that handle (never NULL;
 * with h == NULL the last error of the calling thread's handle-free calls).
 */
#ifndef MPOEVO_H
#define MPOEVO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpoevo_ctx* mpoevo_handle;

enum {
  MPOEVO_OK = 0,
  MPOEVO_EINVAL = -1,       /* bad argument: null pointer, unknown enum, order out of range */
  MPOEVO_ESHAPE = -2,       /* inconsistent or unsupported dimensions */
  MPOEVO_ENOMEM = -3,       /* workspace (or output capacity) too small */
  MPOEVO_EHIP = -4,         /* a HIP runtime call failed */
  MPOEVO_ESOLVER = -5,      /* the FP64 SVD did not converge or a device wait timed out */
  MPOEVO_ENONFINITE = -6,   /* non-finite input (H blocks, tau) or non-finite matrix in truncate */
  MPOEVO_EUNSUPPORTED = -7  /* valid request the library does not implement */
};

enum { MPOEVO_FP64 = 0, MPOEVO_FP32 = 1, MPOEVO_BF16X3 = 2 };
enum { MPOEVO_V1_EXACT = 0, MPOEVO_V2_EXTENDED = 1 };
enum { MPOEVO_LEFT = 0, MPOEVO_RIGHT = 1 };

/* Handle on HIP device `device` (made current by every call that uses it). */
int mpoevo_create(mpoevo_handle* h, int device);
int mpoevo_destroy(mpoevo_handle h);
const char* mpoevo_last_error(mpoevo_handle h);
const char* mpoevo_version(void);

/*
 * mpo_build -- HOST ONLY, synchronous, thread-safe.
 * Order-N MPO for exp(tau H) (Sec. 3 Alg. 1; with variant V2 also Sec. 5 Alg. 3 on H^N before
 * the fold and Sec. 6 Alg. 4 after Sec. 4 Alg. 2).
 *   d, chi      physical dimension and the dimension of the middle level of H (Sec. 2.3).
 *   A, B, C, D  complex128 Jordan blocks of H = [[I, C, D], [0, A, B], [0, 0, I]]:
 *               A[chi][chi][d][d], B[chi][d][d], C[chi][d][d], D[d][d] (D is "Dloc").
 *   order       1..4;  tau_re, tau_im: the complex step (tau = -i dt for exp(-i dt H)).
 *   variant     MPOEVO_V1_EXACT (Alg. 1 + Alg. 2) or MPOEVO_V2_EXTENDED (Alg. 3, 1, 2, 4).
 *   inner_charge[chi], phys_charge[d]: optional U(1) charges (both NULL or both set).
 *   *w_out      receives the MPO bond dimension w.
 *   W_out       complex128 W[w][d][d][w] or NULL (size query: only *w_out is written);
 *               W_capacity = number of complex entries available at W_out.
 *   level_charge_out[w]: optional (needs the charges); charge of every MPO bond index.
 * Level (1,...,1) is bond index 0; the boundary vectors of a finite chain are l = r = e_0.
 * Errors: EINVAL (null blocks, order outside 1..4, bad variant), ENONFINITE (non-finite block
 * entry or tau), ENOMEM (W_capacity < w*d*d*w).
 */
int mpo_build(int d, int chi, const double* A, const double* B, const double* C, const double* D,
              int order, double tau_re, double tau_im, int variant,
              const int* inner_charge, const int* phys_charge,
              int* w_out, double* W_out, size_t W_capacity, int* level_charge_out);

/*
 * Dimensions of one site of the fit (shared by env_update and the workspace query):
 *   dims[0] Dbra_l, dims[1] Dket_l, dims[2] Dbra_r, dims[3] Dket_r, dims[4] d, dims[5] w_l,
 *   dims[6] w_r.  bra[Dbra_l][d][Dbra_r], ket[Dket_l][d][Dket_r], W[w_l][d][d][w_r].
 */

/*
 * env_update -- DEVICE, async on `stream`.
 * One environment step of the sweep (Sec. 2.2; cost O(w d D^3) of Table 1):
 *   side LEFT :  E_out[b'][beta][b]  = sum conj(bra[a'][s'][b']) E_in[a'][alpha][a]
 *                                          W[alpha][s'][s][beta] ket[a][s][b]
 *                E_in (Dbra_l, w_l, Dket_l) -> E_out (Dbra_r, w_r, Dket_r)
 *   side RIGHT:  E_out[a'][alpha][a] = sum conj(bra[a'][s'][b']) W[alpha][s'][s][beta]
 *                                          ket[a][s][b] E_in[b'][beta][b]
 *                E_in (Dbra_r, w_r, Dket_r) -> E_out (Dbra_l, w_l, Dket_l)
 * All tensors complex128 (prec FP64) or complex64 (prec FP32), device pointers. E_out must not
 * alias an input. Workspace: mpoevo_workspace_size(MPOEVO_CALL_ENV_UPDATE, ...).
 * Errors: EINVAL, ESHAPE (non-positive dims), ENOMEM (workspace too small), EHIP.
 */
int env_update(mpoevo_handle h, int side, int prec, const void* E_in, const void* bra,
               const void* W, const void* ket, void* E_out, const int* dims,
               void* workspace, size_t workspace_bytes, void* stream);

/*
 * env_update_noalloc -- DEVICE, async on `stream`. For callers that cannot allocate device
 * memory (code under stream/graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation, arguments and results as env_update, without a workspace argument. Its
 * intermediates live in a scratch array the library holds on each device from its load until
 * the process ends (MPOEVO_NOALLOC_SCRATCH_BYTES = 64 MiB per device); the call itself allocates
 * nothing, host or device, and never synchronises. Dimensions whose intermediates need more than
 * that (mpoevo_workspace_size(MPOEVO_CALL_ENV_UPDATE) minus its 32 MiB split-K share, e.g.
 * D = 256, w = 8 needs 17 MB in FP32 and 34 MB in FP64) are rejected with ENOMEM before any GPU
 * work. What the intermediates leave of the array serves as split-K scratch, so a product may be
 * split fewer ways than under env_update (same result within rounding). All calls on one device
 * share the array: calls that overlap in time on one device (different streams, or handles in
 * different threads) race and give wrong results; serialise them. Nothing in the array needs
 * clearing between calls (every byte read is written first in the same call).
 * Errors: as env_update; ENOMEM for oversized dimensions.
 */
#define MPOEVO_NOALLOC_SCRATCH_BYTES (64u << 20)
int env_update_noalloc(mpoevo_handle h, int side, int prec, const void* E_in, const void* bra,
                       const void* W, const void* ket, void* E_out, const int* dims, void* stream);

/*
 * local_apply -- DEVICE, async on `stream`.
 * nsites = 2: projected two-site tensor of the fit at bond (i, i+1) (the optimal two-site update):
 *   Theta[a'][s'][t'][c'] = sum L[a'][alpha][a] M1[a][s][b] W1[alpha][s'][s][beta]
 *                               M2[b][t][c] W2[beta][t'][t][gamma] R[c'][gamma][c]
 * dims: [0] Dbra_l, [1] Dket_l, [2] Dket_m, [3] Dket_r, [4] Dbra_r, [5] d, [6] w_l, [7] w_m,
 * [8] w_r.  L (Dbra_l, w_l, Dket_l), M1 (Dket_l, d, Dket_m), W1 (w_l, d, d, w_m),
 * M2 (Dket_m, d, Dket_r), W2 (w_m, d, d, w_r), R (Dbra_r, w_r, Dket_r); Theta shaped
 * (Dbra_l*d) x (d*Dbra_r). Workspace: mpoevo_workspace_size(MPOEVO_CALL_LOCAL_APPLY, dims).
 * nsites = 1: projected one-site tensor at site i (the optimal site at fixed bonds, Sec. 2.2,
 * Table 1 (ii)):
 *   Theta[a'][s'][b'] = sum L[a'][alpha][a] M1[a][s][b] W1[alpha][s'][s][beta] R[b'][beta][b]
 * dims: [0] Dbra_l, [1] Dket_l, [2] Dket_r, [3] Dbra_r, [4] d, [5] w_l, [6] w_r.
 * L (Dbra_l, w_l, Dket_l), M1 (Dket_l, d, Dket_r), W1 (w_l, d, d, w_r), R (Dbra_r, w_r, Dket_r);
 * W2 and M2 are not read (may be NULL); Theta shaped (Dbra_l*d) x Dbra_r. Workspace:
 * mpoevo_workspace_size(MPOEVO_CALL_LOCAL_APPLY1, dims).
 * Inputs complex128 (FP64) or complex64 (FP32); Theta is ALWAYS complex128 (the FP32 path
 * accumulates in float and widens on store).
 * Errors: EINVAL (nsites not 1 or 2, NULL pointers), ESHAPE, ENOMEM, EHIP.
 */
int local_apply(mpoevo_handle h, int nsites, int prec, const void* L, const void* W1,
                const void* W2, const void* M1, const void* M2, const void* R, void* Theta,
                const int* dims, void* workspace, size_t workspace_bytes, void* stream);

/*
 * truncate -- DEVICE, async on `stream`. FP64 SVD Theta = U S V^dag of an m x n complex128
 * matrix (row-major) by one-sided Jacobi (for max(m, n) <= 512 on R^dag of a column-pivoted
 * Householder QR of X = Theta^dag for LEFT, Theta for RIGHT, whose right singular vectors are the
 * kept factor; this converges in few sweeps even when the singular values spread over many
 * decades), keeping k = min(Dmax, m, n, #{sigma_i > max(cutoff *
 * sigma_1, 8 eps sqrt(max(m, n)) ||Theta||_F)}) >= 1 singular values (the truncation of the
 * two-site update; the second bound drops singular values at the rounding level of Theta).
 *   direction LEFT  (left-to-right sweep): A_out = U_k (left-orthonormal), B_out = S_k V_k^dag
 *   direction RIGHT (right-to-left sweep): A_out = U_k S_k, B_out = V_k^dag (right-orthonormal)
 * Outputs have the static capacity kcap = min(Dmax, m, n): A_out is m x kcap, B_out is kcap x n
 * (complex128, row-major); columns of A_out and rows of B_out at index >= k are zero.
 * k_dev (int), discarded_dev (double: sum_{i>=k} sigma_i^2 / sum sigma_i^2) and norm_dev
 * (double: ||S_k||) are DEVICE scalars (nullable); sigma_dev (double[min(m,n)], descending,
 * nullable). Theta is not modified. If the SVD does not converge within its sweep limit the
 * result is still written and *k_dev is negated (status is only visible on the device, or
 * through mpoevo_check_solver after a stream synchronisation).
 * Errors: EINVAL, ESHAPE (m or n outside 1..MPOEVO_SVD_MAX_DIM), ENOMEM, EHIP.
 */
#define MPOEVO_SVD_MAX_DIM 1024
int truncate(mpoevo_handle h, const void* Theta, int m, int n, int Dmax, double cutoff,
             int direction, void* A_out, void* B_out, int* k_dev, double* discarded_dev,
             double* norm_dev, double* sigma_dev, void* workspace, size_t workspace_bytes,
             void* stream);

/* After a stream synchronisation: MPOEVO_OK, or ESOLVER if any truncate/step issued on this
 * handle since the previous check did not converge (flag kept in device memory of the handle).
 * *max_sweeps (nullable) receives the largest number of Jacobi sweeps any of those SVDs took. */
int mpoevo_check_solver(mpoevo_handle h, int* max_sweeps);

/*
 * step -- one time step (Sec. 8.2: a variational sweeping optimisation of the time-evolved MPS
 * in every step): the MPS psi is replaced by the normalised two-site variational fit of W|psi>
 * with bonds <= Dmax.  Guess phi = psi brought to right-canonical form (FP64 SVD of each site
 * from the last to the second; skipped if opts->input_right_canonical), then opts->nsweeps
 * sweeps, each a left-to-right pass over the bonds (0,1)..(L-2,L-1) and a right-to-left pass
 * over the same bonds; at every bond the projected two-site tensor is split by `truncate`.
 * Synchronises `stream` once at the end (bond dimensions and statistics are read back).
 *   mps   psi on entry, phi on exit. site[i] is a device pointer to complex128
 *         [bond_dim[i]][d][bond_dim[i+1]] with capacity Dmax*d*Dmax entries; bond_dim (host,
 *         L+1 entries, bond_dim[0] = bond_dim[L] = 1) is updated in place.
 *   mpo   per-site complex128 W_i[w[i]][d][d][w[i+1]] (device); boundaries e_0 on bonds 0, L.
 *   opts  nsweeps in 1..4, prec, cutoff (relative singular value cutoff, e.g. 1e-14),
 *         input_right_canonical (1: psi is already right-canonical, skip the guess SVDs).
 *   stats nullable; filled after the synchronisation.
 * Workspace: mpoevo_workspace_size(MPOEVO_CALL_STEP, dims = {L, d, Dmax, wmax}, prec).
 * Errors: EINVAL, ESHAPE (L < 2, Dmax < 1, Dmax > MPOEVO_SVD_MAX_DIM/d), ENOMEM, EHIP,
 * ESOLVER (an SVD did not converge), ENONFINITE (the fitted norm is not finite).
 */
typedef struct {
  int L, d, Dmax;
  int* bond_dim;
  void** site;
  /* U(1) symmetry (nullable; both or neither): sector_table[b * Dmax + j], j < bond_dim[b], is the
     charge of index j of bond b, nondecreasing in j (the site tensors' bond indices sorted by
     charge), and phys_charge[s] that of physical index s. The site tensors must vanish unless
     q(b) = q(a) + phys_charge[s] (a U(1)-symmetric MPS stored densely in charge order) and the MPO
     must conserve the charge (W[alpha][s'][s][beta] = 0 unless l(alpha) + q(s') = q(s) + l(beta)
     for some level charges l, as mpo_build's level_charge_out gives). step then runs the U(1)
     two-site fit (Sec. 2.4 example; symmetric tensors): every truncation, and the canonical
     guess, factorises each charge block of the bond matrix by its own FP64 SVD and keeps the
     Dmax largest singular values over all blocks (k = min(Dmax, #{sigma > cutoff sigma_max}),
     ties to the lower charge), so the new bond's indices come sorted by charge; the contractions
     are the dense ones (they keep the vanishing blocks exactly zero). The tables of bonds 1..L-1
     are rewritten in place. Two-site updates only (nsites 1 gives EUNSUPPORTED, -1 means 2). */
  int* sector_table;
  const int* phys_charge;
} mpoevo_mps;

typedef struct {
  int L, d;
  const int* w;
  const void* const* site;
} mpoevo_mpo;

typedef struct {
  int nsweeps;
  int prec;
  double cutoff;
  int input_right_canonical;
  int profile;  /* 1: time the kernel classes with HIP events (adds host overhead); 2: time the
                   Jacobi kernel only (the other classes report zero); 0: none */
  int svd_cold_start; /* nonzero: every truncation starts Jacobi from Theta itself. Zero (the
                         default): a square bond matrix is first multiplied by the unitary the
                         previous truncation of the same bond left in the workspace (a singular
                         basis of that matrix), which leaves the same singular values and kept
                         vectors and converges in a few sweeps. The first truncation of a bond
                         in a step (Theta has moved by a whole time step since the last one),
                         rectangular bond matrices, and bonds below Dmax or found numerically
                         rank-deficient by the previous step (whose basis would need
                         completing) instead run Jacobi on R^dag of a column-pivoted QR (up to
                         512). The unitaries persist in the workspace between step calls on one
                         handle with the same workspace and chain shape; the caller must not
                         modify that workspace between such calls. With FP32 or BF16X3
                         contractions the Jacobi iteration ends after the sweep whose largest
                         relative inner product is at most 3e-5 (the next would leave about its
                         square, far below the contraction rounding); with FP64, after a sweep
                         that finds every pair below the rounding tolerance. */
  int nsites;   /* 2 (or 0): two-site updates, bonds adapt up to Dmax by SVD truncation (above).
                   1: one-site updates at the fixed bond dimensions of psi (Sec. 2.2, Table 1 (ii);
                   Sec. 8.2 keeps the bond dimension fixed): each site's projected tensor
                   L_i M_i W_i R_{i+1} becomes its FP64 Householder QR factor (blocked, without
                   pivoting; the left-to-right pass keeps Q of the (D_i d) x D_{i+1} matrix, the
                   right-to-left pass the adjoint Q of the transposed problem), no SVD and no
                   truncation;
                   a sweep is a left-to-right pass over the sites 0..L-2 and a right-to-left pass
                   over L-1..1, and after the last sweep the projected tensor of site 0 completes
                   phi (its norm is the fitted norm). Needs bond[i+1] <= d bond[i] after the guess
                   and d Dmax <= 512 (ESHAPE otherwise); stats: discarded weights 0, visits =
                   2 (L-1) nsweeps + 1 local updates, no Jacobi sweeps.
                   -1: automatic -- one-site when every bond of psi equals its largest possible
                   value min(Dmax, d^i, d^(L-i)) (and d Dmax <= 512); else, when some site has
                   both bonds at that value ("frozen" at the start of the step; d Dmax <= 512,
                   no zip-up guess, no U(1) charges), a mixed sweep: the visits of the two-site
                   sweep, where a position whose site (i going left to right, i + 1 going right
                   to left) has both bonds frozen takes that site's one-site update and the other
                   positions the two-site update; when the last visit is a one-site update, the
                   projected tensor of site 0 completes phi. If a two-site update leaves a frozen
                   bond below its value, the step is redone with two-site updates throughout
                   (stats->two_site_redo). Otherwise two-site. */
  int use_graph; /* 1: the step's device work (everything between the opening check of the
                   workspace and the closing read-back of ranks and statistics) is captured into a
                   HIP graph the second time a step with the same plan runs on this handle (the
                   first runs uncaptured, so that the tile tuner can time new product shapes) --
                   the plan being the shapes, options, buffers (workspace, site and MPO pointers),
                   the truncations' preconditioner state and the tuner's mode -- and replayed by
                   every later step with that plan (one launch instead of thousands). The handle
                   keeps the last 8 graphs; mpoevo_set_tuning starts new ones.
                   Not with profile or U(1) charges (ignored there). In a graph the Jacobi and QR
                   kernels are ordinary launches that need their workgroups resident together (the
                   graph runs one node at a time; other work on the device meanwhile can delay them
                   to their bounded-wait timeout, ESOLVER); the arithmetic is that of the
                   uncaptured step, so the results are the same bit for bit. 0: no graph. */
  int guess;     /* the MPS the sweeps start from. MPOEVO_GUESS_CANONICAL (0): psi, brought to
                   right-canonical form unless input_right_canonical. MPOEVO_GUESS_ZIPUP (1): the
                   zip-up application of W to psi (Sec. 2.2, Table 1 zip-up row), from the right
                   end, in FP64 whatever prec: at site i = L-1 .. 1 the matrix
                   X[(alpha, a), (s', k)] = sum W_i[alpha, s', s, beta] psi_i[a, s, b] C[k, beta, b]
                   (C: the carry, the right boundary level at the start) is split by the FP64 SVD
                   truncation of every bond (Dmax, cutoff), the site becomes V^dag and the carry
                   (U S)^T; site 0 is X at the left boundary level. The guess then has bonds up to
                   Dmax at once instead of growing from psi's during the sweeps (psi need not be
                   canonical). Two-site updates only, no U(1) charges, and every X must have at most
                   d Dmax rows, i.e. bond[i] w[i] <= d Dmax (EUNSUPPORTED otherwise): the zip-up
                   is for states with small bonds (a product state, the first steps of a quench).
                   MPOEVO_GUESS_AUTO (-1): the zip-up where it applies, nsites is not 1 and some
                   bond of psi is below its largest value min(Dmax, d^i, d^(L-i)) (the step then
                   runs two-site updates), else 0. */
} mpoevo_step_opts;

enum { MPOEVO_GUESS_AUTO = -1, MPOEVO_GUESS_CANONICAL = 0, MPOEVO_GUESS_ZIPUP = 1 };

#define MPOEVO_MAX_KERNEL_STATS 16
typedef struct {
  char name[224];   /* the kernel's name as the HIP runtime reports it, demangled (as profilers
                       list it); truncated to 223 characters */
  int kind;         /* 0: Jacobi kernel, 1: complex matrix product, 2: short-leg W contraction,
                       3: Householder QR with the explicit Q (one-site updates; work = its GFLOP) */
  int split_k;      /* 1: each timed interval also holds the sum of the split-K partial tiles */
  int launches;
  double ms;        /* summed durations (HIP events around each launch, on the step's stream) */
  double work;      /* algorithmic GFLOP (kinds 0 and 1; 8 flop per complex multiply-add for the
                       products) or GB read and written (kind 2) */
} mpoevo_kernel_stat;

typedef struct {
  double norm;              /* |<phi_hat|W psi>| = ||S|| at the last bond visit */
  double discarded_max;     /* largest discarded weight of any bond visit */
  double discarded_sum;     /* sum over the bond visits of the discarded weights */
  int visits;               /* number of bond visits (4 (L-1) for two sweeps) */
  int max_bond;             /* largest bond dimension of the result */
  double gflop;             /* algorithmic contraction work of the step (8 flop per complex MAC) */
  int svd_sweeps_max;       /* largest number of Jacobi sweeps any truncation of the step needed */
  /* filled when opts->profile: summed kernel durations (HIP events on the step's stream),
     launch counts and algorithmic work of the three kernel classes of the step */
  double t_jacobi_ms, jacobi_gflop;  /* one-sided Jacobi kernel; 36 mx flop per column pair visit */
  int n_jacobi;
  double t_gemm_ms, gemm_gflop;      /* complex matrix products (8 flop per complex MAC) */
  int n_gemm;
  double t_wmix_ms, wmix_gbyte;      /* short-leg contractions with W (bytes read + written) */
  int n_wmix;
  int svd_sweeps_total;     /* Jacobi sweeps summed over the bond truncations of the step */
  int svd_sweeps_hist[32];  /* number of bond truncations that took s sweeps (index min(s, 31)) */
  /* filled when opts->profile == 1: the timed launches grouped by kernel instance, longest summed
     duration first (at most MPOEVO_MAX_KERNEL_STATS; the rest are counted only in the class
     totals above) */
  int n_kernel_stats;
  mpoevo_kernel_stat kernel_stats[MPOEVO_MAX_KERNEL_STATS];
  int graph;                /* opts->use_graph: 0 the work was issued launch by launch, 1 it was
                               captured into a new graph (then launched), 2 a graph replayed it */
  int guess;                /* the guess the sweeps started from: 0 psi, 1 the zip-up */
  int one_site_visits;      /* visits that took the one-site update (all of them with nsites 1;
                               with nsites -1 those at sites whose two bonds were frozen) */
  int two_site_redo;        /* 1: the automatic mode's mixed sweep found a frozen bond shrunk by a
                               two-site update and the step was redone with two-site updates */
} mpoevo_step_stats;

int step(mpoevo_handle h, mpoevo_mps* mps, const mpoevo_mpo* mpo, const mpoevo_step_opts* opts,
         mpoevo_step_stats* stats, void* workspace, size_t workspace_bytes, void* stream);

/*
 * step_batched -- one time step of each of n independent chains (the method of `step`, Sec. 8.2,
 * applied to every chain), advanced concurrently: data parallelism across chains, each chain's
 * sweep staying sequential over its bonds.
 *   mps[c], mpo[c]  chain c as for step (own L, d, Dmax, MPO); no two chains (and no two sites)
 *                   may share a site buffer or a bond_dim array. Updated in place as by step.
 *   opts            shared by all chains (as for step).
 *   stats           nullable, else n entries (chain order), as for step.
 * Result for each chain: the same as `step` on that chain alone with a fresh workspace (the same
 * kernels run; only their interleaving across chains differs). The per-chain truncation
 * preconditioners persist per chain index in the workspace, as for step.
 * Synchronous: synchronises `stream` on entry (the inputs may have been written on it), runs the
 * chains on the handle's own worker streams and returns when every chain is done. The number of
 * worker streams is 4 (the hardware queues a process gets by default), or MPOEVO_BATCH_STREAMS
 * (1..16) from the environment, lowered if needed so that the truncation kernels of all streams
 * fit on three quarters of the device's compute units at once.
 * Workspace: mpoevo_workspace_size(MPOEVO_CALL_STEP_BATCHED, dims = {n, then L, d, Dmax, wmax of
 * each chain}, prec): the chains' step workspaces, 256-byte aligned, in chain order.
 * Errors: as for step (the message names the chain); EINVAL also for n outside
 * 1..MPOEVO_MAX_CHAINS or shared site buffers / bond arrays.
 */
#define MPOEVO_MAX_CHAINS 4096
int step_batched(mpoevo_handle h, int n, mpoevo_mps* mps, const mpoevo_mpo* mpo,
                 const mpoevo_step_opts* opts, mpoevo_step_stats* stats, void* workspace,
                 size_t workspace_bytes, void* stream);

/*
 * expectation -- <psi| O |psi> for an MPO O = l . O_1 ... O_L . r with boundary vectors l = e_left
 * on MPO bond 0 and r = e_right on MPO bond L: the diagnostics of a time step (Sec. 8.2) -- the
 * energy through the Hamiltonian MPO of Sec. 2.3 (left = 0, right = w - 1), a local observable
 * as a bond-1 MPO with the operator on one site, the norm with identities. FP64 throughout, by
 * the left environment recursion of env_update (E <- E . psi_i . O_i . conj(psi_i)).
 *   mps    as for step; not modified (bond_dim host, site[i] device complex128).
 *   mpo    per-site complex128 O_i[w[i]][d][d][w[i+1]] (device).
 *   left, right  boundary levels, 0 <= left < w[0], 0 <= right < w[L].
 *   out    device complex128 (two doubles), written on `stream`; no synchronisation.
 * Workspace: mpoevo_workspace_size(MPOEVO_CALL_EXPECTATION, dims = {L, d, Dmax, wmax}, FP64).
 * Errors: EINVAL (NULL arguments, levels out of range), ESHAPE, ENOMEM, EHIP.
 */
int expectation(mpoevo_handle h, const mpoevo_mps* mps, const mpoevo_mpo* mpo, int left, int right,
                void* out, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Tile choice of the complex matrix products (a property of the handle; host calls, no GPU work).
 * MPOEVO_TUNE_OFF (the default): every product takes the fixed planner rule -- the largest tile of
 *   the precision's table that gives at least one workgroup per compute unit, else the smallest
 *   tile with K split across workgroups and the partial tiles summed in a fixed order.
 * MPOEVO_TUNE_ON: the first product of each shape (precision, M, N, K, batch, output precision,
 *   operand layout) issued through this handle outside stream capture times every candidate plan
 *   (each tile of the table, unsplit and with the rule's split count; three runs after one warm-up,
 *   HIP events on the call's stream, which is synchronised: such a call blocks) and keeps the
 *   fastest for every later product of that shape. Shapes met during stream capture take the rule.
 * MPOEVO_TUNE_FROZEN: tuned shapes keep their plan; new shapes take the rule and are not tuned.
 * Every plan sums in a fixed order, so results are reproducible for a fixed table, but the rounding
 * of a product depends on the plan it takes. step_batched's chains use the handle's table and
 * never tune. clear != 0 empties the table before setting the mode.
 * Errors: EINVAL (NULL handle, unknown mode).
 */
enum { MPOEVO_TUNE_OFF = 0, MPOEVO_TUNE_ON = 1, MPOEVO_TUNE_FROZEN = 2 };
int mpoevo_set_tuning(mpoevo_handle h, int mode, int clear);

/*
 * The plan a product of M x N x K complex multiply-adds (times batch) in precision prec takes on
 * this handle, for operands contiguous along k (first factor) and n (second factor):
 *   plan[0] tile rows, plan[1] tile columns, plan[2] number of K splits, plan[3] 1 if the plan
 *   comes from the handle's tuned table, else 0 (the fixed rule).
 *   entries (nullable): number of shapes in the tuned table.
 * Errors: EINVAL (NULL handle or plan, unknown precision), ESHAPE (non-positive sizes).
 */
int mpoevo_product_plan(mpoevo_handle h, int prec, int M, int N, int K, int batch, int* plan,
                        int* entries);

/*
 * overlap -- <bra| O |ket> for an MPO O = l . O_1 ... O_L . r (boundary levels as for expectation)
 * and two MPS on the same chain (their bond dimensions may differ): FP64 throughout, by the left
 * environment recursion E <- E . ket_i . O_i . conj(bra_i). The norms and overlaps of the method
 * (Sec. 8.2: fidelities of the evolved state) in double precision whatever the contraction
 * precision of the step that produced the states: with O the evolution MPO, ket = psi and bra the
 * normalised fitted phi, |<phi|W psi>|^2 / ||W psi||^2 = 1 - the step's truncation error.
 *   out   device complex128 (two doubles), written on `stream`; no synchronisation.
 * Workspace: mpoevo_workspace_size(MPOEVO_CALL_EXPECTATION, dims = {L, d, max(bra Dmax, ket Dmax),
 * wmax}, FP64). Errors: as expectation (either MPS).
 */
int overlap(mpoevo_handle h, const mpoevo_mps* bra, const mpoevo_mpo* mpo, const mpoevo_mps* ket, int left,
            int right, void* out, void* workspace, size_t workspace_bytes, void* stream);

/* Workspace sizes in bytes for the device calls (dims as documented for each call). */
enum { MPOEVO_CALL_ENV_UPDATE = 0, MPOEVO_CALL_LOCAL_APPLY = 1, MPOEVO_CALL_TRUNCATE = 2,
       MPOEVO_CALL_STEP = 3, MPOEVO_CALL_EXPECTATION = 4, MPOEVO_CALL_STEP_BATCHED = 5,
       MPOEVO_CALL_LOCAL_APPLY1 = 6 };
/* dims: ENV_UPDATE -> the 7 env_update dims; LOCAL_APPLY -> the 9 local_apply dims;
 * TRUNCATE -> {m, n}; STEP and EXPECTATION -> {L, d, Dmax, wmax};
 * STEP_BATCHED -> {n, L_0, d_0, Dmax_0, wmax_0, ..., L_{n-1}, d_{n-1}, Dmax_{n-1}, wmax_{n-1}}. */
int mpoevo_workspace_size(int call_id, const int* dims, int prec, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* MPOEVO_H */
