/*
 * mpo.h -- C ABI of the MI355X (gfx950) MPO bond-update library (libmpo.so).
 *
 * The library holds one matrix product operator M per handle, in device
 * memory, and applies to it the operations of the middle-MPO contraction of
 * mirrored peaked circuits (Kremer & Dupuis, Sec. II and Alg. 1):
 *
 *   mpo_init_identity     M <- I^{(x)N}                         (Alg. 1, Sec. II.A)
 *   mpo_absorb_gate_pair  two-site absorption + truncated SVD   (Sec. II.B.1)
 *   mpo_unswap_sweep      greedy SWAP extraction, M = P_L M~ P_R (Sec. II.B.2, Eq. (1), App. A.1, A.2)
 *   mpo_extract_peak      M|0...0> as an MPS, greedy peak readout (Alg. 1 last step, Sec. II.C)
 *
 * Representation.  Site i is a tensor B_i[a][s][b] of shape chi_{i-1} x 4 x chi_i
 * (chi_{-1} = chi_{N-1} = 1) with physical index s = 2*o + p, o the output bit
 * and p the input bit.  The MPO is kept in Vidal/Hastings form: every B_i is
 * right-canonical as a vectorised tensor and bond i carries the operator-Schmidt
 * values lambda_i (FP64).  The identity has B_i = (1, 0, 0, 1)/sqrt(2), so the
 * vectorised MPO has unit norm.
 *
 * Gates.  A gate is a 4x4 complex matrix, row-major, interleaved (re, im)
 * doubles (32 doubles), in the basis |q_bond q_bond+1> with site `bond` the
 * most significant bit.  g_out acts on the output legs (M <- G M; gates of the
 * circuit half applied after the midpoint), g_in on the input legs (M <- M G;
 * gates of the half applied before it).  NULL means identity.  Gate data is
 * read before the call returns.
 *
 * Truncation (Sec. II.B.1, App. A.4).  After each SVD the kept rank k is
 *   MPO_CUT_REL_SV:            #{ s_j > cutoff * s_0 }
 *   MPO_CUT_DISCARDED_WEIGHT:  smallest k with sum_{j>=k} s_j^2 <= cutoff * sum_j s_j^2
 * then k <- min(k, chi_max) and k >= 1.  The decision is taken in FP64 in
 * every precision.  Kept values are not renormalised.
 *
 * Streams.  All device work of a handle is enqueued on the HIP stream given at
 * init (NULL = the default stream).  Calls that return host data synchronise
 * that stream.  An absorption waits on the stream too, also with
 * info == NULL: the Jacobi SVD reads its convergence flags back once per sweep
 * (the sweep count is data dependent and decided on the host), and the kept
 * rank k, read back before the write-back, sets the shapes of the write-back
 * launches.  Only the write-back kernels may still be running when an
 * absorption returns; later work on the stream is ordered after them.  A
 * handle is not thread-safe; different handles may be used from different
 * threads on different streams.
 *
 * Errors.  Every call returns an mpo_status_t; no C++ exception crosses the
 * ABI.  On a negative status of an absorption (or of any call that changes a
 * single update) the MPO is unchanged: all checks and allocations happen
 * before the first write, and the device-side failure flags (non-finite
 * singular values, a QR panel barrier that gave up) are read back before the
 * write-back.  mpo_unswap_sweep is a sequence of such updates: after a failure
 * the swaps accepted before it stay applied and are reported in the log.
 * mpo_last_error() gives a message.
 *
 * Memory.  The handle owns its device memory (hipMalloc, or the alloc/free
 * hooks of mpo_config_t); the caller owns every host array passed in.  Site
 * tensors are allocated at init for their largest possible shape, so later
 * calls do not allocate for the MPO itself; SVD workspaces grow on demand and
 * are kept until mpo_free.
 */
#ifndef MPO_H
#define MPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpo_ctx* mpo_handle_t;

typedef enum {
  MPO_OK = 0,
  MPO_WARN_NOCONV = 1,   /* result written, but a Jacobi SVD reached its sweep cap */
  MPO_EINVAL = -1,       /* bad argument (range, NULL, inconsistent sizes)        */
  MPO_ENOMEM = -2,       /* device allocation failed                             */
  MPO_EHIP = -3,         /* HIP runtime error, or a device-side wait that gave up */
  MPO_ENUMERIC = -4,     /* NaN/Inf in a gate or in the singular values          */
  MPO_EOVERFLOW = -5     /* log truncated at log_cap (the sweep itself completed) */
} mpo_status_t;

typedef enum { MPO_CUT_REL_SV = 0, MPO_CUT_DISCARDED_WEIGHT = 1 } mpo_cutoff_mode_t;

/* Arithmetic of the contraction and SVD kernels.  The truncation decision,
 * rotation angles, lambdas and the peak readout are FP64 in all three. */
typedef enum {
  MPO_FP64 = 0,             /* complex128 tensors, FP64 MFMA                          */
  MPO_FP32 = 1,             /* complex64 tensors, FP32 arithmetic                      */
  MPO_MIXED_SPLITBF16 = 2   /* complex64 tensors, Jacobi Gram matrices as
                               split-BF16 MFMA products with FP32 accumulation,
                               converged to a loose tolerance (1e-3); the operand
                               rotated on FP32 MFMA.  (On the accumulate route,
                               theta's operand is rotated in split-BF16 too and
                               updates that keep vectors re-orthogonalise the
                               accumulated rotations in FP64 and recompute the
                               operand from R.)                                */
} mpo_precision_t;
/* SVD of the update (Sec. II.B.1).  FP64: QR of (lambda theta)^dag = Q R, block
 * one-sided Jacobi on L = R^dag with the rotations accumulated (V = Q W).
 * FP32 and mixed: a second QR, L = Q2 R2, and the one-sided Jacobi on R2^dag
 * without accumulation: the right singular vectors are Q times the unit-scaled
 * converged columns, made orthonormal by Newton-Schulz steps after the
 * truncation decision (the environment variable MPO_SVD=accumulate, read when
 * a handle is created, selects the FP64 route for them instead). */

typedef struct {
  int32_t n;              /* number of sites (qubits), >= 2                      */
  int32_t chi_max;        /* bond-dimension cap (App. A.4), 1..1024              */
  double cutoff;          /* SVD cutoff epsilon (App. A.4)                       */
  int32_t cutoff_mode;    /* mpo_cutoff_mode_t                                  */
  int32_t precision;      /* mpo_precision_t                                    */
  int32_t max_sweeps;     /* Jacobi sweep cap per SVD; 0 = default (30)          */
  double jacobi_tol;      /* Jacobi off-diagonal tolerance |g_ij| <= tol sqrt(g_ii g_jj);
                             0 = default: 8 sqrt(m) eps of the working precision
                             (FP64, FP32), 1e-3 for the split-BF16 sweeps of
                             the mixed form (whose values are re-derived to
                             second order in it)                             */
  int64_t tau_elems;      /* Alg. 1 threshold tau on size(M) (App. A.4), read by
                             mpo_tau_reached; <= 0 = never reached            */
  /* Device-memory hooks.  When `alloc` is non-NULL every device buffer of the
   * handle (site tensors, bond vectors, SVD workspaces, temporaries) comes
   * from alloc(bytes, alloc_ctx) and goes back through free(ptr, alloc_ctx);
   * alloc returns NULL on failure (the call then fails with MPO_ENOMEM and the
   * MPO is unchanged).  Buffers must be usable by work on the handle's stream
   * and 256-byte aligned.  NULL hooks: hipMalloc / hipFree. */
  void* (*alloc)(size_t bytes, void* alloc_ctx);
  void (*free)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
} mpo_config_t;

typedef struct {
  int32_t chi_new;          /* kept rank k                                     */
  int32_t sweeps;           /* Jacobi sweeps used                              */
  double discarded_weight;  /* sum of dropped s_j^2 (absolute)                 */
  double total_weight;      /* sum of all s_j^2                                */
  int32_t panel_rotations;  /* 32-column panels rotated over all sweeps        */
  int32_t reserved;
} mpo_update_info_t;

typedef struct {
  int32_t schedule;   /* 0 = sequential (Alg. 1), 1 = parallel (App. A.1)          */
  int32_t relaxed;    /* 1 = also accept swaps that keep the bond (App. A.2)       */
  int32_t max_iters;  /* App. A.4; parallel: full 6-batch cycles, sequential:
                         max_iters * (n-1) accepted swaps; 0 = 20                  */
} mpo_unswap_opts_t;

typedef struct {
  int32_t side;   /* 0 = left (output legs, P_L), 1 = right (input legs, P_R), 2 = both */
  int32_t bond;   /* SWAP acts on sites (bond, bond+1)                                  */
} mpo_swap_t;

/* Alg. 1, "Initialize MPO M <- I^{(x)N}": allocates the handle and all site
 * tensors (shape caps from chi_max and the 4^i edge bounds), writes the
 * identity.  `hip_stream` is a hipStream_t or NULL.  *out receives the handle. */
mpo_status_t mpo_init_identity(const mpo_config_t* cfg, void* hip_stream, mpo_handle_t* out);

/* Sec. II.B.1: absorbs g_out (output legs) and g_in (input legs) at sites
 * (bond, bond+1): theta = (G_out (x) G_in^T) lambda_{bond-1} B_bond B_bond+1
 * as a (4 chi_l) x (4 chi_r) matrix, truncated SVD theta = U S V^dag,
 * B_bond+1 <- V_k^dag, B_bond <- (theta without lambda) V_k, lambda_bond <- s_<k.
 * bond in [0, n-2].  `info` may be NULL. */
mpo_status_t mpo_absorb_gate_pair(mpo_handle_t h, int32_t bond, const double* g_out,
                                  const double* g_in, mpo_update_info_t* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * absorption as mpo_absorb_gate_pair, same kernels and same result, with
 * every SVD workspace carved out of a static device array of 64 MiB (one copy
 * per GPU, held until the process ends) instead of being allocated.  The call
 * makes no hipMalloc/hipFree and no call of the alloc hook.  An update whose
 * workspace does not fit (roughly theta above 512 x 512 in FP64, 724 x 724 in
 * FP32 and in the mixed form) fails with MPO_EINVAL and the MPO unchanged.
 * Kernel timing must be off.  The call synchronises the handle's stream
 * before it returns.  All calls on one GPU share the array: calls that
 * overlap in time on one GPU (from different host threads) race. */
mpo_status_t mpo_absorb_gate_pair_noalloc(mpo_handle_t h, int32_t bond, const double* g_out,
                                          const double* g_in, mpo_update_info_t* info);

/* Batched absorption of `count` updates on pairwise non-adjacent bonds
 * (|bond_a - bond_b| >= 2), which are independent in Vidal form.  g_out / g_in
 * hold `count` gates of 32 doubles each; a NULL array means identity for all,
 * and a gate whose 32 entries are all zero also means identity.  `info` may be
 * NULL or hold `count` entries. */
mpo_status_t mpo_absorb_batch(mpo_handle_t h, int32_t count, const int32_t* bonds,
                              const double* g_out, const double* g_in, mpo_update_info_t* info);

/* Sec. II.B.2 / Alg. 1 (schedule 0) or App. A.1 (schedule 1): SWAP trials from
 * the left, right or both sides, each followed by the truncated SVD; a trial
 * is kept when it lowers (relaxed: does not raise) its bond's dimension.
 * Sequential: largest available bond first (ties: lowest index), best of
 * L/R/B by (k, discarded weight, side order).  Parallel: batches in the order
 * both-even, both-odd, left-even, left-odd, right-even, right-odd until a full
 * cycle lowers nothing.  Trials are values-only SVDs; an accepted swap is then
 * committed with vectors, and the committed rank decides: a commit that does
 * not lower (relaxed: raises) the bond is undone from a copy of the two sites
 * and the bond vector, and neither logged nor counted as a reduction (in the
 * mixed form a trial's rank can differ from the commit's near the cutoff).  A
 * trial whose inputs (B_b, B_b+1, lambda_b-1) are unchanged since its last
 * evaluation on the same side reuses that result (bit-identical).  Accepted
 * swaps are written to log[0..log_cap) in order; *n_accepted gets the total
 * count (which may exceed log_cap, then MPO_EOVERFLOW is returned after the
 * sweep completed). */
mpo_status_t mpo_unswap_sweep(mpo_handle_t h, const mpo_unswap_opts_t* opts, mpo_swap_t* log,
                              int32_t log_cap, int32_t* n_accepted);

/* Alg. 1 last step and Sec. II.C: A_i = B_i[:, s in {0, 2}, :] (input legs
 * projected on |0>), exact right environments, then a left-to-right greedy
 * conditional argmax (ties -> 0).  bits_per_site[n] receives site bits,
 * *prob the product of the chosen conditionals (the normalised probability of
 * that string) and *norm2 = <psi|psi>.  Either pointer may be NULL. */
mpo_status_t mpo_extract_peak(mpo_handle_t h, uint8_t* bits_per_site, double* prob, double* norm2);

/* Sec. II.C (sampling the output state): M|0...0> as an MPS, `count`
 * samples drawn from the left, site i's bit of sample s being 0 when
 * uniforms[s * n + i] < P(bit 0 | the sample's bits at sites < i), the
 * conditionals computed exactly in FP64 from the right environments.  The
 * random numbers are the caller's (count x n doubles in [0, 1), row-major),
 * so a sample is a deterministic function of its row.  site_bits[count * n]
 * receives the bits per site (row s = sample s); probs[count] (may be NULL)
 * the normalised probability of each sampled string.  MPO_ENUMERIC when a
 * conditional weight is not finite.  Device workspace: the environments
 * (sum_i chi_i^2 complex128) plus about 5 * count * max chi complex128. */
mpo_status_t mpo_sample(mpo_handle_t h, int32_t count, const double* uniforms, uint8_t* site_bits,
                        double* probs);

/* ---- helpers ------------------------------------------------------------ */
void mpo_free(mpo_handle_t h);
/* dims[n-1] receives chi_0 .. chi_{n-2}. */
mpo_status_t mpo_bond_dims(mpo_handle_t h, int32_t* dims);
/* size(M) = sum_i chi_{i-1} * 4 * chi_i  (the tau test of Alg. 1). */
mpo_status_t mpo_total_elements(mpo_handle_t h, int64_t* out);
/* lambda_bond into out[0..cap), *count = chi_bond. */
mpo_status_t mpo_singular_values(mpo_handle_t h, int32_t bond, double* out, int32_t cap, int32_t* count);
/* Copies site i (chi_{i-1} x 4 x chi_i complex, interleaved, as complex128)
 * into out (cap doubles); *chi_l / *chi_r receive its shape. */
mpo_status_t mpo_read_site(mpo_handle_t h, int32_t site, double* out, int64_t cap,
                           int32_t* chi_l, int32_t* chi_r);
/* Replaces the whole state: dims[n-1] bond dimensions, sites = concatenation
 * of all site tensors (complex128 interleaved, row-major [a][s][b]), lams =
 * concatenation of all bond vectors.  Values are converted to the handle's
 * precision.  The caller is responsible for the state being in Vidal form. */
mpo_status_t mpo_load_state(mpo_handle_t h, const int32_t* dims, const double* sites,
                            const double* lams);
mpo_status_t mpo_sync(mpo_handle_t h);
/* App. A.3 (adaptive side selection absorbs the next layer of each side into
 * its own copy of the MPO and keeps the smaller): makes dst an exact copy of
 * src's state (bond dimensions, site tensors, bond vectors).  Both handles
 * must have the same n, precision and chi_max.  Waits for src's stream, copies
 * device to device on dst's stream and returns when the copy is complete.
 * dst's counters are kept; its unswap-trial memo no longer applies. */
mpo_status_t mpo_copy_state(mpo_handle_t dst, mpo_handle_t src);
/* Alg. 1's test "size(M) >= tau" with tau = cfg.tau_elems: *reached = 1 when
 * it holds (never when tau_elems <= 0); *size (may be NULL) gets size(M). */
mpo_status_t mpo_tau_reached(mpo_handle_t h, int32_t* reached, int64_t* size);
/* One SWAP trial of Sec. II.B.2 at `bond` (side 0 = L, 1 = R, 2 = B): the
 * values-only truncated SVD that mpo_unswap_sweep decides on; info receives
 * its k and weights.  The MPO is not changed. */
mpo_status_t mpo_trial_swap(mpo_handle_t h, int32_t bond, int32_t side, mpo_update_info_t* info);
/* Counters since init: out[0] committed bond updates, out[1] SWAP-trial SVDs
 * run, out[2] trials served from the unchanged-input memo, out[3] unswap
 * commits undone, out[4] device allocations made through the alloc hook,
 * out[5] Jacobi sweeps replayed from a captured graph, out[6] sweep graphs
 * captured.
 * Up to `cap` entries are written. */
mpo_status_t mpo_counters(mpo_handle_t h, int64_t* out, int32_t cap);

/* ---- groups: one batch of bond updates across several MPOs -------------- *
 * A group owns workspace and a stream but no MPO.  mpo_group_absorb applies
 * `count` updates, update p on handles[p] at bonds[p] with gates g_out/g_in
 * (32 doubles each, all-zero or NULL array = identity), through the same
 * batched kernels as mpo_absorb_batch; the per-update arithmetic is identical
 * to a call on the handle alone.  Every handle must have the group's
 * precision, bonds of one handle must be pairwise non-adjacent, and the
 * handles' own streams must be idle (true between calls, since calls that
 * return results synchronise).  Errors leave every MPO unchanged.  This is the
 * building block of the batched and served forms: updates of many resident
 * circuits share launches. */
typedef struct mpo_group_s* mpo_group_t;
mpo_status_t mpo_group_create(int32_t precision, void* hip_stream, mpo_group_t* out);
void mpo_group_free(mpo_group_t g);
mpo_status_t mpo_group_absorb(mpo_group_t g, int32_t count, const mpo_handle_t* handles, const int32_t* bonds,
                              const double* g_out, const double* g_in, mpo_update_info_t* info);
/* The parallel unswap schedule (App. A.1; schedule must be 1 in opts) run on
 * `count` handles in lockstep: in each (cycle, side, parity) batch the SWAP
 * trials of every handle still in the loop share launches, and so do the
 * accepted commits.  A handle leaves after a cycle without a reduction (or
 * after opts->max_iters cycles), exactly as in mpo_unswap_sweep, and its log,
 * decisions and resulting MPO are those of mpo_unswap_sweep on it alone.
 * logs: count x log_cap_each entries, row p for handles[p]; n_accepted[p]
 * receives the number of accepted swaps of handle p.  Returns MPO_EOVERFLOW
 * when a row was truncated, MPO_WARN_NOCONV when a Jacobi SVD hit its sweep
 * cap.  Handles must be distinct and have the group's precision. */
mpo_status_t mpo_group_unswap(mpo_group_t g, int32_t count, const mpo_handle_t* handles,
                              const mpo_unswap_opts_t* opts, mpo_swap_t* logs, int32_t log_cap_each,
                              int32_t* n_accepted);
/* as mpo_profile, for the group's launches */
mpo_status_t mpo_group_profile(mpo_group_t g, int32_t on, double* ms_out, int64_t* launches_out);
const char* mpo_group_last_error(mpo_group_t g);

/* Kernel timing.  While profiling is on, every kernel launch of the handle is
 * bracketed by HIP events on the handle's stream and its device time is added
 * to one of the classes below.  A call synchronises the stream, writes the
 * accumulated milliseconds and launch counts of each class (either pointer may
 * be NULL), resets them, and then switches profiling on (on != 0) or off. */
enum {
  MPO_PROF_THETA_GEMM = 0,     /* theta0 = B_i B_{i+1} (MFMA complex GEMM)        */
  MPO_PROF_GATE = 1,           /* gate pair + lambda, (lambda theta)^dag          */
  MPO_PROF_JACOBI_INIT = 2,    /* V = I, padding                                  */
  MPO_PROF_JACOBI_GRAM = 3,    /* panel Gram matrices of one round-robin step     */
  MPO_PROF_FINALIZE = 4,       /* column norms, sort, truncation decision         */
  MPO_PROF_WRITEBACK = 5,      /* V_k = Q [W_k; 0], B_{i+1} <- V_k^dag, lambda      */
  MPO_PROF_WRITEBACK_GEMM = 6, /* B_i <- theta_noLambda V_k (MFMA complex GEMM)    */
  MPO_PROF_QR = 7,             /* Householder QR preconditioner of the SVD         */
  MPO_PROF_REORTH = 8,         /* mixed form: FP64 re-orthogonalisation, A = L W   */
  MPO_PROF_JACOBI_EVD = 9,     /* FP64 EVD of every panel Gram matrix of a step    */
  MPO_PROF_JACOBI_ROT = 10,    /* panel rotations of a step                        */
  MPO_PROF_CLASSES = 11
};
mpo_status_t mpo_profile(mpo_handle_t h, int32_t on, double* ms_out, int64_t* launches_out);
/* Launch choices of the Jacobi sweeps (batching form): per bucket (precision,
 * operand width rounded up to a power of two, batch size class) the rotation's
 * row chunk (64, 128 or 256 rows) and whether a sweep is captured as a HIP
 * graph and replayed.  An autotuner in the library measures every choice on
 * the batches it runs (wall time per round-robin step) and keeps the fastest;
 * the choices never change results (bit-identical).  MPO_AUTOTUNE=0 turns it
 * off; MPO_TUNE_CACHE=<file> loads earlier decisions and appends new ones,
 * one line per bucket: "gfx950 <precision> r<width> b<class> rrc=<rows>
 * graph=<0|1> us_per_step=<t>".  Writes the current table (decided buckets
 * and buckets still being measured) into out[0..cap) as text and returns its
 * full length. */
int32_t mpo_tuning_report(char* out, int32_t cap);
/* Sets the sweep launch choices process-wide: -1 = the autotuner, -2 = fixed
 * defaults (no tuning), 0..5 = one choice for every batch (row chunk 64, 128,
 * 256 without capture, then the same three with capture). */
mpo_status_t mpo_tuning_set(int32_t mode);
const char* mpo_last_error(mpo_handle_t h);
/* Library build string (kernels compiled for, precision variants). */
const char* mpo_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPO_H */
