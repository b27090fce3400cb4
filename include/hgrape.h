/*
 * hgrape.h -- C ABI of the hard-coded-gradient (HG) GRAPE cost+gradient
 * library for AMD Instinct MI355X (gfx950).
 *
 * Method: Lu, Joshi, Dinh, Koch, "Optimal control of large quantum systems:
 * assessing memory and runtime performance of GRAPE", arXiv:2304.06200.
 *
 *   H_n   = H_0 + sum_k u[k][n] H_k,  piecewise constant over N steps of dt
 *           (Sec. II; several control channels as in its footnote)
 *   psi_n = exp(-i H_n dt) psi_{n-1}   approximated by (T_m(B_n))^s psi_{n-1},
 *           B_n = -i dt H_n / s, T_m(B) = sum_{q<=m} B^q/q!  (Sec. III.B)
 *   (m_n, s_n): smallest s, then smallest m, with E_A(m, s) <= tau
 *           (Sec. III.B rule, App. C bound; ||A_n||_1 computed exactly in FP64)
 *   cost  C = w_fid (1 - |g|^2) + w_pen C2,
 *           g  = (1/S) sum_h <phi_T^h|psi_N^h>       (Sec. III.A, C1^st / C1^g)
 *           C2 = 1/(N S) sum_h sum_{n=1..N} <psi_n^h|Omega|psi_n^h>   (App. A, C2^st)
 *   grad  dC/du[k][n] = 2 Re sum_h <Lambda_n^h| dU_n/du_k |psi_{n-1}^h>
 *           (Sec. III.A eqs. stgradient/gategradient, App. A eq. C2stgrad),
 *           dU_n/du_k psi by the auxiliary block matrix [[A, E_k],[0, A]]
 *           (Sec. III.B, eq. auxiliary equation), with the forward-backward
 *           sweep of Sec. III.C: states are rebuilt backwards by inverse
 *           propagation, nothing per time step is stored.
 *
 * Conventions
 *   - Every function returns hg_status; no exception crosses the ABI.  On an
 *     error, hg_last_error() returns a thread-local message with the detail.
 *   - Complex numbers are interleaved (re, im) pairs of doubles at the ABI.
 *   - A state block is [S][dim]: state h occupies dim consecutive complex
 *     numbers.  Batched arrays add a leading [n_batch] dimension.
 *   - hg_eval_desc arrays are DEVICE pointers (memory of the context's
 *     device, e.g. from hipMalloc or a torch tensor), except where a field
 *     says "host".  Results' scalar fields are host memory; grad is device.
 *   - The library never takes ownership of caller memory.  Operators are
 *     copied to the device at hg_problem_create.
 *   - Thread safety: a problem is immutable after creation and may be used
 *     by concurrent hg_eval calls on different streams.  A context may be
 *     used from several threads.
 */
#ifndef HGRAPE_H
#define HGRAPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HG_OK = 0,
  HG_ERR_INVALID_ARG = 1,           /* bad size, pointer, flag or unnormalised psi0 */
  HG_ERR_NOT_HERMITIAN = 2,         /* H_0 or some H_k is not Hermitian to 1e-12 relative */
  HG_ERR_NONFINITE = 3,             /* NaN/Inf in operators, amplitudes or dt */
  HG_ERR_TOLERANCE_UNREACHABLE = 4, /* no (m, s) meets E_A <= tau for some step */
  HG_ERR_OUT_OF_MEMORY = 5,         /* device allocation failed / over budget */
  HG_ERR_DEVICE = 6,                /* a HIP runtime call failed */
  HG_ERR_BUSY = 7,                  /* server queue full */
  HG_ERR_CANCELLED = 8,             /* request cancelled before it ran */
  HG_ERR_UNSUPPORTED = 9            /* shape outside what the kernels are built for */
} hg_status;

/* Arithmetic of the Taylor products.  HG_C64: products in FP32; the state
 * vectors the sweeps carry (psi, and Lambda backwards), norms, overlaps,
 * penalty and reductions in FP64.  HG_C128: everything FP64. */
typedef enum { HG_C64 = 0, HG_C128 = 1 } hg_dtype;
typedef enum { HG_MODE_RECONSTRUCT = 0, HG_MODE_CHECKPOINT = 1 } hg_mode;
/* Choice of (m, s) per step under the bound E_A(m, s) <= tau of App. C:
 * the paper's rule (smallest s, then smallest m; Sec. III.B) or the fewest
 * products mu = m s (ties: smaller s), the alternative Sec. III.B mentions and
 * sets aside because the minimisation costs more than it saves there. */
typedef enum { HG_PLAN_SMALLEST_S = 0, HG_PLAN_MIN_MU = 1 } hg_plan_rule_t;
/* How each step's propagator and its derivative are applied:
 *   TAYLOR  the Taylor scaling-and-squaring action with the auxiliary block
 *           matrix (Sec. III.B), any storage;
 *   DIAG    diagonalisation of H_n per step (App. F, eqs. matrix dia and
 *           propagator der): U_n = V e^{-i dt D} V^H, dU_n/du_k from the
 *           divided differences of exp in the eigenbasis; dense storage only;
 *   AUTO    dense storage: DIAG when the Taylor products would cost more
 *           (Sec. V: Taylor ~ mu d^2 S per step against d^3 + d^2 S), i.e. when
 *           mean mu * S >= c (d + S), c = 40 (complex128) or 200 (complex64)
 *           from the measured crossover; else TAYLOR. */
typedef enum { HG_METHOD_TAYLOR = 0, HG_METHOD_DIAG = 1, HG_METHOD_AUTO = 2 } hg_method_t;

/* A host CSR matrix of complex128 values (dim x dim). */
typedef struct {
  int64_t n;                 /* number of rows (= dim) */
  const int64_t* indptr;     /* host, [n + 1] */
  const int32_t* indices;    /* host, [indptr[n]], column indices in [0, n) */
  const double* values;      /* host, [2 * indptr[n]] interleaved complex128 */
} hg_csr;

typedef struct hg_ctx hg_ctx;
typedef struct hg_problem hg_problem;

/* Create a context bound to HIP device `device_ordinal`.  Also raises the
 * release threshold of the device's default memory pool (evaluation
 * workspaces then stay pooled between calls) and looks up, with the device
 * current, the device address of the fixed scratch array of hg_eval_noalloc. */
hg_status hg_create(int device_ordinal, hg_ctx** out);
hg_status hg_destroy(hg_ctx* ctx);
const char* hg_status_string(hg_status s);
const char* hg_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t hg_version(void);

/* Build a problem: drift H0, n_ctrl control operators Hk[k] (all dim x dim,
 * Hermitian) and an optional diagonal penalty operator Omega (host [dim]
 * real, or NULL for no penalty).  The union sparsity pattern of H0 and all
 * Hk is stored on the device by diagonals (DIA: one value per row and union
 * diagonal, zero outside the matrix), each operator's values on it; each Hk
 * also gets its own diagonals for the derivative products.  Duplicate CSR
 * entries are summed, explicit zeros dropped.  The main diagonal and the
 * other diagonals on which every operator is real come first (B is purely
 * imaginary there; App. D's sparse storage, laid out for the GPU).
 * Patterns that are not a few diagonals (more than 13 union diagonals, or
 * more than 4 in a control: e.g. a qubit register's bit flips, offsets
 * +-2^j) are stored row-indexed instead (ELL: per row up to 13 slots of
 * column and value, the main diagonal first; per control at most 2 entries
 * per row), swept by the same kernels with per-row gather columns, one
 * workgroup per column.
 * A state column is swept by one workgroup holding its term vectors in LDS
 * (Sec. III.C's forward-backward sweep per state).  When a column does not
 * fit one workgroup in some precision (complex128 beyond about 2048 rows,
 * either precision beyond 4096), the problem also gets a split layout: the
 * rows, seen as blocks of L (row = t L + c, every union offset either a
 * multiple of L or short and inside its block -- e.g. the cavity index of a
 * transmon x cavity basis), are divided by c-range over P co-resident
 * workgroups that exchange their edge rows after every Taylor term.
 * Errors: INVALID_ARG (bad CSR, dim < 1, n_ctrl < 0), NOT_HERMITIAN,
 * NONFINITE, UNSUPPORTED (a row with more than 13 entries of the union
 * pattern, or a control with more than 2 entries in a row, when the pattern
 * needs row-indexed storage; n_ctrl > 16, dim > 65536, or a column too long
 * for one workgroup in both precisions with no split layout), DEVICE. */
hg_status hg_problem_create(hg_ctx* ctx, int64_t dim, int32_t n_ctrl,
                            const hg_csr* H0, const hg_csr* Hk,
                            const double* omega_diag, hg_problem** out);

/* The same problem with every operator stored as a dense dim x dim matrix, as
 * the paper's runtime and memory benchmarks store the Hamiltonian (Sec. IV.B;
 * Theta(d^2) memory, Sec. IV.A).  hg_eval then runs the dense path: each
 * Taylor term of the forward, reconstruction, co-state and auxiliary-matrix
 * actions (Sec. III.B-C) is one dense complex contraction of the embedded
 * 2d x 2d operator with the whole block of states, on the matrix cores
 * (FP32 MFMA for HG_C64, FP64 MFMA for HG_C128).  Meant for wide state blocks
 * (full-basis gate problems, S = d) and operators that are dense or have
 * more diagonals than the DIA kernels take.  Inputs, validation, sigma' (from
 * the structural pattern), results and precision rules are those of
 * hg_problem_create.  HG_MODE_CHECKPOINT stores whole state blocks every C
 * steps and re-propagates each segment on the matrix cores (Taylor method
 * only: with HG_METHOD_DIAG it returns UNSUPPORTED, and HG_METHOD_AUTO then
 * takes the Taylor method).  Device memory:
 * (n_ctrl+1) dp^2 complex128 here, dp = dim rounded up to 64; per evaluation
 * the embedded operators and the state blocks (hg_eval_footprint).
 * Errors: INVALID_ARG, NOT_HERMITIAN, NONFINITE, UNSUPPORTED (dim > 8192,
 * n_ctrl > 16), OUT_OF_MEMORY, DEVICE. */
hg_status hg_problem_create_dense(hg_ctx* ctx, int64_t dim, int32_t n_ctrl,
                                  const hg_csr* H0, const hg_csr* Hk,
                                  const double* omega_diag, hg_problem** out);
hg_status hg_problem_destroy(hg_problem* p);

/* Problem facts: dim, n_ctrl, number of union diagonals (0 for dense
 * storage), sigma' (the
 * largest number of non-zeros in a row of the union pattern, App. C eq.
 * sigmapdef) and the number of stored union non-zeros.  Any pointer may be NULL. */
hg_status hg_problem_info(const hg_problem* p, int64_t* dim, int32_t* n_ctrl,
                          int32_t* ell_width, int32_t* sigma, int64_t* nnz);

/* Host planner (Sec. III.B rule, App. C bound), FP64.  For each of n norms
 * theta[i] = ||A_i||_1 (host) choose the smallest s, then the smallest
 * m in [1, 60], with E_A(m, s) <= tau, using unit roundoff u (2^-53 for FP64
 * arithmetic).  Writes m_out[i], s_out[i] (host).  Errors: INVALID_ARG,
 * NONFINITE (theta not finite), TOLERANCE_UNREACHABLE (the first failing
 * index and the bound's floor are in hg_last_error()). */
hg_status hg_plan(const double* theta, int64_t n, int32_t sigma, double tau, double u,
                  int32_t* m_out, int32_t* s_out);

/* hg_plan with a choice of rule (hg_plan_rule_t); HG_PLAN_SMALLEST_S is hg_plan. */
hg_status hg_plan_rule(const double* theta, int64_t n, int32_t sigma, double tau, double u,
                       int32_t rule, int32_t* m_out, int32_t* s_out);

/* Error bound E_A(m, s) of App. C at ||A||_1 = theta (host, FP64). */
double hg_error_bound(double theta, int32_t m, int32_t s, int32_t sigma, double u);

/* Exact per-step 1-norms theta[b][n] = dt * max_i sum_j |(H_0 + sum_k u[b][k][n] H_k)_ij|
 * (App. C, eq. norm inequality) for n_batch amplitude sets, FP64, on `stream`
 * (a hipStream_t, NULL = default).  u: device [n_batch][n_ctrl][n_steps];
 * theta_out: device [n_batch][n_steps].  Asynchronous. */
hg_status hg_step_norms(hg_problem* p, const double* u, int32_t n_batch, int32_t n_steps,
                        double dt, double* theta_out, void* stream);

typedef struct {
  int32_t n_steps;           /* N >= 1 */
  int32_t n_batch;           /* B >= 1 independent evaluations of this problem */
  double dt;                 /* step length (ns; H in rad/ns, hbar = 1) */
  const double* u;           /* device [B][n_ctrl][N] amplitudes, FP64 */
  int32_t n_states;          /* S >= 1 */
  const double* psi0;        /* device [B][S][dim] complex128, each column normalised */
  const double* targets;     /* device [B][S][dim] complex128 target states phi_T^h */
  double w_fid, w_pen;       /* cost weights alpha_nu (Sec. II); w_pen ignored without Omega */
  double w_int;              /* weight of the time-integrated infidelity
                                C3 = 1 - (1/N) sum_{n=1..N} |g_n|^2, g_n the overlap
                                (1/S) sum_h <phi_T^h|psi_n^h> after step n (App. A:
                                C3^st for S = 1, C3^g for a full basis); 0 = off */
  double tau;                /* per-step tolerance of the Taylor action (Sec. III.B) */
  hg_dtype dtype;            /* arithmetic of the state products (norms, planner,
                                overlaps and reductions are FP64 in both) */
  hg_mode mode;              /* RECONSTRUCT (HG inverse propagation) or CHECKPOINT */
  int32_t ckpt_every;        /* CHECKPOINT: store psi every C steps (C >= 1) */
  int32_t renorm_every;      /* rescale psi to unit norm every R steps (0 = never);
                                applied to the forward and reconstructed states */
  const int32_t* schedule;   /* NULL, or host [2][B][N]: frozen (m, s) per step
                                (the planner is skipped; norms are still computed) */
  int32_t flags;             /* bit 0 (HG_FLAG_TIMING): time the sweep kernels with
                                HIP events on `stream`, reported in hg_result;
                                bit 1 (HG_FLAG_SPREAD): let several workgroups share
                                one column's backward sweep when the batch leaves
                                compute units idle (each repeats the reconstruction
                                and co-state and takes a share of the controls):
                                lower latency for small batches, more total work;
                                results equal those without it to rounding */
  int32_t rule;              /* hg_plan_rule_t of the planner (0 = the paper's) */
  int32_t method;            /* hg_method_t (0 = Taylor); DIAG/AUTO need dense storage */
} hg_eval_desc;

#define HG_FLAG_TIMING 1
#define HG_FLAG_SPREAD 2

typedef struct {
  double cost;               /* w_fid C1 + w_pen C2 + w_int C3 */
  double infidelity;         /* C1 = 1 - |g|^2 */
  double penalty;            /* C2 */
  double integrated_infidelity;  /* C3 (computed when w_int != 0, else 0) */
  double overlap_re, overlap_im;  /* g */
  int64_t sum_mu;            /* sum over steps of m_n s_n */
  double max_theta;          /* max_n ||A_n||_1 */
  double max_bound;          /* max_n E_A(m_n, s_n) (0 with a frozen schedule) */
  double drift;              /* reconstruction drift: max_h ||psi_0^h(rebuilt) - psi_0^h||;
                                in CHECKPOINT mode only the rounding of psi_0 to the
                                working precision (0 for HG_C128) */
  double ms_forward;         /* with HG_FLAG_TIMING: forward-sweep kernel time (whole batch) */
  double ms_backward;        /* with HG_FLAG_TIMING: backward-sweep kernel time (whole batch) */
} hg_result;

/* Evaluate cost and gradient for B amplitude sets.  results: host [B];
 * grad: device [B][n_ctrl][N] FP64 (may be NULL for cost only).  Work is
 * enqueued on `stream`; the call returns after the stream has finished it,
 * so results and grad are valid on return.  This is synchronous on purpose:
 * the (m, s) schedule is chosen on the host by the FP64 planner from the
 * norms the device computed, so that every decision equals the reference
 * rule's, and the call waits for them mid-way.  The workspace comes
 * stream-ordered from the device's default memory pool (freed blocks stay in
 * the pool, see hg_create) and the host staging is pinned memory kept per
 * calling thread, so repeated calls allocate nothing new.  One workgroup holds
 * one state column's term vectors in LDS, or P workgroups of the problem's
 * split layout (see hg_problem_create; launched cooperatively, so
 * n_batch * n_states * P must not exceed the compute units, else
 * UNSUPPORTED; their bounded waits for each other end in DEVICE if a
 * neighbour does not arrive within 20 s).
 * Errors: INVALID_ARG, NONFINITE, TOLERANCE_UNREACHABLE, UNSUPPORTED,
 * OUT_OF_MEMORY, DEVICE. */
hg_status hg_eval(hg_problem* p, const hg_eval_desc* desc, hg_result* results,
                  double* grad, void* stream);

/* Device memory the library would allocate for one hg_eval call with this
 * shape (workspace only; caller buffers excluded).  Used for admission. */
hg_status hg_eval_footprint(const hg_problem* p, const hg_eval_desc* desc, size_t* bytes);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): hg_eval's evaluation, with the same
 * kernels and same results, with no hipMalloc, hipFree, hipHostMalloc or
 * event creation.  The workspace is a fixed array of 64 MiB of device memory
 * that the library defines once per device (held until the process ends) and
 * the host staging a fixed 2 MiB host array per device; the planner uses its
 * cached threshold table if one exists, else the direct search (same
 * decisions).  Calls that overlap on one device share both arrays and race:
 * one call at a time per device.  The arrays keep the last call's contents;
 * everything that must start at zero is cleared by the kernels.
 * Errors: those of hg_eval; OUT_OF_MEMORY when hg_eval_footprint of the
 * shape exceeds the scratch or the staging (B*N, B*S) exceeds 2 MiB;
 * INVALID_ARG with HG_FLAG_TIMING (it needs events). */
hg_status hg_eval_noalloc(hg_problem* p, const hg_eval_desc* desc, hg_result* results,
                          double* grad, void* stream);
/* Sizes of hg_eval_noalloc's fixed device scratch and host staging (bytes). */
hg_status hg_eval_noalloc_limits(size_t* scratch_bytes, size_t* host_stage_bytes);

/* High-water mark of device memory handed out by the device's default pool,
 * which holds every evaluation workspace (bytes; operators and caller buffers
 * are not in it).  reset != 0 restarts the mark at the current use.  This is
 * the measured peak of hg_eval's own device memory (Table I's comparison). */
hg_status hg_mem_pool_peak(hg_ctx* ctx, int32_t reset, size_t* used_high);

/* ---------------------------------------------------------------- serving ----
 * A server admits cost+gradient requests (any problem, any shape) onto the
 * context's GPU as they arrive: a request starts when one of max_inflight
 * worker slots is free and its device footprint (hg_eval_footprint plus its
 * own u, psi0, targets and grad buffers) fits in hbm_budget_bytes next to the
 * running requests; admission is first come, first served.  Each slot runs on
 * its own HIP stream, so kernels of concurrent requests overlap on the
 * device.  A request's results do not depend on what runs beside it.
 * The desc's device buffers, `results` (host [n_batch]) and `grad` must stay
 * valid until hg_server_wait returns for the request; a frozen schedule is
 * copied at submit.  All server calls are thread-safe. */
typedef struct hg_server hg_server;

hg_status hg_server_create(hg_ctx* ctx, size_t hbm_budget_bytes, int32_t max_inflight,
                           hg_server** out);
/* Queue a request.  The request's device work is ordered after everything
 * queued on `after_stream` (a hipStream_t of the caller, NULL = the null
 * stream) up to this call: the inputs may still be in flight there (e.g.
 * produced by the kernel just launched), the server waits for them on the
 * device.  grad is written on a worker stream and is complete when
 * hg_server_wait returns.  Errors at submit: INVALID_ARG (and the other
 * hg_eval argument checks), OUT_OF_MEMORY (footprint larger than the whole
 * budget), BUSY (queue full or server shutting down), DEVICE.  Writes the
 * request id. */
hg_status hg_server_submit(hg_server* sv, hg_problem* p, const hg_eval_desc* desc,
                           hg_result* results, double* grad, void* after_stream,
                           uint64_t* req_id);
/* done = 1 once the request finished (successfully or not). */
hg_status hg_server_poll(hg_server* sv, uint64_t req_id, int32_t* done);
/* Block until the request finished; returns its hg_eval status (CANCELLED if it
 * was cancelled) and, if non-NULL, the submit-to-finish and submit-to-start
 * times in ms.  The id is released afterwards. */
hg_status hg_server_wait(hg_server* sv, uint64_t req_id, double* latency_ms, double* queued_ms);
/* Cancel a request that has not started (BUSY once it has). */
hg_status hg_server_cancel(hg_server* sv, uint64_t req_id);
/* Device bytes admitted right now, queued and running request counts. */
hg_status hg_server_info(hg_server* sv, size_t* bytes_in_use, int32_t* queued, int32_t* running);
/* Run every queued request to completion, then stop the workers and free. */
hg_status hg_server_destroy(hg_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* HGRAPE_H */
