/*
 * tfmm.h - FFT-based FMM translation with compressed translation operators on
 * one AMD Instinct MI355X (gfx950).
 *
 * The library implements the iterative-solution-stage translation of an
 * FMM-FFT surface-integral-equation matrix-vector product, Eq. (5) of
 * Qian & Yucel, "On the Compression of Translation Operator Tensors in
 * FMM-FFT-Accelerated SIE Simulators via Tensor Decompositions":
 *
 *     B_{s,p} = IFFT3( T~_p  .*  FFT3( zero-pad(A_{s,p}) ) )  cropped to the box grid,
 *
 * for every plane-wave direction p and right-hand side s, where the FFT'ed
 * translation operator T~_p (Eq. (7) sampled on the 2Kx x 2Ky x 2Kz box-offset
 * grid and FFT'ed, Section II-B) is held on the GPU either uncompressed or in one
 * of the paper's five compressed forms (Tucker-3D/4D, Eqs. (8)-(9); H-Tucker-4D,
 * Eq. (11); TT-3D/4D, Eqs. (13)-(14)) and restored per direction inside the
 * translation kernels (Section II-C, Figs. 3-4) without ever being written to
 * device memory.
 *
 * Conventions shared by every entry point:
 *   - Every call returns a tfmm_status; nothing throws across the ABI.
 *     Arguments are validated before any device work is enqueued.  On error the
 *     outputs are left untouched, except the B buffer of a translation that
 *     failed on the device, whose contents are then undefined.
 *   - Complex numbers are interleaved (re, im) pairs: complex64 = two floats,
 *     complex128 = two doubles.  Arrays are C order, last index fastest.
 *   - A tfmm_ctx owns one HIP device, one device-memory budget and one
 *     scheduler thread.  Calls on one context are serialised by an internal
 *     mutex and may come from any thread.
 *   - The library owns operator memory (allocated at setup, charged to the
 *     context's budget, freed at release).  Callers own A and B.
 *   - All enqueues are asynchronous with respect to the host: the call returns
 *     once the work is queued on the given stream.
 *   - tfmm_last_error() returns a human-readable detail string for the last
 *     failing call made by the calling thread.
 */
#ifndef TFMM_H
#define TFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfmm_ctx_s* tfmm_ctx;
typedef struct tfmm_op_s* tfmm_op;
typedef struct tfmm_basis_s* tfmm_basis;
typedef struct tfmm_near_s* tfmm_near;
typedef uint64_t tfmm_ticket;

typedef enum {
  TFMM_OK = 0,
  TFMM_ERR_INVALID_ARG = 1,  /* null pointer, out-of-range size or enum           */
  TFMM_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement       */
  TFMM_ERR_BUDGET = 3,       /* the context's device-memory budget is exhausted   */
  TFMM_ERR_OOM = 4,          /* hipMalloc or host allocation failed               */
  TFMM_ERR_HIP = 5,          /* a HIP runtime call or kernel launch failed        */
  TFMM_ERR_BUSY = 6,         /* operator still referenced by queued jobs          */
  TFMM_ERR_UNKNOWN_TICKET = 7,
  TFMM_ERR_QUEUE_FULL = 8,
  TFMM_ERR_INTERNAL = 9,
  TFMM_ERR_NO_DEVICE = 10,   /* no HIP device (the library has no CPU fallback)    */
  TFMM_ERR_NOT_CONVERGED = 11 /* an iterative solve stopped at its iteration limit */
} tfmm_status;

/* Operator storage formats (Section II-B). */
typedef enum {
  TFMM_FMT_FULL = 0,       /* uncompressed FFT'ed operator, n_dir x n1 x n2 x n3        */
  TFMM_FMT_TUCKER3D = 1,   /* per direction: core r1 x r2 x r3, factors n_i x r_i, Eq. (8) */
  TFMM_FMT_TT3D = 2,       /* per direction: U1 n1 x r1, C r1 x n2 x r2, U3 n3 x r2, Eq. (13) */
  TFMM_FMT_TUCKER4D = 3,   /* one core r1 x r2 x r3 x r4 and four factors, Eq. (9)      */
  TFMM_FMT_TT4D = 4,       /* U1 n1 x r1, C1 r1 x n2 x r2, C2 r2 x n3 x r3, U3 n_dir x r3, Eq. (14) */
  TFMM_FMT_HTUCKER4D = 5   /* leaves U1..U4, C12 r1 x r2 x r12, C34 r3 x r4 x r34,
                              root r12 x r34, Eq. (11), balanced tree {1,2}{3,4}       */
} tfmm_format;

/* Arithmetic of the per-direction restoration contractions (the FFTs and the
 * pointwise product are always FP32).  BF16X3 splits each FP32 operand into a
 * bf16 high part and a bf16 remainder and accumulates hi*hi + hi*lo + lo*hi in
 * FP32 on the matrix cores.  The once-per-call GEMMs (the per-direction cores
 * of the 4-D formats and the formed x-mode / x-y products) use BF16X3 too for
 * an operator set up by tfmm_setup_compressed at tol >= 1e-5, else FP32. */
typedef enum { TFMM_PREC_FP32 = 0, TFMM_PREC_BF16X3 = 1 } tfmm_precision;

/* Near-field rule (Section II-A): box pairs closer than the rule are handled
 * classically, so their operator samples are zero.  CHEB: max_i |d_i| <=
 * near_param (default 1, the 27 nearest boxes).  KAPPA: R < kappa R^s with
 * kappa = near_param (4 in the paper) and R^s = a sqrt(3)/2. */
typedef enum { TFMM_NEAR_CHEB = 0, TFMM_NEAR_KAPPA = 1 } tfmm_near_rule;

/* Direction grid (Section II-A, text after Eq. (4)): n_theta Gauss-Legendre
 * nodes in cos(theta), ascending, times n_phi uniform nodes phi_j = 2 pi j /
 * n_phi; direction index p = i_theta * n_phi + j_phi.  An explicit list of
 * directions may replace the grid (the restoration does not depend on how the
 * directions were chosen). */
typedef struct {
  int32_t K[3];            /* box grid Kx, Ky, Kz; each one of 4, 8, 12, 16, 24, 32,
                              Kx also 64 or 128, with Kx * Ky <= 2048
                              (FFT grid n_i = 2 K_i)                                */
  double box_size;         /* box edge a, in the length unit of 1/k                  */
  double k_re, k_im;       /* wavenumber k = k_re + i k_im (Section II-A, Eq. (7));
                              k_re > 0.  A lossy medium (Section III-A-5:
                              k = k0 sqrt(eps_r) with eps_r = eps' - j sigma/(w eps0))
                              has k_im < 0 under the e^{jwt} convention, so that
                              e^{-jkR} decays; k_im > 0 is rejected                 */
  int32_t L;               /* multipole order; 0 => derive it from `digits`         */
  double digits;           /* accurate digits, used only when L == 0:
                              L = ceil(x + 1.8 digits^(2/3) x^(1/3)), x = |k| a sqrt(3) */
  int32_t n_theta, n_phi;  /* 0,0 => L+1 and 2(L+1)                                   */
  const double* dirs;      /* optional: n_dir x 3 unit vectors k_p (host memory, read
                              during the call only); when set it replaces the
                              n_theta x n_phi grid and direction p is dirs[3p..3p+2] */
  int32_t n_dir;           /* number of rows of `dirs`; for tfmm_op_import, which
                              samples nothing, a direction count without `dirs`    */
  tfmm_near_rule near_rule;
  double near_param;       /* 0 => 1 for CHEB, 4 for KAPPA                            */
  double scale_re, scale_im; /* global prefactor of Eq. (7); 0,0 => 1                 */
  tfmm_format fmt;
  double tol;              /* gamma: relative Frobenius tolerance of the
                              decomposition (per direction for 3-D formats, over
                              the whole 4-D tensor otherwise); ignored for FULL   */
  tfmm_precision prec;
} tfmm_problem;

typedef struct {
  tfmm_format fmt;
  tfmm_precision prec;
  int32_t K[3], n[3];
  int32_t n_dir, L;
  size_t bytes_full;       /* complex64 bytes of the uncompressed operator           */
  size_t bytes_stored;     /* device bytes of the stored operator                    */
  size_t elems_stored;     /* complex entries of cores and factors                   */
  size_t bytes_scratch;    /* device bytes of translation scratch a one-RHS
                              tfmm_translate of this operator takes from the
                              context (half spectrum of one chunk of directions,
                              per-direction cores of the 4-D formats, z-major
                              copies); it grows with the RHS count up to the
                              context's chunk size                                  */
  double rel_err_fro;      /* ||T~ - T~hat||_F / ||T~||_F over all directions, estimated at
                              setup from ||T~||^2 - ||core||^2 in FP64 (below ~1e-6 the
                              cancellation leaves it uncertain by about gamma)        */
  double max_dir_rel_err;  /* max over directions of the same ratio                  */
  int32_t ranks[8];        /* format ranks; 3-D formats: maximum over directions     */
  double setup_seconds;
} tfmm_op_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` with a device-memory budget for
 * operators and translation scratch (0 => 90% of the device's free memory).
 * Fails with TFMM_ERR_NO_DEVICE when no device is visible.  Environment
 * variables read at creation select implementation variants (results agree
 * within FP32 rounding):
 *   TFMM_NO_FUSED=1  always use the three-pass kernel pipeline instead of the
 *                    fused one-kernel-per-direction path available for cubic
 *                    grids up to 16^3 boxes;
 *   TFMM_NO_TK2=1    restore Tucker-family operators through LDS-staged
 *                    products instead of the register-chained restoration;
 *   TFMM_HCAP_MB=n   bytes (MiB) of the three-pass pipeline's half-spectrum
 *                    scratch per chunk of directions (default: an eighth of
 *                    the budget, within 64 MiB .. 1 GiB);
 *   TFMM_GRAPH=0|1   never / always replay tfmm_translate from a captured
 *                    hipGraph (default: only multi-launch translations). */
tfmm_status tfmm_ctx_create(int device, size_t hbm_budget_bytes, tfmm_ctx* out);

/* Wait for every submitted job, stop the scheduler, free all operators and
 * scratch.  The handle is invalid afterwards. */
tfmm_status tfmm_ctx_destroy(tfmm_ctx ctx);

/* Bytes charged to the budget so far and the budget itself. */
tfmm_status tfmm_ctx_memory(tfmm_ctx ctx, size_t* used, size_t* budget);

/* ---- operator setup (Section II-B; Algorithms 1-3) ------------------------ */

/* Build the FFT'ed translation operator for `prob` and store it in the
 * requested format: directions and L on the host, Eq. (7) sampled in FP64 on
 * the device, FFT'ed and compressed in FP64 on the host (truncation: keep the
 * smallest rank whose discarded singular values have root-sum-square <=
 * gamma/sqrt(m) ||X||_F, m = d, d-1, 6 for Tucker, TT, H-Tucker), then packed
 * for the device in the requested precision.  Blocks until the operator is
 * resident.  TFMM_ERR_BUDGET if it does not fit the remaining budget. */
tfmm_status tfmm_setup_compressed(tfmm_ctx ctx, const tfmm_problem* prob, tfmm_op* out);

/* Build an operator from caller-supplied factors instead of sampling and
 * compressing.  `prob` supplies K, the direction count (n_theta * n_phi, or
 * L-derived), fmt and prec, and optionally in `tol` the tolerance the factors
 * were compressed at (0: unknown; it only selects the arithmetic of the
 * once-per-call GEMMs, see tfmm_precision); the physical fields are ignored.  `ranks` and
 * `data` (complex128, host memory, caller-owned, read during the call only)
 * are laid out as follows, all arrays C order:
 *   FULL      ranks: none (nranks 0);  data: T~[n_dir][n1][n2][n3]
 *   TUCKER3D  ranks: n_dir x {r1,r2,r3}; data per direction p in order:
 *             C[r1][r2][r3], U1[n1][r1], U2[n2][r2], U3[n3][r3]
 *   TT3D      ranks: n_dir x {r1,r2};   data per p: U1[n1][r1], C[r1][n2][r2], U3[n3][r2]
 *   TUCKER4D  ranks: {r1,r2,r3,r4};     data: C[r1][r2][r3][r4], U1, U2, U3, U4[n_dir][r4]
 *   TT4D      ranks: {r1,r2,r3};        data: U1[n1][r1], C1[r1][n2][r2], C2[r2][n3][r3], U3[n_dir][r3]
 *   HTUCKER4D ranks: {r1,r2,r3,r4,r12,r34}; data: U1, U2, U3, U4, C12[r1][r2][r12],
 *             C34[r3][r4][r34], B[r12][r34]
 * T~_p[x,y,z] is then sum C[a,b,c] U1[x,a] U2[y,b] U3[z,c] (Tucker, with the
 * 4-D core contracted with row p of U4), sum U1[x,a] C[a,y,b] U3[z,b] (TT-3D),
 * sum U1[x,a] C1[a,y,b] C2[b,z,c] U3[p,c] (TT-4D), and the Tucker form with core
 * sum_{b,b'} C12[a1,a2,b] B[b,b'] C34[a3,a4,b'] contracted with row p of U4
 * (H-Tucker).  `ndata` is the number of doubles in `data`. */
tfmm_status tfmm_op_import(tfmm_ctx ctx, const tfmm_problem* prob, const int32_t* ranks,
                           size_t nranks, const double* data, size_t ndata, tfmm_op* out);

tfmm_status tfmm_op_info_get(tfmm_op op, tfmm_op_info* out);

/* Per-direction ranks of a 3-D format (n_dir x 3 for Tucker-3D, n_dir x 2 for
 * TT-3D) or the format's ranks for 4-D formats.  `need` receives the count. */
tfmm_status tfmm_op_ranks(tfmm_op op, int32_t* ranks, size_t cap, size_t* need);

/* Copy the operator's factors to host memory in the tfmm_op_import layout
 * (complex128), for saving and reloading an operator.  With host_buf NULL
 * only `need` (number of doubles) is returned. */
tfmm_status tfmm_op_export(tfmm_op op, double* host_buf, size_t cap, size_t* need);

/* Free the operator.  TFMM_ERR_BUSY while submitted jobs still use it. */
tfmm_status tfmm_op_release(tfmm_ctx ctx, tfmm_op op);

/* ---- translation, Eq. (5) --------------------------------------------------- */

/* Enqueue B = translate(A) for `nrhs` right-hand sides on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  A and B are device pointers to
 * complex64 arrays [nrhs][n_dir][Kx][Ky][Kz], caller-owned; they must not
 * alias and must stay valid until the stream reaches the end of the work.
 * Translation scratch comes from the context (charged to its budget on first
 * use and kept) and is shared by every tfmm_translate call of the context:
 * calls on different streams must not overlap on the device.  The first call
 * for a given (op, nrhs, A, B) runs eagerly and records the launch sequence in
 * a hipGraph that later calls with the same arguments replay (see
 * TFMM_GRAPH); at most four graphs are kept per operator, and a graph is
 * dropped when the scratch it uses moves.  The kernels are persistent: they
 * take (direction, pencil tile) work items from a device counter, costliest
 * directions first, so results do not depend on the launch shape.  On the
 * three-pass path the per-call GEMMs (the 4-D formats' direction cores and
 * formed products, TT-3D's formed products) run on an internal stream forked
 * from `hip_stream` and joined back into it before the first z-stage, beside
 * the first x pass; everything the call enqueues has finished when
 * `hip_stream` reaches the end of its work. */
tfmm_status tfmm_translate(tfmm_ctx ctx, tfmm_op op, const void* A, void* B, int32_t nrhs,
                           void* hip_stream);

/* ---- translation without device allocation -------------------------------- */

/* Bytes of the fixed device scratch of tfmm_translate_noalloc (per device). */
#define TFMM_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * translation as tfmm_translate, enqueued on `hip_stream`, with every byte of
 * scratch taken from a fixed device array of TFMM_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device it runs on until the process ends (its
 * address is looked up at context creation).  The call makes no hipMalloc or
 * hipFree and no allocating library call, never captures or replays a graph
 * (so it may itself be captured), and enqueues all of its work on
 * `hip_stream` (no internal stream).  The direction chunk of the three-pass
 * pipeline shrinks until the scratch fits; a translation that does not fit
 * even with one direction per chunk (the per-direction cores of a 4-D format
 * plus one direction's x-FFT'ed planes for all RHS) fails
 * with TFMM_ERR_UNSUPPORTED before any work is enqueued.  Every call on a
 * device shares that device's array, which keeps the last call's contents:
 * calls that overlap on one device (other streams, other threads, other
 * contexts) race and must be serialised by the caller.  Operators, A and B as
 * for tfmm_translate; the tile plan is the operator's current one. */
tfmm_status tfmm_translate_noalloc(tfmm_ctx ctx, tfmm_op op, const void* A, void* B, int32_t nrhs,
                                   void* hip_stream);

/* ---- far-field matrix-vector product around the translation ---------------- */

/* Basis functions of the far-field product (Section II-A): point dipoles
 * b_n(r) = u_n delta(r - r_n) in the box grid of `op` (grid corner at the
 * origin, box v = floor(r / a), centre (v + 1/2) a).  Their far-field patterns,
 * Eq. (3) for a delta-function basis,
 *     P+(k_p, b_n) = (I - k_p k_p) u_n exp(+jk k_p . (r_n - r_v)),
 * kept as theta and phi components, are computed on the device in FP64 for
 * every direction of `op` and stored as complex64 (16 B per direction and
 * basis function); the receive patterns of Eq. (6) are
 * P-(k_p, b_m) = (I - k_p k_p) u_m exp(-jk k_p . (r_m - r_v')), the conjugates
 * of P+ for a real k.  `pos` and `orient` are host arrays n_basis x 3 (read
 * during the call; orientations unit vectors).  The operator must come from
 * tfmm_setup_compressed with a direction grid (its quadrature weights w_p are
 * used); it stays referenced until tfmm_basis_release.  Charged to the budget. */
tfmm_status tfmm_basis_setup(tfmm_ctx ctx, tfmm_op op, int32_t n_basis, const double* pos, const double* orient,
                             tfmm_basis* out);
tfmm_status tfmm_basis_release(tfmm_ctx ctx, tfmm_basis basis);

/* Aggregation, Eq. (4): A_v(k_p) = sum_{n in box v} P+(k_p, b_n) I_n.
 * I: device complex64 [nrhs][n_basis] (caller order); A: device complex64
 * [2 nrhs][n_dir][Kx][Ky][Kz], field 2 r + c = component c (0 theta, 1 phi) of
 * RHS r (each component is one right-hand side of tfmm_translate); empty boxes
 * are written as zero.  Enqueued on `hip_stream`. */
tfmm_status tfmm_aggregate(tfmm_ctx ctx, tfmm_basis basis, const void* I, void* A, int32_t nrhs, void* hip_stream);

/* Projection with the direction quadrature, Eq. (6):
 * y_m = sum_p w_p sum_c P-_c(k_p, b_m) B_c,v'(m)(k_p).  B: device complex64
 * [2 nrhs][n_dir][Kx][Ky][Kz] as for tfmm_aggregate; y: device complex64
 * [nrhs][n_basis].  Enqueued on `hip_stream`. */
tfmm_status tfmm_disaggregate(tfmm_ctx ctx, tfmm_basis basis, const void* B, void* y, int32_t nrhs,
                              void* hip_stream);

/* The far-field part of the matrix-vector product of Eq. (2): aggregation,
 * the translation of Eq. (5) through `op` (compressed or not), projection.
 * I, y as above; `op` is the basis's operator.  The intermediate A and B
 * (2 x 2 nrhs x n_dir x Kx x Ky x Kz complex64) are context scratch, charged to
 * the budget and kept; calls on one context must not overlap on the device. */
tfmm_status tfmm_farfield_matvec(tfmm_ctx ctx, tfmm_op op, tfmm_basis basis, const void* I, void* y, int32_t nrhs,
                                 void* hip_stream);

/* ---- iterative solution of Eq. (2) ---------------------------------------- */

/* Near-field matrix of the system (the classically computed interactions of
 * Section II-A; this library takes it as given): n x n, CSR on the host
 * (row_ptr[n + 1], cols[nnz], vals[2 nnz] complex128 interleaved; read during
 * the call), stored on the device as complex64.  Charged to the budget. */
tfmm_status tfmm_near_setup(tfmm_ctx ctx, int32_t n, const int32_t* row_ptr, const int32_t* cols,
                            const double* vals, tfmm_near* out);
tfmm_status tfmm_near_release(tfmm_ctx ctx, tfmm_near near);
/* y = Zn x for nrhs device complex64 vectors of n entries each (x, y [nrhs][n]). */
tfmm_status tfmm_near_matvec(tfmm_ctx ctx, tfmm_near near, const void* x, void* y, int32_t nrhs, void* hip_stream);

/* Solve (Zn + Zfar) I = V by TFQMR (transpose-free quasi-minimal residual,
 * Section II-A), Zfar = tfmm_farfield_matvec of (op, basis).  V, I: device
 * complex64 vectors of n_basis entries (I is written only on success).  The
 * Krylov vectors are complex128 on the device; initial guess 0, shadow
 * residual V.  Stops when ||V - Z I|| / ||V|| <= tol (checked whenever
 * Freund's bound tau sqrt(m + 1) on the residual of half step m passes tol),
 * else fails with TFMM_ERR_NOT_CONVERGED after maxit iterations (two products
 * with Z each).  iters / relres (may be NULL) receive the iteration count and
 * the last true relative residual.  Blocks until done; uses its own stream. */
tfmm_status tfmm_solve_tfqmr(tfmm_ctx ctx, tfmm_op op, tfmm_basis basis, tfmm_near near, const void* V, void* I,
                             double tol, int32_t maxit, int32_t* iters, double* relres);

/* ---- serving: continuous batching (submit / poll) ------------------------ */

/* Queue a translation job for the context's scheduler thread (continuous
 * batching of the translation of Eq. (5)).  A and B as for tfmm_translate and
 * caller-owned until the job is reported done; A must be complete on the
 * device when the job is submitted (the scheduler's streams do not wait for
 * the caller's streams).  The job keeps a reference on `op`.
 * Admission, in arrival order: a job is started on one of two scheduler
 * streams once a stream is free and its memory fits the context's budget --
 * its A and B bytes (2 x nrhs x n_dir x Kx x Ky x Kz complex64) plus the
 * stream's translation scratch (whose direction chunk shrinks, down to one
 * direction, to fit).  A job that does not fit waits at the head of the queue
 * until a running job completes and returns its memory; it fails with
 * TFMM_ERR_BUDGET only if it cannot fit with no other job running.  Queued
 * jobs on the same operator are started together in one batched launch.
 * Returns at once with a ticket. */
tfmm_status tfmm_submit(tfmm_ctx ctx, tfmm_op op, const void* A, void* B, int32_t nrhs,
                        tfmm_ticket* out);

/* Non-blocking completion check.  done = 1 once B is complete (or the job
 * failed; then job_status says why).  latency_us = submit-to-completion time. */
tfmm_status tfmm_poll(tfmm_ctx ctx, tfmm_ticket t, int32_t* done, tfmm_status* job_status,
                      double* latency_us);

/* Block until the job is done; the ticket is then retired. */
tfmm_status tfmm_wait(tfmm_ctx ctx, tfmm_ticket t, tfmm_status* job_status, double* latency_us);

/* Scheduler counters since the context was created: {launches started, times
 * the head of the queue waited for memory, jobs completed, jobs failed, jobs
 * queued now}; writes min(cap, 5) values. */
tfmm_status tfmm_sched_stats(tfmm_ctx ctx, uint64_t* out, size_t cap);

/* ---- batching: tile autotuner ------------------------------------------------ */

/* Time every tile configuration the operator's grid admits (fused
 * one-kernel path vs three-pass pipeline, three-pass pencil tile of 64*cb
 * pencils, and for compressed operators the register-chained vs LDS-staged
 * restoration) on `nrhs` right-hand sides, `reps` timed runs each
 * (median of HIP-event durations on an internal stream, after two warm-up
 * runs), and adopt the fastest for this operator.  Temporary A/B buffers
 * (2 x nrhs x n_dir x Kx x Ky x Kz complex64) are charged to the budget for
 * the duration of the call.  The choice is remembered by the context under a
 * key of (format, precision, FFT grid, direction count, maximum rank rounded up
 * to 8, RHS bucket 1 | 2-4 | 5-16 | >16); later translations of any operator
 * with the same key use it, and with TFMM_TUNE_CACHE=<path> set at context
 * creation the choices are read from and appended to that text file.
 * `choice_out` (may be NULL) receives {fused 0/1, cb, register-chained 0/1};
 * `best_ms` (may be NULL) the winning median.  TFMM_ERR_BUSY while submitted
 * jobs use the operator. */
/* The first time one of the operator's batched GEMMs (per-direction cores,
 * formed x-mode or x-y products) runs during this call, its shape's block tile
 * and LDS buffering are chosen by timing each once; the choice is kept for
 * the process (every choice gives bitwise-identical results). */
tfmm_status tfmm_autotune(tfmm_ctx ctx, tfmm_op op, int32_t nrhs, int32_t reps, int32_t* choice_out,
                          double* best_ms);

/* The operator's current plan: {fused 0/1, three-pass cb, register-chained
 * restoration 0/1, 1 if chosen by the autotuner, 1 if the x-mode product of the
 * per-direction cores (Fig. 3(a) step 1) is formed by a batched GEMM ahead of
 * the z-stage (Tucker-4D / H-Tucker-4D on the three-pass path)}; writes
 * min(cap, 5) values. */
tfmm_status tfmm_op_plan(tfmm_op op, int32_t* out, size_t cap);

/* ---- diagnostics ------------------------------------------------------------ */

const char* tfmm_status_str(tfmm_status s);
const char* tfmm_last_error(void);

/* Kernel-level timing: when enabled, tfmm_translate brackets each kernel it
 * launches with HIP events on the launch stream.  tfmm_kernel_times waits for
 * those events and reports, per kernel name (newline-separated in `names`),
 * the average duration in ms and the launch count since the last reset; at
 * most `cap` entries are written, `count` receives the number of names, and a
 * negative `cap` clears the statistics after reporting. */
tfmm_status tfmm_set_profiling(tfmm_ctx ctx, int32_t on);
tfmm_status tfmm_kernel_times(tfmm_ctx ctx, char* names, size_t names_cap, double* avg_ms,
                              int32_t* launches, int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* TFMM_H */
