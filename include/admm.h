/*
 * admm.h -- C ABI of the MI355X split-lasso ADMM library (libadmm.so).
 *
 * Solves  min_u  1/2 |g - H u|^2 + lambda |u|_1  over complex u with the
 * consensus-and-sectioning ADMM of Heredia-Juesas et al. (arXiv 1811.05571,
 * Sec. III-C): H (m x n) is cut into Q row blocks and P column blocks; block
 * (i,j) keeps a replica u_j^i of image section j, a scaled dual s_j^i and its
 * estimated data ghat_ij = H_ij u_j^i.  Q = 1 is the sectioning scheme
 * (Sec. III-B), P = 1 the consensus scheme (Sec. III-A).  One iteration is
 *   g'_ij = g_i - sum_{q!=j} ghat_iq                     (eq. g_rows_columns)
 *   u_j^i = (H_ij^H H_ij + rho I)^{-1}(H_ij^H g'_ij + rho(v_j - s_j^i))
 *                                   (eq. x_solution_rows_columns, evaluated
 *                                    with the inversion lemma, eq. inversion_lemma3)
 *   v_j   = S_{lambda/(Q rho)}(mean_i u_j^i + mean_i s_j^i) (eq. v_variable_rows_columns,
 *                                    soft threshold eq. softhresholding, sign(a)=a/|a|)
 *   s_j^i += u_j^i - v_j                                  (eq. s_variable_rows_columns)
 * All blocks live on one GPU.  The solver output is v = [v_1; ...; v_P].
 *
 * Conventions for every entry point:
 *   - Complex data are interleaved single precision (re, im) pairs, i.e. the
 *     layout of C99 `float _Complex` / numpy complex64, unless stated.
 *   - "device" pointers are HIP device (or managed) memory; "host" pointers
 *     are ordinary host memory.  The library never allocates device memory:
 *     the caller passes one workspace buffer sized by admm_workspace_bytes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that return host values synchronise it.
 *   - Every call returns 0 (ADMM_OK) or a negative status; admm_strerror
 *     names the code and admm_last_error() (per thread) gives the detail.
 *   - A plan must not be used from two host threads at once.
 */
#ifndef ADMM_H
#define ADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define ADMM_OK            0
#define ADMM_EINVAL       (-1) /* bad argument: NULL, size, split, rho, lambda, iters   */
#define ADMM_EWORKSPACE   (-2) /* workspace NULL, too small or not 256-byte aligned     */
#define ADMM_EHIP         (-3) /* a HIP runtime call failed (detail in last_error)      */
#define ADMM_ENOTPD       (-4) /* Gram matrix not positive definite (non-finite H)     */
#define ADMM_ENONFINITE   (-5) /* NaN/Inf found in H, g or the iterates                 */
#define ADMM_ESTATE       (-6) /* call out of order (e.g. backward without a record)   */
#define ADMM_EUNSUPPORTED (-7) /* valid but not implemented combination                */

/* ---- storage of H inside the plan ------------------------------------ */
#define ADMM_STORAGE_C64   0   /* complex64, as given                                  */
#define ADMM_STORAGE_BF16  1   /* bfloat16 real and imaginary planes, each value the   */
                               /* round-to-nearest-even bfloat16 of the fp32 value     */
#define ADMM_STORAGE_FP8   2   /* OCP fp8 e4m3 (bias 7, max 448) real and imaginary    */
                               /* planes of x / s_r, round to nearest even, saturating;*/
                               /* s_r = max over row r of |Re|,|Im|, divided by 448    */
                               /* (1 for an all-zero row).  The Gram factors are built */
                               /* in FP64 from the dequantised values; products       */
                               /* accumulate in FP32.                                  */
/* Flag OR-ed into `storage` (admm_workspace_bytes, admm_setup) or passed as
 * `flags` to the batched setup: besides the complex64 inverses, keep a copy of
 * each block's packed inverse G_ij^{-1} (formed in FP64, Sec. III-C, eq.
 * inversion_lemma3) rounded to bfloat16 (nearest even, Re and Im) and apply
 * that copy in every iteration and in the reverse sweep: half the bytes of the
 * Gram apply, at an inverse perturbation of at most 2^-9 relative per entry.
 * admm_backward's d/drho then differentiates through the unrounded inverse
 * (the rounding counts as the identity). */
#define ADMM_INVERSE_BF16  16
/* Flag, OR-ed in the same way: apply the complex64 inverses in patches of
 * 4 x 4 tiles (one workgroup per patch keeps its row and column sums across
 * the patch's tiles, so the partial stores shrink 4x) in every case.  Without
 * it the library uses patches when a split has at least 4096 of them (fewer
 * leave the GPU under-occupied) and single tiles otherwise.  No effect with
 * ADMM_INVERSE_BF16, whose copy is applied per tile. */
#define ADMM_GRAM_PATCHES  32
/* Flag, OR-ed in the same way (single plan only): always iterate with the
 * two-pass kernels, which read H once for the forward products H_ij c and
 * once for the adjoint products H_ij^H y.  Without it, complex64 plans with
 * at most 16 row blocks that fit 16 waves of at most six 64-row groups each,
 * every row block on whole waves (so at most 6144 rows, row blocks padded to
 * multiples of 64), iterate in a single pass over H: the plan also keeps a
 * copy of H cut into slabs of two columns over all rows, and one kernel
 * visit of a slab forms u = c + H^H y on its columns, applies the z- and
 * dual updates there (eqs. v_variable_rows_columns, s_variable_rows_columns)
 * and accumulates the next iteration's H c from the same registers.  Both
 * give the same iterates up to FP32 rounding order; the single pass reads
 * each element of H once per iteration instead of twice. */
#define ADMM_TWO_PASS      64
/* Flags, OR-ed in the same way (single plan only), fixing the form of the
 * x-update (eq. x_solution_rows_columns) for every block of the split.
 * ADMM_XUPDATE_LEMMA: the inversion-lemma form (eq. inversion_lemma3) in
 * push-through order, y_ij = G_ij^{-1}(g'_ij - H_ij c), u = c + H_ij^H y,
 * ghat_ij = g'_ij - rho y, with G_ij = rho I + H_ij H_ij^H (m_i x m_i).
 * ADMM_XUPDATE_DIRECT: the original inversion that Sec. III-B recommends for
 * tall blocks, u = A_ij^{-1}(H_ij^H g'_ij + rho c), ghat_ij = H_ij u, with
 * A_ij = rho I + H_ij^H H_ij (n_j x n_j): two passes over H per iteration
 * (an adjoint product, then the forward product of u), never the single
 * pass.  It is evaluated as a correction of the previous iteration's u,
 * u = u_prev + A^{-1}(H^H r_i + rho (c - u_prev)) with r_i = g_i - sum_q
 * ghat_iq the row block's residual (the same u; the inverse's rounding then
 * scales with the step), and from u_prev = 0 after a reset or a state
 * import.  Both inverses are formed in FP64 and stored as complex64.
 * Without either flag (both: EINVAL) the plan takes the form whose iteration
 * streams fewer bytes: H once (single pass) or twice plus the packed
 * m_i x m_i inverses, against H twice plus the packed n_j x n_j inverses;
 * with the single pass the direct form wins from about m_i >= (1 + sqrt 2) n_j,
 * without it from m_i > n_j.  Direct-form plans have no reverse sweep
 * (admm_solve_record and admm_backward return ADMM_EUNSUPPORTED). */
#define ADMM_XUPDATE_LEMMA  128
#define ADMM_XUPDATE_DIRECT 256

typedef struct admm_plan admm_plan;

/* Library version as an integer (major*10000 + minor*100 + patch). */
int admm_version(void);

/* Static name of a status code (never NULL). */
const char* admm_strerror(int status);

/* Detail of the last failing call on this thread ("" when none). */
const char* admm_last_error(void);

/*
 * admm_workspace_bytes -- device workspace needed by admm_setup.
 *   m, n      rows (measurements) and columns (pixels) of H, both >= 1.
 *   Q, P      number of row and column blocks, 1 <= Q <= m, 1 <= P <= n.
 *   row_off   host int64[Q+1] block boundaries, strictly increasing from 0
 *             to m, or NULL for the equal split (the first m mod Q blocks
 *             get one extra row).  col_off likewise with P and n.
 *   storage   ADMM_STORAGE_*, optionally | ADMM_INVERSE_BF16 | ADMM_GRAM_PATCHES
 *             | ADMM_TWO_PASS | ADMM_XUPDATE_LEMMA or ADMM_XUPDATE_DIRECT.
 *   out_bytes host, receives the size.
 * Errors: EINVAL for any bad size or split, an unknown flag, or both
 * x-update flags.  Every block shape is served, by one of the two forms of
 * the x-update (see ADMM_XUPDATE_DIRECT).
 * Launch-shape overrides, read from the environment when the split is
 * planned (sizing, setup, cost model), for tuning sweeps; results stay
 * within rounding of the defaults:
 *   ADMM_FZ_NT=1024     1024-thread slab workgroups even where 512 would do;
 *   ADMM_FZ_WGS=N       about N slab workgroups (default 512 of 512 threads,
 *                       256 of 1024);
 *   ADMM_FZR_LOADS=N    at most N workgroup parts of H c added by one thread
 *                       of the row kernel (default 16).
 */
int admm_workspace_bytes(int64_t m, int64_t n, int Q, const int64_t* row_off,
                         int P, const int64_t* col_off, int storage,
                         size_t* out_bytes);

/*
 * admm_split_cost -- cost model of one split (host computation, no GPU call).
 *   m..storage  as for admm_workspace_bytes, with the same errors.
 *   out16     host double[16]:
 *     [0] elements one computational node sends and receives per iteration
 *         when each block is its own node (Sec. IV, table of exchanged
 *         elements): 2 n with row blocks only, P m with column blocks only,
 *         P m_i + 2 n_j with both (the largest blocks when uneven), 0 unsplit;
 *     [1] HBM bytes one iteration of this library moves (algorithmic), for
 *         the kernels this split gets: with the single pass H once, the
 *         packed inverses once, the block vectors and the slab workgroups'
 *         row parts of H c (written and read once); with the two-pass
 *         kernels H twice, the inverses, the vectors and, with Q > 32, the
 *         z-update's second read of c and the partials; in the direct form
 *         H twice, the packed n_j x n_j inverses and the vectors;
 *     [2] FP64 flops of the setup (lower half of H_ij H_ij^H, or of
 *         H_ij^H H_ij in the direct form, Cholesky, triangular inverse and
 *         W^H W, 8 per complex multiply-add);
 *     [3] bytes of the packed complex64 inverses, [4] bytes of stored H,
 *     [5] workspace bytes, [6] largest m_i, [7] largest n_j, [8] row chunks
 *     of the adjoint product, [9] 4 x 4 tile patches of the Gram apply (0:
 *     single tiles), [10] 1 if the split iterates in a single pass over H,
 *     [11] workgroups of the single-pass slab kernel, [12] 1 if the split
 *     takes the direct x-update (see ADMM_XUPDATE_DIRECT), [13] the single
 *     pass's wave load factor (64-row group slots of all waves over the row
 *     groups, >= 1; 0 without the single pass), [14] its workgroup size
 *     (512, 1024; 0), [15] the Gram build's span (see admm_choose_split).
 */
int admm_split_cost(int64_t m, int64_t n, int Q, const int64_t* row_off,
                    int P, const int64_t* col_off, int storage, double* out16);

/*
 * Timing model of a plan, for choosing a split (Sec. IV weighs splits by
 * what the nodes exchange; on one GPU the price is time).  Setup seconds =
 *   c[0] flops + c[1] span + c[2] steps + c[3] blocks + c[4],
 * iteration seconds =
 *   c[5] h512 + c[6] h1024 + c[7] bytes + c[8] blocks + c[9],
 * where flops is admm_split_cost's [2]; span the Gram build's serial length,
 * ceil(K / 32) K-chunks of one tile's workgroup times ceil(tiles / 512)
 * rounds of workgroups (K = n_j, or m_i in the direct form); steps the tile-
 * padded Gram edge / 64 (serial Cholesky and triangular-inverse panels);
 * blocks Q P; h512 / h1024 the bytes of H a single-pass iteration streams
 * with 512- / 1024-thread workgroups, times its wave load factor ([13]);
 * bytes every other algorithmic byte of the iteration ([1], all of it for
 * the two-pass and direct forms).  `coef` is host double[10].
 *
 * admm_model_coefficients -- the built-in coefficients: a non-negative
 *   least-squares fit (relative error) to the setup and 50-iteration times
 *   of all 169 candidate splits of 2160 x 22500 and 6144 x 32000 on MI355X.
 *   Errors: EINVAL.
 * admm_calibrate -- coefficients measured on the current device for this
 *   shape: times the setup and 20 iterations of up to seven probe splits
 *   ((4,4), (16,16), (2,1), (32,32), (20,4), (4,4) with the two-pass kernels,
 *   (8,2)) of H with measurements g (device, as for admm_setup / admm_solve;
 *   any finite g) in the caller's workspace (probes that do not fit are
 *   skipped), and fits four scale factors of the built-in coefficients by
 *   non-negative least squares (relative error): setup work (c[0..2]),
 *   setup overhead (c[3..4]), iteration bytes (c[5..7]) and iteration
 *   overhead (c[8..9]).  A short pass: tens to a few hundred ms.  Synchronises `stream`.  Errors: EINVAL,
 *   EWORKSPACE (fewer than three probes fit), the errors of admm_setup and
 *   admm_solve.
 * admm_choose_split -- the equal split (Q, P), Q and P from {1, 2, 3, 4, 5,
 *   6, 8, 10, 12, 16, 20, 24, 32}, whose modelled setup plus `iters`
 *   iterations is least, among the splits admm_workspace_bytes accepts whose
 *   exchange count [0] is at most max_exchange (<= 0: no limit; the limit
 *   stands for the link budget of a distributed run, Sec. IV).  coef: host
 *   double[10], or NULL for the built-in values.  The model prices a fixed
 *   number of iterations; how many a split needs to converge depends on the
 *   problem and is the caller's input.  Host computation.
 *     Q_out, P_out  host, receive the split; model_s host or NULL, receives
 *                   the modelled seconds.
 *   Errors: EINVAL (NULL outputs, iters < 0, a negative or non-finite
 *   coefficient), EUNSUPPORTED (no candidate meets the exchange limit; the
 *   unsplit (1, 1) exchanges nothing, so only when its workspace would be
 *   too large).
 * admm_shortlist -- the same ranking: the k cheapest candidates into host
 *   Qs[k], Ps[k] and (host or NULL) model_s[k], their number into *count
 *   (<= k), and the workspace bytes the largest of them needs into
 *   *max_workspace (host or NULL).  Host computation.  Errors: as
 *   admm_choose_split, EINVAL (k < 1, NULL outputs).
 * admm_choose_split_measure -- the same ranking, then the `shortlist`
 *   cheapest candidates that fit the workspace are set up and timed on the
 *   device (setup plus 20 iterations after a warm-up solve, in the caller's
 *   workspace, with H and g as for admm_calibrate); the pick is the one with
 *   the least measured setup + iters x iteration time, returned in
 *   measured_s (host or NULL).  Synchronises `stream`.  Errors: those of
 *   admm_choose_split, EINVAL (shortlist < 1, NULL H, g or workspace),
 *   EWORKSPACE (no shortlisted split fits), the errors of admm_setup and
 *   admm_solve.
 */
int admm_model_coefficients(double* coef);
int admm_calibrate(const void* H, const void* g, int64_t m, int64_t n,
                   int storage, void* workspace, size_t workspace_bytes,
                   void* stream, double* coef);
int admm_choose_split(int64_t m, int64_t n, int iters, int storage,
                      double max_exchange, const double* coef, int* Q_out,
                      int* P_out, double* model_s);
int admm_shortlist(int64_t m, int64_t n, int iters, int storage,
                   double max_exchange, const double* coef, int k, int* Qs,
                   int* Ps, double* model_s, int* count,
                   size_t* max_workspace);
int admm_choose_split_measure(const void* H, const void* g, int64_t m,
                              int64_t n, int iters, int storage,
                              double max_exchange, const double* coef,
                              int shortlist, void* workspace,
                              size_t workspace_bytes, void* stream,
                              int* Q_out, int* P_out, double* measured_s);

/*
 * admm_setup -- build a plan: copy/quantise H into the workspace and factor
 * every block's Gram matrix G_ij = rho I + H_ij H_ij^H once (FP64 Gram,
 * Cholesky and inverse on the GPU, stored as an FP32 Hermitian inverse), or
 * A_ij = rho I + H_ij^H H_ij for a plan in the direct form (see
 * ADMM_XUPDATE_DIRECT).  This is the paper's one-off "inversion" step
 * (Sec. III, inversion lemma; Table tab:timing, "Inversion time").
 *   out       host, receives the plan (host memory, free with admm_destroy).
 *   H         device, m x n complex64, row-major with leading dimension n.
 *             Read only during this call; the caller may free it afterwards.
 *   m..storage  as for admm_workspace_bytes.
 *   rho       augmented-Lagrangian parameter, finite and > 0.
 *   lambda    l1 weight, finite and >= 0 (changeable by admm_set_lambda).
 *   workspace device, >= admm_workspace_bytes, 256-byte aligned; owned by the
 *             caller and must outlive the plan.
 *   stream    hipStream_t (void*).
 * Synchronises `stream`.  Errors: EINVAL, EWORKSPACE, ENONFINITE (NaN/Inf
 * in H), ENOTPD, EHIP.  On error *out is set to NULL.
 */
int admm_setup(admm_plan** out, const void* H, int64_t m, int64_t n,
               int Q, const int64_t* row_off, int P, const int64_t* col_off,
               double rho, double lambda, int storage,
               void* workspace, size_t workspace_bytes, void* stream);

/* Change lambda (finite, >= 0) of a plan; the Gram factors do not depend on
 * it.  Errors: EINVAL. */
int admm_set_lambda(admm_plan* plan, double lambda);

/*
 * admm_solve -- run ADMM iterations on measurements g.
 *   g          device complex64[m]; must stay valid until the stream reaches
 *              the end of this call's work.
 *   iters      >= 0 iterations to run (0 only copies the current image).
 *   tol        <= 0: run exactly `iters`.  > 0: after every `check_every`-th
 *              iteration stop when |r_p| <= tol max(|(u^i)|, sqrt(Q)|v|) and
 *              |r_d| <= tol rho |(s^i)| (residuals of Sec. III-C).
 *   check_every >= 1 (ignored when tol <= 0).
 *   v_out      device complex64[n], receives the image v after the last
 *              iteration.
 *   iters_done host int or NULL: iterations actually run.
 *   resid_hist device double[2*iters] or NULL: per iteration |r_p|^2 and
 *              |r_d|^2 (r_d uses rho^2 Q |v^k - v^{k-1}|^2).
 *   warm       0: start from u = v = s = ghat = 0.  1: continue from the
 *              plan's current state (previous solve or admm_set_state).
 *   stream     hipStream_t.
 * Synchronises `stream` at the end (and at every check when tol > 0).
 * Errors: EINVAL, ENONFINITE (a NaN/Inf reached the image), EHIP.
 */
int admm_solve(admm_plan* plan, const void* g, int iters, double tol,
               int check_every, void* v_out, int* iters_done,
               double* resid_hist, int warm, void* stream);

/*
 * admm_set_graphs -- graph replay in admm_solve on (enable != 0) or off (the
 * default: on MI355X dependent plain launches ran faster than the replayed
 * graph, 1 % at 6144 x 32000 and 9 % at 256 x 4096).  When on, and no kernel timing is enabled (admm_profile), a solve
 * captures the launches of a run of iterations (10, or check_every when
 * tol > 0) once as a HIP graph on a stream of the plan (default priority)
 * and replays it; the captured launches depend on g, resid_hist and lambda,
 * so a solve with other values captures again.  The solve's work is ordered
 * after earlier work on `stream` and before later work on it by events.
 * Results are bitwise those of plain launches.  Errors: EINVAL.
 */
int admm_set_graphs(admm_plan* plan, int enable);

/*
 * Reverse mode of K unrolled iterations (the differentiable map
 * (g, lambda, rho) -> v^K from the zero state).
 *
 * admm_tape_bytes   -- size of the tape for `iters` iterations with a
 *                      checkpoint of (v, s, ghat) every `interval` iterations.
 * admm_solve_record -- admm_solve from the zero state for exactly `iters`
 *                      iterations, writing the checkpoints to `tape` (device,
 *                      >= admm_tape_bytes, 256-byte aligned, caller-owned) and
 *                      v^K to v_out (device complex64[n]).
 * admm_backward     -- given grad_v = dL/dv^K (device complex64[n]), writes
 *                      grad_g = dL/dg (device complex64[m]) and the host
 *                      doubles dL/dlambda, dL/drho.  Complex gradients use the
 *                      convention dL/dRe z + j dL/dIm z.  `g` must be the
 *                      measurements the tape was recorded with.  Each
 *                      checkpoint interval is recomputed forward (storing the
 *                      Gram-apply output y and the pre-threshold mean a of
 *                      each iteration in the tape) and then swept in reverse:
 *                      soft-threshold Jacobian, H u, G^{-1} (its rho
 *                      derivative -G^{-2}), H^H r, estimated-data and
 *                      local-data adjoints.  FP32 vectors, FP64 scalar sums.
 *                      The tape is also the sweep's scratch: backward writes
 *                      the recomputed y and a records into it (the
 *                      checkpoints stay), so a tape serves any number of
 *                      backward calls.  Leaves the plan's iteration state at
 *                      the end of the first checkpoint interval (iteration
 *                      min(interval, iters), reported by admm_get_state).
 * Errors: EINVAL; EWORKSPACE (tape too small); ESTATE (tape not recorded by
 * this plan, or lambda changed since); ENONFINITE; EHIP; EUNSUPPORTED for a
 * plan in the direct form (the sweep is built for the inversion-lemma form).
 * All synchronise `stream`.
 */
int admm_tape_bytes(const admm_plan* plan, int iters, int interval,
                    size_t* out_bytes);
int admm_solve_record(admm_plan* plan, const void* g, int iters, int interval,
                      void* tape, size_t tape_bytes, void* v_out,
                      void* stream);
int admm_backward(admm_plan* plan, const void* g, const void* grad_v,
                  void* tape, void* grad_g, double* grad_lambda,
                  double* grad_rho, void* stream);

/*
 * admm_get_state / admm_set_state -- the iteration state (k, v, s, ghat),
 * which fixes every later iterate (c = v - s and g'_ij follows from ghat).
 *   v     device complex64[n];  s device complex64[Q*n] (replica i at i*n);
 *   ghat  device complex64[P*m] (for column block j, entry j*m + row holds
 *         ghat_ij for the row's block i);  k host int.
 * get may pass NULL for any output it does not want.  Errors: EINVAL, EHIP.
 */
int admm_get_state(admm_plan* plan, void* v, void* s, void* ghat, int* k,
                   void* stream);
int admm_set_state(admm_plan* plan, const void* v, const void* s,
                   const void* ghat, int k, void* stream);

/*
 * admm_kkt -- lasso optimality check of an image in FP64 (one pass over the
 * stored H, accumulated in double):  z = H^H (g - H v);  the result is
 * max_n dist(z_n, lambda * subdifferential of |v_n|) / lambda, i.e.
 * |z_n - lambda v_n/|v_n|| on the support and max(0, |z_n| - lambda) off it.
 * Zero at the lasso minimiser; every splitting's fixed point satisfies it.
 *   g, v    device complex64[m], complex64[n].
 *   out     host double.
 *   lambda must be > 0.  Synchronises `stream`.  Errors: EINVAL, EHIP.
 */
int admm_kkt(admm_plan* plan, const void* g, const void* v, double* out,
             void* stream);

/*
 * admm_kkt_noalloc -- admm_kkt for callers that cannot allocate device memory
 * at the call (code near HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same check and result, but its scratch (v in the
 * padded column space, the FP64 residual, the FP64 adjoint partials and the
 * per-workgroup maxima) lives in one static device array of the library,
 * 16 MiB per GPU, held until the process ends, instead of in the plan's
 * workspace.  It calls no allocating routine.  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (two streams, two
 * threads) race and must be serialised by the caller.
 *   Arguments, synchronisation and result as admm_kkt.
 *   Errors: EINVAL, EHIP; EWORKSPACE when the plan's check needs more than
 *   the 16 MiB: 8 n_pad + 16 m + 16 n_pad Q KH + 8 T bytes, each term
 *   rounded up to 256 (n_pad, KH = "chunks" of admm_plan_info, T = 64-column
 *   tiles of the column blocks); 6144 x 32000 with Q = 4, P = 8 needs
 *   8.8 MB.  EUNSUPPORTED on a device index of 64 or more.
 */
int admm_kkt_noalloc(admm_plan* plan, const void* g, const void* v, double* out,
                     void* stream);

/*
 * admm_hty_absmax -- ||H^H g||_inf over the stored H, accumulated in FP64:
 * the scale of the regularisation weight (the lasso minimiser is 0 for
 * lambda >= ||H^H g||_inf; workloads set lambda as a fraction of it).  Uses
 * the same pass as admm_kkt with v = 0 (for bf16 / fp8 storage, over the
 * dequantised H).
 *   g    device complex64[m].   out  host double.
 *   Synchronises `stream`.  Errors: EINVAL, EHIP.
 */
int admm_hty_absmax(admm_plan* plan, const void* g, double* out, void* stream);

/*
 * admm_get_stored_h -- copy the plan's stored H back out as dense m x n
 * row-major planes (for checking the quantiser):
 *   C64:  re_out receives complex64[m*n]; im_out and scale_out are ignored.
 *   BF16: re_out, im_out receive uint16 bfloat16 codes [m*n].
 *   FP8:  re_out, im_out receive uint8 e4m3 codes [m*n]; scale_out receives
 *         float[m], the row scales s_r (value = s_r * e4m3(code)).
 * All outputs are device memory.  Synchronises `stream`.  Errors: EINVAL, EHIP.
 */
int admm_get_stored_h(admm_plan* plan, void* re_out, void* im_out,
                      float* scale_out, void* stream);

/*
 * Profiling.  admm_profile(plan, every) with every >= 1 makes later solves
 * time the kernels of every every-th iteration (iteration index k of each
 * solve with k % every == 0) with HIP events carried by the kernels' own
 * dispatch packets on the solve's stream; admm_profile_read returns the
 * summed duration in ms and the number of timed launches of one kernel class
 * since profiling was enabled (ADMM_K_* below).  admm_profile(plan, 0) stops
 * and clears.  Reading synchronises the recorded events.  Timing adds a few
 * microseconds between the timed kernels, so sample (every > 1) inside a
 * throughput measurement.  Errors: EINVAL (every < 0), EHIP.
 */
#define ADMM_K_GEMV_N   0   /* r_ij = g'_ij - H_ij c_j^i (two-pass);            */
                            /* direct form: ghat_ij = H_ij u_j^i                */
#define ADMM_K_GRAM     1   /* y_ij = G_ij^{-1} r_ij, ghat update;              */
                            /* direct form: the pieces of A_ij^{-1} d_ij        */
#define ADMM_K_GEMV_H   2   /* partial H_ij^H y_ij (two-pass);                  */
                            /* direct form: partial H_ij^H r_i                  */
#define ADMM_K_ZUPDATE  3   /* mean, soft threshold, duals, norms (two-pass);   */
                            /* direct form: u from the pieces, then the same    */
#define ADMM_K_FZ_ROWS  4   /* single pass: r_ij from the slab parts of H c      */
#define ADMM_K_FZ_SLAB  5   /* single pass: H^H y, z- and dual update, next H c */
#define ADMM_K_DIRECT_GP  6 /* direct form: row residuals r_i (or g') from ghat */
#define ADMM_K_DIRECT_RHS 7 /* direct form: d = H^H r_i + rho (c - u_prev)     */
#define ADMM_K_COUNT    8
int admm_profile(admm_plan* plan, int every);
int admm_profile_read(admm_plan* plan, int kernel, double* total_ms,
                      int64_t* launches);

/* Static description of the plan: fills host int64 info[16] with
 * m, n, Q, P, storage, chunks of the adjoint product, workspace bytes,
 * bytes of stored H, bytes of stored inverses, iterations done, padded row
 * and column space lengths, 4 x 4 tile patches of the Gram apply (0: one
 * tile per workgroup), 1 if the plan iterates in a single pass over H (else
 * 0), workgroups of the single-pass slab kernel, 1 if the plan takes the
 * direct x-update (else 0). */
int admm_plan_info(const admm_plan* plan, int64_t* info16);

/* Release the plan (host memory only; the workspace stays the caller's). */
void admm_destroy(admm_plan* plan);

/* ======================================================================
 * Batched multi-scene form.
 *
 * S scenes measured by one instrument matrix H0 (m0 x n).  The rows of H0
 * come in tiles of `tile_rows` consecutive rows (one frequency each; 64,
 * 128 or 256, dividing m0).  Scene s measures the tiles
 * tiles[tiles_off[s] .. tiles_off[s+1]) (strictly increasing tile indices),
 * each of its rows multiplied by a unit phase, so its sensing matrix is
 *     H_s = diag(phase_s) H0[rows of its tiles, :]
 * (a subsampling of frequencies with a per-row code).  Its Q_s row blocks
 * are cut at tile boundaries: cuts[cuts_off[s] .. cuts_off[s+1]) = Q_s + 1
 * increasing tile counts from 0 to its number of tiles.  All scenes share
 * the column split (P, col_off, NULL = equal) and rho; each has its own
 * lambda.  Every scene runs the same consensus-and-sectioning iteration as
 * admm_solve (Sec. III-C).  The products of all scenes with the shared H0
 * are dense GEMMs per (tile, column block) run on MFMA: H0 is stored in
 * bfloat16 (round to nearest even) and the FP32 vector operands are split
 * into three bfloat16 terms, with FP32 accumulation.  Each scene block's Gram
 * inverse is built in FP64 from the shared Gram of H0's tiles.
 *   H0       device complex64 m0 x n, row-major (read during setup only).
 *   phases   device complex64, the scenes' rows packed scene after scene.
 *   lambdas  host double[S].
 *   g        device complex64, packed like phases.
 *   v_out    device complex64 S x n (scene s at s*n).
 *   use_graph  1: replay one captured hipGraph of the iteration per step.
 * Errors: EINVAL, EUNSUPPORTED (a block with m_i >= (1 + sqrt 2) n_j: the
 * batch applies the inversion-lemma x-update only), EWORKSPACE, ENONFINITE,
 * ENOTPD, EHIP.  setup and solve synchronise `stream`.
 * ====================================================================== */
typedef struct admm_batch admm_batch;

/* flags: 0, ADMM_INVERSE_BF16 and/or ADMM_GRAM_PATCHES (the same value in both
 * calls). */
int admm_batch_workspace_bytes(int64_t m0, int64_t n, int tile_rows, int S,
                               const int32_t* tiles, const int64_t* tiles_off,
                               const int32_t* cuts, const int64_t* cuts_off,
                               int P, const int64_t* col_off, int flags,
                               size_t* out_bytes);
int admm_batch_setup(admm_batch** out, const void* H0, int64_t m0, int64_t n,
                     int tile_rows, int S, const int32_t* tiles,
                     const int64_t* tiles_off, const int32_t* cuts,
                     const int64_t* cuts_off, const void* phases, int P,
                     const int64_t* col_off, int flags, double rho,
                     const double* lambdas, void* workspace,
                     size_t workspace_bytes, void* stream);
int admm_batch_solve(admm_batch* batch, const void* g, int iters,
                     void* v_out, int use_graph, void* stream);
/* Kernel event timing as admm_profile (solves run without the graph while
 * on): 0 forward GEMM, 1 Gram apply, 2 adjoint GEMM, 3 z-update. */
int admm_batch_profile(admm_batch* batch, int enable);
int admm_batch_profile_read(admm_batch* batch, int kernel, double* total_ms,
                            int64_t* launches);
/* info16: m0, n, S, P, row blocks, scene tiles, workspace bytes, bytes of
 * the complex64 packed inverses, chosen forward k-chunks per column block, chosen adjoint columns per
 * workgroup, their work items, packed rows, chosen forward rows per
 * workgroup, 4 x 4 tile patches of the Gram apply (0: one tile per
 * workgroup), 0 */
int admm_batch_info(const admm_batch* batch, int64_t* info16);
/* Autotuner timings (ms): the three forward GEMM shapes [0..2] (rows per
 * workgroup, k-chunks per column block: (128, 1), (128, 2), (64, 2), rows
 * capped at tile_rows); the adjoint GEMM with 64, 128, 256 columns per
 * workgroup [3..5]. */
int admm_batch_tuning(const admm_batch* batch, double* ms6);
void admm_batch_destroy(admm_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* ADMM_H */
