/*
 * shlr.h -- C ABI of the MI355X separable low-rank Hankel (SHLR) library.
 *
 * The library reconstructs undersampled multi-coil k-space with the
 * separable Hankel low-rank models of Zhang et al., "Accelerated MRI
 * Reconstruction with Separable and Enhanced Low-Rank Hankel Regularization"
 * (arXiv 2107.11650):
 *   - parallel imaging (model SHLR_MODEL_PI): SHLR, SHLR-S, SHLR-V, SHLR-SV
 *     (Eqs. 2, 3, 5, 6), solved by the ADMM of Eqs. 9-17 in the order of
 *     Algorithm S1 (inputs Y, U, G, lambda, lambda1, beta, tau; output X,
 *     returned here as its k-space K = F^2D X, Eq. 2);
 *   - parameter imaging (model SHLR_MODEL_PARAM): SHLR-P and SHLR-VP
 *     (Eqs. 7, 8), solved by Eqs. S1-S9 in the order of Algorithm S2 for every
 *     frequency-encode position (inputs Y^Parameter, U, lambda, lambda2, beta,
 *     tau).
 *
 * Conventions shared by every entry point
 *   - Complex data are interleaved (re, im): float pairs (complex64) when
 *     precision is SHLR_PREC_MIXED or SHLR_PREC_MIXED_R32, double pairs
 *     (complex128) when precision == SHLR_PREC_FP64.
 *   - k-space is centred: the DC sample of an axis of length n sits at index
 *     n / 2 (integer division).  Every DFT is unitary.
 *   - "dev" pointers are device (HBM) pointers owned by the caller; "host"
 *     pointers are host memory owned by the caller.  The library never frees
 *     caller memory and never keeps a caller pointer past the call, except the
 *     workspace bound by shlr_bind, which must outlive the plan's use.
 *   - Every function returns a shlr_status; none throws or aborts.  The text
 *     of the last error of the calling thread is shlr_last_error().
 *   - Work is enqueued on the stream given to shlr_bind (a hipStream_t passed
 *     as void*).  Functions that return results to the host synchronise that
 *     stream.  A plan must not be used from two threads at once.
 */
#ifndef SHLR_H
#define SHLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHLR_MODEL_PI 0     /* parallel imaging: SHLR(-S/-V/-SV)          */
#define SHLR_MODEL_PARAM 1  /* parameter imaging: SHLR-P / SHLR-VP         */

/* Precision forms.  In every form the Gram matrices are accumulated to FP64 and the
 * eigenvalue count above the threshold (the decision of Eq. 16) is a Sturm count in FP64
 * arithmetic on the tridiagonal form; the forms differ in the data type and in the
 * arithmetic of the Householder reduction that produces that tridiagonal form. */
#define SHLR_PREC_MIXED 0     /* complex64 data; FP32 MFMA Gram and reprojection products with FP32
                                 accumulation; the whole Hermitian eigen-solve (Householder reduction,
                                 eigenvalues, threshold decision, eigenvectors, S) in FP64          */
#define SHLR_PREC_FP64 1      /* complex128 data; FP64 everywhere                                    */
#define SHLR_PREC_MIXED_R32 2 /* opt-in: as SHLR_PREC_MIXED but the Householder reduction to
                                 tridiagonal form runs in FP32 (FP64 scalars), so the tridiagonal
                                 whose eigenvalues are counted carries FP32 rounding (backward error
                                 about 1e-7 of the Gram norm); faster, not the default.  Not
                                 accepted by the reverse-mode calls.                                 */

#define SHLR_MAX_SLICES 4096

typedef enum {
    SHLR_OK = 0,
    SHLR_E_INVALID_ARG = 1,   /* a size, window, weight or pointer is out of range         */
    SHLR_E_SINGULAR = 2,      /* Eq. 15 / Eq. S7 has a zero pivot (e.g. the k-space centre  */
                              /* is not sampled while W vanishes there)                     */
    SHLR_E_NONFINITE = 3,     /* NaN or Inf met in the input or in the iterate               */
    SHLR_E_WORKSPACE = 4,     /* no workspace bound, or the bound one is too small          */
    SHLR_E_DEVICE = 5,        /* a HIP runtime call failed                                  */
    SHLR_E_UNSUPPORTED = 6,   /* a combination the library does not implement               */
    SHLR_E_STATE = 7,         /* call out of order (e.g. iterate before init)               */
    SHLR_E_EIG_NOCONV = 8     /* an eigenpair of the eigen-solve behind the threshold of    */
                              /* Eq. 16 / Eqs. S8-S9 failed its residual check              */
} shlr_status;

/*
 * Problem description.  All host arrays are read during shlr_plan_create only.
 *
 * SHLR_MODEL_PI: n_slices independent slices, slice s of size M[s] x N[s]
 *   (rows x columns, Table I), J coils.  Row lifts (P_m, Eq. 2) act on lines of
 *   length N with window k_row; column lifts (Q_n) on lines of length M with
 *   window k_col.  Data layout [slice][J][M][N] with N fastest, slices packed
 *   back to back; mask layout [slice][M][N] (uint8, nonzero = acquired,
 *   shared by all coils).
 * SHLR_MODEL_PARAM: one series of L echoes (parameter dimension), M
 *   frequency-encode positions (fully sampled) and N phase-encode positions
 *   (n_slices must be 1).  PE lifts (Q_l with W, F and optionally H_vc, Eq. 8)
 *   use window k_row on lines of length N; parameter-direction lifts (P_n, H
 *   only) use window k_col on lines of length L.  Data layout [L][J][M][N];
 *   mask layout [L][N] (acquired PE lines of each echo).
 */
typedef struct {
    int32_t model;          /* SHLR_MODEL_PI or SHLR_MODEL_PARAM                        */
    int32_t precision;      /* SHLR_PREC_MIXED, SHLR_PREC_FP64 or SHLR_PREC_MIXED_R32     */
    int32_t n_slices;       /* PI: 1..SHLR_MAX_SLICES; PARAM: 1                           */
    const int32_t* M;       /* host [n_slices]: rows (PARAM: FE positions)                */
    const int32_t* N;       /* host [n_slices]: columns (PARAM: PE positions)             */
    int32_t J;              /* coils, >= 1                                                */
    int32_t L;              /* echoes (PARAM), >= 2; ignored for PI                       */
    int32_t k_row;          /* window of row (PI) / PE (PARAM) lifts, 1..line length      */
    int32_t k_col;          /* window of column (PI) / parameter-direction lifts           */
    int32_t use_vc;         /* 1: virtual-coil lifts H_vc (Eq. 4; SHLR-V/-SV/-VP)         */
    int32_t use_w;          /* 1: weighting W (Eq. 2); 0: plain Hankel of F^1D lines      */
    int32_t spirit_ksize;   /* PI only: 0 = no SPIRiT term; odd kernel size (e.g. 5)       */
    int32_t hard_dc;        /* 1: lambda = +inf, acquired samples kept exactly             */
    int32_t normalize;      /* 1: divide Y by max|Y| before iterating, scale back after    */
    int32_t max_iter;       /* iteration cap used by shlr_reconstruct                      */
    int32_t n_cg;           /* PCG steps per X-update when the SPIRiT term is on           */
    double lambda;          /* data-consistency weight (Eq. 2), > 0 unless hard_dc         */
    double lambda1;         /* SPIRiT weight (Eq. 3), >= 0                                 */
    double lambda2;         /* parameter-direction weight (Eq. 7), > 0 for PARAM           */
    double beta;            /* ADMM penalty (Eq. 9), > 0                                   */
    double tau;             /* multiplier step (Eqs. 13-14), > 0                           */
    double tol;             /* relative-change stop of Algorithm S1/S2; <= 0: fixed count;  */
                            /* checked per unit (slice of PI, FE position of PARAM)         */
    double d0;              /* initial multiplier value (Algorithms S1/S2 use 1)           */
    int64_t slot_budget;    /* bytes of eigen-solver slots per chunk of a run of lifted     */
                            /* matrices (G, S and solver scratch per matrix); 0: 16 GiB.   */
                            /* A run larger than the budget is solved in chunks, one set   */
                            /* of launches each (results do not depend on it); >= 0        */
} shlr_params;

typedef struct {
    int32_t iters_done;     /* iterations run by the last call (with tol > 0: the most any  */
                            /* unit ran in that call)                                       */
    int32_t converged;      /* 1 if the tol test has stopped every unit                     */
    double rel_change;      /* with tol > 0: the largest over units of the last             */
                            /* ||K^{k+1}-K^k||^2 / ||K^k||^2 of each unit; else 0           */
    double scale;           /* max|Y| used for normalisation (1 if off)                     */
    uint32_t device_flags;  /* bit0: non-finite value met; bit1: an eigenpair failed the     */
                            /* residual check of shlr_set_eig_check (SHLR_E_EIG_NOCONV)      */
} shlr_info;

typedef struct shlr_plan shlr_plan;

/* Fill *p with the paper's settings for a model (Algorithms S1 / S2): iteration cap 50
 * (SHLR_MODEL_PI) or 100 (SHLR_MODEL_PARAM), relative-change tolerance 1e-6, initial
 * multipliers D = 1 (Z = 0), weighting W on, virtual coils off, no SPIRiT term, soft data
 * consistency, normalisation on, precision SHLR_PREC_MIXED, one slice.  Sizes (M, N, J, L,
 * windows) and the weights lambda, lambda1, lambda2, beta, tau, which the paper sets per
 * experiment, are left 0 / NULL for the caller to fill. */
shlr_status shlr_params_default(int32_t model, shlr_params* p);

/* Validate p and build the plan (host only, no device call).  *out is NULL on error. */
shlr_status shlr_plan_create(const shlr_params* p, shlr_plan** out);

/* Free the plan's host memory (the workspace belongs to the caller).  NULL is accepted. */
void shlr_plan_destroy(shlr_plan* plan);

/* Bytes of device workspace the plan needs (host only). */
shlr_status shlr_workspace_size(const shlr_plan* plan, size_t* bytes);

/* Bind a caller-owned device workspace of at least shlr_workspace_size bytes
 * (256-byte aligned) and the stream to enqueue on; uploads the plan's tables. */
shlr_status shlr_bind(shlr_plan* plan, void* ws_dev, size_t bytes, void* stream);

/* Replace the weighting W of Eq. 2 (the diagonal filter applied to every lifted line; by default
 * the DFT of the circular first difference, w(f) = 1 - exp(-2 pi i f / n) at the centred frequency
 * f) with caller values, and rebuild what depends on it: the Gram diagonals of the Eq. 15 / Eq. S7
 * denominators and the adjoint lift of the initial multipliers.  w_row_dev: device, complex128,
 * the row-line (PI) or PE-line (PARAM) weights of every slice back to back (N[s] values per
 * slice); w_col_dev: device, complex128, the column-line weights (M[s] per slice) for PI, NULL
 * for PARAM (the parameter-direction lifts are unweighted, Eq. 7).  The plan must have
 * use_w = 1 (else SHLR_E_STATE) and be bound; the iterate is discarded, so shlr_init must
 * follow.  A point where both directions' weights vanish must be sampled (SHLR_E_SINGULAR
 * at shlr_init otherwise).  Synchronises the stream. */
shlr_status shlr_set_weights(shlr_plan* plan, const void* w_row_dev, const void* w_col_dev);

/* SPIRiT kernel (Eq. 3) from host memory: g_host[t][s][dm][dn], complex128,
 * J x J x ks x ks, with K_t(x) ~ sum_{s,d} g[t][s][d] K_s(x + d) (circular).
 * The per-pixel image-domain operator (G - I)^H (G - I) is built on the device. */
shlr_status shlr_set_spirit_kernel(shlr_plan* plan, const void* g_host);

/* Calibrate the SPIRiT kernel by Tikhonov least squares on the fully sampled
 * acs x acs centre of the (normalised) data given to shlr_init, then install it.
 * Weight reg * trace(A^H A) / n_unknowns.  Requires shlr_init first. */
shlr_status shlr_calibrate_spirit(shlr_plan* plan, int32_t acs, double reg);

/* Start a reconstruction: copy Y (device, layout above) and the mask
 * (device, uint8), normalise, set Z = 0, D = d0 and K = Y (Algorithm S1/S2
 * initialisation). */
shlr_status shlr_init(shlr_plan* plan, const void* y_dev, const uint8_t* mask_dev);

/* Run up to n ADMM iterations (X-update Eq. 15 / S7, Z-updates Eqs. 16-17 / S8-S9,
 * multiplier updates Eqs. 13-14 / S5-S6).  With tol > 0 the stop test of Algorithms S1 / S2
 * runs on the device after every iteration, per unit (each slice of SHLR_MODEL_PI, each FE
 * position of SHLR_MODEL_PARAM): a unit whose relative change ||K^{k+1}-K^k||^2 / ||K^k||^2
 * falls below tol keeps its K from then on, as if its own loop had ended.  The host reads
 * only the number of active units, every 8 iterations, and returns once it is 0.  With
 * tol <= 0 nothing is read back.  info (may be NULL) is filled after a stream
 * synchronisation. */
shlr_status shlr_iterate(shlr_plan* plan, int32_t n, shlr_info* info);

/* The same n iterations as replays of a HIP graph of one iteration, captured at the first
 * call (stop test included when tol > 0; no early return to the host). */
shlr_status shlr_iterate_graph(shlr_plan* plan, int32_t n, shlr_info* info);

/* Residual check of the eigen-solve behind every singular-value threshold (Eq. 16; Eqs.
 * S8-S9): each eigenpair (l, z) of the real tridiagonal form T of a Gram matrix that enters
 * S must satisfy ||T z - l z|| <= rel_residual_limit * ||T|| * ||z|| (||T||: Gershgorin
 * bound); a failure, or an eigenvector that had to be replaced because it came out zero
 * or non-finite, sets bit 1 of shlr_info.device_flags, and the iterate / reconstruct call
 * returns SHLR_E_EIG_NOCONV (the iterate is still written).  Default 1e-6 (converged pairs
 * sit near 1e-14 in FP64 and below 1e-10 in the mixed forms); 0 makes every pair with a
 * non-zero residual fail.  rel_residual_limit must be finite and >= 0. */
shlr_status shlr_set_eig_check(shlr_plan* plan, double rel_residual_limit);

/* Per-unit state of the stop test since shlr_init: units are the slices (SHLR_MODEL_PI)
 * or the FE positions (SHLR_MODEL_PARAM); n_units must equal that count.  iters_host
 * [n_units] receives the iterations each unit ran (counted only when tol > 0),
 * rel_host [n_units] its last relative change, active_host [n_units] 1 while it still
 * iterates.  Any output pointer may be NULL.  Synchronises the stream. */
shlr_status shlr_unit_status(const shlr_plan* plan, int32_t n_units, int32_t* iters_host, double* rel_host,
                             int32_t* active_host);

/* Write the current k-space estimate (scaled back) to k_out_dev (layout of Y). */
shlr_status shlr_get_kspace(const shlr_plan* plan, void* k_out_dev);

/* shlr_init + shlr_iterate(max_iter) + shlr_get_kspace. */
shlr_status shlr_reconstruct(shlr_plan* plan, const void* y_dev, const uint8_t* mask_dev,
                             void* k_out_dev, shlr_info* info);

/* Per-phase device timing of later shlr_iterate calls, measured with HIP events
 * recorded on the plan's stream around every launch of a phase.  enable != 0
 * starts (and resets) the accumulation; enable == 0 stops it.  shlr_iterate_graph
 * is not timed. */
#define SHLR_TIMING_PHASES 6
shlr_status shlr_timing_enable(shlr_plan* plan, int32_t enable);

/* As shlr_timing_enable, for the phases whose bits are set in phase_mask (bit p: phase p
 * of shlr_timing_read); the other phases record no events, so their launches run as
 * untimed.  phase_mask == 0 stops the accumulation; bits at or above SHLR_TIMING_PHASES
 * are rejected with SHLR_E_INVALID_ARG. */
shlr_status shlr_timing_enable_phases(shlr_plan* plan, uint32_t phase_mask);

/* Read the accumulated times (synchronises the stream).  Phase index:
 * 0 transforms and X-update (Eq. 15 / S7), 1 lift + Gram, 2 eigen-solve and
 * threshold (Eq. 16), 3 reprojection + multiplier update (Eq. 13) + adjoint
 * lift, 4 SPIRiT PCG, 5 register-resident Householder reduction of the Gram
 * matrices (the first stage of the eigen-solve where it applies).
 * ms_out[6] milliseconds, launches_out[6] launch counts. */
shlr_status shlr_timing_read(shlr_plan* plan, double* ms_out, int32_t* launches_out);

/* Choose the launch parameters of the batched low-rank step by timing them on this
 * plan's own shapes: per bucket of identical lifted-matrix shapes the rows staged per
 * chunk of the lift + Gram and reprojection products, per run of buckets the
 * Householder reduction (register-resident or in memory).  Candidates run on
 * seeded pseudo-random data written into the bound workspace and timed with HIP
 * events on the plan's stream; reps (1..100) runs each, the best counts.  The
 * workspace then holds no iterate: call shlr_init before iterating.  report
 * (host, may be NULL) receives a NUL-terminated text of the choices and times,
 * truncated to report_len bytes.  The iteration computes the same quantities
 * with any choice (rounding order aside). */
shlr_status shlr_autotune(shlr_plan* plan, int32_t reps, char* report, size_t report_len);

/* ---------------------------------------------------------------------------
 * Reverse mode through unrolled iterations.
 *
 * The paper states no derivative; these calls differentiate the fixed map of
 * n_iter iterations of Algorithm S1 (X-update of Eq. 15, SVT of Eq. 16,
 * multiplier update of Eq. 13, for rows and columns) from the acquired
 * k-space Y and the data-consistency weight lambda (Eq. 2) to the k-space
 * K after the n_iter-th X-update.  Scope: SHLR_MODEL_PI with finite lambda
 * (hard_dc = 0), no SPIRiT term (spirit_ksize = 0) and normalize = 0 (the
 * caller scales Y); virtual coils and any number of slices are covered.
 * Gradients follow the real inner product: for the loss L = Re <gK, K>
 * (sum over entries of conj(gK) K) the call returns gY with dL = Re <gY, dY>
 * and dL/dlambda.  The SVT derivative is the spectral-function derivative
 * of the Gram form (Daleckii-Krein divided differences, exact at repeated
 * singular values); it is undefined where a singular value equals the
 * threshold.
 * ------------------------------------------------------------------------- */

/* Bytes of the checkpoint buffer (K after every X-update, the multipliers
 * before every low-rank step) and of the backward work buffer for n_iter
 * iterations.  SHLR_E_UNSUPPORTED outside the scope above. */
shlr_status shlr_unrolled_sizes(const shlr_plan* plan, int32_t n_iter, size_t* ckpt_bytes,
                                size_t* work_bytes);

/* shlr_init(y_dev, mask_dev), then n_iter iterations that fill ckpt_dev
 * (device, >= ckpt_bytes of shlr_unrolled_sizes, 256-byte aligned), then
 * K_n to k_out_dev (layout of Y).  The low-rank step of the last iteration
 * does not reach K_n and is skipped. */
shlr_status shlr_unrolled_forward(shlr_plan* plan, int32_t n_iter, const void* y_dev,
                                  const uint8_t* mask_dev, void* k_out_dev, void* ckpt_dev,
                                  size_t ckpt_bytes);

/* Reverse pass of the last shlr_unrolled_forward on this plan (same n_iter
 * and checkpoint buffer, else SHLR_E_STATE).  gk_dev: cotangent of K_n
 * (layout of Y); gy_dev: output gradient with respect to Y (layout of Y,
 * overwritten); g_lambda_host (may be NULL): dL/dlambda.  work_dev: device,
 * >= work_bytes of shlr_unrolled_sizes, 256-byte aligned.  The plan's
 * iterate state is consumed: call shlr_init before iterating again. */
shlr_status shlr_unrolled_backward(shlr_plan* plan, int32_t n_iter, const void* gk_dev,
                                   const void* ckpt_dev, size_t ckpt_bytes, void* work_dev,
                                   size_t work_bytes, void* gy_dev, double* g_lambda_host);

/* ---------------------------------------------------------------------------
 * Stage entry points (the steps of one iteration, callable on their own).
 * ------------------------------------------------------------------------- */

/* Centred unitary 1D DFT (F^1D, Eq. 2) of n_lines contiguous lines of length n
 * (inverse when inverse != 0).  in_dev and out_dev may alias.  n in [1, 4096]. */
shlr_status shlr_fft_lines(int32_t precision, int32_t n, int32_t n_lines, int32_t inverse,
                           const void* in_dev, void* out_dev, void* stream);

/* Workspace bytes for shlr_lowrank_lines with these shapes. */
shlr_status shlr_lowrank_workspace_size(int32_t precision, int32_t n_mat, int32_t J, int32_t n,
                                        int32_t k, int32_t use_vc, size_t* bytes);

/* One low-rank step on n_mat independent lines (Eqs. 16 and 13, plus the
 * adjoint lift that feeds Eq. 15), with the default eigenpair check (returns
 * SHLR_E_EIG_NOCONV or SHLR_E_NONFINITE after writing its outputs):
 *   T   = lift(h) + D / beta          lift = H~ W~ or H~_vc W~ (Eqs. 2, 4)
 *   Z   = S_thr(T)                     singular-value threshold (Eq. 16)
 *   D  <- D + tau (lift(h) - Z)        (Eq. 13), in place
 *   b   = lift^*(Z - D / beta)         (the term of the Eq. 15 right-hand side)
 * h_dev: [n_mat][J][n] lines (k-space along the line); d_dev: [n_mat][p][q]
 * with p = n-k+1, q = k*J*(1+use_vc), column index (v*J + j)*k + b; b_dev:
 * [n_mat][J][n] output.  use_w selects W.  ranks_dev (may be NULL) receives
 * the number of singular values above thr of each matrix (int32). */
shlr_status shlr_lowrank_lines(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k,
                               int32_t use_vc, int32_t use_w, double beta, double tau, double thr,
                               const void* h_dev, void* d_dev, void* b_dev, int32_t* ranks_dev,
                               void* ws_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Evaluation step after a reconstruction (Section IV and Supplement S2): the coil combination,
 * the two quality measures and the T2 map of the parameter-imaging experiment.  Real images are
 * float (SHLR_PREC_MIXED, SHLR_PREC_MIXED_R32) or double (SHLR_PREC_FP64), [M][N] row-major;
 * sums are accumulated in FP64 in a fixed order, so results repeat bit for bit.  work_dev is a
 * caller-owned device buffer of SHLR_EVAL_WORK_BYTES (8-byte aligned) for partial sums, except
 * where stated.  Calls are enqueued on `stream`; those returning a host value synchronise it.
 * ------------------------------------------------------------------------- */
#define SHLR_EVAL_WORK_BYTES 65536
#define SHLR_T2_MAX_ECHOES 32

/* SSOS coil combination (Section IV, first paragraph): img[i] = sqrt(sum_j |x_ij|^2) with x_ij
 * the centred unitary inverse 2D DFT of coil j of image i.  k_dev: [n_img][J][M][N] complex
 * k-space; work_dev: n_img*J*M*N complex of the precision (receives the coil images); img_dev:
 * [n_img][M][N] real output. */
shlr_status shlr_ssos(int32_t precision, int32_t n_img, int32_t J, int32_t M, int32_t N, const void* k_dev,
                      void* work_dev, void* img_dev, void* stream);

/* RLNE of Eq. S10: ||x - x_hat||_2 / ||x||_2 over count real values (x = ref_dev, the fully
 * sampled image; x_hat = rec_dev), restricted to roi_dev != 0 when roi_dev (uint8, count) is not
 * NULL.  SHLR_E_INVALID_ARG if the reference is zero there. */
shlr_status shlr_rlne(int32_t precision, int64_t count, const void* ref_dev, const void* rec_dev,
                      const uint8_t* roi_dev, void* work_dev, double* rlne_host, void* stream);

/* MSSIM of Eq. S11 between the reference ref_dev and rec_dev (both M x N, M, N >= 11): the mean
 * over every 11 x 11 window position inside the image of the SSIM of the window, with Gaussian
 * window weights (sigma 1.5, unit sum), C1 = (0.01 L)^2 and C2 = (0.03 L)^2, L = dyn_range, or the
 * reference's maximum when dyn_range <= 0 (the window and the constants are the cited SSIM
 * paper's; Eq. S11 states neither). */
shlr_status shlr_mssim(int32_t precision, int32_t M, int32_t N, const void* ref_dev, const void* rec_dev,
                       double dyn_range, void* work_dev, double* mssim_host, void* stream);

/* Pixel-wise T2 map (Section IV-B: nonlinear least squares per pixel inside a region of interest,
 * values outside a reasonable range excluded).  img_dev: [L][n_pix] real echo images (e.g. SSOS
 * magnitudes), te_host[L] echo times; per pixel S(TE) = rho exp(-TE / T2) is fitted in FP64 from
 * the log-linear least-squares start by Levenberg-Marquardt.  The ROI is every pixel whose first
 * echo is >= roi_frac times that image's maximum; outside it, where the fit fails, or where T2
 * falls outside [t2_min, t2_max], t2 (and rho) are 0 and roi is 0.  t2_dev [n_pix] real output;
 * rho_dev [n_pix] real and roi_dev [n_pix] uint8 outputs may be NULL.  2 <= L <= 32. */
shlr_status shlr_t2_fit(int32_t precision, int32_t L, int64_t n_pix, const double* te_host, const void* img_dev,
                        double roi_frac, double t2_min, double t2_max, void* t2_dev, void* rho_dev,
                        uint8_t* roi_dev, void* work_dev, void* stream);

/* shlr_lowrank_lines without the workspace argument, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid hipMalloc): the
 * eigen-solver slots, descriptors, weights and flags live in a fixed 64 MiB device array of the
 * library (one copy per GPU, taken at module load and held until the process ends), so no call
 * allocates.  Same arguments, outputs and status codes as shlr_lowrank_lines; lines that need
 * more than the array for one eigen-solver slot plus their tables are refused with
 * SHLR_E_WORKSPACE, and a batch larger than the array holds at once runs in more chunks.  All
 * calls on one GPU share its array: calls that overlap in time on that GPU (other threads or
 * streams) race and must be serialised by the caller; each call synchronises its stream before
 * it returns. */
shlr_status shlr_lowrank_lines_noalloc(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k,
                                       int32_t use_vc, int32_t use_w, double beta, double tau, double thr,
                                       const void* h_dev, void* d_dev, void* b_dev, int32_t* ranks_dev,
                                       void* stream);

/* Text of the calling thread's last error ("" if none). */
const char* shlr_last_error(void);

/* Library version string. */
const char* shlr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHLR_H */
