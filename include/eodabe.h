/*
 * eodabe.h -- C ABI of the MI355X (gfx950) EOD-ABE library.
 *
 * EOD-ABE (efficient orthogonal decomposition with automatic basis
 * extraction; Xu, Shen, Liu, Jia, arXiv 2506.22713) computes
 *     A ~= U_hat * D_hat * V_hat^T
 * for a real m x n matrix A, with U_hat (m x r) and V_hat (n x r) having
 * orthonormal columns and D_hat (r x r) upper triangular, where the rank r
 * is found on the fly by the blocked randomized basis extraction of
 * Alg. 1 (BasisExt) and the factorization is closed out by Alg. 2 (power
 * iteration, C = Q^T A, QR of C^T, QR of R^T).
 *
 * Conventions for every entry point:
 *   - Matrix arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *     tensors) unless stated otherwise.  Sizes are element counts.
 *   - A is row-major: element (i, j) at A[i*lda + j], lda >= n.  A is read
 *     only; the caller keeps ownership of every buffer it passes.
 *   - Work is enqueued on the stream given in eodabe_opts (0 = the null
 *     stream).  eodabe_factor returns after one final stream
 *     synchronisation, with the rank valid in *info.
 *   - The library allocates no device memory: the caller passes a
 *     workspace of at least eodabe_workspace_size() bytes.
 *   - Return value: 0 = EODABE_OK, < 0 error (nothing useful written),
 *     > 0 warning (results written).  No exception crosses the ABI.
 *   - One context per stream; a context is not thread safe.
 */
#ifndef EODABE_H
#define EODABE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eodabe_ctx eodabe_ctx;

/* ---- status codes ---------------------------------------------------- */
#define EODABE_OK             0
#define EODABE_EINVAL        -1   /* bad size, leading dimension, tol, option or NULL pointer */
#define EODABE_EWORKSPACE    -2   /* workspace NULL or smaller than eodabe_workspace_size() */
#define EODABE_ECAPACITY     -3   /* the rank found exceeds r_cap (outputs too small) */
#define EODABE_ENONFINITE    -4   /* A holds NaN or Inf (||A||_F is not finite) */
#define EODABE_EHIP          -5   /* a HIP runtime call failed (see eodabe_last_hip_error) */
#define EODABE_ENODEVICE     -6   /* no gfx950 device visible */
#define EODABE_ESCRATCH      -7   /* eodabe_factor_noalloc: the problem needs more workspace than
                                     EODABE_NOALLOC_SCRATCH_BYTES */
#define EODABE_ESYNC         -8   /* a barrier between the workgroups of one launch did not see all of
                                     them within ~1 s (another process held the device's CUs); the
                                     outputs of the call are void, the context stays usable */
#define EODABE_WTOL_FLOOR     1   /* warning: tol is below the data-type floor 8 u sqrt(n);
                                     rank decisions there are dominated by rounding */

/* ---- element types ---------------------------------------------------- */
#define EODABE_F32  0
#define EODABE_F64  1

/* ---- sketch precision (steps that read A inside the basis loop) -------
 * The low-precision form (not part of the paper) is defined as: blocks 1
 * and 2 of Alg. 1 sketch A in FP32 (block 1 records max|A| for the FP16
 * scale, block 2 also writes the FP16/BF16 copy A_lp); blocks 3, 4, ...
 * sketch A_lp with FP16/BF16 MFMA operands and FP32 accumulation.  The
 * Grams, Cholesky factors and the stopping test stay FP64.  When a block
 * read A_lp, Alg. 2 runs one subspace iteration more than opts.power_iters
 * (Q~ = orth(A^T Q), Q = orth(A Q~)), and in each iteration the projection
 * A^T Q takes A_lp and Q rounded to the same format on MFMA (FP32
 * accumulation) while A Q~ and the final projection C = Q^T A run in FP32:
 * the FP32 re-orthogonalisation and projection win back the accuracy the
 * rounded copy costs.  Below tol = 2 u_lp the form is not used (status
 * bit 3). */
#define EODABE_SKETCH_NATIVE 0    /* same type as A */
#define EODABE_SKETCH_F16    1    /* FP16 operands on MFMA, FP32 accumulation (A must be F32) */
#define EODABE_SKETCH_BF16   2    /* BF16 operands on MFMA, FP32 accumulation (A must be F32) */

typedef struct eodabe_opts {
  int      block;        /* b: columns per basis block (the paper's k), 1..128; default 32   */
  int      power_iters;  /* q: subspace iterations of Alg. 2, 0..16; default 0               */
  uint64_t seed;         /* Philox4x32-10 key; column c of Omega is a pure function of (seed, c) */
  int      a_dtype;      /* EODABE_F32 or EODABE_F64                                         */
  int      sketch_dtype; /* EODABE_SKETCH_*                                                   */
  int      blocks_per_sync; /* basis blocks enqueued between host checks of the stop flag;
                              0 = automatic                                                   */
  void*    stream;       /* hipStream_t                                                       */
} eodabe_opts;

typedef struct eodabe_info {
  int64_t rank;          /* r: columns accepted by Alg. 1                                     */
  int     blocks;        /* basis blocks executed (J)                                         */
  int     status_flags;  /* bit 0: tol below floor (WTOL_FLOOR); bit 1: A was transposed (m<n);
                            bit 2: a Cholesky pivot was floored in the final QRs;
                            bit 3: a low-precision sketch was requested with tol below 2 u_lp
                            (u_lp = 2^-11 FP16, 2^-8 BF16), where its rounding noise would mask
                            the stop test; every block sketched in FP32 (the plain path);
                            bit 4: a block read the low-precision copy, and one more subspace
                            iteration (A^T Q from the copy) refined the basis before the FP32
                            projection                                                         */
  double  norm_a;        /* ||A||_F (FP64 accumulation)                                       */
  double  eps;           /* tol * ||A||_F, the absolute stopping threshold                    */
  double  relres_est;    /* |T(l,l)| / ||A||_F for the column l whose test stopped the loop:
                            a one-sample estimate of ||A - Q Q^T A||_F / ||A||_F before the
                            basis grew past l (its square has that expectation, Sec. 3.1 and
                            the Gaussian-moment lemma of Sec. 3.3); 0 when the loop ran to the
                            last column or ||A||_F = 0                                         */
} eodabe_info;

/* Fill *o with defaults (block 32, q 0, seed 0, F32, native sketch, stream 0). */
void eodabe_default_opts(eodabe_opts* o);

/* Create a context bound to the current HIP device.  *out receives the
 * handle.  Errors: EINVAL (NULL out/opts or option out of range), ENODEVICE. */
int eodabe_create(eodabe_ctx** out, const eodabe_opts* opts);

/* Create a host-only context: options are validated and workspace sizes
 * can be queried without a device (e.g. on a build host); every call that
 * would touch the GPU returns EODABE_ENODEVICE.  Errors: EINVAL. */
int eodabe_create_host(eodabe_ctx** out, const eodabe_opts* opts);

/* Release the context (host memory only). NULL is ignored. */
void eodabe_destroy(eodabe_ctx* ctx);

/* Bytes of device workspace eodabe_factor needs for an m x n problem whose
 * outputs have r_cap columns (r_cap <= min(m, n); 0 = min(m, n)).
 * Returns 0 for invalid sizes. */
size_t eodabe_workspace_size(const eodabe_ctx* ctx, int64_t m, int64_t n, int64_t r_cap);

/* Factor A (Alg. 2 around Alg. 1).
 *   A      m x n, row-major, leading dimension lda >= n, type opts.a_dtype.
 *   tol    relative tolerance: the basis loop stops at the first column l
 *          with |T(l,l)| <= eps = tol * ||A||_F (Alg. 1 stopping test,
 *          Remark rem3.6).  tol > 0 and finite.
 *   ws     device workspace of ws_bytes >= eodabe_workspace_size(m, n, r_cap).
 *   Ut     output, r_cap x m row-major: row a holds column a of U_hat.
 *   core   output, r_cap x r_cap row-major: D_hat (upper triangular, diag >= 0)
 *          in its leading r x r block.
 *   Vt     output, r_cap x n row-major: row a holds column a of V_hat.
 *   info   host pointer; rank, blocks, ||A||_F, eps.
 * Rows r..r_cap-1 of the outputs are left unspecified.  For m < n the
 * factorization of A^T is computed and transposed back (the core is
 * re-triangularised by one more QR).  Errors: EINVAL, EWORKSPACE,
 * ECAPACITY (rank > r_cap; info->rank holds the rank found so far),
 * ENONFINITE, EHIP.  Warning: WTOL_FLOOR. */
int eodabe_factor(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda,
                  double tol, void* ws, size_t ws_bytes,
                  void* Ut, void* core, void* Vt, int64_t r_cap, eodabe_info* info);

/* ---- factorization without device allocation ---------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * factorization as eodabe_factor, with the workspace taken from a static
 * device array of EODABE_NOALLOC_SCRATCH_BYTES inside the library (one copy
 * per GPU, held until the process ends; its address is looked up once per
 * device by eodabe_create).  The call allocates nothing and calls no
 * hipMalloc/hipFree; per-kernel timing (eodabe_profile) is suspended for it.
 * The caller still owns A and the outputs, laid out as for eodabe_factor.
 * Every call on a GPU shares that GPU's scratch, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one
 * GPU, from any context or stream, race and must be serialised by the
 * caller.  Errors: those of eodabe_factor, and ESCRATCH when
 * eodabe_workspace_size(m, n, r_cap) exceeds the scratch (e.g. 4096 x 4096
 * with r_cap = 0 needs 3.3 GiB; with r_cap = 64, 2048 x 2048 FP32 needs
 * 46 MiB and fits). */
#define EODABE_NOALLOC_SCRATCH_BYTES (64ull << 20)
int eodabe_factor_noalloc(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda,
                          double tol, void* Ut, void* core, void* Vt, int64_t r_cap, eodabe_info* info);

/* ---- complex input (the paper's setting, A in C^{m x n}) ----------------
 * A ~= U_hat D_hat V_hat^H with U_hat, V_hat column-orthonormal (complex),
 * D_hat upper triangular with a real non-negative diagonal, the rank found
 * by Alg. 1 with a complex standard Gaussian test matrix (column c =
 * (g_2c + i g_2c+1) / sqrt(2), g_j the FP64 Box-Muller column j of the
 * real test matrix, each part rounded to FP32) and the stopping test
 * |T(l,l)| <= tol ||A||_F.  A is interleaved (real, imaginary) pairs,
 * row-major m x n with row stride lda >= n complex elements: complex64 for an
 * F32 context, complex128 for F64.  Outputs, interleaved complex of the
 * same type: Ut (r_cap x m, row a = column a of U_hat), core (r_cap x r_cap,
 * D_hat), Vt (r_cap x n, row a = conjugate of column a of V_hat, so A ~=
 * U_hat core Vt).  opts.block counts complex columns per block (up to 64).
 * The work runs on the realification [[Re A, -Im A], [Im A, Re A]] with
 * the test columns in pairs (omega, i omega) and the stopping test on the
 * leading column of each pair: real Gram-Schmidt over pair-ordered realified
 * columns is complex Gram-Schmidt, so every factor is the realification of
 * the complex one; the workspace holds the 2m x 2n realification.  Requires
 * the native sketch (EINVAL otherwise).  Errors: those of eodabe_factor;
 * info->rank, eps and relres_est refer to A itself. */
size_t eodabe_complex_workspace_size(eodabe_ctx* ctx, int64_t m, int64_t n, int64_t r_cap);
int eodabe_factor_complex(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, double tol,
                          void* ws, size_t ws_bytes, void* Ut, void* core, void* Vt, int64_t r_cap,
                          eodabe_info* info);

/* Human-readable text for a status code (static storage). */
const char* eodabe_strerror(int status);

/* Last hipError_t seen by the context (0 if none). */
int eodabe_last_hip_error(const eodabe_ctx* ctx);

/* ---- live kernel timing ------------------------------------------------ */
#define EODABE_PROF_SKETCH  0   /* a2: Y = A Omega_j, one launch per executed block */
#define EODABE_PROF_PROJECT 1   /* a9: C = Q^T A, one launch per factorization      */
#define EODABE_PROF_TILES   2   /* eodabe_factor_batched: one persistent launch per call
                                   (timed with its descriptor and result copies)   */
#define EODABE_PROF_KINDS   3

/* Turn HIP-event timing of the dominant kernels on (enable != 0) or off,
 * and reset the accumulated totals.  The events are attached to the timed
 * kernel's own dispatch (start and end of its execution on the context's
 * stream); launches of speculative blocks or gated closing steps that
 * returned early are not counted. */
int eodabe_profile(eodabe_ctx* ctx, int enable);

/* Accumulated timing of one kernel kind since the last eodabe_profile():
 * total milliseconds, number of launches, and algorithmic bytes moved
 * (sketch: A + Omega_j + Y_j; projection: A + Q + C, in the data type;
 * tiles: per tile 4 h w (J + 1) for the J sketch passes and C^T = A^T Q,
 * plus 4 r (h + w + r) for U, core and V^T). */
int eodabe_profile_read(const eodabe_ctx* ctx, int kind, double* total_ms, int64_t* launches,
                        double* bytes);

/* ---- building blocks, exposed for kernel-level parity tests ----------- */

/* Raw Philox4x32-10 words: for i < count, counter (ctr0 + i, ctr1, ctr2, 0)
 * and key (seed lo, seed hi) -> out[4*i .. 4*i+3] (device, uint32).
 * (Salmon et al., SC'11.) */
int eodabe_philox(eodabe_ctx* ctx, uint64_t seed, uint32_t ctr0, uint32_t ctr1, uint32_t ctr2,
                  int64_t count, uint32_t* out);

/* Columns col0 .. col0+ncols-1 of the n x n Gaussian test matrix of Alg. 1,
 * written transposed: out[j*ldo + i] = Omega(i, col0 + j) for i < n, 0 for
 * n <= i < ldo (ldo >= n).  Entry (i, c) comes from Philox counter
 * (i/4, c, 0, 0) and Box-Muller in FP64, rounded to FP32 (dtype F32) or
 * kept as that FP32 value (dtype F64). */
int eodabe_omega(eodabe_ctx* ctx, int dtype, int64_t n, int64_t col0, int64_t ncols,
                 int64_t ldo, void* out);

/* Y = A * Omega(:, col0 : col0+ncols-1), the sketch of Alg. 1 (Y_j before
 * projection).  A as in eodabe_factor; Y column-major m x ncols (ldy >= m).
 * ncols <= 128.  ws >= eodabe_sketch_workspace_size(m, n, ncols). */
size_t eodabe_sketch_workspace_size(const eodabe_ctx* ctx, int64_t m, int64_t n, int64_t ncols);
int eodabe_sketch(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda,
                  int64_t col0, int64_t ncols, void* Y, int64_t ldy, void* ws, size_t ws_bytes);

/* Alg. 1 only: the basis Q (column-major m x r_cap, ldq = m) and the
 * examined |T(l,l)| values (host array diagT of capacity diag_cap; the
 * count written is min(info->rank + 1, n)).  Same workspace as eodabe_factor. */
int eodabe_basis(eodabe_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda,
                 double tol, void* ws, size_t ws_bytes, void* Q, int64_t r_cap,
                 double* diagT, int64_t diag_cap, eodabe_info* info);

/* ---- many small matrices (tiles) in one launch -------------------------
 * Each tile A_t (m[t] x n[t] FP32, row-major, lda[t] >= n[t], device
 * pointer A[t]; 1 <= m[t], n[t] <= 1024) is factored exactly as
 * eodabe_factor would with q = 0, the context's seed and a block width per
 * tile-size bucket (opts.block clamped to 64, or the width chosen by
 * eodabe_tune_batched).  The tiles run in one persistent launch (one
 * workgroup per tile at a time, largest tiles first), replayed from a
 * hipGraph when the same workspace, pool, tile count, tol and seed come
 * back.  Outputs go to the device pool out_pool (FP32, pool_len elements)
 * at element offset out_offsets[t]: Ut (r_caps[t] x m[t] row-major), then core
 * (r_caps[t] x r_caps[t]), then Vt (r_caps[t] x n[t]), laid out as for
 * eodabe_factor; r_caps[t] <= min(m[t], n[t]), 0 = min(m[t], n[t]); each
 * tile's r_cap * (m + r_cap + n) elements must lie inside the pool (tiles
 * must not overlap each other or the inputs: not checked).
 * Host outputs: ranks[t], status[t] (0 ok, 2 non-finite, 3 rank > r_cap)
 * and, when non-NULL, blocks_used[t] (the block width used).  A tile whose
 * rank exceeds 64 is finished by the single-matrix path within the same
 * call.  All arrays except A's targets and out_pool are host arrays.
 * Errors: EINVAL (sizes, tol, dtype not F32, NULL arrays), EWORKSPACE,
 * EHIP; the call returns after the batch has completed. */
size_t eodabe_batched_workspace_size(eodabe_ctx* ctx, int ntiles);
int eodabe_factor_batched(eodabe_ctx* ctx, int ntiles, const void* const* A, const int64_t* m,
                          const int64_t* n, const int64_t* lda, double tol, void* ws, size_t ws_bytes,
                          void* out_pool, int64_t pool_len, const int64_t* out_offsets,
                          const int64_t* r_caps, int64_t* ranks, int32_t* status, int32_t* blocks_used);

/* Autotuner of the batched launch: for each tile-size bucket present
 * (max side <= 128, 256, 512, 1024) it times eodabe_factor_batched on the
 * given tiles with block widths 16, 32 and 64 and keeps the fastest in the
 * context (chosen[4] receives the widths, 0 for absent buckets).  Same
 * arguments and errors as eodabe_factor_batched. */
int eodabe_tune_batched(eodabe_ctx* ctx, int ntiles, const void* const* A, const int64_t* m,
                        const int64_t* n, const int64_t* lda, double tol, void* ws, size_t ws_bytes,
                        void* out_pool, int64_t pool_len, const int64_t* out_offsets, const int64_t* r_caps,
                        int32_t* chosen);

/* ---- learned warm start of the basis size ------------------------------
 * A GELU MLP 67 -> 256 -> 256 -> 256 -> 2 (FP32, EODABE_MLP_NPARAM
 * parameters, flat: W1 256x67 row-major, b1, W2 256x256, b2, W3, b3,
 * W4 2x256, b4) predicts log(1 + rank) (head 0) and its 0.9-quantile
 * (head 1) from the first 64 values d_c = |T(c,c)| of the stopping test of
 * Alg. 1 (log10(d_c / d_0) clamped at -16, over 16), log2 m / 16,
 * log2 n / 16 and log10(eps / d_0) / 16 (clamped to [-1, 1]), eps =
 * tol ||A||_F the threshold of the test.  The warm start sizes the basis loop from
 * head 1: d0 = b ceil((rhat (1 + margin) + 1) / b), rhat = exp(y1) - 1.
 * The predictor is not part of the paper; the loop of Alg. 1 stays the
 * judge: blocks past d0 run as usual if the test has not fired, and the
 * rank is the one of the plain loop.  All pointers below are device
 * pointers unless marked host. */
#define EODABE_MLP_NIN 67

int64_t eodabe_mlp_param_count(void);
/* Workspace (bytes) of a forward or gradient call on a batch of B samples. */
size_t eodabe_mlp_workspace_size(int batch);
/* Y (batch x 2, row-major) = network(X) for X batch x 67 (row-major).
 * Errors: EINVAL, EWORKSPACE, ENODEVICE, EHIP.  Asynchronous on the
 * context's stream. */
int eodabe_mlp_forward(eodabe_ctx* ctx, const float* params, const float* X, int batch, float* Y,
                       void* ws, size_t ws_bytes);
/* Gradient of the loss (1/B) sum_b [(y_b0 - t_b)^2 + rho_0.9(t_b - y_b1)]
 * (rho_tau(u) = max(tau u, (tau - 1) u), t_b = log(1 + rank_b), T device,
 * batch entries) with respect to the flat parameters, written to grads;
 * *loss (host, optional) receives the loss (the call then synchronises). */
int eodabe_mlp_grad(eodabe_ctx* ctx, const float* params, const float* X, const float* T, int batch,
                    float* grads, void* ws, size_t ws_bytes, double* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * counted from 1) on params with moments m, v (all EODABE_MLP_NPARAM). */
int eodabe_mlp_adam(eodabe_ctx* ctx, float* params, const float* grads, float* m, float* v, float lr,
                    int step);
/* The 67 network inputs (host out) from the stopping-test values d_0..d_63
 * (host, as returned in the diag output of eodabe_basis) of an m x n matrix
 * (m >= n) with threshold eps = tol ||A||_F (eodabe_info.eps); the same
 * function the device inference uses. */
int eodabe_mlp_features(const double* diag, int64_t m, int64_t n, double eps, float* out67);
/* Attach (params non-NULL) or detach (NULL) the predictor.  The parameters
 * must stay valid while the context factors matrices.  Workspace sizes
 * depend on it: size workspaces after attaching.  margin in [0, 10].
 * Used for FP32/FP64 data with the native sketch, block <= 64 and more than
 * 64 columns (after orientation); otherwise factorization is unchanged. */
int eodabe_set_predictor(eodabe_ctx* ctx, const float* params, double margin);
/* The last factorization's prediction (host outputs, each optional): width
 * d0, both heads, and used = 0 (no prediction: the probe of the first 64
 * columns stopped, or no predictor), 1 (the stop fell within d0), 2 (the
 * loop went on past d0). */
int eodabe_last_prediction(const eodabe_ctx* ctx, int64_t* d0, double* log_rank, double* log_rank_q,
                           int* used);

/* ---- application: colour-image compression ------------------------------
 * The introduction's storage criterion and the quality criteria of section
 * 4.1.  Each channel of a planar image img (channels x h x w FP32, device,
 * channel c at img + c h w, values nominally in [0, 255]) is factored by
 * EOD-ABE exactly as eodabe_factor would (one call per channel: the
 * context's block width, power iterations and seed), reconstructed as
 * U_hat D_hat V_hat^T into recon (device, same
 * layout), and compared with the original:
 *   PSNR   = 10 log10(255^2 N / ||A_hat - A||_F^2), N = channels h w values
 *            (+inf when the reconstruction is exact);
 *   SSIM   = (2 mu_x mu_y + c1)(2 s_xy + c2) / ((mu_x^2 + mu_y^2 + c1)(s_x^2 + s_y^2 + c2))
 *            over the vectorised images (one global window, as section 4.1
 *            defines it), c1 = (0.01 255)^2, c2 = (0.03 255)^2, (co)variances
 *            with 1 / (N - 1);
 *   RelErr = ||A - A_hat||_F / ||A||_F;
 * all accumulated in FP64 in a fixed order (deterministic).  Storage: a
 * channel's factors keep (h + w) r + r (r + 1) / 2 entries against h w, and
 * keeping them pays while r < sqrt(h^2 + w^2 + 4hw + h + w + 1/4) - (h + w + 1/2)
 * (rank_bound).  factors: device FP32 pool of channels * r_cap (h + r_cap + w)
 * elements, r_cap = min(h, w); channel c's Ut (r_cap x h), core (r_cap x
 * r_cap) and Vt (r_cap x w) start at c r_cap (h + r_cap + w), laid out as for
 * eodabe_factor.  Requires an F32 context; 1 <= channels <= 4.  Errors:
 * EINVAL, EWORKSPACE, ECAPACITY, ENONFINITE, EHIP.  Returns after the
 * stream has synchronised. */
#define EODABE_IMAGE_MAX_CHANNELS 4
typedef struct eodabe_image_info {
  int64_t rank[EODABE_IMAGE_MAX_CHANNELS];   /* adaptive rank of each channel              */
  int     channels;
  double  relerr, psnr, ssim;                /* criteria over the whole image              */
  double  stored;                            /* entries of all factors                     */
  double  full;                              /* channels h w                               */
  double  reduction;                         /* 1 - stored / full                          */
  double  rank_bound;                        /* factors smaller than a channel below this  */
} eodabe_image_info;
size_t eodabe_image_workspace_size(eodabe_ctx* ctx, int channels, int64_t h, int64_t w);
int eodabe_compress_image(eodabe_ctx* ctx, const float* img, int channels, int64_t h, int64_t w, double tol,
                          void* ws, size_t ws_bytes, float* factors, int64_t factors_len, float* recon,
                          eodabe_image_info* info);

/* ---- application: hyperspectral dimensionality reduction (section 4.2) ---
 * Features of the m pixels of a factored pixels x bands matrix: the rows of
 * U_hat D_hat (F, m x r FP32 row-major, leading dimension ldf >= r, device),
 * i.e. each pixel's spectrum in the r-dimensional basis, from the Ut
 * (r_cap x m) and core (r_cap x r_cap) outputs of eodabe_factor.  Errors:
 * EINVAL, ENODEVICE, EHIP; asynchronous on the context's stream. */
int eodabe_features(eodabe_ctx* ctx, const float* Ut, const float* core, int64_t m, int64_t r, int64_t r_cap,
                    float* F, int64_t ldf);

/* KNN classification with cross-validation (section 4.2): every point i of
 * F (m x d FP32, row-major ldf, device; d <= 32) is classified by its k
 * nearest points (k <= 16) among those whose fold (device int32, m) differs
 * from fold[i]; so with folds 0..9 this is ten-fold cross-validation, each
 * point tested once.  Squared Euclidean distances are summed feature by
 * feature in FP64 with a separate multiply and add per term; the nearest are
 * the smallest (distance, index) pairs; the vote goes to the most frequent
 * label (device int32 in [0, nclass), nclass <= 64), ties to the smallest.
 * pred (device, m) receives the classes; confusion (host, optional, nclass x
 * nclass row-major) receives n[i][j] = points of class j classified as i and
 * oa (host, optional) the overall accuracy sum_i n_ii / sum_ij n_ij.  The
 * workspace holds the device counters (eodabe_knn_workspace_size bytes).
 * Errors: EINVAL, EWORKSPACE, ENODEVICE, EHIP.  Returns after the stream has
 * synchronised. */
size_t eodabe_knn_workspace_size(int nclass);
int eodabe_knn_cv(eodabe_ctx* ctx, const float* F, int64_t m, int d, int64_t ldf, const int32_t* labels,
                  const int32_t* fold, int k, int nclass, int32_t* pred, void* ws, size_t ws_bytes,
                  int64_t* confusion, double* oa);

#ifdef __cplusplus
}
#endif
#endif /* EODABE_H */
