/*
 * hyres.h -- C ABI of the MI355X (gfx950) HyRes denoising library.
 *
 * HyRes is the low-rank, wavelet-based, parameter-free Gaussian denoiser of
 * hyperspectral cubes that the HyDe paper moves onto GPUs (Section 2.1, the
 * list of conventional methods; Table 1 and Table 2 report its speed and
 * energy).  The path implemented here is:
 *
 *   per-band noise by multiple regression -> whitening -> band Gram Y^T Y and
 *   its FP64 eigendecomposition (rank-r spectral subspace) -> projection ->
 *   L-level periodised 2-D Daubechies-4 transform of every component image ->
 *   per-component soft threshold minimising SURE -> inverse transform ->
 *   back-projection.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller, unless a
 *    comment says "host".  Compute calls never allocate device memory; all
 *    scratch comes from the caller's workspace, whose size the matching
 *    *_workspace_size call returns.  Workspaces must be 256-byte aligned.
 *  - Every compute call is stream-ordered on the caller's hipStream_t and
 *    never synchronises the host, so a sequence of calls may be captured in
 *    a HIP graph.
 *  - The return value is a synchronous status from host-side validation or
 *    from the kernel launches.  Conditions found on the device are OR-ed into
 *    the optional device word `status` (HYRES_DEV_* bits); read it after your
 *    own synchronisation.
 *  - Cube layout: Y is H x W x p, band-fastest.  `pitch` is the number of
 *    elements between the band vectors of two neighbouring pixels (>= p) and
 *    `row_pitch` the number between two image rows (>= W * pitch), so a tile
 *    of a larger cube is addressed in place.
 *  - Element type of cubes, component images and coefficients: HYRES_F32 or
 *    HYRES_F64.  Noise levels, eigenvectors, eigenvalues, thresholds and SURE
 *    values are always double.
 *  - V is p x r, column-major (column i is eigenvector i).
 *  - Wavelet coefficients of one image of size H x W with L levels are stored
 *    flat: [LH_1 HL_1 HH_1 LH_2 HL_2 HH_2 ... LH_L HL_L HH_L LL_L], each block
 *    row-major of size h_l x w_l with h_l = ceil(h_{l-1}/2), w_l likewise;
 *    the first letter names the filter along y, the second along x.  The
 *    number of coefficients is hyres_coeff_count(H, W, L).
 *  - No C++ exception crosses this interface.
 */
#ifndef HYRES_H
#define HYRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hyres_stream_t;   /* same type as hipStream_t */

typedef enum {
    HYRES_OK = 0,
    HYRES_E_NULL = 1,         /* a required pointer is NULL */
    HYRES_E_SHAPE = 2,        /* r < 1, r >= p (r > p where allowed), p < 2, p > 224,
                                 r > 16, a level length < 4, pitch < p, ... */
    HYRES_E_DTYPE = 3,        /* unknown element type or precision */
    HYRES_E_WORKSPACE = 4,    /* workspace NULL, too small or misaligned */
    HYRES_E_HIP = 5,          /* a HIP runtime call or kernel launch failed */
    HYRES_E_UNSUPPORTED = 6   /* valid request this build does not handle */
} hyres_status;

typedef enum { HYRES_F32 = 0, HYRES_F64 = 1 } hyres_dtype;

typedef enum {
    HYRES_PREC_NATIVE = 0,    /* every large product in the element type (FP32 or FP64) */
    HYRES_PREC_MIXED = 1      /* FP32 cubes only: band Gram from split-BF16 MFMA products
                                 (hi/lo operands, FP32 accumulation, FP64 across chunks);
                                 FP64 noise regression and eigensolve; FP32 MFMA projection
                                 and back-projection; one FP32 Rayleigh-Ritz refinement of
                                 the subspace (r x r FP64 eigensolve of the projected Gram) */
} hyres_precision;

typedef enum {
    HYRES_SCOPE_ALL = 0,      /* one threshold over every coefficient of a component */
    HYRES_SCOPE_DETAIL = 1    /* coarsest approximation LL_L is left untouched */
} hyres_scope;

/* Device status bits (OR-ed into the caller's `status` word). */
#define HYRES_DEV_NOT_PD        1   /* band Gram not positive definite (zero or dependent band) */
#define HYRES_DEV_NONFINITE     2   /* NaN or Inf in the input cube */
#define HYRES_DEV_EIGH_NOCONV   4   /* eigensolver produced a non-finite value */
#define HYRES_DEV_DEGENERATE    8   /* warning: evals[r-1] / evals[r] < 1 + 1e-6 */
#define HYRES_DEV_SURE_INEXACT 16   /* SURE search stopped before isolating the exact minimiser;
                                       the threshold is the best exact candidate seen */

typedef struct hyres_handle hyres_handle;

/* Options of one solve.  rank: r; levels: L (1..8); precision: hyres_precision;
 * scope: hyres_scope; flags: HYRES_FLAG_* bits. */
typedef struct {
    int rank;
    int levels;
    int precision;
    int scope;
    int flags;
} hyres_options;

/* Compute all p eigenvalues of the whitened Gram (otherwise only the top r+1,
 * which the solve needs, are computed and written to hyres_outputs.evals). */
#define HYRES_FLAG_ALL_EVALS 1
/* Data-chosen rank (Section 2.1: HyRes is parameter-free, and HySime, the
 * subspace identification the section names beside it, chooses the subspace
 * from the data).  With either flag, options.rank is the largest rank r_max
 * and the rank k used is chosen on the device from the eigenvalues lambda of
 * the whitened Gram C (n = H W pixels); components k..r_max-1 are zero (their
 * columns of V are zero and they contribute nothing to X), and k is written
 * to hyres_outputs.rank.
 *   HYRES_FLAG_RANK_HYSIME: HySime in the whitened frame, where the noise
 *     correlation is the identity: k = #{i : lambda_i > 2 n}, the directions
 *     whose data power exceeds twice the noise power, clamped to [1, r_max].
 *   HYRES_FLAG_RANK_SURE: the k in [1, r_max] minimising Stein's unbiased
 *     risk estimate of the rank-k truncation of the whitened cube,
 *     sum_{j>k} lambda_j - n p + 2 df(k), df(k) = k (n - p + 1) + k (k - 1)
 *     + 2 sum_{i<=k<j} lambda_i / (lambda_i - lambda_j) (smallest k on ties;
 *     needs every eigenvalue, so it implies HYRES_FLAG_ALL_EVALS).
 * The two flags exclude each other (HYRES_E_UNSUPPORTED), as do they and
 * hyres_denoise_backward. */
#define HYRES_FLAG_RANK_HYSIME 2
#define HYRES_FLAG_RANK_SURE 4

/* Optional device outputs of a solve (any pointer may be NULL). */
typedef struct {
    double* sigma;   /* [p]   noise standard deviation per band */
    double* V;       /* [p*r] top-r eigenvectors of the whitened Gram, column-major, sign rule:
                              the entry of largest magnitude is positive */
    double* evals;   /* [p]   eigenvalues of the whitened Gram, descending: entries 0..r always,
                              all p with HYRES_FLAG_ALL_EVALS */
    double* lambda;  /* [r]   soft thresholds */
    double* sure;    /* [r]   SURE at the thresholds */
    double* gap;     /* [1]   evals[k-1] / evals[k] for the rank k used (Inf when k == p) */
    int*    status;  /* [1]   HYRES_DEV_* bits, OR-ed (the caller zeroes it) */
    int*    rank;    /* [1]   the rank used (options.rank unless a HYRES_FLAG_RANK_* flag chose it) */
    double* eig_check; /* [2] accuracy of the FP64 eigensolve, on the whitened Gram C it decomposed
                              (before the Rayleigh-Ritz refinement of the mixed path), over the k
                              eigenpairs used: [0] ||C V - V Lambda||_F / ||C||_F, [1] max |V^T V - I|;
                              computed only when this pointer is set (a few microseconds) */
} hyres_outputs;

/* ---- handle ------------------------------------------------------------- */

/* Create a handle bound to HIP device `device` (it becomes current during calls).
 * The handle owns a few side streams (default priority) and events: the small
 * solves of cubes in different band-count classes run on them beside the
 * caller's stream, forked from and joined back into it, so every call stays
 * ordered on the caller's stream (and a capture of it records the branches).
 * Use a handle from one host thread at a time.
 * Fails with HYRES_E_HIP when no such device exists or the streams cannot be
 * created. */
hyres_status hyres_create(hyres_handle** handle, int device);
void hyres_destroy(hyres_handle* handle);
const char* hyres_status_string(int status);
/* Number of wavelet coefficients of one H x W image with L levels (0 on bad shape). */
int64_t hyres_coeff_count(int H, int W, int L);

/* ---- noise estimation (regression of each band on the others) ----------- */

/* Defined by: Section 2.1 -- HyRes removes Gaussian noise and is parameter-free,
 * so the per-band noise level is estimated from the cube; the estimator is the
 * multiple-regression one of HySime, which the same section names as part of
 * the toolbox. */
/* sigma_i^2 = RSS_i / n where RSS_i is the residual of the least-squares
 * regression, without intercept, of band i on the other p-1 bands, n = H*W.
 * Computed from the FP64 band Gram G = Y^T Y as 1 / (n [G^-1]_ii).
 * sigma_out [p] (device double); gram_out [p*p] (device double, may be NULL). */
hyres_status hyres_estimate_noise_workspace_size(int H, int W, int p, int dtype, size_t* bytes);
hyres_status hyres_estimate_noise(hyres_handle* h, const void* Y, int H, int W, int p,
                                  int64_t pitch, int64_t row_pitch, int dtype,
                                  double* sigma_out, double* gram_out, int* status,
                                  void* workspace, size_t workspace_bytes, hyres_stream_t stream);

/* ---- spectral subspace -------------------------------------------------- */

/* Defined by: Section 2.1 -- HyRes is a low-rank method: the cube is modelled
 * in the span of the leading eigenvectors of the whitened band Gram. */
/* Eigendecomposition of the whitened Gram C = D^-1 Y^T Y D^-1, D = diag(sigma)
 * (sigma == NULL means D = I).  V_out receives the top-r eigenvectors
 * (column-major p x r, sign rule as in hyres_outputs), evals_out all p
 * eigenvalues in descending order.  Solved in FP64 on the device. */
hyres_status hyres_subspace_workspace_size(int H, int W, int p, int r, int dtype, size_t* bytes);
hyres_status hyres_subspace(hyres_handle* h, const void* Y, int H, int W, int p,
                            int64_t pitch, int64_t row_pitch, int dtype,
                            const double* sigma, int r, double* V_out, double* evals_out,
                            int* status, void* workspace, size_t workspace_bytes,
                            hyres_stream_t stream);

/* ---- wavelet transforms ------------------------------------------------- */

/* Defined by: Section 2.1 -- HyRes is wavelet-based: every component image is
 * represented by its 2-D orthogonal wavelet coefficients. */
/* Forward L-level periodised 2-D db2 transform of `batch` images x[batch][H][W]
 * (contiguous) into coeffs[batch][Nc], Nc = hyres_coeff_count(H, W, L).  An
 * odd length is extended by repeating its last sample before each step. */
hyres_status hyres_dwt2_workspace_size(int batch, int H, int W, int L, int dtype, size_t* bytes);
hyres_status hyres_dwt2(hyres_handle* h, const void* x, int batch, int H, int W, int L,
                        int dtype, void* coeffs, void* workspace, size_t workspace_bytes,
                        hyres_stream_t stream);
/* Inverse transform.  When lambda (device double [batch]) is not NULL each
 * coefficient is first soft-thresholded, sign(b) max(|b| - lambda_i, 0)
 * (every coefficient for scope ALL, details only for scope DETAIL). */
hyres_status hyres_idwt2(hyres_handle* h, const void* coeffs, int batch, int H, int W, int L,
                         int dtype, const double* lambda, int scope, void* x_out,
                         void* workspace, size_t workspace_bytes, hyres_stream_t stream);

/* ---- SURE threshold ----------------------------------------------------- */

/* Defined by: Section 2.1 -- HyRes is parameter-free: the per-component
 * threshold is not a user parameter but the minimiser of Stein's unbiased
 * risk estimate. */
/* For each of `batch` coefficient vectors of length Nc (stride `stride`
 * elements) the exact minimiser, over t in {0} U {|b_k|}, of Stein's unbiased
 * risk estimate of soft thresholding at unit noise,
 *   SURE(t) = Nc - 2 #{k : |b_k| <= t} + sum_k min(b_k^2, t^2),
 * smallest t on ties.  lambda_out, sure_min_out: device double [batch]. */
hyres_status hyres_sure_workspace_size(int batch, int64_t Nc, int dtype, size_t* bytes);
hyres_status hyres_sure_threshold(hyres_handle* h, const void* coeffs, int batch, int64_t Nc,
                                  int64_t stride, int dtype, double* lambda_out,
                                  double* sure_min_out, int* status, void* workspace,
                                  size_t workspace_bytes, hyres_stream_t stream);

/* ---- the whole denoiser ------------------------------------------------- */

/* Defined by: Section 2.1 (the HyRes method) and Section 3 (a cube resident on
 * the GPU is processed there; Table 1 times this solve on the Houston 2013
 * cube, Table 2 gives its energy). */
/* X = HyRes(Y).  sigma_in (device [p]) and lambda_in (device [r]) override the
 * estimates when not NULL.  X has its own pitch and row pitch (same rules as
 * Y) and must not overlap Y. */
hyres_status hyres_denoise_workspace_size(int H, int W, int p, const hyres_options* opt,
                                          int dtype, size_t* bytes);
hyres_status hyres_denoise(hyres_handle* h, const void* Y, int H, int W, int p,
                           int64_t pitch, int64_t row_pitch, int dtype,
                           const hyres_options* opt, const double* sigma_in,
                           const double* lambda_in, void* X, int64_t x_pitch,
                           int64_t x_row_pitch, const hyres_outputs* out,
                           void* workspace, size_t workspace_bytes, hyres_stream_t stream);

/* ---- the whole denoiser without a workspace ------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 * hyres_denoise with the same arguments minus the workspace: the scratch is a
 * fixed array of HYRES_NOALLOC_SCRATCH_BYTES in the library's code object, one
 * per device, resolved when a handle is created on that device and held until
 * the process ends.  The call allocates nothing (no hipMalloc, no library
 * allocation).  Solves whose hyres_denoise_workspace_size exceeds the array
 * return HYRES_E_WORKSPACE (the 349 x 1905 x 144 cube at rank 8 needs 61 MiB
 * in FP32 and 71 MiB in mixed precision).  Every call on a device shares that
 * device's array and leaves its last contents there (the solve rewrites
 * everything it reads before reading it): calls that overlap on one device,
 * on different streams or from different handles, race and must be ordered
 * by the caller.  X, sigma, V, evals, lambda and gap equal hyres_denoise's bit
 * for bit; the SURE minima agree to rounding (their FP64 sums are formed with
 * device atomics in either call). */
#define HYRES_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
hyres_status hyres_denoise_noalloc(hyres_handle* h, const void* Y, int H, int W, int p,
                                   int64_t pitch, int64_t row_pitch, int dtype,
                                   const hyres_options* opt, const double* sigma_in,
                                   const double* lambda_in, void* X, int64_t x_pitch,
                                   int64_t x_row_pitch, const hyres_outputs* out,
                                   hyres_stream_t stream);

/* ---- HyMiNoR: HyRes, then the sparse-noise stage ------------------------- */

/* Defined by: Section 2.1 -- HyMiNoR is built on HyRes: after HyRes has removed
 * the Gaussian noise, the sparse noise that remains is removed by an l1-l1
 * problem solved with split Bregman.  The paper states neither the problem nor
 * the iteration; this library takes, per pixel spectrum h (p bands),
 *     x = argmin_x ||h - x||_1 + lam ||D x||_1,   (D x)_i = x_{i+1} - x_i,
 * (l1 data term: a few bands may move far; l1 first-order spectral roughness:
 * spectral edges are kept), by split Bregman with s = h - x and u = D x,
 * penalties mu1 and mu2, every auxiliary and Bregman variable starting at 0:
 *     x  <- (mu1 I + mu2 D^T D)^-1 (mu1 (h - s + b1) + mu2 D^T (u - b2))
 *     s  <- soft(h - x + b1, 1/mu1),   u <- soft(D x + b2, lam/mu2)
 *     b1 <- b1 + h - x - s,            b2 <- b2 + D x - u
 * for `iters` sweeps; the result is the x of the last sweep.  lam is
 * dimensionless (the problem is 1-homogeneous in h); 1/mu1 and lam/mu2 are
 * thresholds in the units of h.  An isolated one-band spike is removed when
 * lam > 1/2. */
typedef struct {
    double lam;      /* >= 0 */
    double mu1;      /* > 0 */
    double mu2;      /* > 0 */
    int    iters;    /* >= 1 */
} hyres_l1l1_options;

/* The sparse-noise stage alone on an H x W x p cube Hc (device, dtype
 * HYRES_F32 or HYRES_F64, pitch / row_pitch as for Y, 1 <= p <= 224; FP64
 * cubes of more than 224 bands are not handled).  Each pixel's spectrum is read
 * whole before its result is written, so X may be Hc itself (same pitches);
 * otherwise X must not overlap Hc.  Needs no workspace.  Computed in the
 * cube's precision (the tridiagonal factors are formed in FP64).
 * HYRES_E_SHAPE for bad sizes, pitches or options (mu1 or mu2 <= 0, lam < 0,
 * iters < 1, non-finite values). */
hyres_status hyres_l1l1_spectral(hyres_handle* h, const void* Hc, int H, int W, int p,
                                 int64_t pitch, int64_t row_pitch, int dtype,
                                 const hyres_l1l1_options* opt, void* X, int64_t x_pitch,
                                 int64_t x_row_pitch, hyres_stream_t stream);

/* HyMiNoR: hyres_denoise (same arguments, options, outputs and workspace:
 * hyres_denoise_workspace_size gives its size), then hyres_l1l1_spectral on
 * its output, in place in X.  The outputs describe the HyRes stage. */
hyres_status hyres_hyminor(hyres_handle* h, const void* Y, int H, int W, int p,
                           int64_t pitch, int64_t row_pitch, int dtype,
                           const hyres_options* opt, const double* sigma_in,
                           const double* lambda_in, const hyres_l1l1_options* l1,
                           void* X, int64_t x_pitch, int64_t x_row_pitch,
                           const hyres_outputs* out, void* workspace, size_t workspace_bytes,
                           hyres_stream_t stream);

/* ---- WSRRR: wavelet-based sparse reduced-rank regression ----------------- */

/* Defined by: Section 2.1 -- WSRRR is a low-rank, wavelet-based method for
 * Gaussian noise that can also extract features; the paper prints nothing
 * more, and this library takes, in the whitened frame of HyRes (Yw = Y / sigma):
 * the model Yw = W F V^T + noise with F the wavelet coefficients of r component
 * images and V^T V = I, fitted by minimising 1/2 ||Yw - W F V^T||^2 +
 * sum_i lambda_i ||f_i||_1; it starts from the HyRes solve (its sigma,
 * subspace, SURE thresholds, which then stay fixed, and coefficients) and
 * alternates `iters` times the Procrustes step V <- polar factor of
 * Yw^T W F with the soft-threshold step F <- soft(W^T Yw V, lambda);
 * X = W F V^T sigma.  iters = 0 is hyres_denoise.  Native precision only
 * (HYRES_PREC_MIXED and the HYRES_FLAG_RANK_* flags: HYRES_E_UNSUPPORTED);
 * other arguments, outputs (V: the final subspace) and the layout rules as for
 * hyres_denoise; the workspace comes from hyres_wsrrr_workspace_size.  A
 * component thresholded to zero leaves the polar factor rank deficient:
 * HYRES_DEV_DEGENERATE in the status word. */
hyres_status hyres_wsrrr_workspace_size(int H, int W, int p, const hyres_options* opt, int dtype,
                                        size_t* bytes);
hyres_status hyres_wsrrr(hyres_handle* h, const void* Y, int H, int W, int p,
                         int64_t pitch, int64_t row_pitch, int dtype, const hyres_options* opt,
                         int iters, const double* sigma_in, const double* lambda_in, void* X,
                         int64_t x_pitch, int64_t x_row_pitch, const hyres_outputs* out,
                         void* workspace, size_t workspace_bytes, hyres_stream_t stream);

/* ---- FORPDN: first-order spectral roughness penalty denoising ------------ */

/* Defined by: Section 2.1 -- FORPDN is a full-rank, wavelet-based method for
 * additive Gaussian noise (first-order spectral roughness penalty); the paper
 * prints nothing more, and this library takes:
 *   sigma: the per-band noise of the HyRes estimator (sigma_in overrides);
 *   the whitened bands Y / sigma are transformed by the same L-level periodised
 *   2-D db2 wavelet as HyRes; the coefficients of one position across the p
 *   bands form a vector, and the vectors fall into L + 1 groups (the three
 *   detail subbands of level l = 1..L, then the coarsest approximation);
 *   every vector c of group j becomes (I + lam_j D^T D)^-1 c, D the
 *   first-order spectral difference (the minimiser of ||c - x||^2 +
 *   lam_j ||D x||^2); lam_j minimises Stein's unbiased risk estimate of that
 *   smoother at unit noise over lam = 10^(t/10), t = -40..40 (the smallest on
 *   ties; lambda_in [L+1] overrides); X is the inverse transform times sigma.
 * Y, X: H x W x p cubes (dtype HYRES_F32 or HYRES_F64, pitches as for Y in
 * hyres_denoise; X must not overlap Y), 2 <= p <= 224, 1 <= levels <= 8 with
 * every level's input at least 4 x 4.  Outputs (device, any may be NULL):
 * sigma_out [p], lambda_out [L+1], sure_out [L+1] (SURE at the chosen lam),
 * status (HYRES_DEV_* bits of the noise estimate, OR-ed; the caller zeroes it).
 * The workspace (hyres_forpdn_workspace_size; sigma_given != 0 when sigma_in
 * will be passed) holds the position-major coefficients (about one cube),
 * two approximation buffers and the per-group Gram partial sums. */
hyres_status hyres_forpdn_workspace_size(int H, int W, int p, int levels, int dtype, int sigma_given,
                                         size_t* bytes);
hyres_status hyres_forpdn(hyres_handle* h, const void* Y, int H, int W, int p,
                          int64_t pitch, int64_t row_pitch, int dtype, int levels,
                          const double* sigma_in, const double* lambda_in, void* X,
                          int64_t x_pitch, int64_t x_row_pitch, double* sigma_out,
                          double* lambda_out, double* sure_out, int* status,
                          void* workspace, size_t workspace_bytes, hyres_stream_t stream);

/* ---- batches of cubes ---------------------------------------------------- */

/* Defined by: Section 3 (device residency) applied to many cubes at once; the
 * paper times one cube per call, the batch is an execution form of the same
 * solve (each cube's result is that of hyres_denoise). */
/* One cube of a batch.  The struct itself is host memory; Y, X, sigma_in,
 * lambda_in and the pointers in `out` are device pointers with the meaning
 * they have in hyres_denoise.  Cubes may differ in H, W, p, rank and levels. */
typedef struct {
    const void* Y; int H, W, p; int64_t pitch, row_pitch;
    void* X; int64_t x_pitch, x_row_pitch;
    int rank, levels;
    const double* sigma_in;    /* [p] or NULL: estimate */
    const double* lambda_in;   /* [rank] or NULL: SURE */
    hyres_outputs out;
} hyres_cube;

/* A planned batch: the solve of `count` independent cubes as one sequence of
 * persistent launches (each kernel class is one launch over a prefix-summed
 * list of work items spanning every cube of the class), with the noise
 * regression and eigensolve of every cube in one launch per band-count class.
 * The cubes run in up to four groups by band-count class, the first on the
 * caller's stream and the others on the handle's side streams (forked from
 * and joined back into it), a group's Gram stage after the previous group's,
 * so that one group's eigensolves overlap the other groups' bandwidth-bound
 * stages.
 * Each cube's results equal those of hyres_denoise on that cube alone.
 * All cubes share dtype and opt's precision, scope and flags (opt's rank and
 * levels are not used: each cube carries its own). */
typedef struct hyres_batch hyres_batch;

/* Workspace of a batch; only the shape fields of `cubes` are read (host array). */
hyres_status hyres_batch_workspace_size(const hyres_cube* cubes, int count, int dtype,
                                        const hyres_options* opt, size_t* bytes);
/* Validates and plans the batch and writes its descriptor and work tables
 * into `workspace` (stream-ordered on `stream`).  The host object keeps the
 * plan; the workspace belongs to the batch until hyres_batch_destroy, and the
 * cubes' device buffers must stay valid as long as the batch is run. */
hyres_status hyres_batch_create(hyres_handle* h, const hyres_cube* cubes, int count, int dtype,
                                const hyres_options* opt, void* workspace, size_t workspace_bytes,
                                hyres_stream_t stream, hyres_batch** batch);
/* Enqueues one solve of every cube on `stream` (no host synchronisation). */
hyres_status hyres_batch_run(hyres_batch* batch, hyres_stream_t stream);
/* Launches the solve as one HIP graph: the first call captures the launch
 * sequence on a private stream and instantiates it (host work only), every
 * call then launches the graph on `stream`.  Run calls on one batch in stream
 * order: the replays share the workspace. */
hyres_status hyres_batch_launch_graph(hyres_batch* batch, hyres_stream_t stream);
void hyres_batch_destroy(hyres_batch* batch);
/* One-shot batched solve: create, run, destroy. */
hyres_status hyres_denoise_batched(hyres_handle* h, const hyres_cube* cubes, int count, int dtype,
                                   const hyres_options* opt, void* workspace, size_t workspace_bytes,
                                   hyres_stream_t stream);

/* ---- sliding-window denoising ------------------------------------------- */

/* Defined by: Section 2.2.2 -- large cubes are denoised in spatial sections by
 * a sliding window, and the sections are blended into one output (the paper
 * uses it for network inference; here every section is a HyRes solve). */
/* Tile starts along an axis of length `size`: 0, tile - overlap, 2 (tile -
 * overlap), ..., the last start clamped to size - tile so that the last tile
 * ends at the border (one tile at 0 when tile >= size).  starts: host array of
 * up to 64 ints, or NULL to query `count` only.  Needs tile >= 4 and
 * 0 <= 2 overlap <= tile; more than 64 tiles is HYRES_E_UNSUPPORTED. */
hyres_status hyres_tile_grid(int size, int tile, int overlap, int* starts, int* count);

/* X = sum_t w_t HyRes(Y_t) / sum_t w_t over the grid of min(tile,H) x
 * min(tile,W) tiles Y_t of Y (starts from hyres_tile_grid on each axis), each
 * denoised independently (own noise estimate, subspace and thresholds, rank
 * and levels from opt).  w_t is separable; along an axis it is 1 except for
 * sin^2(pi/2 (k + 1/2) / overlap) ramps over the first and the last `overlap`
 * samples of the tile, with no ramp on a side that touches the image border.
 * All tiles run as one batch (tiles are addressed in place through pitch and
 * row_pitch, nothing is copied), in four groups of consecutive tiles on
 * streams of their own.  The back-projection applies the blend: FP32 in one
 * pass over X (each pixel sums its covering tiles in raster order and is
 * written once), FP64 in passes of non-overlapping tiles; either way the sums
 * are formed in a fixed order.  lambda_out [ntiles * rank] and sigma_out [ntiles * p] (device
 * double, tile t = row-major index over the grid) may be NULL. */
hyres_status hyres_tiled_workspace_size(int H, int W, int p, int tile, int overlap,
                                        const hyres_options* opt, int dtype, size_t* bytes);
hyres_status hyres_denoise_tiled(hyres_handle* h, const void* Y, int H, int W, int p,
                                 int64_t pitch, int64_t row_pitch, int dtype, int tile, int overlap,
                                 const hyres_options* opt, void* X, int64_t x_pitch,
                                 int64_t x_row_pitch, double* lambda_out, double* sigma_out,
                                 int* status, void* workspace, size_t workspace_bytes,
                                 hyres_stream_t stream);

/* ---- adjoint (reverse-mode derivative) ----------------------------------- */

/* Defined by: Section 2.2 -- a HyRes step is trained inside a network (the
 * MemNet variant with a trainable HyRes step before its layers), which needs
 * the derivative of the solve with respect to its input and thresholds.
 * Forward solves in HYRES_PREC_MIXED are refused (HYRES_E_UNSUPPORTED): their
 * Ritz basis is not an eigenbasis of the Gram the adjoint differentiates. */
/* Vector-Jacobian product of X = HyRes(Y; lambda) with the thresholds held as
 * inputs: given dX (same layout rules as Y) it writes dY = (dX/dY)^T dX
 * (through the noise estimate, the whitening, the eigenvectors, the
 * projections, the transforms and the soft threshold) and dlambda [rank]
 * (device double, may be NULL).  The forward call must have been
 * hyres_denoise with the same Y, shape, opt and dtype, whose outputs
 * sigma, V, evals and lambda were requested (fwd_out, device), and whose
 * workspace has not been used since (it holds the band Gram, the
 * coefficients and the denoised component images that the adjoint reads;
 * the intermediate approximation levels of the transforms are recomputed).
 * The SURE choice of the thresholds is piecewise constant in Y: with
 * thresholds chosen by SURE the derivative is the one at fixed thresholds.
 * The eigen-derivative needs simple top-r eigenvalues (a degenerate gap makes
 * it unbounded).  The small systems are solved in FP64; a singular one sets
 * HYRES_DEV_NOT_PD in `status`. */
hyres_status hyres_denoise_backward_workspace_size(int H, int W, int p, const hyres_options* opt,
                                                   int dtype, size_t* bytes);
hyres_status hyres_denoise_backward(hyres_handle* h, const void* Y, int H, int W, int p,
                                    int64_t pitch, int64_t row_pitch, int dtype,
                                    const hyres_options* opt, const void* fwd_workspace,
                                    size_t fwd_workspace_bytes, const hyres_outputs* fwd_out,
                                    const void* dX, int64_t dx_pitch, int64_t dx_row_pitch,
                                    void* dY, int64_t dy_pitch, int64_t dy_row_pitch,
                                    double* dlambda, int* status, void* workspace,
                                    size_t workspace_bytes, hyres_stream_t stream);

/* Derivative of SURE(t) = Nc - 2 #{|b| <= t} + sum min(b^2, t^2) with respect
 * to t at t = lambda_i, for each of `batch` coefficient vectors (stride
 * `stride`): 2 lambda_i #{k : |b_k| > lambda_i} (the risk is piecewise
 * quadratic in t; at a candidate t = |b_k| this is the right derivative).
 * dsure_out: device double [batch]. */
hyres_status hyres_sure_grad_workspace_size(int batch, int64_t Nc, size_t* bytes);
hyres_status hyres_sure_grad(hyres_handle* h, const void* coeffs, int batch, int64_t Nc, int64_t stride,
                             int dtype, const double* lambda, double* dsure_out, void* workspace,
                             size_t workspace_bytes, hyres_stream_t stream);

/* ---- DWT tile autotuner -------------------------------------------------- */

/* An execution aid with no counterpart in the paper: it changes launch shapes
 * only, never a result. */
/* Chooses, for every (element type, direction, level-width class) that the
 * batch's transforms use, the workgroup tile shape of the transform kernels
 * (64x4, 32x8, 16x16 or 128x2 threads) that runs fastest.  A level of width w
 * belongs to class ceil(log2 w).  Choices found in the JSON file `cache_path`
 * for this device are taken from it; the rest are timed with HIP events on the
 * batch's own data (one solve, then each candidate per level) and written
 * back to the file (NULL: no file).  The choices are kept in the handle and
 * used by every later call on it; the batch is re-planned (its graph, if any,
 * is captured again on its next launch).  Unlike the compute calls this one
 * synchronises the host with `stream`; it must not be captured. */
hyres_status hyres_autotune(hyres_handle* h, hyres_batch* batch, const char* cache_path,
                            hyres_stream_t stream);
/* The tile the handle uses for a level of width `width` (tuned: 1 if it came
 * from the tuner or its cache, 0 for the built-in choice). */
hyres_status hyres_tile_choice(hyres_handle* h, int dtype, int inverse, int width, int* tx, int* ty,
                               int* tuned);

/* ---- host-only checks of a launch program ------------------------------- */

/* What a launch program enqueues (counts over one solve). */
typedef struct {
    int launches;   /* kernel launches */
    int records;    /* event records */
    int waits;      /* stream waits on events */
    int streams;    /* streams used, the caller's included */
    int groups;     /* cube groups */
} hyres_program_stats;

/* Plans the launch program of a batch (only the shape fields, rank, levels and
 * lambda_in of `cubes` are read; no pointer is dereferenced) or of a tile grid
 * and walks it without touching a device, checking its stream order: every
 * wait on an event follows a record of that event in the same program (a wait
 * on an older record would, inside a graph capture, depend on work outside
 * the capture), every side stream first waits on an event of the caller's
 * stream and ends with a record that the caller's stream waits on.  Returns
 * HYRES_E_HIP when the order breaks one of these rules, a planning error as
 * the matching create call would, and fills `stats` (may be NULL).  The
 * executor applies the same record-before-wait rule at run time and refuses
 * (HYRES_E_HIP) to enqueue a program that breaks it. */
hyres_status hyres_batch_check_program(const hyres_cube* cubes, int count, int dtype,
                                       const hyres_options* opt, hyres_program_stats* stats);
hyres_status hyres_tiled_check_program(int H, int W, int p, int tile, int overlap,
                                       const hyres_options* opt, int dtype, hyres_program_stats* stats);

/* ---- stage timing (benchmarks) ------------------------------------------ */

/* Stages of a solve, as bit positions of the mask below. */
#define HYRES_STAGE_GRAM        0   /* band Gram (first pass over Y) */
#define HYRES_STAGE_SMALL       1   /* FP64 noise regression and eigensolve */
#define HYRES_STAGE_PROJECT     2   /* projection (second pass over Y) */
#define HYRES_STAGE_DWT         3   /* forward transforms */
#define HYRES_STAGE_SURE        4   /* SURE threshold search */
#define HYRES_STAGE_IDWT        5   /* soft threshold + inverse transforms */
#define HYRES_STAGE_BACKPROJECT 6   /* back-projection (write of X) */
#define HYRES_NUM_STAGES        7

/* When stage bit s of `mask` is set, every later solve on this handle records
 * a HIP event pair around stage s on the stream that runs it: the caller's,
 * or a cube group's (mask 0: off).  The events are host objects owned by the
 * handle; no device memory is used. */
hyres_status hyres_profile_enable(hyres_handle* h, unsigned mask);
/* Wait for the recorded events, then add the elapsed milliseconds and the
 * number of timed solves of each stage to ms_out[s] and count_out[s] (host
 * arrays of HYRES_NUM_STAGES) and forget them.  Where the cubes of a batch or
 * tile grid run in groups on streams of their own, each group's stage is timed
 * on its stream and the groups' times of one solve add up. */
hyres_status hyres_profile_read(hyres_handle* h, double* ms_out, int* count_out);

#ifdef __cplusplus
}
#endif
#endif /* HYRES_H */
