/*
 * swift.h -- C ABI of libswift: signal-whitened FFT window matching on MI355X.
 *
 * Method: Wetzel et al., "Registering large volume serial-section electron
 * microscopy image sets for neural circuit reconstruction using FFT signal
 * whitening" (arXiv 1612.04787), Section III.  Large sections are matched as
 * tiled local windows; each window pair is correlated in the frequency domain
 * with Fourier amplitudes scaled by a power 0..1 (0 = plain correlation, 1 =
 * phase-only), edges apodized with a cosine taper, and the match is scored as
 * a Z-score (SNR) against the background of the correlation surface.  The
 * reference of a section is the rounded mean of its z-neighbours ("model").
 *
 * Conventions shared by every entry point
 *  - All functions return 0 (SWIFT_OK) or a negative SWIFT_E_* code and never
 *    abort or throw.  swift_last_error() gives a message for the calling thread.
 *  - Validation of host-side arguments is synchronous.  Device work is queued
 *    on the caller's stream; faults in device work surface at the caller's next
 *    synchronisation.  No function synchronises the stream except
 *    swift_create/swift_destroy/swift_autotune.
 *  - The caller owns every buffer.  Pointers documented "device" must be
 *    device memory of the context's GPU; "host" pointers are read during the
 *    call only.  The library keeps no pointer beyond a call.
 *  - Images are row-major [y][x] with a pitch in bytes.  Window pixel (i, j)
 *    (column i, row j) of a window of edge n has window coordinates
 *    u = i - n/2, v = j - n/2 and samples the image at
 *        x = cx + a11*u + a12*v + tx,   y = cy + a21*u + a22*v + ty
 *    with bilinear interpolation and clamp-to-edge reads.
 *  - Correlation sign: if window B equals window A moved by +d, the peak is
 *    at +d.  Shifts are wrapped to [-n/2, n/2).
 */
#ifndef SWIFT_H
#define SWIFT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWIFT_OK             0
#define SWIFT_E_INVAL       -1 /* bad argument (NULL, size, range, ordering)   */
#define SWIFT_E_UNSUPPORTED -2 /* valid request the library does not implement */
#define SWIFT_E_WORKSPACE   -3 /* workspace or saved buffer too small          */
#define SWIFT_E_HIP         -4 /* HIP runtime error (message has its string)   */
#define SWIFT_E_CAPTURE     -5 /* hipGraph capture/instantiate/launch failed    */

#define SWIFT_U8  0 /* uint8 pixels   */
#define SWIFT_F32 1 /* float32 pixels */

/* match status bits */
#define SWIFT_ST_NEAR_TIE   1 /* best and second-best surface values within 2e-4 relative */
#define SWIFT_ST_DEGENERATE 2 /* surface standard deviation 0 (e.g. a constant window)    */
#define SWIFT_ST_CLAMPED    4 /* a window sample fell outside an image (edge clamped)     */

/* Number of supported window edges and their values: n in {64,128,256,512,1024}. */
#define SWIFT_NSIZES 5

typedef struct swift_ctx swift_ctx;

/* An image in device memory (32 bytes).  Width, height >= 2. */
typedef struct {
  const void* data;    /* device pointer to pixel (0, 0)                 */
  int32_t width;
  int32_t height;
  int64_t pitch;       /* bytes between consecutive rows (>= width*elem) */
  int32_t dtype;       /* SWIFT_U8 or SWIFT_F32                          */
  int32_t reserved;    /* must be 0                                      */
} swift_image;

/* A batch of window pairs, structure of arrays in device memory.  Pairs are
 * sorted by window edge ascending; size_count (host) gives how many pairs
 * have each edge 64, 128, 256, 512, 1024, in that order. */
typedef struct {
  int32_t n_pairs;                   /* host: total, = sum(size_count)          */
  int32_t size_count[SWIFT_NSIZES];  /* host                                    */
  const int32_t* img_a;              /* device [P]: index into the image table  */
  const int32_t* img_b;              /* device [P]                              */
  const float* theta_a;              /* device [P][8]: cx,cy,a11,a12,tx,a21,a22,ty */
  const float* theta_b;              /* device [P][8]                           */
} swift_pairs;

/* Matching parameters (host).
 *  p          whitening exponent in [0, 1] (Section III: the 0..1 exponent of
 *             the amplitude power function; 0 = NCC-like, 1 = phase-only).
 *  eps_rel    relative floor of the whitening denominator, >= 0: the cross
 *             power X is scaled by (|X|^2 + eps^2)^(-p/2) with
 *             eps = eps_rel * ||w_A||_2 * ||w_B||_2 (w = tapered windows).
 *  taper_frac fraction of the window edge covered by the raised-cosine taper,
 *             both edges together, in [0, 1] (Section III, apodization).
 *  centroid_r half-width of the sub-pixel centroid box; only 1 is supported.
 *  flags      an OR of
 *             SWIFT_FLAG_CONCURRENT_SIZES: the size groups of a ragged batch
 *               that are too small to fill the GPU (forward row pass below
 *               8192 workgroups, i.e. pairs x n / rows per block) run
 *               concurrently on the context's own streams, forked from and
 *               joined back into the call's stream with events, so the call
 *               stays stream-ordered and capturable; larger groups run on the
 *               call's stream one after another (beside each other they would
 *               only share the CUs);
 *             SWIFT_FLAG_JAC_TRANSLATION: swift_centroid_jacobian computes
 *               only the translation columns (tx, ty) of the Jacobian, the
 *               ones the Newton refinement step uses, and writes zeros in
 *               the other four (fewer per-pixel sums); other calls ignore it;
 *             SWIFT_FLAG_PEARSON: Pearson-normalised correlation instead of
 *               the whitened match (Section II: NCC via an FFT correlation
 *               and a cumulative-area correction).  The central n/2 x n/2
 *               template of window A is scored against every placement
 *               inside window B, shifts |sx|, |sy| <= n/4, by the Pearson
 *               coefficient of the two patches (in [-1, 1]; 0 where the patch
 *               of B is constant).  Windows are gathered without taper; p,
 *               eps_rel and taper_frac are ignored and max_shift must be 0.
 *               The record's peak is the best coefficient (first row-major
 *               maximum of the wrapped index, as usual), mean/std/snr are
 *               taken over the (n/2+1)^2 placements, and the centroid weighs
 *               max(coefficient - mean, 0) over the placements among the 3x3
 *               neighbours (curvatures 0 when a neighbour lies beyond the
 *               range).  A constant template is degenerate.  surfaces and
 *               saved must be NULL; the adjoint entry points reject it
 *               (SWIFT_E_UNSUPPORTED).
 *  max_shift  radius r >= 0 of the expected-shift neighbourhood (the pruned
 *             inverse FFT, an algorithmic speed-up named in Section V).  For a
 *             window edge n with 0 < r < n/2 the integer peak is the first
 *             row-major maximum among the surface entries with wrapped shifts
 *             |sx|, |sy| <= r, and only the surface rows within r + 1 of the
 *             origin (rounded out to the inverse row blocks) are transformed
 *             back.  The SNR background stays the whole surface: mean 0 (the
 *             DC bin is 0) and the population std from the whitened spectrum
 *             by Parseval, std^2 = sum_k |C(k)|^2 / n^4.  r = 0, or r >= n/2,
 *             searches the whole surface.  With 0 < r < n/2 for some size in
 *             the batch, `surfaces` must be NULL.
 *  snr_exclude_r  R in [0, 8] (Section III, Z-score paragraph: the peak is
 *             scored against the background distribution of the surface).
 *             R = 0: the background is the whole surface.  R > 0: the mean
 *             and population std of the record (and so the SNR and the
 *             centroid weights c - mean) are taken over the n^2 - (2R+1)^2
 *             entries outside the box of half-width R around the integer peak
 *             (wrapped).  Not with SWIFT_FLAG_PEARSON; the adjoint entry
 *             points reject R > 0 (SWIFT_E_UNSUPPORTED).
 *
 * Samples.  Window samples a are taken about an offset o, the source pixel
 * nearest the window centre, before the taper-weighted mean is removed (which
 * makes the result independent of o).  A window is degenerate (status
 * SWIFT_ST_DEGENERATE, SNR 0, surface 0) when its taper-weighted variance
 * ||w||^2 is at most 1e-6 of sum((a - o) T)^2: its samples are equal up to
 * rounding (a constant window always is).  The cross power is formed from
 * the spectra divided by ||w||, so no input scale overflows the FP32
 * arithmetic: SWIFT_F32 pixels may take any finite values whose window sums
 * sum((a - o) T)^2 stay below 1e36 (|a - o| below about 1e15 at n = 1024);
 * the results (surface values, peak) carry the input's scale. */
#define SWIFT_FLAG_CONCURRENT_SIZES 1
#define SWIFT_FLAG_JAC_TRANSLATION 2
#define SWIFT_FLAG_PEARSON 4
typedef struct {
  float p;
  float eps_rel;
  float taper_frac;
  int32_t centroid_r;
  int32_t flags;
  int32_t max_shift;
  int32_t snr_exclude_r;
  int32_t reserved;  /* must be 0 */
} swift_params;

/* One match record (64 bytes). */
typedef struct {
  float dx, dy;      /* sub-pixel shift: wrapped integer peak + 3x3 centroid   */
  int32_t ix, iy;    /* integer peak index in the n x n surface (first maximum) */
  float peak;        /* surface value at the peak                               */
  float snr;         /* (peak - mean) / std                                     */
  double mean, std;  /* background mean and population std (FP64 reduction): the
                        whole surface, or without the snr_exclude_r box         */
  int32_t status;    /* SWIFT_ST_* bits                                         */
  int32_t n;         /* window edge of this pair                                */
  float hxx, hyy;    /* surface curvature at the peak: second differences in x, y */
  float hxy;         /* and the mixed difference (c11 - c1-1 - c-11 + c-1-1) / 4  */
  int32_t reserved;
} swift_match;

/* Context: owns the device twiddle table of one GPU.  Allocates (once).
 * tune_cache_path: host string or NULL.  When given, the plan (the kernel
 * variants per window size, see swift_plan) is read from that text file for
 * this device (its architecture name and compute-unit count) if the file
 * exists, and swift_autotune writes the plans it finds back into it (other
 * devices' lines are kept).  A missing file is not an error; unreadable lines
 * are ignored. */
int swift_create(int device, const char* tune_cache_path, swift_ctx** out);
void swift_destroy(swift_ctx* ctx);

/* Bytes of device workspace swift_match_batch needs for this batch
 * (*ws_bytes), and of the optional buffer that swift_match_batch fills for
 * swift_match_backward (*saved_bytes). */
int swift_workspace_size(swift_ctx* ctx, const swift_pairs* pairs,
                         const swift_params* params, size_t* ws_bytes,
                         size_t* saved_bytes);

/* Whitened FFT matching of a batch of window pairs (Section III).  For each
 * pair: gather A and B through their affines, subtract the taper-weighted mean
 * and taper, 2-D FFT both, X = conj(F_A) F_B, C = X (|X|^2+eps^2)^(-p/2) with
 * the DC bin set to 0, inverse FFT to the n x n surface c (scaled 1/n^2), then
 * the first maximum, mean/std (FP64), SNR and the 3x3 centroid.
 *  imgs      device [n_imgs] image table, indexed by pairs->img_a/img_b.
 *  out       device [P] records.
 *  surfaces  device float, NULL or room for sum over pairs of n^2 values; pair
 *            k's surface starts after those of pairs 0..k-1, row-major.
 *  saved     device, NULL or swift_workspace_size's saved_bytes: the state
 *            swift_match_backward reads.
 *  ws        device workspace of ws_bytes >= swift_workspace_size's ws_bytes.
 * Errors: SWIFT_E_INVAL (NULL pointers, counts, params out of range),
 * SWIFT_E_UNSUPPORTED (centroid_r != 1, unknown flags), SWIFT_E_WORKSPACE,
 * SWIFT_E_HIP.  Calls on one context must not overlap in time from several
 * host threads (the context's streams and events are shared). */
int swift_match_batch(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs,
                      const swift_pairs* pairs, const swift_params* params,
                      swift_match* out, float* surfaces, void* saved, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* swift_match_batch for callers that cannot allocate (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): no
 * workspace argument, no surfaces, no saved state.  The workspace is a
 * fixed device array of SWIFT_NOALLOC_SCRATCH_BYTES (128 MiB) that the library
 * holds on every GPU it runs on until the process ends; the call creates,
 * allocates and frees nothing (one launch sequence per size group on
 * `stream`; kernel timing does not apply).  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other streams, other
 * host threads, other contexts) race and must not be issued.  The kernels
 * write every scratch byte they read within the call, so nothing needs
 * clearing between calls.  Records are those of swift_match_batch.
 * Errors: as swift_match_batch; SWIFT_E_WORKSPACE when the batch needs more
 * than the array holds (swift_workspace_size tells how much it needs). */
#define SWIFT_NOALLOC_SCRATCH_BYTES (128u << 20)
int swift_match_batch_noalloc(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs,
                              const swift_pairs* pairs, const swift_params* params,
                              swift_match* out, hipStream_t stream);

/* swift_match_batch as one hipGraph launch (ragged batching, not in the
 * paper): the first call with a given argument tuple (every pointer, n_imgs,
 * size_count, params) captures the whole batch, scheduled as with
 * SWIFT_FLAG_CONCURRENT_SIZES (groups too small to fill the GPU as concurrent
 * branches), and instantiates it; later calls with the same tuple
 * only launch the cached graph on `stream`.  Buffer contents may change
 * between calls (the image table, pairs and thetas are read when the graph
 * runs); pointers and counts may not without a new capture.  Up to 16 graphs
 * are cached per context (least recently used evicted).  Kernel timing
 * (swift_profile_enable) does not apply to graph launches.
 * Errors: as swift_match_batch, plus SWIFT_E_CAPTURE. */
int swift_match_graph(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs,
                      const swift_pairs* pairs, const swift_params* params,
                      swift_match* out, float* surfaces, void* saved, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* Adjoint of swift_match_batch (not in the paper): for J = sum_k g_peak[k] *
 * peak_k + g_snr[k] * snr_k, the gradient with respect to the six affine
 * entries (a11, a12, tx, a21, a22, ty) of every window, the integer peak held
 * fixed.  Inputs and params must be those of the forward call that filled
 * `saved`.  g_peak / g_snr: device [P] or NULL (= 0).  g_theta_a: device [P][6];
 * g_theta_b: device [P][6] or NULL.  peak_hess: device [P][3] or NULL, receives
 * the Hessian (d2c/dx2, d2c/dy2, d2c/dxdy) of the surface's trigonometric
 * interpolant at the integer peak, sum_k C(k) (2 pi i k/n)^2 e^{2 pi i k.s/n} / n^2
 * over signed frequencies (the Nyquist frequency contributes (n/2)^2 to the
 * pure terms and nothing to the mixed one).  ws as for the forward call. */
int swift_match_backward(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs,
                         const swift_pairs* pairs, const swift_params* params,
                         const void* saved, const float* g_peak, const float* g_snr,
                         float* g_theta_a, float* g_theta_b, float* peak_hess, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/* Z-projection "model" of every section of a stack (Section III, model
 * paragraph; the remod program): out[s] = round-half-up of the mean of the
 * included sections j with 1 <= |j - s| <= k (self always omitted, sections
 * with exclude[j] != 0 omitted), computed exactly in integers.  A section with
 * no included neighbour gets all zeros.
 *  stack     device uint8, S sections of height x width; pixel (s, y, x) at
 *            stack[s*section_stride + y*pitch + x].
 *  exclude   device [S] uint8 or NULL.
 *  out       device uint8 with the same geometry rules (out_pitch,
 *            out_section_stride); must not overlap stack.
 *  k         1..8.
 * Errors: SWIFT_E_INVAL (NULL, S < 1, sizes, pitches smaller than width,
 * strides smaller than height*pitch, k out of range), SWIFT_E_HIP. */
int swift_project(swift_ctx* ctx, const uint8_t* stack, int32_t S, int32_t height, int32_t width,
                  int64_t pitch, int64_t section_stride, const uint8_t* exclude, int32_t k,
                  uint8_t* out, int64_t out_pitch, int64_t out_section_stride, hipStream_t stream);

/* Jump repair (Section III, model paragraphs).  An abrupt change of content
 * or magnification can make a section's match lock to one side of its model.
 * The sections involved are then fitted against a left-only and a right-only
 * model, and the affines across the failed span follow a smooth curve between
 * the two fits.
 *
 * One-sided models: as swift_project, but out[s] is the rounded mean of the
 * included sections s-k..s-1 (side = -1) or s+1..s+k (side = +1) only.
 * Errors: as swift_project, and SWIFT_E_INVAL for side not -1 or +1. */
int swift_project_side(swift_ctx* ctx, const uint8_t* stack, int32_t S, int32_t height, int32_t width,
                       int64_t pitch, int64_t section_stride, const uint8_t* exclude, int32_t k,
                       int32_t side, uint8_t* out, int64_t out_pitch, int64_t out_section_stride,
                       hipStream_t stream);

/* The smoothing curve across a failed span [a, b] of sections: for s in
 * [a, b], aff[s] = (1 - w) aff_left[s] + w aff_right[s] entry by entry, where
 * w = 3 t^2 - 2 t^3 is the cubic Bezier with control values 0, 0, 1, 1 and
 * t = (s - a + 1) / (b - a + 2) (the span's good neighbours a - 1 and b + 1
 * sit at t = 0 and 1).  aff_left / aff_right: the section affines [S][6]
 * fitted against the left / right one-sided models; aff [S][6] receives the
 * span's entries (others untouched).  All device, double.  Errors:
 * SWIFT_E_INVAL (NULL, span outside [0, S)), SWIFT_E_HIP. */
int swift_blend_span(swift_ctx* ctx, int32_t S, int32_t a, int32_t b, const double* aff_left,
                     const double* aff_right, double* aff, hipStream_t stream);

/* Joins the sections after a break to the frame before it: with A_j the
 * affine of section j and L_j = aff_left[j] its fit against the left
 * one-sided model, the aligned-frame correction D = A_j^-1 L_j is composed
 * into every section s >= j (out[s] = A_s o D, so out[j] = L_j); sections
 * before j are copied.  aff, aff_left, out: device [S][6] double; out must not
 * alias aff.  A singular A_j gives non-finite output.  Errors: SWIFT_E_INVAL
 * (NULL, aliasing, j outside [0, S)), SWIFT_E_HIP. */
int swift_join_break(swift_ctx* ctx, int32_t S, int32_t j, const double* aff, const double* aff_left,
                     double* out, hipStream_t stream);

/* Search with an SNR stop (Section III, SNR paragraph: an SNR above 15 marks
 * a correct match, so a search for better matches can stop there).  After a
 * round that matched the n active windows idx[i] (of P) at candidate `cand`
 * (records recs[i], device [n]), every such window keeps the higher-SNR of
 * its kept record best[w] and the new one (its candidate in best_cand[w];
 * the earlier candidate on equal SNR) and gets done[w] = 1 once the kept
 * SNR reaches `accept`.  Before the first round the caller sets best_cand to
 * -1 and done to 0.  idx: device [n]; best: device [P] records; best_cand:
 * device [P] int32; done: device [P] uint8.  Entries of idx outside [0, P),
 * and windows already done, are left alone, so a caller may match several
 * candidates ahead and keep them one candidate at a time.  The other entries
 * must be distinct (one thread owns each window's record), as
 * swift_search_next's output is.  Errors: SWIFT_E_INVAL (NULL,
 * n outside [0, P], cand < 0), SWIFT_E_HIP. */
int swift_search_keep(swift_ctx* ctx, int32_t P, int32_t n, const int32_t* idx, const swift_match* recs,
                      int32_t cand, float accept, swift_match* best, int32_t* best_cand, uint8_t* done,
                      hipStream_t stream);

/* Next round of the search with an SNR stop (Section III, SNR paragraph):
 * gathers the windows w with done[w] == 0, in ascending order, into
 * idx[0..n) (their indices), img_a_out/img_b_out and theta_a_out/theta_b_out
 * [n][8], window A's translation (entries 4 and 7) moved by (ox, oy); n is
 * written to count (device int32).  A batch sorted by window edge stays
 * sorted.  done: device [P] uint8; img_a/img_b: device [P] int32;
 * theta_a/theta_b: device [P][8]; the outputs: device, room for P entries,
 * not aliasing the inputs.  Runs as one workgroup (cost grows with P / 1024).
 * Errors: SWIFT_E_INVAL (NULL, P < 0, aliasing), SWIFT_E_HIP. */
int swift_search_next(swift_ctx* ctx, int32_t P, const uint8_t* done, float ox, float oy, const int32_t* img_a,
                      const int32_t* img_b, const float* theta_a, const float* theta_b, int32_t* idx,
                      int32_t* img_a_out, int32_t* img_b_out, float* theta_a_out, float* theta_b_out,
                      int32_t* count, hipStream_t stream);

/* One level of the x2 source pyramid (Section III: iscale): dst(x, y) =
 * (sum of the 2x2 block at (2x, 2y) + 2) >> 2 for uint8 images; dst must be
 * (src.width/2) x (src.height/2).  Descriptors are host structs whose data
 * pointers are device memory. */
int swift_pyramid(swift_ctx* ctx, const swift_image* src, const swift_image* dst,
                  hipStream_t stream);

/* Peak, SNR and centroid of given correlation surfaces (the scoring step of
 * swift_match_batch alone; Section III, Z-score paragraph).
 *  surfaces  device [batch][n][n] float; out device [batch].  params: only
 *            snr_exclude_r is used (the rest is validated).
 * Errors: SWIFT_E_INVAL (NULL, n outside [4, 4096], batch < 0, params). */
int swift_snr(swift_ctx* ctx, const float* surfaces, int32_t n, int32_t batch,
              const swift_params* params, swift_match* out, hipStream_t stream);

/* Jacobian of the centroid shift (not in the paper; for the Newton refinement
 * below): jac [P][2][6] receives d(dx)/d theta_A and d(dy)/d theta_A, the
 * six affine entries (a11, a12, tx, a21, a22, ty) of window A, with the integer
 * peak and the set of positive centroid weights (3x3 box, weight = c - mean)
 * held fixed.  One adjoint pass: the two objectives share one packed inverse
 * 2-D FFT.  A pair whose record is degenerate, or whose box has no positive
 * weight, gets zeros.  With SWIFT_FLAG_JAC_TRANSLATION in params->flags only
 * the tx and ty columns (jac[.][.][2], jac[.][.][5], the ones the Newton step
 * reads) are computed and the other four are written as zeros; the computed
 * columns equal those of the full pass.  Inputs, params and `saved` as for
 * swift_match_backward; jac is device memory.  Errors as for
 * swift_match_backward. */
int swift_centroid_jacobian(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs,
                            const swift_pairs* pairs, const swift_params* params,
                            const void* saved, float* jac, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* One step of iterative window refinement (Section IV: matching is iterated
 * until the scores stabilise), applied in place to the window-A parameters
 * theta [P][8] on the device, one thread per pair:
 *  mode SWIFT_REFINE_CENTROID: t <- t - d with d = (dx, dy), the record's
 *    sub-pixel shift;
 *  mode SWIFT_REFINE_NEWTON: Newton's method on the centroid.  Within the
 *    cell of the integer peak s the centroid moves as d = s + J (t - t* - s)
 *    with J = [[jac[2], jac[5]], [jac[8], jac[11]]] (d d / d (tx, ty) from
 *    swift_centroid_jacobian), so t <- t - (s + J^-1 (d - s)).  Used when s
 *    is the origin, or one of its eight neighbours with J^-1 (d - s) inside
 *    [-0.6, 0.6]^2, the record is not degenerate and det J > 1e-6; otherwise
 *    the centroid step.
 * Steps longer than max_step pixels are scaled down to max_step (> 0); a
 * Newton step may be longer by |s| (its whole-pixel part is never cut).
 * step_out: device [P] receives the length of each applied step (may be NULL).
 * recs, jac: device, as produced for the same pairs; jac may be NULL in
 * centroid mode. */
#define SWIFT_REFINE_CENTROID 0
#define SWIFT_REFINE_NEWTON   1
int swift_refine_update(swift_ctx* ctx, int32_t P, const swift_match* recs, const float* jac,
                        float* theta, int32_t mode, float max_step, float* step_out,
                        hipStream_t stream);

/* ---- Stack loop (Sections III-IV: swim matches a section to its remod model,
 * mir renders it by the least-squares affine of the matches, repeated over
 * iscale levels).  A section affine maps aligned-frame points p to raw-section
 * points q, both in level-0 pixels: q = L p + t, stored as double
 * (a11, a12, tx, a21, a22, ty).  Pixel x_l of pyramid level l has its centre at
 * level-0 coordinate 2^l x_l + (2^l - 1)/2. */

/* mir rendering of S sections: dst(s, y, x) = bilinear value (clamp to edge)
 * of the level-l raw section src(s) at the raw point of aligned pixel (x, y),
 * rounded half up to uint8.  Coordinates and interpolation are FP64 with every
 * operation rounded separately, so the result is reproducible bit for bit.
 *  src   device uint8, pixel (s, y, x) at src[s*src_stride + y*src_pitch + x].
 *  aff   device double [S][6], level-0 affines.
 *  dst   device uint8 [S] x dst_h x dst_w with dst_pitch, dst_stride; must not
 *        overlap src.
 * Errors: SWIFT_E_INVAL (NULL, sizes < 1, pitches/strides too small, level
 * outside 0..12), SWIFT_E_HIP. */
int swift_render(swift_ctx* ctx, const uint8_t* src, int32_t S, int32_t src_h, int32_t src_w,
                 int64_t src_pitch, int64_t src_stride, const double* aff, int32_t level,
                 uint8_t* dst, int32_t dst_h, int32_t dst_w, int64_t dst_pitch, int64_t dst_stride,
                 hipStream_t stream);

/* swim window set-up for S sections at level l: a grid x grid tiling of n x n
 * windows of the h_l x w_l aligned frame (tile size h_l/grid, w_l/grid, centres
 * at half a tile).  Pair i = s*grid^2 + k (k row-major).  Window B reads the
 * model at the tile centre at identity: theta_b = (px, py, 1, 0, 0, 0, 1, 0).
 * Window A reads the raw section around the raw point c of that centre with
 * the section's linear part: theta_a = (rint(cx), rint(cy), a11, a12,
 * cx - rint(cx), a21, a22, cy - rint(cy)).  img_a[i] = img_a0 + s, img_b[i] =
 * img_b0 + s.  All outputs are device arrays of S*grid^2 entries (theta [8]).
 * Errors: SWIFT_E_INVAL. */
int swift_stack_windows(swift_ctx* ctx, int32_t S, const double* aff, int32_t level, int32_t grid,
                        int32_t h_l, int32_t w_l, int32_t img_a0, int32_t img_b0,
                        float* theta_a, float* theta_b, int32_t* img_a, int32_t* img_b,
                        hipStream_t stream);

/* mir's affine of each section from its `per_section` window matches (pairs
 * s*per_section .. (s+1)*per_section - 1): model point p = centre of window B,
 * raw point q = window A's point -(dx, dy) (a pair with B(x) = A(x - d) aligns
 * them), both mapped to level 0; weight = snr, or 0 when the record is
 * degenerate or snr < min_snr.  aff [S][6] (device, double) holds the previous
 * affines and receives the weighted least-squares fit q ~ L p + t; a section
 * with fewer than three weighted points, or with collinear points, keeps its
 * previous affine and gets status 1 (else 0).  status: device [S] or NULL.
 * Errors: SWIFT_E_INVAL. */
int swift_fit_sections(swift_ctx* ctx, int32_t S, int32_t per_section, const float* theta_a,
                       const float* theta_b, const swift_match* recs, int32_t level, float min_snr,
                       double* aff, int32_t* status, hipStream_t stream);

/* ---- Local-affine triangle mesh (mir at the finest stages, Section IV; texture
 * mapping of a triangulated mesh, Section III).
 *
 * The mesh of a section lives on an h_l x w_l level-l aligned frame with a
 * grid x grid layout (2 <= grid <= 1024, grid <= h_l, w_l <= 65535): node (i, j), index
 * k = j*grid + i, sits at the centre of swim window k, (sx/2 + i*sx, sy/2 +
 * j*sy) with sx = w_l/grid, sy = h_l/grid (integer division).  Cell (ci, cj),
 * 0 <= ci, cj < grid-1, is cut along the diagonal from node (ci+1, cj) to node
 * (ci, cj+1) into triangle 2c (nodes (ci,cj), (ci+1,cj), (ci,cj+1)) and
 * triangle 2c+1 (nodes (ci+1,cj), (ci+1,cj+1), (ci,cj+1)), c = cj*(grid-1) + ci;
 * T = 2*(grid-1)^2 triangles per section.  Level-l pixel (x, y) belongs to cell
 * (clamp(floor((x - sx/2)/sx)), clamp(floor((y - sy/2)/sy))), clamped to the
 * cells so that the border triangles reach the frame edges, and to its first
 * triangle iff (x - x_c)*sy + (y - y_c)*sx <= sx*sy, (x_c, y_c) the cell's node
 * (ci, cj).  Triangle affines are level-0 maps from aligned-frame points to
 * raw-section points, like the section affines: tri_aff [S][T][6] doubles
 * (a11, a12, tx, a21, a22, ty), device. */

/* mir texture mapping: as swift_render, except that every output pixel takes
 * the affine of its triangle in the mesh of the dst_h x dst_w output frame.
 * Output is bit-exact to that definition (FP64, fixed operation order).
 * Errors: SWIFT_E_INVAL (sizes as swift_render; grid out of range or larger
 * than dst_h or dst_w), SWIFT_E_HIP. */
int swift_render_mesh(swift_ctx* ctx, const uint8_t* src, int32_t S, int32_t src_h, int32_t src_w,
                      int64_t src_pitch, int64_t src_stride, const double* tri_aff, int32_t grid,
                      int32_t level, uint8_t* dst, int32_t dst_h, int32_t dst_w, int64_t dst_pitch,
                      int64_t dst_stride, hipStream_t stream);

/* swim window set-up through a mesh: the windows of swift_stack_windows (same
 * layout, pair i = s*grid^2 + k at node k, same outputs), except that window A
 * reads the raw section through the affine of the triangle node k's pixel
 * belongs to.  Errors: SWIFT_E_INVAL. */
int swift_mesh_windows(swift_ctx* ctx, int32_t S, const double* tri_aff, int32_t level, int32_t grid,
                       int32_t h_l, int32_t w_l, int32_t img_a0, int32_t img_b0, float* theta_a,
                       float* theta_b, int32_t* img_a, int32_t* img_b, hipStream_t stream);

/* mir's local affines (Section IV): each triangle's affine is the weighted
 * least-squares fit q ~ L p + t of the window matches in its band, the
 * triangle's three nodes and every node sharing a mesh edge with one of them
 * (12 nodes inside the mesh, fewer at its border).  Matches are pairs
 * s*grid^2 + k (node k), read as in swift_fit_sections (p, q, weights).  A
 * triangle with fewer than three weighted band points, or collinear ones,
 * takes its section's affine aff [S][6] (device, double, read only) and status
 * 1, else 0.  tri_aff: device [S][T][6] output; status: device [S][T] or NULL.
 * Errors: SWIFT_E_INVAL (S outside [1, 65535], grid outside [2, 1024]). */
int swift_fit_mesh(swift_ctx* ctx, int32_t S, int32_t grid, const float* theta_a, const float* theta_b,
                   const swift_match* recs, int32_t level, float min_snr, const double* aff,
                   double* tri_aff, int32_t* status, hipStream_t stream);

/* The plan: kernel variants of the match per window size (a tuning choice,
 * not in the paper; the results agree to rounding).
 *  - Row-count variants: two row counts per block for the forward row pass
 *    and two for the inverse row pass (variant 0 = the default, 1 = the
 *    alternative).
 *  - Forward variant 2, for n <= 128 (whitened match; a Pearson batch keeps
 *    the five-kernel path): the whole pair in one workgroup, its packed
 *    spectrum resident in LDS from the gather to the record, so no spectrum
 *    crosses device memory (the inverse variant is then unused and the rows
 *    per block reported are n).  A new context uses it at n = 64 and the
 *    five-kernel path (variants 0, 0, one chunk) at the other sizes.
 *  - Chunks (1, 2, 4, 8): a size group of P pairs is split into that many
 *    chunks of consecutive pairs whose kernel sequences alternate between two
 *    streams of the context (forked from and joined back into the call's
 *    stream), so that one chunk's forward row pass runs beside another's
 *    column pass.  The records are identical to those of one chunk.  A batch
 *    with size groups running beside each other (SWIFT_FLAG_CONCURRENT_SIZES,
 *    or swift_match_graph, with several sizes one of which is too small to
 *    fill the GPU) runs every group as one chunk.
 * swift_plan sets the variants of size n (a value < 0 keeps the current one)
 * and reports the rows per block and the chunks (any output may be NULL).
 * Plans are per context; cached graphs are keyed by them.  Errors:
 * SWIFT_E_INVAL. */
int swift_plan(swift_ctx* ctx, int32_t n, int32_t fwd_variant, int32_t inv_variant, int32_t chunks,
               int32_t* fwd_rows, int32_t* inv_rows, int32_t* chunks_out);

/* Times plan variants of each listed window size on a synthetic batch
 * (pairs_per_size translation windows of hashed uint8 noise, p = 0.65;
 * <= 0 means 512) and keeps the fastest in the context's plan (and, with a
 * tune cache path, in that file).  Each variant's time is the fastest of 3
 * rounds that visit the variants in turn, a round timing the mean of 3
 * batches; a variant replaces the defaults (slot 0), and a chunk count the
 * best row variant, only when at least 2% faster.  Synchronous; allocates
 * and frees its own device buffers, so it is a set-up call, not one for a
 * capture or a serving loop.  times_ms: host [n_sizes][SWIFT_TUNE_SLOTS] or
 * NULL, receives those times per batch for: slots 0..3 the row variants
 * (fwd + 2 inv) in one chunk, slots 4..6 the chosen row variant in 2, 4 and
 * 8 chunks, slot 7 the one-workgroup kernel (n <= 128); -1 where a variant
 * equals another or does not apply.  Errors: SWIFT_E_INVAL, SWIFT_E_HIP. */
#define SWIFT_TUNE_SLOTS 8
int swift_autotune(swift_ctx* ctx, const int32_t* sizes, int32_t n_sizes, int32_t pairs_per_size,
                   float* times_ms);

/* Kernel timing (instrumentation, not in the paper).  While enabled, every
 * kernel the context launches is bracketed by a pair of HIP events recorded on
 * the launch stream (a few microseconds per launch; no work is skipped).
 * swift_profile_read waits for those events and returns, per kernel name
 * ("k_col<512>" ...), the number of launches and their summed duration in ms,
 * then forgets them.  names: host [max_kernels][64] chars; launches, total_ms:
 * host [max_kernels]; *n_kernels receives the number of distinct kernels (may
 * exceed max_kernels).  Not thread-safe with concurrent calls on one context. */
int swift_profile_enable(swift_ctx* ctx, int enable);
int swift_profile_read(swift_ctx* ctx, int32_t max_kernels, char* names, int32_t* launches,
                       double* total_ms, int32_t* n_kernels);

/* Message of the last failing call on this thread ("" if none). */
const char* swift_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SWIFT_H */
