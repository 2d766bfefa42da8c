/*
 * htsvd.h -- C ABI of the MI355X (gfx950) Haar-tSVD denoising library.
 *
 * Method: "Image Denoising Using Global and Local Circulant Representation"
 * (Kong, Yang, Zhang).  For every reference patch on a regular grid the
 * library groups the K most similar patches inside a search window
 * (Sec. III-A, Eq. 9), projects the group with the shared t-SVD basis and a
 * Haar transform along the group (Sec. III-D, Eq. 19), hard-thresholds the
 * coefficients (Eq. 20), inverts the transform (Eq. 21) and averages the
 * patches back into the image (Algorithm 1).  The noise level comes from the
 * caller, from a plain patch-covariance estimator adjusted by the
 * circulant-eigenvalue vote of Eq. 22-23 (Sec. III-E-1), or from a small
 * learned network.
 *
 * Conventions for every entry point:
 *  - Image pointers named d_* are DEVICE pointers (HIP global memory) owned
 *    by the caller; h_* pointers are host memory.  Buffers must not alias.
 *  - Input images are uint8, row-major, channels interleaved (HWC):
 *    pixel (y, x, ch) at d_in[y*in_stride + x*c + ch]; in_stride is in bytes
 *    and >= w*c.  Outputs are float32 HWC on the 0..255 scale, unclipped,
 *    out_stride in elements and >= w*c.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work asynchronously on it and return a status synchronously for
 *    argument errors; device faults surface from the next call or from
 *    htsvd_sync().  A context is not thread-safe; use one per thread.
 *  - On any non-OK status nothing has been enqueued, and
 *    htsvd_last_error() returns a message for the calling thread.
 *  - The context owns its workspace (grown on demand, freed by
 *    htsvd_destroy); buffers passed in are never freed by the library.
 */
#ifndef HTSVD_H
#define HTSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HTSVD_OK = 0,
    HTSVD_EINVAL = -1,  /* null pointer, bad parameter value */
    HTSVD_ESHAPE = -2,  /* image too small, too few candidates for K, stride too small */
    HTSVD_ENOMEM = -3,  /* device allocation failed */
    HTSVD_EDEVICE = -4, /* HIP runtime error (including deferred kernel faults) */
    HTSVD_ENOTSUP = -5, /* parameter combination the library does not support */
    HTSVD_ESTATE = -6   /* missing basis or network weights */
} htsvd_status;

/* Pass as `sigma` to estimate the noise level from the image. */
#define HTSVD_SIGMA_AUTO (-1.0f)

/* Method parameters (htsvd_default_params fills the paper's defaults). */
typedef struct {
    int32_t ps;          /* patch side; 8 (Sec. IV-A) is the only supported value */
    int32_t stride;      /* reference-grid step in pixels, >= 1 (grid: 0, s, 2s, ..., plus the last position) */
    int32_t window;      /* odd search-window side W, 3..31, clipped at the image border */
    int32_t K;           /* group size, a power of two in {4, 8, 16, 32} (Sec. III-C-2 needs 2^n) */
    double tau_mult;     /* tau = sigma * tau_mult; <= 0 selects sqrt(2 ln(c K ps^2)) (Sec. IV-A) */
    int32_t adaptive;    /* 1: adjust sigma per sub-image by the vote of Eq. 23 */
    double beta;         /* Eq. 23 divisor, 1.2 */
    int32_t gamma_rank;  /* Eq. 23 rank bound, 13 */
    int32_t gcp_num;     /* Eq. 9 green-prior weight gamma = gcp_num/gcp_den (6/5 = 1.2) */
    int32_t gcp_den;
    int32_t estimator;   /* sigma source under HTSVD_SIGMA_AUTO: 0 plain covariance-eigenvalue estimator
                            per sub-image; 1 learned per-8x8-block sigma map, judged per sub-image by the
                            plain estimator, which replaces it where they differ by more than 1.5x */
    int32_t subimage;    /* sub-image side for sigma estimation and votes, 128 */
    int32_t n_vote;      /* sampled groups per sub-image for the vote, 15 */
    uint64_t vote_seed;  /* seed of the counter-based SplitMix64 sampler of the vote */
    int32_t ra;          /* 1: RA-Haar-tSVD (Sec. III-E-2, Eq. 24-25): the refinement network of
                            htsvd_ra_set_weights replaces the first Haar row of every group whose
                            noise level tau / tau-multiplier exceeds ra_sigma (single-image calls) */
    double ra_sigma;     /* 30 (Sec. IV-B applies the enhancement where sigma > 30) */
} htsvd_params;

typedef struct htsvd_ctx htsvd_ctx;

/* Creates a context on HIP device `device` (allocates nothing large). */
htsvd_status htsvd_create(htsvd_ctx **out, int device);
/* Frees the context, its workspace, graphs and weights.  NULL is ignored. */
void htsvd_destroy(htsvd_ctx *ctx);
/* Fills `out` with the defaults for c channels: ps 8, stride 4, window 31 (c=3) or 21 (c=1),
 * K 32 (c=3) or 16 (c=1), tau_mult 0, adaptive 0, beta 1.2, gamma_rank 13, gcp 6/5,
 * estimator 0, subimage 128, n_vote 15, vote_seed 0, ra 0, ra_sigma 30. */
htsvd_status htsvd_default_params(int32_t c, htsvd_params *out);

/* Sets the shared t-SVD basis pair (U, V) for c channels (Sec. III-B, "globally reused"
 * bases, Eq. 11): host FP64 arrays of ps*ps*c values each, slice-major:
 * U[(k*ps + i)*ps + j] = U(i, j, k).  Both tensors must be orthogonal (U^T * U = I);
 * the library copies them (FP32 Fourier-domain slices for the transform, FP64 for the
 * threshold guard band).  Returns HTSVD_EINVAL if they are not orthogonal to 1e-9.
 * c = 2 or 4 .. 64 sets the basis of the hyperspectral path (htsvd_denoise_bands; one band
 * count at a time). */
htsvd_status htsvd_set_basis(htsvd_ctx *ctx, int32_t ps, int32_t c, const double *h_U, const double *h_V);

/* Channel Gram sums of all reference patches of one image (the sums behind the learned basis
 * of Sec. III-B, Eq. 10-11).  Over the reference grid of step `stride` (Algorithm 1) and patches
 * P of ps = 8, into the DEVICE int64 array d_gram of 2*c*c*64 entries:
 *   d_gram[((0*c + a)*c + b)*64 + i*8 + k] = sum_P sum_j P(i, j, a) P(k, j, b)   (patch rows)
 *   d_gram[((1*c + a)*c + b)*64 + i*8 + k] = sum_P sum_j P(j, i, a) P(j, k, b)   (patch columns)
 * Exact integers.  Asynchronous on `stream` (clears d_gram first); the caller owns d_gram.
 * Errors: HTSVD_EINVAL (null pointers, c not 1/3, stride < 1, in_stride < w*c), HTSVD_ENOTSUP
 * (ps != 8, more than 2^30 pixels), HTSVD_ESHAPE (image smaller than one patch). */
htsvd_status htsvd_basis_gram(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                              int64_t in_stride, int32_t ps, int32_t stride, int64_t *d_gram, void *stream);

/* Learns the t-SVD basis pair (U, V) from one image (Sec. III-B, Eq. 10-11) and installs it as
 * the context's basis for c channels, exactly as htsvd_set_basis would.  Per slice f of the
 * channel DFT (Eq. 5), U_hat^(f) holds the eigenvectors of C_row = sum_P P_hat P_hat^H and
 * V_hat^(f) those of C_col = sum_P P_hat^H P_hat over all reference patches of the grid of
 * step `stride`, by descending eigenvalue, each with the phase that makes its entry of largest
 * modulus (the first among equals) real and positive; slices f and c-f are conjugate, so U and
 * V are real.  The sums run on the device (see htsvd_basis_gram); the 8x8 eigendecompositions
 * run on the host.  h_U, h_V (host, ps*ps*c FP64 each, slice-major as in htsvd_set_basis) receive
 * the pair when not NULL.  Synchronises `stream`; like htsvd_set_basis, it must not overlap a
 * running call that uses the basis for c channels.  Errors as htsvd_basis_gram, plus those of
 * htsvd_set_basis and HTSVD_EDEVICE / HTSVD_ENOMEM from the device. */
htsvd_status htsvd_learn_basis(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, int32_t ps, int32_t stride, double *h_U, double *h_V,
                               void *stream);

/* Number of reference positions along a side of length n (grid 0, s, 2s, ..., n-ps). */
int32_t htsvd_ref_count(int32_t n, int32_t ps, int32_t stride);

/* Grouping only (Sec. III-A, Eq. 9; Algorithm 1 "Grouping"): for every reference
 * r = iy*nx + ix, the K most similar patches in ascending (distance, row, column) order.
 * d_idx[r*K + k] = y*w + x (int32) of member k; d_dist[r*K + k] = its squared distance
 * (green-channel or channel-sum distance, chosen per reference by Eq. 9), may be NULL.
 * Distances are exact integers (int8 / fp16 matrix-core dot products). */
htsvd_status htsvd_block_match(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, const htsvd_params *p, int32_t *d_idx, int32_t *d_dist,
                               void *stream);

/* Full denoising (Algorithm 1 with Eq. 19-21).  sigma > 0: known noise level;
 * HTSVD_SIGMA_AUTO: estimated (p->estimator).  With p->adaptive the per-sub-image vote of
 * Eq. 23 adjusts it.  d_out: h*w*c float32 (HWC, out_stride elements per row). */
htsvd_status htsvd_denoise(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                           int64_t in_stride, float sigma, const htsvd_params *p, float *d_out,
                           int64_t out_stride, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): htsvd_denoise with every scratch buffer it needs
 * (groups, thresholds, the filter's aggregation regions, the noise-level arrays) taken from a
 * fixed device array of HTSVD_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on, from htsvd_create until the process ends.  It allocates nothing (no hipMalloc, hipFree or
 * allocating library call); the caller still owns d_in and d_out.  Arguments, layout and
 * results are those of htsvd_denoise, with sigma known or HTSVD_SIGMA_AUTO with the plain
 * estimator (p->estimator 0) and p->ra 0 (HTSVD_ENOTSUP otherwise).  An image whose scratch
 * exceeds the array returns HTSVD_ENOMEM before anything is launched (at stride 4, window 31,
 * K 32 an RGB image of about one megapixel fits).  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads, other contexts) race on it, so
 * issue them one at a time per device. */
#define HTSVD_NOALLOC_SCRATCH_BYTES (64u << 20)
htsvd_status htsvd_denoise_noalloc(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                                   int64_t in_stride, float sigma, const htsvd_params *p, float *d_out,
                                   int64_t out_stride, void *stream);

/* Denoising with a caller-provided threshold per reference (tau of reference r in
 * d_tau_ref[r], FP64, n_ref entries).  Used to check the transform path against the oracle. */
htsvd_status htsvd_denoise_tau(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, const double *d_tau_ref, const htsvd_params *p, float *d_out,
                               int64_t out_stride, void *stream);

/* ---- Hyperspectral tube patches (Sec. IV-D) ----
 * A cube of `bands` uint8 bands per pixel (HWC, in_stride bytes per row) is grouped on a gray
 * guide, the band mean rounded half up ((sum + bands/2) / bands), with the block matcher of the
 * other paths (window, stride, K of p), and its 8 x 8 x bands tube patches are filtered with the
 * t-product along the band axis (Eq. 19-21; basis from htsvd_set_basis or htsvd_learn_basis
 * with c = bands) and tau = sigma * (p->tau_mult, or sqrt(2 ln(bands K ps^2))), then
 * aggregated uniformly (Algorithm 1). */
/* The guide image: d_guide[y*w + x] (uint8, h*w, device). */
htsvd_status htsvd_band_guide(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t bands,
                              int64_t in_stride, uint8_t *d_guide, void *stream);
/* Memory of htsvd_denoise_bands: its groups are filtered in passes whose three FP64 patch
 * matrices (K*64*bands doubles per group each) stay below `bytes` each (default 4 GiB, at least
 * 1 MiB, at least one group per pass).  The output does not depend on it. */
htsvd_status htsvd_set_band_memory(htsvd_ctx *ctx, int64_t bytes);
/* Band-wise noise levels (Sec. IV-D): sigma_b of every band, the mean over the band's 128 x 128
 * sub-images of the plain estimate htsvd_estimate_sigma gives for the band alone.  h_sigma:
 * `bands` doubles (host).  Synchronises the stream. */
htsvd_status htsvd_band_sigma(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t bands,
                              int64_t in_stride, double *h_sigma, void *stream);
/* Denoises the cube into d_out (float32 HWC, out_stride elements per row) with a known sigma, or
 * with sigma = HTSVD_SIGMA_AUTO by the band-wise rule of Sec. IV-D: with the levels sigma_b of
 * htsvd_band_sigma and their mean sigma_mean, the cube is filtered at sigma_mean, and the bands
 * with sigma_b > 2 sigma_mean take their values from the cube filtered at max_b sigma_b (one
 * grouping serves both; AUTO synchronises the stream).  Errors: HTSVD_ESTATE (no basis for this
 * band count), HTSVD_ENOTSUP (adaptive or ra set), HTSVD_EINVAL / HTSVD_ESHAPE as for
 * htsvd_denoise. */
htsvd_status htsvd_denoise_bands(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t bands,
                                 int64_t in_stride, float sigma, const htsvd_params *p, float *d_out,
                                 int64_t out_stride, void *stream);

/* ---- Video (Sec. IV-C) ----
 * T frames of h x w x c uint8 (c = 1 or 3, HWC) stacked vertically in one buffer: frame t is rows
 * t*h .. t*h + h - 1 of d_in, in_stride bytes per row.  The patch search runs over space and
 * time: each reference of frame t (frame-major, then the grid of Algorithm 1) takes the K
 * nearest patches, by the distance of Eq. 9 as decided by the reference, among the positions of
 * its clipped search window (p->window) in every frame f with |f - t| <= radius, 0 <= f < T,
 * ordered by (distance, frame, row, column).  radius = 0 gives the groups of each frame alone.
 * Errors as for htsvd_block_match, plus HTSVD_ESHAPE for T < 1, HTSVD_EINVAL for a radius
 * outside [0, 31] and HTSVD_ENOTSUP for more than 2^30 pixels in all. */
/* Groups: d_idx[r*K + k] = (f*h + y)*w + x of member k of reference r (T * ny * nx references,
 * int32, device), d_dist (may be NULL) its distance. */
htsvd_status htsvd_block_match_video(htsvd_ctx *ctx, const uint8_t *d_in, int32_t T, int32_t h, int32_t w,
                                     int32_t c, int64_t in_stride, int32_t radius, const htsvd_params *p,
                                     int32_t *d_idx, int32_t *d_dist, void *stream);
/* Denoises the frames: the spatio-temporal groups are filtered with the global t-SVD basis of c
 * channels and the Haar transform (Eq. 19-21; the matrix-core transform of htsvd_denoise,
 * coefficients near the threshold re-decided in FP64) and aggregated uniformly over the stacked
 * frames (Algorithm 1) into d_out (float32, T*h rows of out_stride elements).  The threshold is
 * tau = sigma_hat * (p->tau_mult, or sqrt(2 ln(c K ps^2))), with sigma_hat set frame by frame
 * (Sec. IV-C) as htsvd_denoise sets it for one image: the known sigma; or HTSVD_SIGMA_AUTO, the
 * frame's per-sub-image estimate (p->estimator); and p->adaptive = 1 adjusts either by the vote
 * over the frame's spatial groups (Eq. 22-23).  p->ra = 1 refines the spatio-temporal groups'
 * mean patches as htsvd_denoise does (Sec. III-E-2).  Errors: HTSVD_ESTATE (no basis for c, or
 * no network for ra or the learned estimator), the others as above. */
htsvd_status htsvd_denoise_video(htsvd_ctx *ctx, const uint8_t *d_in, int32_t T, int32_t h, int32_t w, int32_t c,
                                 int64_t in_stride, int32_t radius, float sigma, const htsvd_params *p, float *d_out,
                                 int64_t out_stride, void *stream);

/* ---- RA-Haar-tSVD refinement network (Sec. III-E-2, Eq. 24-25) ----
 * The first Haar row of a group is sqrt(K) times its mean patch p (Eq. 24); a fully connected
 * network refines p (Eq. 25), trained by residual learning on mean patches of noisy/clean
 * groups.  With P = 64c values per patch (slice-major: p[(k*8 + i)*8 + j] = p(i, j, k)) and
 * H = 256 (c = 3) or 128 (c = 1) hidden units:
 *   x = (p - 128)/128, h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), r = W3 h2 + b3,
 *   p_est = p - 128 r.
 * Parameters: FP32, flattened W1 (H x P), b1, W2 (H x H), b2, W3 (P x H), b3, row-major.
 * Inference runs on the matrix cores (fp16 hi/lo products, FP32 accumulation); training in FP32. */
int32_t htsvd_ra_param_count(int32_t c);
/* Copies n = htsvd_ra_param_count(c) host parameters into the context (resets Adam). */
htsvd_status htsvd_ra_set_weights(htsvd_ctx *ctx, int32_t c, const float *h_params, int64_t n);
/* Copies the current parameters (after training steps too) to the host. */
htsvd_status htsvd_ra_get_weights(htsvd_ctx *ctx, int32_t c, float *h_params, int64_t n);
/* Mean patches of n_ref groups over the image d_in: d_idx[r*K + k] = y*w + x of member k (as
 * htsvd_block_match gives them; the image may be another one than the groups were matched on,
 * e.g. the clean image of a training pair).  d_means: n_ref * P FP32, slice-major per group. */
htsvd_status htsvd_ra_means(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                            int64_t in_stride, const int32_t *d_idx, int32_t K, int64_t n_ref, float *d_means,
                            void *stream);
/* Network output r (n * P FP32) for n mean patches (n * P FP32), on the device. */
htsvd_status htsvd_ra_forward(htsvd_ctx *ctx, int32_t c, const float *d_means, int64_t n, float *d_r, void *stream);
/* Loss (mean of (r - (noisy - clean)/128)^2) and its gradient (d_grad: param_count FP32) for a
 * batch of n pairs of mean patches.  Synchronises `stream` for the loss (h_loss may be NULL). */
htsvd_status htsvd_ra_gradients(htsvd_ctx *ctx, int32_t c, const float *d_noisy, const float *d_clean, int32_t n,
                                float *d_grad, double *h_loss, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on a batch; h_loss as above. */
htsvd_status htsvd_ra_train_step(htsvd_ctx *ctx, int32_t c, const float *d_noisy, const float *d_clean, int32_t n,
                                 float lr, double *h_loss, void *stream);

/* One setting of a parameter sweep. */
typedef struct {
    float sigma;          /* known noise level (> 0); tau = sigma * (p->tau_mult, or sqrt(2 ln(c K ps^2))) */
    int32_t K;            /* group size of this setting: 4, 8, 16 or 32, at most p->K */
    float *d_out;         /* device, float32 HWC */
    int64_t out_stride;   /* elements per row */
} htsvd_sweep_item;

/* Denoises one image under n parameter settings (sigma, K) with a single grouping pass (the
 * cached patch indices of the paper's fast implementation, Sec. III-D-3): groups are matched
 * once with p->K members; a setting with K < p->K uses the first K members of each group, which
 * are exactly its K-member groups (members are ordered by distance, then position).  Each
 * output equals the one htsvd_denoise gives for that sigma with that K (p->adaptive must be 0:
 * the vote of Eq. 23 depends on the group size).  Asynchronous on `stream`.  Errors:
 * HTSVD_EINVAL (n < 1, null items or outputs, sigma <= 0, K > p->K or not a power of two in
 * 4..32, out_stride < w*c), HTSVD_ENOTSUP (p->adaptive), and those of htsvd_denoise. */
htsvd_status htsvd_denoise_sweep(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                                 int64_t in_stride, int32_t n, const htsvd_sweep_item *items,
                                 const htsvd_params *p, void *stream);

/* One image of a batched call. */
typedef struct {
    const uint8_t *d_in;  /* device, uint8 HWC */
    int32_t h, w, c;
    int64_t in_stride;    /* bytes per row */
    float sigma;          /* > 0: known noise level; HTSVD_SIGMA_AUTO: estimated (p->estimator) */
    int32_t K;            /* group size for this image: 0 = p->K; HTSVD_K_AUTO = chosen on the device
                             between 16 and 32 from the image's mean estimated sigma (opts->k_sigma_cutoff) */
    float *d_out;         /* device, float32 HWC */
    int64_t out_stride;   /* elements per row */
} htsvd_image;

#define HTSVD_K_AUTO (-1)

typedef struct {
    int32_t use_graph;      /* 1: capture the launches in a hipGraph; an identical batch replays it */
    int32_t blocks_per_cu;  /* persistent workgroups per compute unit for the work-queue kernels (0 = 1) */
    float k_sigma_cutoff;   /* HTSVD_K_AUTO images whose mean sigma is below this use K = 16, else 32 */
    int32_t tile_side;      /* largest side of a filter reference tile, 0..16 (0 = 16); LDS may cap it lower */
} htsvd_batch_opts;

/* Denoises n images of any sizes (one channel count) with shared method parameters.  Block
 * matching, filtering and aggregation run as persistent kernels that pull (image, tile) units
 * from work queues, so one launch covers the whole batch; with use_graph the whole sequence is
 * captured once in a hipGraph and replayed while the batch (pointers, shapes, sigma, K) and
 * the parameters stay the same.  An HTSVD_K_AUTO image is matched with 32 members; after its
 * noise level is known a device kernel keeps 32 or the first 16 members (the 16 nearest under
 * the same order), so the choice needs no host round trip and stays inside the graph.
 * opts may be NULL (defaults: graph on, 1 block per CU, cutoff 0 = always 32, tile side 16). */
htsvd_status htsvd_denoise_batch(htsvd_ctx *ctx, int32_t n, const htsvd_image *imgs, const htsvd_params *p,
                                 const htsvd_batch_opts *opts, void *stream);

/* State of image `image` (index into the imgs array) of the last htsvd_denoise_batch call on
 * this context, for checking the batched decisions from outside (Algorithm 1 with Eq. 20, 23):
 * *h_K (host, may be NULL): the group size the image was filtered with -- for an HTSVD_K_AUTO
 * image the device's choice (waits for `stream`); d_tau_ref (device, n_ref FP64, may be NULL):
 * the per-reference thresholds the filter applied (for an HTSVD_K_AUTO image that took 16,
 * already scaled to the 16-member multiplier).  It reads the context's workspace, so call it
 * after the batch's work and before any other call that uses the context.
 * HTSVD_ESTATE if no batch has been planned since the workspace last changed. */
htsvd_status htsvd_batch_inspect(htsvd_ctx *ctx, int32_t image, int32_t *h_K, double *d_tau_ref, void *stream);

/* Noise levels (Sec. III-E-1, Eq. 22-23).  Per sub-image (ceil(h/S) * ceil(w/S) tiles,
 * S = p->subimage, row-major): d_sigma_est: sigma_est before the vote (FP64) -- the known level,
 * the plain estimate, or under the learned estimator the tile's judged level (the mean learned
 * sigma of its 8x8 blocks where it lies within a factor 1.5 of the plain estimate, else the
 * plain estimate); d_sigma_hat: after Eq. 23 (FP64, equals d_sigma_est when p->adaptive is 0);
 * d_votes: "adjust" votes per tile (int32).
 * d_sigma_map: the effective noise level per 8x8 block (ceil(h/8) * ceil(w/8), row-major, FP64)
 * -- the sigma that the thresholds tau = sigma * multiplier of the references whose top-left
 * pixel lies in the block use: sigma_hat of the block's tile, or under the learned estimator
 * where the tile accepted the map, exp(z) of the block times the tile's vote factor
 * sigma_hat / sigma_est.
 * sigma > 0 uses the known level as sigma_est.  Any output pointer may be NULL.  All outputs
 * are device buffers owned by the caller. */
htsvd_status htsvd_estimate_sigma(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                                  int64_t in_stride, float sigma, const htsvd_params *p, double *d_sigma_est,
                                  double *d_sigma_hat, int32_t *d_votes, double *d_sigma_map, void *stream);

/* Waits for `stream` and reports deferred device errors. */
htsvd_status htsvd_sync(htsvd_ctx *ctx, void *stream);

/* Message for the last non-OK status of the calling thread ("" if none). */
const char *htsvd_last_error(void);

/* Counters of the last denoise call, copied to the host (synchronises the device):
 * h_count[0] = coefficients re-decided in FP64 because they fell within the guard band of
 * tau, h_count[1] = near-threshold coefficients beyond the per-group FP64 list (decided in
 * FP32).  h_count must hold 2 values. */
htsvd_status htsvd_last_guard_count(htsvd_ctx *ctx, int64_t *h_count);

/* ---- Learned noise-level network (replaces the paper's CNN estimator, Sec. III-E-1) ----
 * Six 3x3 convolutions, 32 channels, ReLU: C->32 stride 2, 32->32 stride 2, 32->32 stride 2,
 * 32->32, 32->32, 32->1; the output z is log(sigma) (0..255 scale) for every 8x8 block, i.e.
 * a ceil(h/8) x ceil(w/8) map.  Input normalisation (u8 - 128) / 64.  Weights are kept in
 * FP32 (master copy and Adam moments) and used in bf16; activations are bf16 with FP32
 * accumulation.  Parameter layout: per layer w[co][ky][kx][ci] then b[co]. */
int32_t htsvd_cnn_param_count(int32_t c);
/* He-normal weights from a counter-based generator of `seed`, zero biases (last bias log 20),
 * Adam state and step counter reset.  Makes c (1 or 3) the network's channel count. */
htsvd_status htsvd_cnn_init(htsvd_ctx *ctx, int32_t c, uint64_t seed);
/* Host FP32 parameters in, n = htsvd_cnn_param_count(c); resets Adam state. */
htsvd_status htsvd_cnn_set_weights(htsvd_ctx *ctx, int32_t c, const float *h_params, int64_t n);
/* Host FP32 master parameters out (synchronises the device). */
htsvd_status htsvd_cnn_get_weights(htsvd_ctx *ctx, float *h_params, int64_t n);
/* Inference on one image: d_log_sigma = ceil(h/8)*ceil(w/8) floats, row-major. */
htsvd_status htsvd_cnn_forward(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, float *d_log_sigma, void *stream);
/* Forward and backward on a batch of n crops (device, contiguous NHWC u8, each h x w x c) with
 * per-block targets d_target_log (n * ceil(h/8) * ceil(w/8) floats, log sigma): mean absolute
 * error in *h_loss (synchronises; may be NULL) and its gradient in d_grad (device, FP32,
 * htsvd_cnn_param_count(c) values). */
htsvd_status htsvd_cnn_gradients(htsvd_ctx *ctx, const uint8_t *d_crops, int32_t n, int32_t h, int32_t w,
                                 int32_t c, const float *d_target_log, float *d_grad, double *h_loss, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on a batch, as above. */
htsvd_status htsvd_cnn_train_step(htsvd_ctx *ctx, const uint8_t *d_crops, int32_t n, int32_t h, int32_t w,
                                  int32_t c, const float *d_target_log, float lr, double *h_loss, void *stream);
/* Checkpoint: parameters, Adam moments and the step counter (binary file). */
htsvd_status htsvd_cnn_save(htsvd_ctx *ctx, const char *path);
htsvd_status htsvd_cnn_load(htsvd_ctx *ctx, const char *path);

/* Stage timing.  With timing enabled each call records a HIP event pair around each of its
 * stages on its stream; htsvd_stage_times() waits for the pending pairs and returns, per
 * stage, the summed milliseconds and the number of timed calls since htsvd_set_timing().
 * h_ms (and h_calls if not NULL) must hold HTSVD_N_STAGES values. */
enum {
    HTSVD_STAGE_BM = 0,        /* grouping (block matching + top-K) */
    HTSVD_STAGE_CLEAR = 1,     /* clearing the accumulators */
    HTSVD_STAGE_FILTER = 2,    /* transform, threshold, inverse, aggregation */
    HTSVD_STAGE_NORMALIZE = 3, /* division by the patch counts */
    HTSVD_STAGE_SIGMA = 4,     /* noise estimation (plain or learned) and the vote */
    HTSVD_N_STAGES = 5
};
htsvd_status htsvd_set_timing(htsvd_ctx *ctx, int32_t enable);
htsvd_status htsvd_stage_times(htsvd_ctx *ctx, double *h_ms, int64_t *h_calls);

#ifdef __cplusplus
}
#endif

#endif /* HTSVD_H */
