// Internal declarations shared by the HIP translation units of libhtsvd.
// Not part of the public ABI (include/htsvd.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace htsvd {

constexpr int PS = 8;             // patch side (Sec. IV-A); the kernels are written for 8
constexpr int MAX_WINDOW = 31;    // largest supported odd search-window side
constexpr int MAX_BANDS = 64;     // largest band count of the hyperspectral path
constexpr int MAX_CAND = MAX_WINDOW * MAX_WINDOW;
constexpr int REF_TILE = 4;       // references per tile side in block matching (4 x 4 = 16 = MFMA M)
constexpr int MAX_UNION = 64;     // largest union of search windows per tile side (candidates)

// Geometry of one image and its reference grid.
struct ImageGeom {
    const uint8_t *img;  // HWC uint8
    int64_t stride;      // bytes per row
    int h, w, c;
    int ny, nx;          // reference grid size
    int s;               // grid step
};

// Method parameters after validation.
struct MethodParams {
    int W, K, gnum, gden;
};

// Basis constants for the FP32 transform (device memory):
//   c = 3: U0, V0 (slice f=0, real 8x8), U1r, U1i, V1r, V1i (slice f=1, complex 8x8),
//          row-major [row][col]; slice f=2 is the conjugate of f=1.
//   c = 1: U0, V0 only.
// Plus the FP64 matrix T (P x P, P = 64c) with s = T g for one patch in slice-major
// vector form, used to re-decide coefficients near the threshold.
struct BasisDev {
    float *f32;        // 6*64 floats
    double *T64;       // P*P doubles
    const void *frag;  // MFMA operand fragments of the per-slice transform matrices (fp16 hi/lo)
};

// Maps of the t-product along B bands (bands.hip): the real band DFT D (rows Re0, Re1, Im1, ...,
// and Re(B/2) last for even B; D[c*nb + b]) and its inverse Dinv (Dinv[b*nb + c]), both nb x nb
// with zeros beyond B, and per frequency f <= B/2 the v_mfma_f64_16x16x4f64 operands of the two
// slice products of each direction (forward U_hat_f^H * P * V_hat_f, inverse U_hat_f * S *
// V_hat_f^H) in their real 16 x 16 embeddings: frag[f*512 + s*64 + lane] is the left factor's A
// operand of k-step s (s < 4) and the right factor's B operand of k-step s - 4 (s >= 4).
struct BandMaps {
    const double *D = nullptr, *Dinv = nullptr, *frag_fwd = nullptr, *frag_inv = nullptr;
    int nb = 32;
};
// Padded band count of the band kernels: 32 for B <= 32, else 64.
inline int band_nb(int B) { return B <= 32 ? 32 : 64; }

// Device copy of the RA-Haar-tSVD refinement network for inference (ra.hip).
struct RaWeightsDev {
    const void *frag = nullptr;     // fp16 hi/lo operand fragments of W1, W2, W3
    const void *frag3t = nullptr;   // of 128 T W3 (the last layer folded with the patch transform)
    const float *bias = nullptr;    // b1, b2, b3
    const float *bias3t = nullptr;  // 128 T b3
};

// Reference tiles of the filter kernel and the image regions their groups reach.
struct TileGeom {
    int TY, TX;          // references per tile
    int tiles_y, tiles_x;
    int RH, RW;          // region capacity (rows, cols) per tile
    int RP;              // row pitch of a region plane in floats (>= RW, RP % 16 == 8)
    int FS;              // fixed-point shift of the LDS accumulation (sums in int32 units of 2^-FS)
    int R;               // search radius (W-1)/2
};

// A tile's region is C + 1 planes of RH x RP floats: the channel sums, then the number of
// patches covering each pixel.  Planar, with the pitch chosen so that the 4 x 8 pixels of a
// patch half fall on 32 distinct LDS banks.  In LDS the planes hold int32 (fixed point for the
// sums, see FS); the global copy is float.
__host__ __device__ inline int region_plane(const TileGeom &tg) { return tg.RH * tg.RP; }
__host__ __device__ inline int region_elems(const TileGeom &tg, int C) { return (C + 1) * tg.RH * tg.RP; }

// One image of a batched call, as the persistent kernels see it.
struct BatchItem {
    ImageGeom g;
    MethodParams mp;
    TileGeom tg;
    int bm_tiles_x;
    int32_t *idx;          // groups, n_ref * idx_stride (the first mp.K of each row are used)
    const double *tau;     // thresholds, n_ref
    float *regions;        // per-tile regions of the filter
    float *out;            // output image
    int64_t out_stride;
    int idx_stride;        // members stored per reference (>= mp.K)
    double tau_mul;        // factor applied to tau (threshold multiplier of this K over the stored one)
    const int *ksel;       // device: this image's entry of the chosen group sizes (nullptr: fixed mp.K)
    int k_alt;             // the other group size the image may take, and its tiling
    TileGeom tg_alt;
};

// One image of the batched noise-level stages (sub-images of side `tile`, Sec. III-E-1).
enum SigmaMode { SIGMA_KNOWN = 0, SIGMA_PLAIN = 1, SIGMA_LEARNED = 2 };
struct SigmaItem {
    ImageGeom g;
    int K;                  // members per stored group
    const int *ksel;        // group size chosen on the device (auto images; the vote reads the first
                            // *ksel members of each group), or nullptr: the vote reads all K
    int mode;               // SigmaMode
    int adaptive;           // Eq. 22-23 vote on
    int n_tiles;            // sub-images
    double sigma;           // known sigma (SIGMA_KNOWN)
    double mult;            // threshold multiplier: tau = mult * sigma
    const int32_t *idx;     // groups, n_ref * K
    double *tau;            // per-reference thresholds (written)
    double *sig_est, *sig_hat, *cov, *sig_plain;   // per sub-image (cov: c per sub-image)
    int32_t *votes, *use_plain;
    const float *zmap;      // learned log-sigma per 8x8 block (SIGMA_LEARNED)
};

// Index i of the unit range [start[i], start[i+1]) holding u (start has n+1 entries).
__device__ inline int find_unit(const int *start, int n, int u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Value of v in lane (lane ^ j) for j = 1, 2, 4, 8, 16, 32, by register moves between lanes
// (DPP within a row of 16 lanes, the row-swap instructions across rows), no LDS round trip.
//   j = 1, 2: quad permutations; j = 4, 8: row shift left (lane i reads i + j) for lanes with
//   bit j clear, row shift right (reads i - j) for the others; j = 16, 32: permlane swaps.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int j, int lane) {
    if (j == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);   // [1,0,3,2]
    if (j == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);   // [2,3,0,1]
    if (j == 4) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x104, 0xF, 0xF, true);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x114, 0xF, 0xF, true);
        return (lane & 4) ? dn : up;
    }
    if (j == 8) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x108, 0xF, 0xF, true);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x118, 0xF, 0xF, true);
        return (lane & 8) ? dn : up;
    }
    if (j == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? r[0] : r[1];
}

// Value of v in lane lane ^ (k - 1), k = 2, 4, ..., 64: the mirror image of the lane within its
// aligned block of k lanes (quad permutations, the half-row and row mirrors of DPP, then the
// row swaps for the blocks of 32 and 64).
__device__ __forceinline__ uint32_t mirror_lane(uint32_t v, int k, int lane) {
    if (k == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);   // [1,0,3,2]
    if (k == 4) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x1B, 0xF, 0xF, true);   // [3,2,1,0]
    if (k == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);  // half-row mirror
    const uint32_t m = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true);  // row mirror: ^15
    if (k == 16) return m;
    const uint32_t m2 = xor_lane(m, 16, lane);   // lane ^ 31
    if (k == 32) return m2;
    return xor_lane(m2, 32, lane);               // lane ^ 63
}

// Ascending sort of one key per lane across the 64 lanes (bitonic network in the form whose
// every comparator is ascending: each merge of two sorted halves of a block of k lanes starts
// with lane i against its mirror i ^ (k - 1), then half-cleaners i ^ j; the lower lane of a
// pair keeps the minimum).  T is uint32_t or uint64_t.
template <typename T>
__device__ __forceinline__ T lane_exchange(T v, int k_or_j, int lane, bool mirror) {
    if constexpr (sizeof(T) == 4) {
        return mirror ? mirror_lane(v, k_or_j, lane) : xor_lane(v, k_or_j, lane);
    } else {
        const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        const uint32_t plo = mirror ? mirror_lane(lo, k_or_j, lane) : xor_lane(lo, k_or_j, lane);
        const uint32_t phi = mirror ? mirror_lane(hi, k_or_j, lane) : xor_lane(hi, k_or_j, lane);
        return ((uint64_t)phi << 32) | plo;
    }
}

template <typename T>
__device__ inline T wave_sort_asc(T v, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
        {
            const T p = lane_exchange<T>(v, k, lane, true);
            v = (lane & (k >> 1)) ? (v < p ? p : v) : (p < v ? p : v);
        }
#pragma unroll
        for (int j = k >> 2; j > 0; j >>= 1) {
            const T p = lane_exchange<T>(v, j, lane, false);
            v = (lane & j) ? (v < p ? p : v) : (p < v ? p : v);
        }
    }
    return v;
}

// Value of v in lane l (l uniform over the wavefront), as a scalar.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l), hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Reference position along one side: 0, s, 2s, ... and the last position n-ps.
__host__ __device__ inline int ref_pos(int i, int n_ref, int n, int s) {
    return (i == n_ref - 1) ? (n - PS) : i * s;
}

__host__ __device__ inline int ref_count(int n, int s) {
    if (n < PS || s < 1) return 0;
    int c = (n - PS) / s + 1;
    if ((n - PS) % s) c += 1;
    return c;
}

// Image rows / columns reached by the groups of reference tile (ty, tx): the references'
// window reach plus the patch extent, clipped to the image.
__device__ __host__ inline void region_rows(const ImageGeom &g, const TileGeom &tg, int ty, int *r0, int *r1) {
    const int i0 = ty * tg.TY;
    const int i1 = min(i0 + tg.TY, g.ny) - 1;
    *r0 = max(0, ref_pos(i0, g.ny, g.h, g.s) - tg.R);
    *r1 = min(g.h - 1, ref_pos(i1, g.ny, g.h, g.s) + tg.R + PS - 1);
}

__device__ __host__ inline void region_cols(const ImageGeom &g, const TileGeom &tg, int tx, int *c0, int *c1) {
    const int i0 = tx * tg.TX;
    const int i1 = min(i0 + tg.TX, g.nx) - 1;
    *c0 = max(0, ref_pos(i0, g.nx, g.w, g.s) - tg.R);
    *c1 = min(g.w - 1, ref_pos(i1, g.nx, g.w, g.s) + tg.R + PS - 1);
}

// Makes `bytes` of dynamic LDS available to `kernel` (static LDS comes on top); fails with
// hipErrorInvalidValue if the device cannot give a workgroup that much.
hipError_t prepare_dynamic_lds(const void *kernel, int bytes, int static_bytes);

// Launchers (stream-ordered, no synchronisation).
hipError_t launch_block_match(const ImageGeom &g, const MethodParams &mp, int32_t *idx, int32_t *dist,
                              hipStream_t st);
hipError_t launch_block_match_video(const ImageGeom &g, const MethodParams &mp, int T, int radius, int32_t *idx,
                                    int32_t *dist, hipStream_t st);
hipError_t launch_fill_tau(double *tau_ref, int64_t n_ref, const double *sigma_tile, double sigma_const,
                           double mult, const ImageGeom &g, int tile, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// out[r*kout + k] = in[r*kin + k] for k < kout <= kin.
hipError_t launch_idx_prefix(const int32_t *in, int kin, int32_t *out, int kout, int64_t n_ref, hipStream_t st);

// Noise estimation (plain): per sub-image covariance eigenvalues and the tail rule.
// mom: sigma_mom_ints() int32 per (sub-image, channel) of scratch; cov_work: c doubles per sub-image.
int sigma_mom_ints();
// The per-(sub-image, channel) noise variances of units unit0 .. unit0 + n_units - 1 (unit
// t*c + ch) into sigma2[0 .. n_units); mom holds n_units * sigma_mom_ints() int32.
hipError_t launch_sigma2_units(const ImageGeom &g, int tile, int unit0, int n_units, int32_t *mom, double *sigma2,
                               hipStream_t st);
hipError_t launch_sigma_est(const ImageGeom &g, int tile, int32_t *mom, double *cov_work, double *sigma_est,
                            hipStream_t st);
hipError_t launch_vote(const ImageGeom &g, const MethodParams &mp, const int32_t *idx, int tile, int n_vote,
                       uint64_t seed, int gamma_rank, double beta, const double *sigma_est, double *sigma_hat,
                       int32_t *votes, hipStream_t st);

// ---- batched (persistent, work-queue) forms ----
hipError_t launch_block_match_batched(const BatchItem *items, int n_items, const int *unit_start, int max_s,
                                      int max_W, int max_h, int max_w, int *queue, int grid, hipStream_t st);
hipError_t launch_filter_batched(int C, int K, const BatchItem *items, int n_items, const int *unit_start, int lds,
                                 const BasisDev &b, unsigned long long *gc, int *queue, int grid, hipStream_t st);
hipError_t launch_gather_batched(int C, const BatchItem *items, int n_items, const int *pix_start, int total_px,
                                 hipStream_t st);
int select_k_chunks(int64_t max_refs);
hipError_t launch_select_k(const BatchItem *items, const int *auto_list, int n_auto, int n_chunk, double *partial,
                           const double *mult, double cutoff, int *ksel, hipStream_t st);
hipError_t launch_fill_tau_batched(const BatchItem *items, int n_items, const int *ref_start, int total_refs,
                                   const double *sigma, const double *mult, hipStream_t st);
// Reference tiling of the filter: the largest square tile (side <= max_side, 0 = 16) whose
// region and group buffers fit in LDS.
TileGeom plan_filter_tiles(const ImageGeom &g, int W, int K, int max_side);
int filter_lds_bytes_for(const TileGeom &tg, int C, int K);
// matrix-core filter (filter_mfma.hip)
int filter_mfma_lds_bytes(const TileGeom &tg, int C);
int filter_mfma_group_bytes(int C);  // LDS besides the region
int filter_mfma_static_bytes();
// ra_d (n_ref x 64C, may be NULL) and ra_flag (n_ref): RA-Haar-tSVD corrections of the first Haar
// row, applied to the groups whose flag is set.
hipError_t launch_filter_mfma(const ImageGeom &g, const TileGeom &tg, int K, const BasisDev &b, const int32_t *idx,
                              const double *tau_ref, float *regions, unsigned long long *gc, hipStream_t st,
                              const float *ra_d = nullptr, const uint8_t *ra_flag = nullptr);
size_t filter_mfma_global_bytes(const ImageGeom &g, int T, int radius, int W, int K, bool force_direct = false);
hipError_t launch_filter_mfma_global(const ImageGeom &g, int T, int radius, int W, int K, const BasisDev &b,
                                     const int32_t *idx, const double *tau_ref, void *accum, int *ghist,
                                     unsigned long long *gc, float *out, int64_t out_stride, hipStream_t st,
                                     const float *ra_d = nullptr, const uint8_t *ra_flag = nullptr,
                                     bool force_direct = false);
hipError_t launch_filter_mfma_batched(int C, int K, const BatchItem *items, int n_items, const int *unit_start,
                                      int lds, const BasisDev &b, unsigned long long *gc, int *queue, int grid,
                                      hipStream_t st);
int filter_lds_budget();

// ---- learned noise-level network ----
void cnn_layout(int c, int *w_off, int *b_off, int *total);
size_t cnn_act_elems(int l, int N, int H, int W, int c);   // elements of activation l (1..6)
struct CnnBuffers {
    const float *wq;      // bf16-rounded weights as FP32
    const uint16_t *wbf;  // bf16 weights
    uint16_t *act[6];     // act[1..5], NHWC bf16, 32 channels
    float *z;             // layer-6 output (log sigma per block)
};
hipError_t cnn_forward(const CnnBuffers &b, const uint8_t *img, int64_t img_stride, int64_t img_batch_stride,
                       int N, int H, int W, int c, hipStream_t st);
// The same for N images of one size in separate buffers: image n at img_tab[n] (device table),
// row stride stride_tab[n]; the outputs of image n follow those of image n - 1 in b.z.
hipError_t cnn_forward_tab(const CnnBuffers &b, const uint8_t *const *img_tab, const int64_t *stride_tab, int N,
                           int H, int W, int c, hipStream_t st);
hipError_t cnn_backward(const CnnBuffers &b, const uint8_t *img, int64_t img_stride, int64_t img_batch_stride,
                        int N, int H, int W, int c, const float *target, float *grads, float *d0, float *d1,
                        double *loss_sum, hipStream_t st);
hipError_t cnn_adam(float *w, float *m, float *v, const float *g, int n, float lr, int64_t step, float *wq,
                    uint16_t *wbf, hipStream_t st);
hipError_t cnn_quantize(const float *w, int n, float *wq, uint16_t *wbf, hipStream_t st);

// Batched noise-level stages.  Each launch walks a list of items: sel[j] is the item of list
// entry j, start[j] .. start[j+1] its units (sub-images x channels for the covariance stage,
// sub-images for the tile and vote stages, references for the thresholds).
hipError_t launch_sigma_est_batched(const SigmaItem *items, const int *sel, const int *start, int n, int total,
                                    int tile, int32_t *mom, hipStream_t st);   // mom: total units of scratch
hipError_t launch_sigma_tiles_batched(const SigmaItem *items, const int *sel, const int *start, int n, int total,
                                      int tile, double ratio_bound, hipStream_t st);
hipError_t launch_vote_batched(int K, const SigmaItem *items, const int *sel, const int *start, int n, int total,
                               int tile, int n_vote, uint64_t seed, int gamma_rank, double beta, hipStream_t st);
hipError_t launch_fill_tau_sigma_batched(const SigmaItem *items, const int *sel, const int *start, int n,
                                         int total, int tile, hipStream_t st);

// Learned sigma map -> thresholds: per-tile judge against the plain estimate, per-reference tau.
hipError_t launch_learned_judge(const ImageGeom &g, int tile, const float *zmap, const double *sigma_plain,
                                double ratio_bound, int32_t *use_plain, double *sigma_tile, hipStream_t st);
hipError_t launch_fill_tau_learned(double *tau, const ImageGeom &g, int tile, const float *zmap,
                                   const int32_t *use_plain, const double *sigma_est, const double *sigma_hat,
                                   double mult, hipStream_t st);
// Effective sigma of every 8x8 block (the sigma the thresholds of references with their top-left
// pixel in the block use): block_sigma over ceil(h/8) x ceil(w/8) blocks; zmap may be NULL.
hipError_t launch_sigma_map(double *map, const ImageGeom &g, int tile, const float *zmap, const int32_t *use_plain,
                            const double *sigma_est, const double *sigma_hat, hipStream_t st);
// out[r] = tau[r] * (ksel && *ksel == k_alt ? mul_alt : 1): the thresholds a batched image was
// filtered with, after the device's group-size choice.
hipError_t launch_scale_tau(const double *tau, double *out, int64_t n, const int *ksel, int k_alt, double mul_alt,
                            hipStream_t st);

// Hyperspectral tube patches (bands.hip).
hipError_t launch_band_guide(const uint8_t *cube, int64_t stride, int h, int w, int B, uint8_t *guide, hipStream_t st);
hipError_t launch_select_bands(const float *alt, int64_t alt_stride, const uint8_t *sel, int h, int w, int B,
                               float *out, int64_t out_stride, hipStream_t st);
// The filter works in chunks of groups whose FP64 patch matrices stay below cap bytes each.
size_t band_ws_bytes(int h, int w, int B, int K, int64_t n_group, int64_t cap);
hipError_t launch_band_filter(const BandMaps &bm, const uint8_t *cube, int64_t stride, int h, int w, int B,
                              const int32_t *idx, int64_t n_group, int K, double tau, int64_t cap, void *ws,
                              float *out, int64_t out_stride, hipStream_t st);

// RA-Haar-tSVD refinement network (ra.hip).
int ra_hidden(int c);
int ra_param_count(int c);
size_t ra_frag_halves(int c);    // fp16 values of the W1, W2, W3 fragment tables (hi and lo)
hipError_t launch_ra_means(const uint8_t *img, int64_t stride, int h, int w, int c, const int32_t *idx,
                           int idx_stride, int K, int64_t n_ref, float *out, hipStream_t st);
// Network output for n inputs: from mean patches (means) or from groups (img, idx, K; then
// flags[r] = tau[r] / mult > sigma_min when flags is not NULL).  folded: the last layer gives
// 128 T r (the first-Haar-row correction), else r.
hipError_t launch_ra_forward(int c, const RaWeightsDev &wd, bool folded, const float *means, const uint8_t *img,
                             int64_t stride, int h, int w, const int32_t *idx, int idx_stride, int K, int64_t n,
                             const double *tau, double mult, double sigma_min, uint8_t *flags, float *out,
                             hipStream_t st);
size_t ra_train_ws_floats(int c, int n);
hipError_t ra_gradients(int c, const float *w, const float *noisy, const float *clean, int n, float *grad,
                        float *ws, double *partial, int *n_partial, hipStream_t st);
hipError_t ra_adam(float *w, float *m, float *v, const float *g, int n, float lr, int64_t step, hipStream_t st);

// Channel Gram sums of the reference patches (rows, then columns) into out[2][c][c][8][8].
hipError_t launch_gram(const uint8_t *img, int64_t stride, int h, int w, int c, int s, int64_t *out, hipStream_t st);

}  // namespace htsvd
