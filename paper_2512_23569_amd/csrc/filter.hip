// Aggregation regions and the gather (normalisation) of Algorithm 1, and the tiling of the
// reference grid for the filter kernel (filter_mfma.hip).
//
// The filter processes the references of a T x T tile in one workgroup and adds every
// reconstructed patch into an LDS copy of the image region those references' groups can reach
// (their search windows plus the patch extent).  The region is written, without atomics, to the
// tile's own slot of a global buffer as C + 1 planes: the channel sums and the number of patches
// covering each pixel.  The gather kernel then sums, for every pixel, the (at most a few)
// regions covering it and divides (uniform weights, "average" aggregation); a pixel no patch
// covers keeps its noisy value.
#include "common.h"

namespace htsvd {
namespace {

// out = (sum of the regions covering the pixel) / (their count); noisy value where no patch landed.
template <int C>
__device__ __forceinline__ void gather_px(const ImageGeom &g, const TileGeom &tg, const float *__restrict__ regions,
                                          float *__restrict__ out, int64_t out_stride, int64_t e) {
    constexpr int CH = C + 1;
    const int y = (int)(e / g.w), x = (int)(e % g.w);
    const int span_y = tg.TY * g.s, span_x = tg.TX * g.s;
    const int ty_lo = max(0, (y - tg.R - PS - span_y) / span_y - 1);
    const int ty_hi = min(tg.tiles_y - 1, (y + tg.R) / span_y + 1);
    const int tx_lo = max(0, (x - tg.R - PS - span_x) / span_x - 1);
    const int tx_hi = min(tg.tiles_x - 1, (x + tg.R) / span_x + 1);
    float acc[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) acc[k] = 0.f;
    const int plane = region_plane(tg), elems = region_elems(tg, C);
    for (int ty = ty_lo; ty <= ty_hi; ++ty) {
        int r0, r1;
        region_rows(g, tg, ty, &r0, &r1);
        if (y < r0 || y > r1) continue;
        for (int tx = tx_lo; tx <= tx_hi; ++tx) {
            int c0, c1;
            region_cols(g, tg, tx, &c0, &c1);
            if (x < c0 || x > c1) continue;
            const float *src = regions + (int64_t)(ty * tg.tiles_x + tx) * elems + (y - r0) * tg.RP + (x - c0);
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[k] += src[k * plane];
        }
    }
    float *o = out + (int64_t)y * out_stride + (int64_t)x * C;
    const uint8_t *px = g.img + (int64_t)y * g.stride + (int64_t)x * C;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) o[ch] = acc[C] > 0.f ? acc[ch] / acc[C] : (float)px[ch];
}

template <int C>
__global__ void gather_kernel(ImageGeom g, TileGeom tg, const float *__restrict__ regions, float *__restrict__ out,
                              int64_t out_stride) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)g.h * g.w) return;
    gather_px<C>(g, tg, regions, out, out_stride, e);
}

// All pixels of all images of a batch; pix_start holds the prefix sums of the pixel counts.
template <int C>
__global__ void gather_kernel_batched(const BatchItem *__restrict__ items, int n_items,
                                      const int *__restrict__ pix_start) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pix_start[n_items]) return;
    const int i = find_unit(pix_start, n_items, e);
    const BatchItem &it = items[i];
    const bool alt = it.ksel && *it.ksel == it.k_alt;
    gather_px<C>(it.g, alt ? it.tg_alt : it.tg, it.regions, it.out, it.out_stride, e - pix_start[i]);
}

// Smallest pitch >= w with pitch % 16 == 8: four consecutive rows then start 8 banks apart
// (mod 32), so the 4 x 8 pixels one half-wave adds to hit distinct banks.
int region_pitch(int w) { return w + ((8 - w % 16) + 16) % 16; }

// Largest reference tile (side <= max_side) whose region and the filter's other buffers fit in LDS.
TileGeom plan_tiles(const ImageGeom &g, int W, int lds_budget, int max_side) {
    TileGeom tg;
    tg.FS = 0;
    tg.R = (W - 1) / 2;
    const int CH = g.c + 1;
    const int other = filter_mfma_group_bytes(g.c);
    int T = max(1, min(16, max_side));
    for (; T > 1; --T) {
        const int RH = min((T - 1) * g.s + 2 * tg.R + PS, g.h);
        const int RW = min((T - 1) * g.s + 2 * tg.R + PS, g.w);
        if (CH * RH * region_pitch(RW) * 4 + other <= lds_budget) break;
    }
    tg.TY = tg.TX = T;
    tg.RH = min((T - 1) * g.s + 2 * tg.R + PS, g.h);
    tg.RW = min((T - 1) * g.s + 2 * tg.R + PS, g.w);
    tg.RP = region_pitch(tg.RW);
    tg.tiles_y = (g.ny + T - 1) / T;
    tg.tiles_x = (g.nx + T - 1) / T;
    return tg;
}

}  // namespace

int filter_lds_budget() { return 160 * 1024 - filter_mfma_static_bytes() - 64; }

int filter_lds_bytes_for(const TileGeom &tg, int C, int K) {
    (void)K;
    return filter_mfma_lds_bytes(tg, C);
}

// Fixed-point shift of the region sums: a pixel of a tile's region receives at most T^2 K
// contributions (every member of every group of the tile), each clamped to |v| <= 1024, so
// T^2 K 1024 2^FS must stay below 2^31.  Tiles are capped so that FS >= 9: a contribution
// is rounded by at most 2^-10, and so is the average of a pixel's contributions.  FS <= 12
// keeps every scaled contribution below 2^22, the range of the filter's rounding by
// addition of 1.5 * 2^23.
constexpr double FX_CLAMP = 1024.0;
constexpr int FX_MIN_SHIFT = 9;
constexpr int FX_MAX_SHIFT = 12;

int accumulation_shift(int T, int K) {
    const double worst = (double)T * T * K * FX_CLAMP;
    int fs = 0;
    while (fs < FX_MAX_SHIFT && worst * (double)(1 << (fs + 1)) < 2147483647.0) ++fs;
    return fs;
}

TileGeom plan_filter_tiles(const ImageGeom &g, int W, int K, int max_side) {
    int side = max_side > 0 ? max_side : 16;
    while (side > 1 && accumulation_shift(side, K) < FX_MIN_SHIFT) --side;
    TileGeom tg = plan_tiles(g, W, filter_lds_budget(), side);
    tg.FS = accumulation_shift(tg.TY, K);
    return tg;
}

size_t filter_region_bytes(const ImageGeom &g, int W, int K) {
    const TileGeom tg = plan_filter_tiles(g, W, K, 0);
    return (size_t)tg.tiles_y * tg.tiles_x * region_elems(tg, g.c) * sizeof(float);
}

hipError_t launch_filter_batched(int C, int K, const BatchItem *items, int n_items, const int *unit_start, int lds,
                                 const BasisDev &b, unsigned long long *gc, int *queue, int grid, hipStream_t st) {
    return launch_filter_mfma_batched(C, K, items, n_items, unit_start, lds, b, gc, queue, grid, st);
}

hipError_t launch_gather_batched(int C, const BatchItem *items, int n_items, const int *pix_start, int total_px,
                                 hipStream_t st) {
    const unsigned grid = (unsigned)((total_px + 255) / 256);
    if (C == 3)
        hipLaunchKernelGGL(gather_kernel_batched<3>, dim3(grid), dim3(256), 0, st, items, n_items, pix_start);
    else
        hipLaunchKernelGGL(gather_kernel_batched<1>, dim3(grid), dim3(256), 0, st, items, n_items, pix_start);
    return hipGetLastError();
}

hipError_t launch_filter(const ImageGeom &g, int W, int K, const BasisDev &b, const int32_t *idx,
                         const double *tau_ref, float *regions, unsigned long long *gc, float *out, int64_t out_stride,
                         hipStream_t st, bool gather, const float *ra_d, const uint8_t *ra_flag) {
    const TileGeom tg = plan_filter_tiles(g, W, K, 0);
    if (!gather) return launch_filter_mfma(g, tg, K, b, idx, tau_ref, regions, gc, st, ra_d, ra_flag);
    const int64_t n = (int64_t)g.h * g.w;
    if (g.c == 3)
        hipLaunchKernelGGL(gather_kernel<3>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, tg, regions, out,
                           out_stride);
    else
        hipLaunchKernelGGL(gather_kernel<1>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, tg, regions, out,
                           out_stride);
    return hipGetLastError();
}

}  // namespace htsvd
