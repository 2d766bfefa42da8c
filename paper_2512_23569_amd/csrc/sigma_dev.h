// Per-tile and per-reference noise-level arithmetic shared by the one-image kernels and the
// batched kernels (same code, hence bit-identical results on both paths).
#pragma once

#include <math.h>

#include "common.h"

namespace htsvd {

// Image-level sigma from the per-channel sigma^2 of one sub-image: sqrt(mean_c sigma_c^2).
__device__ inline double combine_sigma_tile(const double *sigma2, int c, int t) {
    double s = 0.0;
    for (int ch = 0; ch < c; ++ch) s += sigma2[t * c + ch];
    s /= (double)c;
    return s > 0.0 ? sqrt(s) : 0.0;
}

// The learned map judged on sub-image t: the mean learned sigma over the tile's 8x8 blocks is
// kept when it lies within a factor `bound` of the plain estimate sp on either side
// (sp / bound <= mean <= bound * sp, both products in FP64; finite, positive), else the plain
// estimate stands in.  Returns the sigma the tile then stands for; *use_plain says which.
__device__ inline double judge_tile(const ImageGeom &g, int tile, int t, const float *zmap, double sp,
                                    double bound, int32_t *use_plain) {
    const int ntx = (g.w + tile - 1) / tile;
    const int hb = (g.h + PS - 1) / PS, wb = (g.w + PS - 1) / PS, bpt = tile / PS;
    const int ty = t / ntx, tx = t % ntx;
    double sum = 0.0;
    int n = 0;
    for (int by = ty * bpt; by < min(hb, (ty + 1) * bpt); ++by)
        for (int bx = tx * bpt; bx < min(wb, (tx + 1) * bpt); ++bx) {
            sum += exp((double)zmap[by * wb + bx]);
            ++n;
        }
    const double mean = n > 0 ? sum / n : 0.0;
    const bool ok = isfinite(mean) && mean > 0.0 && sp > 0.0 && mean <= bound * sp && mean * bound >= sp;
    *use_plain = ok ? 0 : 1;
    return ok ? mean : sp;
}

// Sub-image holding the top-left pixel of reference r.
__device__ inline int ref_tile(const ImageGeom &g, int tile, int64_t r, int *y, int *x) {
    const int iy = (int)(r / g.nx), ix = (int)(r % g.nx);
    *y = ref_pos(iy, g.ny, g.h, g.s);
    *x = ref_pos(ix, g.nx, g.w, g.s);
    const int ntx = (g.w + tile - 1) / tile;
    return (*y / tile) * ntx + *x / tile;
}

// Effective noise level of the 8x8 block (by, bx), which lies in sub-image t: under the learned
// map, the block's learned sigma scaled by its tile's vote (sigma_hat / sigma_est), or the
// tile's plain sigma_hat where the judge rejected the map (zmap == nullptr: sigma_hat).
__device__ inline double block_sigma(const ImageGeom &g, int t, int by, int bx, const float *zmap,
                                     const int32_t *use_plain, const double *sigma_est, const double *sigma_hat) {
    if (!zmap || use_plain[t]) return sigma_hat[t];
    const int wb = (g.w + PS - 1) / PS;
    return exp((double)zmap[by * wb + bx]) * (sigma_hat[t] / sigma_est[t]);
}

// Noise level of reference r under the learned map: that of the 8x8 block holding its top-left
// pixel (block_sigma).
__device__ inline double learned_ref_sigma(const ImageGeom &g, int tile, int64_t r, const float *zmap,
                                           const int32_t *use_plain, const double *sigma_est,
                                           const double *sigma_hat) {
    int y, x;
    const int t = ref_tile(g, tile, r, &y, &x);
    return block_sigma(g, t, y / PS, x / PS, zmap, use_plain, sigma_est, sigma_hat);
}

}  // namespace htsvd
