// Small utility kernels: buffer clearing and per-reference thresholds.
#include "common.h"

namespace htsvd {
namespace {

__global__ void zero_rows_kernel(float *p, int64_t rows, int64_t cols, int64_t stride) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    p[(e / cols) * stride + e % cols] = 0.f;
}

__global__ void zero_words_kernel(uint32_t *p, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0u;
}

__global__ void fill_tau_kernel(double *tau, int64_t n_ref, const double *sigma_tile, double sigma_const,
                                double mult, ImageGeom g, int tile) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_ref) return;
    double s = sigma_const;
    if (sigma_tile) {
        const int iy = (int)(r / g.nx), ix = (int)(r % g.nx);
        const int y = ref_pos(iy, g.ny, g.h, g.s), x = ref_pos(ix, g.nx, g.w, g.s);
        const int ntx = (g.w + tile - 1) / tile;
        s = sigma_tile[(y / tile) * ntx + x / tile];
    }
    tau[r] = s * mult;
}

// Per sub-image: the mean of the learned sigma over the tile's 8x8 blocks is compared with the
// plain estimate; the plain value replaces the learned map where they differ by more than
// ratio_bound (or the map is not finite).  sigma_tile = the value the tile then stands for.
__global__ void learned_judge_kernel(ImageGeom g, int tile, const float *zmap, const double *sigma_plain,
                                     double log_bound, int32_t *use_plain, double *sigma_tile) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntx = (g.w + tile - 1) / tile, nty = (g.h + tile - 1) / tile;
    if (t >= ntx * nty) return;
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
    const double sp = sigma_plain[t];
    const bool ok = isfinite(mean) && mean > 0.0 && sp > 0.0 && fabs(log(mean / sp)) <= log_bound;
    use_plain[t] = ok ? 0 : 1;
    sigma_tile[t] = ok ? mean : sp;
}

// tau of every reference: the learned sigma of the 8x8 block holding its top-left pixel, scaled
// by its tile's vote (sigma_hat / sigma_est), or the tile's plain sigma_hat where the judge
// rejected the map.
__global__ void fill_tau_learned_kernel(double *tau, ImageGeom g, int tile, const float *zmap,
                                        const int32_t *use_plain, const double *sigma_est,
                                        const double *sigma_hat, double mult) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (int64_t)g.ny * g.nx) return;
    const int iy = (int)(r / g.nx), ix = (int)(r % g.nx);
    const int y = ref_pos(iy, g.ny, g.h, g.s), x = ref_pos(ix, g.nx, g.w, g.s);
    const int ntx = (g.w + tile - 1) / tile;
    const int t = (y / tile) * ntx + x / tile;
    double s;
    if (use_plain[t]) {
        s = sigma_hat[t];
    } else {
        const int wb = (g.w + PS - 1) / PS;
        s = exp((double)zmap[(y / PS) * wb + x / PS]) * (sigma_hat[t] / sigma_est[t]);
    }
    tau[r] = s * mult;
}

// Known noise levels of a batch: tau of every reference of image i = sigma[i] * mult[i].
__global__ void fill_tau_batched_kernel(const BatchItem *items, int n_items, const int *ref_start,
                                        const double *sigma, const double *mult) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ref_start[n_items]) return;
    const int i = find_unit(ref_start, n_items, e);
    const_cast<double *>(items[i].tau)[e - ref_start[i]] = sigma[i] * mult[i];
}

// Group size of each image in auto mode: the mean threshold over its references, divided by
// the multiplier it was filled with, is the image's mean noise level; below the cutoff the
// image is filtered with 16-member groups (the first half of its 32-member groups), else 32.
// One block per image; a fixed-order tree keeps the decision deterministic.
__global__ __launch_bounds__(256) void select_k_kernel(const BatchItem *__restrict__ items,
                                                       const int *__restrict__ auto_list,
                                                       const double *__restrict__ mult, double cutoff,
                                                       int *__restrict__ ksel) {
    __shared__ double part[256];
    const int i = auto_list[blockIdx.x];
    const BatchItem &it = items[i];
    const int64_t n = (int64_t)it.g.ny * it.g.nx;
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) acc += it.tau[e];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) ksel[i] = (part[0] / (double)n) / mult[i] < cutoff ? 16 : 32;
}

}  // namespace

hipError_t launch_select_k(const BatchItem *items, const int *auto_list, int n_auto, const double *mult,
                           double cutoff, int *ksel, hipStream_t st) {
    if (n_auto <= 0) return hipSuccess;
    hipLaunchKernelGGL(select_k_kernel, dim3(n_auto), dim3(256), 0, st, items, auto_list, mult, cutoff, ksel);
    return hipGetLastError();
}

hipError_t launch_fill_tau_batched(const BatchItem *items, int n_items, const int *ref_start, int total_refs,
                                   const double *sigma, const double *mult, hipStream_t st) {
    hipLaunchKernelGGL(fill_tau_batched_kernel, dim3((total_refs + 255) / 256), dim3(256), 0, st, items, n_items,
                       ref_start, sigma, mult);
    return hipGetLastError();
}

hipError_t launch_learned_judge(const ImageGeom &g, int tile, const float *zmap, const double *sigma_plain,
                                double ratio_bound, int32_t *use_plain, double *sigma_tile, hipStream_t st) {
    const int n = ((g.h + tile - 1) / tile) * ((g.w + tile - 1) / tile);
    hipLaunchKernelGGL(learned_judge_kernel, dim3((n + 255) / 256), dim3(256), 0, st, g, tile, zmap, sigma_plain,
                       log(ratio_bound), use_plain, sigma_tile);
    return hipGetLastError();
}

hipError_t launch_fill_tau_learned(double *tau, const ImageGeom &g, int tile, const float *zmap,
                                   const int32_t *use_plain, const double *sigma_est, const double *sigma_hat,
                                   double mult, hipStream_t st) {
    const int64_t n = (int64_t)g.ny * g.nx;
    hipLaunchKernelGGL(fill_tau_learned_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tau, g, tile,
                       zmap, use_plain, sigma_est, sigma_hat, mult);
    return hipGetLastError();
}

hipError_t launch_zero_rows(float *p, int64_t rows, int64_t cols, int64_t stride, hipStream_t st) {
    const int64_t n = rows * cols;
    hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, rows, cols, stride);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t *)p, n);
    return hipGetLastError();
}

hipError_t launch_fill_tau(double *tau_ref, int64_t n_ref, const double *sigma_tile, double sigma_const,
                           double mult, const ImageGeom &g, int tile, hipStream_t st) {
    hipLaunchKernelGGL(fill_tau_kernel, dim3((unsigned)((n_ref + 255) / 256)), dim3(256), 0, st, tau_ref, n_ref,
                       sigma_tile, sigma_const, mult, g, tile);
    return hipGetLastError();
}

}  // namespace htsvd
