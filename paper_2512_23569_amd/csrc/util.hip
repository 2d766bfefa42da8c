// Small utility kernels: buffer clearing and per-reference thresholds.
#include "common.h"
#include "sigma_dev.h"

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
        int y, x;
        s = sigma_tile[ref_tile(g, tile, r, &y, &x)];
    }
    tau[r] = s * mult;
}

// Per sub-image: the learned map judged by the plain estimate (see judge_tile).
__global__ void learned_judge_kernel(ImageGeom g, int tile, const float *zmap, const double *sigma_plain,
                                     double bound, int32_t *use_plain, double *sigma_tile) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntx = (g.w + tile - 1) / tile, nty = (g.h + tile - 1) / tile;
    if (t >= ntx * nty) return;
    sigma_tile[t] = judge_tile(g, tile, t, zmap, sigma_plain[t], bound, use_plain + t);
}

// tau of every reference under the learned map (see learned_ref_sigma).
__global__ void fill_tau_learned_kernel(double *tau, ImageGeom g, int tile, const float *zmap,
                                        const int32_t *use_plain, const double *sigma_est,
                                        const double *sigma_hat, double mult) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (int64_t)g.ny * g.nx) return;
    tau[r] = learned_ref_sigma(g, tile, r, zmap, use_plain, sigma_est, sigma_hat) * mult;
}

// Effective sigma per 8x8 block (see block_sigma); the tile is a multiple of the block size.
__global__ void sigma_map_kernel(double *map, ImageGeom g, int tile, const float *zmap, const int32_t *use_plain,
                                 const double *sigma_est, const double *sigma_hat) {
    const int hb = (g.h + PS - 1) / PS, wb = (g.w + PS - 1) / PS;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= hb * wb) return;
    const int by = b / wb, bx = b % wb;
    const int ntx = (g.w + tile - 1) / tile;
    const int t = (by * PS / tile) * ntx + bx * PS / tile;
    map[b] = block_sigma(g, t, by, bx, zmap, use_plain, sigma_est, sigma_hat);
}

__global__ void scale_tau_kernel(const double *tau, double *out, int64_t n, const int *ksel, int k_alt,
                                 double mul_alt) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    out[r] = tau[r] * ((ksel && *ksel == k_alt) ? mul_alt : 1.0);
}

// Batched thresholds of the images whose noise level went through the sub-image stages.
__global__ void fill_tau_sigma_batched_kernel(const SigmaItem *__restrict__ items, const int *__restrict__ sel,
                                              const int *__restrict__ start, int n, int total, int tile) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= total) return;
    const int j = find_unit(start, n, u);
    const SigmaItem &it = items[sel[j]];
    const ImageGeom g = it.g;
    const int64_t r = u - start[j];
    double s;
    if (it.mode == SIGMA_LEARNED) {
        s = learned_ref_sigma(g, tile, r, it.zmap, it.use_plain, it.sig_est, it.sig_hat);
    } else {
        int y, x;
        s = it.sig_hat[ref_tile(g, tile, r, &y, &x)];
    }
    it.tau[r] = s * it.mult;
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
// Two passes with fixed-order trees keep the decision deterministic: chunks of SK_CHUNK
// references are summed by one block each, then one block per image adds its chunk sums.
constexpr int SK_CHUNK = 8192;

__device__ inline double block_sum_256(double v, double *part) {
    part[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    return part[0];
}

__global__ __launch_bounds__(256) void select_k_partial_kernel(const BatchItem *__restrict__ items,
                                                               const int *__restrict__ auto_list, int n_chunk,
                                                               double *__restrict__ partial) {
    __shared__ double part[256];
    const int a = blockIdx.y, c = blockIdx.x;
    const BatchItem &it = items[auto_list[a]];
    const int64_t n = (int64_t)it.g.ny * it.g.nx;
    const int64_t e0 = (int64_t)c * SK_CHUNK, e1 = min(n, e0 + SK_CHUNK);
    double acc = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) acc += it.tau[e];
    const double tot = block_sum_256(acc, part);
    if (threadIdx.x == 0) partial[(int64_t)a * n_chunk + c] = tot;
}

__global__ __launch_bounds__(256) void select_k_kernel(const BatchItem *__restrict__ items,
                                                       const int *__restrict__ auto_list, int n_chunk,
                                                       const double *__restrict__ partial,
                                                       const double *__restrict__ mult, double cutoff,
                                                       int *__restrict__ ksel) {
    __shared__ double part[256];
    const int a = blockIdx.x, i = auto_list[a];
    const BatchItem &it = items[i];
    const int64_t n = (int64_t)it.g.ny * it.g.nx;
    const int used = (int)((n + SK_CHUNK - 1) / SK_CHUNK);
    double acc = 0.0;
    for (int c = threadIdx.x; c < used; c += 256) acc += partial[(int64_t)a * n_chunk + c];
    const double tot = block_sum_256(acc, part);
    if (threadIdx.x == 0) ksel[i] = (tot / (double)n) / mult[i] < cutoff ? 16 : 32;
}

}  // namespace

int select_k_chunks(int64_t max_refs) { return (int)((max_refs + SK_CHUNK - 1) / SK_CHUNK); }

hipError_t launch_select_k(const BatchItem *items, const int *auto_list, int n_auto, int n_chunk, double *partial,
                           const double *mult, double cutoff, int *ksel, hipStream_t st) {
    if (n_auto <= 0) return hipSuccess;
    if (n_chunk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(select_k_partial_kernel, dim3(n_chunk, n_auto), dim3(256), 0, st, items, auto_list, n_chunk,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_k_kernel, dim3(n_auto), dim3(256), 0, st, items, auto_list, n_chunk, partial, mult,
                       cutoff, ksel);
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
                       ratio_bound, use_plain, sigma_tile);
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

hipError_t launch_sigma_map(double *map, const ImageGeom &g, int tile, const float *zmap, const int32_t *use_plain,
                            const double *sigma_est, const double *sigma_hat, hipStream_t st) {
    if (tile % PS != 0) return hipErrorInvalidValue;
    const int n = ((g.h + PS - 1) / PS) * ((g.w + PS - 1) / PS);
    hipLaunchKernelGGL(sigma_map_kernel, dim3((n + 255) / 256), dim3(256), 0, st, map, g, tile, zmap, use_plain,
                       sigma_est, sigma_hat);
    return hipGetLastError();
}

hipError_t launch_scale_tau(const double *tau, double *out, int64_t n, const int *ksel, int k_alt, double mul_alt,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_tau_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tau, out, n, ksel,
                       k_alt, mul_alt);
    return hipGetLastError();
}

hipError_t launch_fill_tau_sigma_batched(const SigmaItem *items, const int *sel, const int *start, int n,
                                         int total, int tile, hipStream_t st) {
    if (n <= 0 || total <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_tau_sigma_batched_kernel, dim3((total + 255) / 256), dim3(256), 0, st, items, sel, start,
                       n, total, tile);
    return hipGetLastError();
}

hipError_t launch_zero_rows(float *p, int64_t rows, int64_t cols, int64_t stride, hipStream_t st) {
    const int64_t n = rows * cols;
    hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, rows, cols, stride);
    return hipGetLastError();
}

// The first kout members of every group stored with kin members per reference.
__global__ void idx_prefix_kernel(const int32_t *__restrict__ in, int kin, int32_t *__restrict__ out, int kout,
                                  int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * kout) return;
    const int64_t r = e / kout;
    out[e] = in[r * kin + (int)(e - r * kout)];
}

hipError_t launch_idx_prefix(const int32_t *in, int kin, int32_t *out, int kout, int64_t n_ref, hipStream_t st) {
    const int64_t n = n_ref * kout;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(idx_prefix_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, kin, out, kout,
                       n_ref);
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
