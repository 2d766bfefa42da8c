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

}  // namespace

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
