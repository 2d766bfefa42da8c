// Collaborative filtering and aggregation for Haar-tSVD on gfx950.
//
// Per group of K patches (one wavefront per group):
//   Eq. 19  S = U^T * G * V  x_4  H_K      (t-product through the channel DFT, Eq. 4-5)
//   Eq. 20  hard threshold: keep |S| >= tau
//   Eq. 21  G_est = U * S_trunc * V^T  x_4  H_K^T
//   Algorithm 1: uniform ("average") aggregation of every patch of G_est.
//
// The t-product with 3 channels is evaluated slice-wise after a 3-point DFT along the
// channel mode: slice 0 is real, slice 1 complex, slice 2 its conjugate, so per patch the
// forward transform is X = G_hat V_hat (rows) and S_hat = U_hat^H X (columns), then the
// inverse DFT returns the real coefficients S that Eq. 20 thresholds.  With 1 channel it is
// the plain U^T G V.
//
// Layout of one wavefront's work: phase 1/5 give each lane a few rows of one member patch
// (K=32: 2 lanes per member, 4 rows each), phases 2/4 the same lanes a few columns, phase 3
// one coefficient position across all K members (the Haar butterflies run in registers).
// The group lives in LDS between phases as K x (64 c) floats.
//
// Threshold guard band: an FP32 coefficient within GUARD of tau is recomputed in FP64 from
// the uint8 group and the FP64 transform matrix by the whole wave, and that decides.
#include "common.h"

namespace htsvd {
namespace {

constexpr float R2F = 0.70710678118654752440f;
constexpr double R2D = 0.70710678118654752440;
constexpr float SQ3_2 = 0.86602540378443864676f;  // sqrt(3)/2
constexpr float THIRD = 0.33333333333333333333f;
constexpr float SQ3 = 1.73205080756887729353f;
constexpr float GUARD_F = 0.05f;  // >> worst-case FP32 error of a coefficient (~1e-2 for 8-bit input)
constexpr int NEAR_CAP = 256;

__device__ inline void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// Eq. 8 recursion applied to a K-vector in registers: the first half of each level holds
// the scaled pair sums (recursed on), the second half the scaled pair differences.
template <int K>
__device__ inline void haar_fwd(float (&v)[K]) {
#pragma unroll
    for (int n = K; n > 1; n >>= 1) {
        float t[K];
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            t[i] = (v[2 * i] + v[2 * i + 1]) * R2F;
            t[n / 2 + i] = (v[2 * i] - v[2 * i + 1]) * R2F;
        }
#pragma unroll
        for (int i = 0; i < n; ++i) v[i] = t[i];
    }
}

template <int K>
__device__ inline void haar_inv(float (&v)[K]) {
#pragma unroll
    for (int n = 2; n <= K; n <<= 1) {
        float t[K];
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            t[2 * i] = (v[i] + v[n / 2 + i]) * R2F;
            t[2 * i + 1] = (v[i] - v[n / 2 + i]) * R2F;
        }
#pragma unroll
        for (int i = 0; i < n; ++i) v[i] = t[i];
    }
}

// Entry (k, m) of H_n from the recursion H_n = 1/sqrt2 [H_{n/2} (x) [1,1]; I_{n/2} (x) [1,-1]].
__device__ inline double haar_weight(int k, int m, int n) {
    double w = 1.0;
    while (n > 1) {
        if (k < n / 2) {
            w *= R2D;
            m >>= 1;
            n >>= 1;
        } else {
            const int i = k - n / 2;
            return m == 2 * i ? w * R2D : (m == 2 * i + 1 ? -w * R2D : 0.0);
        }
    }
    return w;
}

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int C, int K>
__global__ __launch_bounds__(64) void group_kernel(ImageGeom g, const float *__restrict__ B,
                                                   const double *__restrict__ T64, const int32_t *__restrict__ idx,
                                                   const double *__restrict__ tau_ref, float *__restrict__ num,
                                                   int64_t num_stride, int32_t *__restrict__ hits,
                                                   unsigned long long *__restrict__ guard_count, int64_t n_ref) {
    constexpr int P = 64 * C;                    // coefficients per patch
    constexpr int LPM = (64 / K) < 8 ? (64 / K) : 8;  // lanes per member
    constexpr int RPL = 8 / LPM;                 // rows (or columns) per lane
    __shared__ float buf[K * P];
    __shared__ int near_k[NEAR_CAP], near_q[NEAR_CAP];
    __shared__ int near_n;

    const int lane = threadIdx.x;
    const int64_t r = blockIdx.x;
    if (r >= n_ref) return;
    const int m = lane / LPM, part = lane % LPM;
    const bool active = m < K;
    const int32_t lin = active ? idx[r * K + m] : 0;
    const int ym = lin / g.w, xm = lin % g.w;
    const double tau = tau_ref[r];
    const float tauf = (float)tau;
    // tau = 0 keeps every coefficient whatever its rounding, so no FP64 re-decision is needed
    const bool guard_on = tau > (double)GUARD_F;
    if (lane == 0) near_n = 0;

    const float *U0 = B, *V0 = B + 64, *U1r = B + 128, *U1i = B + 192, *V1r = B + 256, *V1i = B + 320;

    // ---- phase 1: gather rows, channel DFT, right product with V_hat ----
    if (active) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int a = part * RPL + t;
            const uint8_t *px = g.img + (int64_t)(ym + a) * g.stride + (int64_t)xm * C;
            float *dst = buf + m * P + a * 8;
            if (C == 3) {
                float g0[8], gr[8], gi[8];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const float R = px[3 * b], G = px[3 * b + 1], Bc = px[3 * b + 2];
                    g0[b] = R + G + Bc;
                    gr[b] = R - 0.5f * (G + Bc);
                    gi[b] = SQ3_2 * (Bc - G);
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    float x0 = 0.f, xr = 0.f, xi = 0.f;
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        x0 += g0[b] * V0[b * 8 + j];
                        xr += gr[b] * V1r[b * 8 + j] - gi[b] * V1i[b * 8 + j];
                        xi += gr[b] * V1i[b * 8 + j] + gi[b] * V1r[b * 8 + j];
                    }
                    dst[j] = x0;
                    dst[64 + j] = xr;
                    dst[128 + j] = xi;
                }
            } else {
                float g0[8];
#pragma unroll
                for (int b = 0; b < 8; ++b) g0[b] = px[b];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    float x0 = 0.f;
#pragma unroll
                    for (int b = 0; b < 8; ++b) x0 += g0[b] * V0[b * 8 + j];
                    dst[j] = x0;
                }
            }
        }
    }
    wave_lds_sync();

    // ---- phase 2: left product with U_hat^H, inverse channel DFT -> real S ----
    if (active) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int j = part * RPL + t;
            float *col = buf + m * P + j;
            if (C == 3) {
                float x0[8], xr[8], xi[8];
#pragma unroll
                for (int a = 0; a < 8; ++a) { x0[a] = col[a * 8]; xr[a] = col[64 + a * 8]; xi[a] = col[128 + a * 8]; }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    float s0 = 0.f, sr = 0.f, si = 0.f;
#pragma unroll
                    for (int a = 0; a < 8; ++a) {
                        s0 += U0[a * 8 + i] * x0[a];
                        sr += U1r[a * 8 + i] * xr[a] + U1i[a * 8 + i] * xi[a];
                        si += U1r[a * 8 + i] * xi[a] - U1i[a * 8 + i] * xr[a];
                    }
                    col[i * 8] = (s0 + 2.f * sr) * THIRD;
                    col[64 + i * 8] = (s0 - sr - SQ3 * si) * THIRD;
                    col[128 + i * 8] = (s0 - sr + SQ3 * si) * THIRD;
                }
            } else {
                float x0[8];
#pragma unroll
                for (int a = 0; a < 8; ++a) x0[a] = col[a * 8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    float s0 = 0.f;
#pragma unroll
                    for (int a = 0; a < 8; ++a) s0 += U0[a * 8 + i] * x0[a];
                    col[i * 8] = s0;
                }
            }
        }
    }
    wave_lds_sync();

    // ---- phase 3: Haar along the group, threshold, guard band ----
#pragma unroll 1
    for (int t = 0; t < C; ++t) {
        const int q = lane + 64 * t;
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = buf[k * P + q];
        haar_fwd<K>(v);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float a = fabsf(v[k]);
            if (guard_on && fabsf(a - tauf) < GUARD_F) {
                const int e = atomicAdd(&near_n, 1);
                if (e < NEAR_CAP) { near_k[e] = k; near_q[e] = q; }
                else if (!(a >= tauf)) v[k] = 0.f;
            } else if (!(a >= tauf)) {
                v[k] = 0.f;
            }
            buf[k * P + q] = v[k];
        }
    }
    wave_lds_sync();
    const int n_near = near_n;
    if (n_near > 0) {
        if (lane == 0) {
            atomicAdd(guard_count, (unsigned long long)(n_near < NEAR_CAP ? n_near : NEAR_CAP));
            if (n_near > NEAR_CAP) atomicAdd(guard_count + 1, (unsigned long long)(n_near - NEAR_CAP));
        }
        const int ne = n_near < NEAR_CAP ? n_near : NEAR_CAP;
        for (int e = 0; e < ne; ++e) {
            const int k = near_k[e], q = near_q[e];
            double part_sum = 0.0;
            for (int p = lane; p < P; p += 64) {
                // Haar-weighted pixel sum of position p over the members, then row q of T
                const int ch = p / 64, i = (p / 8) % 8, j = p % 8;
                double acc = 0.0;
                for (int mm = 0; mm < K; ++mm) {
                    const double w = haar_weight(k, mm, K);
                    if (w == 0.0) continue;
                    const int32_t l2 = idx[r * K + mm];
                    const int y2 = l2 / g.w, x2 = l2 % g.w;
                    acc += w * (double)g.img[(int64_t)(y2 + i) * g.stride + (int64_t)(x2 + j) * C + ch];
                }
                part_sum += T64[(int64_t)q * P + p] * acc;
            }
            const double s = wave_sum_f64(part_sum);
            if (lane == 0 && !(fabs(s) >= tau)) buf[k * P + q] = 0.f;
        }
        wave_lds_sync();
    }
#pragma unroll 1
    for (int t = 0; t < C; ++t) {
        const int q = lane + 64 * t;
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = buf[k * P + q];
        haar_inv<K>(v);
#pragma unroll
        for (int k = 0; k < K; ++k) buf[k * P + q] = v[k];
    }
    wave_lds_sync();

    // ---- phase 4: channel DFT of S', left product with U_hat ----
    if (active) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int j = part * RPL + t;
            float *col = buf + m * P + j;
            if (C == 3) {
                float s0[8], sr[8], si[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float a = col[i * 8], b = col[64 + i * 8], c = col[128 + i * 8];
                    s0[i] = a + b + c;
                    sr[i] = a - 0.5f * (b + c);
                    si[i] = SQ3_2 * (c - b);
                }
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    float y0 = 0.f, yr = 0.f, yi = 0.f;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        y0 += U0[a * 8 + i] * s0[i];
                        yr += U1r[a * 8 + i] * sr[i] - U1i[a * 8 + i] * si[i];
                        yi += U1r[a * 8 + i] * si[i] + U1i[a * 8 + i] * sr[i];
                    }
                    col[a * 8] = y0;
                    col[64 + a * 8] = yr;
                    col[128 + a * 8] = yi;
                }
            } else {
                float s0[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) s0[i] = col[i * 8];
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    float y0 = 0.f;
#pragma unroll
                    for (int i = 0; i < 8; ++i) y0 += U0[a * 8 + i] * s0[i];
                    col[a * 8] = y0;
                }
            }
        }
    }
    wave_lds_sync();

    // ---- phase 5: right product with V_hat^H, inverse channel DFT, aggregation ----
    if (active) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int a = part * RPL + t;
            const float *row = buf + m * P + a * 8;
            float *dst = num + (int64_t)(ym + a) * num_stride + (int64_t)xm * C;
            if (C == 3) {
                float y0[8], yr[8], yi[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) { y0[j] = row[j]; yr[j] = row[64 + j]; yi[j] = row[128 + j]; }
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    float p0 = 0.f, pr = 0.f, pi = 0.f;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        p0 += y0[j] * V0[b * 8 + j];
                        pr += yr[j] * V1r[b * 8 + j] + yi[j] * V1i[b * 8 + j];
                        pi += yi[j] * V1r[b * 8 + j] - yr[j] * V1i[b * 8 + j];
                    }
                    atomicAdd(dst + 3 * b, (p0 + 2.f * pr) * THIRD);
                    atomicAdd(dst + 3 * b + 1, (p0 - pr - SQ3 * pi) * THIRD);
                    atomicAdd(dst + 3 * b + 2, (p0 - pr + SQ3 * pi) * THIRD);
                }
            } else {
                float y0[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) y0[j] = row[j];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    float p0 = 0.f;
#pragma unroll
                    for (int j = 0; j < 8; ++j) p0 += y0[j] * V0[b * 8 + j];
                    atomicAdd(dst + b, p0);
                }
            }
        }
        if (part == 0) atomicAdd(hits + (int64_t)ym * g.w + xm, 1);
    }
}

// cnt(y, x) = number of aggregated patches covering the pixel = 8x8 box sum of the patch
// hit counts; out = num / cnt, or the noisy value where no patch landed.
__global__ void normalize_kernel(ImageGeom g, const int32_t *__restrict__ hits, float *__restrict__ out,
                                 int64_t out_stride) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)g.h * g.w) return;
    const int y = (int)(e / g.w), x = (int)(e % g.w);
    int cnt = 0;
    for (int i = 0; i < PS; ++i) {
        const int yy = y - i;
        if (yy < 0) break;
        if (yy > g.h - PS) continue;
        for (int j = 0; j < PS; ++j) {
            const int xx = x - j;
            if (xx < 0) break;
            if (xx > g.w - PS) continue;
            cnt += hits[(int64_t)yy * g.w + xx];
        }
    }
    float *o = out + (int64_t)y * out_stride + (int64_t)x * g.c;
    const uint8_t *px = g.img + (int64_t)y * g.stride + (int64_t)x * g.c;
    for (int ch = 0; ch < g.c; ++ch) o[ch] = cnt > 0 ? o[ch] / (float)cnt : (float)px[ch];
}

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

template <int C, int K>
hipError_t launch_groups_t(const ImageGeom &g, const BasisDev &b, const int32_t *idx, const double *tau_ref,
                           float *num, int64_t num_stride, int32_t *hits, unsigned long long *gc, hipStream_t st) {
    const int64_t n_ref = (int64_t)g.ny * g.nx;
    hipLaunchKernelGGL((group_kernel<C, K>), dim3((unsigned)n_ref), dim3(64), 0, st, g, b.f32, b.T64, idx, tau_ref,
                       num, num_stride, hits, gc, n_ref);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_denoise_groups_impl(const ImageGeom &g, int K, const BasisDev &b, const int32_t *idx,
                                      const double *tau_ref, float *num, int64_t num_stride, int32_t *hits,
                                      unsigned long long *gc, hipStream_t st) {
#define HT_CASE(CC, KK) \
    if (g.c == CC && K == KK) return launch_groups_t<CC, KK>(g, b, idx, tau_ref, num, num_stride, hits, gc, st);
    HT_CASE(1, 4) HT_CASE(1, 8) HT_CASE(1, 16) HT_CASE(1, 32)
    HT_CASE(3, 4) HT_CASE(3, 8) HT_CASE(3, 16) HT_CASE(3, 32)
#undef HT_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_normalize(const ImageGeom &g, const int32_t *hits, float *out, int64_t out_stride,
                            hipStream_t st) {
    const int64_t n = (int64_t)g.h * g.w;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, hits, out, out_stride);
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
