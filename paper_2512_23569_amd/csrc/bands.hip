// Hyperspectral tube patches (Sec. IV-D): Haar-tSVD on an h x w x B cube with 8 x 8 x B patches.
//
// Grouping runs on a gray guide, the band mean rounded half up (the block matcher of the other
// paths, Eq. 9 on one channel).  The members of every group are gathered into a patch matrix
// X (n = group*K + member, e = 8i + j, b = band; FP64, the full-rate vector precision of this
// device, so that keep/kill decisions agree with an FP64 reference without a guard band), and
// the t-product S = U^T * P * V
// (Eq. 19) is taken along the band axis through its DFT (Eq. 4-5), as three dense products:
//   band DFT      Xd = X D^T                 (B Fourier reals Re0, Re1, Im1, ..., each stored as
//                                             one contiguous block over the rows n*64 + e)
//   slice maps    per frequency f, vec(S_hat_f) = M_f vec(P_hat_f), M_f((i',j'),(i,j)) =
//                 conj(U_hat_f(i,i')) V_hat_f(j,j') (64 x 64, real for f = 0 and f = B/2)
//   inverse DFT   S = Sd Dinv^T              (the real slices S^(k), where the threshold acts)
// then the Haar transform along each group with the hard threshold (Eq. 20), the inverse path
// with M_f^H (Eq. 21), and uniform aggregation (Algorithm 1) in 64-bit fixed point (exact sums,
// so the result does not depend on the order of the additions).
#include "common.h"

namespace htsvd {

namespace {

constexpr int BFS = 16;   // aggregation fixed point: values in units of 2^-16

__global__ void guide_kernel(const uint8_t *__restrict__ cube, int64_t stride, int h, int w, int B,
                             uint8_t *__restrict__ guide) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= (int64_t)h * w) return;
    const int y = (int)(q / w), x = (int)(q % w);
    const uint8_t *p = cube + (int64_t)y * stride + (int64_t)x * B;
    int s = 0;
    for (int b = 0; b < B; ++b) s += p[b];
    guide[q] = (uint8_t)((s + B / 2) / B);
}

// X[(n*64 + e)*B + b] = cube(y_n + i, x_n + j, b), n = r*K + k.
__global__ void gather_kernel(const uint8_t *__restrict__ cube, int64_t stride, int w, int B,
                              const int32_t *__restrict__ idx, int64_t n_patch, double *__restrict__ X) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_patch * 64 * B) return;
    const int b = (int)(t % B);
    const int64_t ne = t / B;
    const int e = (int)(ne & 63);
    const int64_t n = ne >> 6;
    const int32_t lin = idx[n];
    X[t] = (double)cube[(int64_t)(lin / w + (e >> 3)) * stride + (int64_t)(lin % w + (e & 7)) * B + b];
}

// C(m, n) (+)= sum_k A(m, k) B(k, n): A(m, k) at A[m*sam + k*sak], B(k, n) at Bm[k*sbk + n*sbn],
// C(m, n) at Cm[m*scm + n*scn]; 64 x 64 tiles, 4 x 4 outputs per thread, FP64.
__global__ __launch_bounds__(256) void gemm_kernel(const double *__restrict__ A, int64_t sam, int64_t sak,
                                                   const double *__restrict__ Bm, int64_t sbk, int64_t sbn,
                                                   double *__restrict__ Cm, int64_t scm, int64_t scn, int64_t M, int N,
                                                   int Kd, double alpha, int accumulate) {
    __shared__ double As[16][64 + 1];
    __shared__ double Bs[16][64 + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 64;   // rows on x: the grid's y extent is limited
    const int n0 = blockIdx.y * 64;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < Kd; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int gk = k0 + kk;
            const int64_t gm = m0 + mm;
            As[kk][mm] = (gm < M && gk < Kd) ? A[gm * sam + (int64_t)gk * sak] : 0.0;
            const int gn = n0 + mm;
            Bs[kk][mm] = (gn < N && gk < Kd) ? Bm[(int64_t)gk * sbk + (int64_t)gn * sbn] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gm = m0 + ty * 4 + i;
            const int gn = n0 + tx * 4 + j;
            if (gm < M && gn < N) {
                double *c = Cm + gm * scm + (int64_t)gn * scn;
                *c = accumulate ? *c + alpha * acc[i][j] : alpha * acc[i][j];
            }
        }
}

// Haar transform along each group (orthonormal butterflies), hard threshold |s| >= tau, inverse.
// One thread per (group, position e, slice b); S[((g*K + k)*64 + e)*B + b].
template <int K>
__global__ void haar_threshold_kernel(double *__restrict__ S, int64_t n_group, int B, double tau) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_group * 64 * B) return;
    const int b = (int)(t % B);
    const int64_t ge = t / B;
    const int e = (int)(ge & 63);
    const int64_t g = ge >> 6;
    double v[K];
    const int64_t stride_k = (int64_t)64 * B;
    double *base = S + ((g * K) * 64 + e) * B + b;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = base[k * stride_k];
    constexpr double R2 = 0.70710678118654752440;
    // forward: at each level the pair sums move to the front, the differences stay in place
#pragma unroll
    for (int st = 1; st < K; st <<= 1)
#pragma unroll
        for (int i = 0; i < K; i += 2 * st) {
            const double a = v[i], c = v[i + st];
            v[i] = (a + c) * R2;
            v[i + st] = (a - c) * R2;
        }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = fabs(v[k]) >= tau ? v[k] : 0.0;
#pragma unroll
    for (int st = K / 2; st >= 1; st >>= 1)
#pragma unroll
        for (int i = 0; i < K; i += 2 * st) {
            const double a = v[i], c = v[i + st];
            v[i] = (a + c) * R2;
            v[i + st] = (a - c) * R2;
        }
#pragma unroll
    for (int k = 0; k < K; ++k) base[k * stride_k] = v[k];
}

// Uniform aggregation in 64-bit fixed point; counts per pixel from the band-0 thread.
__global__ void aggregate_kernel(const double *__restrict__ Pe, const int32_t *__restrict__ idx, int64_t n_patch,
                                 int w, int B, unsigned long long *__restrict__ acc, int *__restrict__ cnt) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_patch * 64 * B) return;
    const int b = (int)(t % B);
    const int64_t ne = t / B;
    const int e = (int)(ne & 63);
    const int64_t n = ne >> 6;
    const int32_t lin = idx[n];
    const int64_t pix = (int64_t)(lin / w + (e >> 3)) * w + (lin % w + (e & 7));
    const double v = fmin(fmax(Pe[t], -1024.0), 1024.0);
    const long long q = __double2ll_rn(v * (double)(1 << BFS));
    atomicAdd(acc + pix * B + b, (unsigned long long)q);
    if (b == 0) atomicAdd(cnt + pix, 1);
}

__global__ void normalize_kernel(const unsigned long long *__restrict__ acc, const int *__restrict__ cnt,
                                 const uint8_t *__restrict__ cube, int64_t stride, int h, int w, int B,
                                 float *__restrict__ out, int64_t out_stride) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)h * w * B) return;
    const int b = (int)(t % B);
    const int64_t pix = t / B;
    const int y = (int)(pix / w), x = (int)(pix % w);
    const int n = cnt[pix];
    out[(int64_t)y * out_stride + (int64_t)x * B + b] =
        n > 0 ? (float)((double)(long long)acc[t] / ((double)n * (double)(1 << BFS)))
              : (float)cube[(int64_t)y * stride + (int64_t)x * B + b];
}

// Band planes: planes[(b*h + y)*w + x] = cube(y, x, b), for the band-wise noise estimate.
__global__ void planes_kernel(const uint8_t *__restrict__ cube, int64_t stride, int h, int w, int B,
                              uint8_t *__restrict__ planes) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= (int64_t)h * w) return;
    const int y = (int)(q / w), x = (int)(q % w);
    const uint8_t *p = cube + (int64_t)y * stride + (int64_t)x * B;
    for (int b = 0; b < B; ++b) planes[(int64_t)b * h * w + q] = p[b];
}

// out(y, x, b) = alt(y, x, b) for the bands with sel[b] != 0.
__global__ void select_bands_kernel(const float *__restrict__ alt, int64_t alt_stride, const uint8_t *__restrict__ sel,
                                    int h, int w, int B, float *__restrict__ out, int64_t out_stride) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)h * w * B) return;
    const int b = (int)(t % B);
    if (!sel[b]) return;
    const int64_t pix = t / B;
    const int y = (int)(pix / w), x = (int)(pix % w);
    out[(int64_t)y * out_stride + (int64_t)x * B + b] = alt[(int64_t)y * alt_stride + (int64_t)x * B + b];
}

unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t gemm(const double *A, int64_t sam, int64_t sak, const double *Bm, int64_t sbk, int64_t sbn, double *Cm,
                int64_t scm, int64_t scn, int64_t M, int N, int Kd, double alpha, bool accumulate, hipStream_t st) {
    hipLaunchKernelGGL(gemm_kernel, dim3((unsigned)((M + 63) / 64), nb(N, 64)), dim3(256), 0, st, A, sam, sak, Bm, sbk,
                       sbn, Cm, scm, scn, M, N, Kd, alpha, accumulate ? 1 : 0);
    return hipGetLastError();
}

// One direction of the t-product on the patch matrix (rows n*64 + e, B columns):
//   X -> Xd = X D^T -> per frequency the slice maps into Sd -> Y = Sd Dinv^T.
// Xd and Sd hold one contiguous block of rows per Fourier component, so the slice maps read and
// write whole rows.  Forward uses M_f, inverse M_f^H (M stored as real and imaginary 64 x 64
// parts per slice).
hipError_t tproduct(const BandMaps &bm, int B, int64_t n_patch, const double *X, double *Xd, double *Sd, double *Y,
                    bool inverse, hipStream_t st) {
    const int64_t rows = n_patch * 64;
    hipError_t e;
    if ((e = gemm(X, B, 1, bm.D, 1, B, Xd, 1, rows, rows, B, B, 1.0, false, st)) != hipSuccess) return e;
    const int NF = B / 2 + 1;
    for (int f = 0; f < NF; ++f) {
        const double *Mr = bm.M + (size_t)f * 2 * 4096, *Mi = Mr + 4096;
        const bool real = f == 0 || 2 * f == B;
        const int cr = f == 0 ? 0 : 2 * f - 1, ci = 2 * f;   // columns of Re, Im of frequency f
        // C(n, e') = sum_e A(n, e) M(e', e)  [forward]   or   M(e, e')  [inverse, M^T; M^H flips Mi's sign]
        const int64_t sbk = inverse ? 64 : 1, sbn = inverse ? 1 : 64;
        const double *ar = Xd + cr * rows, *ai = Xd + ci * rows;
        double *cre = Sd + cr * rows, *cim = Sd + ci * rows;
        if (real) {
            if ((e = gemm(ar, 64, 1, Mr, sbk, sbn, cre, 64, 1, n_patch, 64, 64, 1.0, false, st)) != hipSuccess) return e;
            continue;
        }
        const double si = inverse ? -1.0 : 1.0;   // Im of M or of M^H
        // Re out = Mr Re - (si Mi) Im;  Im out = (si Mi) Re + Mr Im
        if ((e = gemm(ar, 64, 1, Mr, sbk, sbn, cre, 64, 1, n_patch, 64, 64, 1.0, false, st)) != hipSuccess ||
            (e = gemm(ai, 64, 1, Mi, sbk, sbn, cre, 64, 1, n_patch, 64, 64, -si, true, st)) != hipSuccess ||
            (e = gemm(ar, 64, 1, Mi, sbk, sbn, cim, 64, 1, n_patch, 64, 64, si, false, st)) != hipSuccess ||
            (e = gemm(ai, 64, 1, Mr, sbk, sbn, cim, 64, 1, n_patch, 64, 64, 1.0, true, st)) != hipSuccess)
            return e;
    }
    return gemm(Sd, 1, rows, bm.Dinv, 1, B, Y, B, 1, rows, B, B, 1.0, false, st);
}

}  // namespace

hipError_t launch_band_planes(const uint8_t *cube, int64_t stride, int h, int w, int B, uint8_t *planes,
                              hipStream_t st) {
    hipLaunchKernelGGL(planes_kernel, dim3(nb((int64_t)h * w, 256)), dim3(256), 0, st, cube, stride, h, w, B, planes);
    return hipGetLastError();
}

hipError_t launch_select_bands(const float *alt, int64_t alt_stride, const uint8_t *sel, int h, int w, int B,
                               float *out, int64_t out_stride, hipStream_t st) {
    hipLaunchKernelGGL(select_bands_kernel, dim3(nb((int64_t)h * w * B, 256)), dim3(256), 0, st, alt, alt_stride, sel,
                       h, w, B, out, out_stride);
    return hipGetLastError();
}

hipError_t launch_band_guide(const uint8_t *cube, int64_t stride, int h, int w, int B, uint8_t *guide,
                             hipStream_t st) {
    hipLaunchKernelGGL(guide_kernel, dim3(nb((int64_t)h * w, 256)), dim3(256), 0, st, cube, stride, h, w, B, guide);
    return hipGetLastError();
}

// Groups per pass of the filter: each of the three FP64 patch matrices stays below cap bytes.
int64_t band_chunk_groups(int B, int K, int64_t n_group, int64_t cap) {
    const int64_t per = (int64_t)K * 64 * B * (int64_t)sizeof(double);
    return std::max<int64_t>(1, std::min<int64_t>(n_group, cap / per));
}

size_t band_ws_bytes(int h, int w, int B, int K, int64_t n_group, int64_t cap) {
    const int64_t n_patch = band_chunk_groups(B, K, n_group, cap) * K;
    const size_t mat = sizeof(double) * (size_t)n_patch * 64 * B;
    return 3 * ((mat + 255) & ~(size_t)255) + (((size_t)h * w * B * 8 + 255) & ~(size_t)255) +
           (((size_t)h * w * 4 + 255) & ~(size_t)255);
}

hipError_t launch_band_filter(const BandMaps &bm, const uint8_t *cube, int64_t stride, int h, int w, int B,
                              const int32_t *idx, int64_t n_group, int K, double tau, int64_t cap, void *ws,
                              float *out, int64_t out_stride, hipStream_t st) {
    const int64_t chunk = band_chunk_groups(B, K, n_group, cap);
    const size_t mat = ((sizeof(double) * (size_t)(chunk * K) * 64 * B) + 255) & ~(size_t)255;
    double *X = (double *)ws, *Xd = (double *)((char *)ws + mat), *Sd = (double *)((char *)ws + 2 * mat);
    unsigned long long *acc = (unsigned long long *)((char *)ws + 3 * mat);
    int *cnt = (int *)((char *)acc + (((size_t)h * w * B * 8 + 255) & ~(size_t)255));
    hipError_t e;
    if ((e = launch_zero(acc, (size_t)h * w * B * 8, st)) != hipSuccess) return e;
    if ((e = launch_zero(cnt, (size_t)h * w * 4, st)) != hipSuccess) return e;
    for (int64_t g0 = 0; g0 < n_group; g0 += chunk) {
        const int64_t ng = std::min<int64_t>(chunk, n_group - g0), n_patch = ng * K;
        const int32_t *ix = idx + g0 * K;
        const int64_t nel = n_patch * 64 * B;
        hipLaunchKernelGGL(gather_kernel, dim3(nb(nel, 256)), dim3(256), 0, st, cube, stride, w, B, ix, n_patch, X);
        if ((e = tproduct(bm, B, n_patch, X, Xd, Sd, X, false, st)) != hipSuccess) return e;   // S into X
        const int64_t nt = ng * 64 * B;
        switch (K) {
            case 4: hipLaunchKernelGGL(haar_threshold_kernel<4>, dim3(nb(nt, 256)), dim3(256), 0, st, X, ng, B, tau); break;
            case 8: hipLaunchKernelGGL(haar_threshold_kernel<8>, dim3(nb(nt, 256)), dim3(256), 0, st, X, ng, B, tau); break;
            case 16: hipLaunchKernelGGL(haar_threshold_kernel<16>, dim3(nb(nt, 256)), dim3(256), 0, st, X, ng, B, tau); break;
            case 32: hipLaunchKernelGGL(haar_threshold_kernel<32>, dim3(nb(nt, 256)), dim3(256), 0, st, X, ng, B, tau); break;
            default: return hipErrorInvalidValue;
        }
        if ((e = tproduct(bm, B, n_patch, X, Xd, Sd, X, true, st)) != hipSuccess) return e;    // estimates into X
        hipLaunchKernelGGL(aggregate_kernel, dim3(nb(nel, 256)), dim3(256), 0, st, X, ix, n_patch, w, B, acc, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(normalize_kernel, dim3(nb((int64_t)h * w * B, 256)), dim3(256), 0, st, acc, cnt, cube, stride, h,
                       w, B, out, out_stride);
    return hipGetLastError();
}

}  // namespace htsvd
