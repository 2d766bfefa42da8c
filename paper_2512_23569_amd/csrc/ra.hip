// RA-Haar-tSVD (Sec. III-E-2, Eq. 24-25): the mean patch of every group, the refinement network
// that maps it to a cleaner one, and the network's training.
//
// Network (residual learning on mean patches; P = 64c inputs and outputs, H hidden units):
//   x = (p - 128) / 128,  h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  r = W3 h2 + b3,
//   p_est = p - 128 r.
// Inference runs 64 groups per workgroup on the matrix cores: every layer is a 64 x (outputs)
// product over the inputs in steps of v_mfma_f32_32x32x16_f16 (each wave takes one 32-column
// tile for both 32-row tiles, so a weight fragment read from L2 serves 64 rows, and the next
// step's fragments are loaded while the current products run), with activations and weights
// split into fp16 hi + lo and three products (hi.hi + hi.lo + lo.hi, about 22 bits), FP32
// accumulation, bias and ReLU in FP32.  Activations stay in LDS between layers, already split:
// each layer's epilogue writes the hi and lo halves, so operands are read, not re-split.  Inside the
// denoiser the last layer's weights are folded with the forward patch transform T (times 128),
// so the kernel writes the change of the group's first Haar row directly:
//   sqrt(K) T p_est = sqrt(K) T p - sqrt(K) * (128 T r).
// Training runs in FP32 on the vector units (tiled products, the loss and Adam).
#include "common.h"

namespace htsvd {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

namespace {

constexpr int FR = 64;            // groups per workgroup
constexpr int FMT = FR / 32;      // 32-row tiles
constexpr int FWAVES = 8;
constexpr int FTHREADS = FWAVES * 64;
constexpr int APITCH = 256 + 8;   // halves per activation row in LDS (16 bytes of padding)
constexpr int ABUF = FR * APITCH;  // halves of one split activation array (hi, then lo)

// Stores v as fp16 hi + lo at row m, column n of a split activation buffer.
__device__ inline void put_split(_Float16 *buf, int m, int n, float v) {
    const _Float16 hv = (_Float16)v;
    buf[m * APITCH + n] = hv;
    buf[ABUF + m * APITCH + n] = (_Float16)(v - (float)hv);
}

// One layer for the FR rows held in LDS: out(m, n) = act(sum_k in(m, k) W(n, k) + b(n)).
// Fragments: frag[((nt * KS + ks) * 2 + part) * 64 + lane], part 0 = hi, 1 = lo, holding
// W(nt*32 + lane%32, ks*16 + 8*(lane/32) + e), e = 0..7.
template <int KIN, int NOUT, bool RELU, bool TO_GLOBAL>
__device__ inline void fcn_layer(const _Float16 *in, _Float16 *out_lds, float *out_g, int64_t out_row0, int nrows,
                                 const v8h *__restrict__ frag, const float *__restrict__ bias) {
    constexpr int KS = KIN / 16, NT = NOUT / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, kh = 8 * (lane >> 5);
    for (int nt = wave; nt < NT; nt += FWAVES) {
        v16f acc[FMT];
#pragma unroll
        for (int mt = 0; mt < FMT; ++mt) acc[mt] = (v16f){};
        const v8h *f = frag + (size_t)(nt * KS * 2) * 64;
        v8h bhi = f[lane], blo = f[64 + lane];
        for (int ks = 0; ks < KS; ++ks) {
            v8h nhi = bhi, nlo = blo;
            if (ks + 1 < KS) {
                nhi = f[(size_t)(ks + 1) * 128 + lane];
                nlo = f[(size_t)(ks + 1) * 128 + 64 + lane];
            }
#pragma unroll
            for (int mt = 0; mt < FMT; ++mt) {
                const _Float16 *row = in + (mt * 32 + m) * APITCH + ks * 16 + kh;
                const v8h ahi = *reinterpret_cast<const v8h *>(row);
                const v8h alo = *reinterpret_cast<const v8h *>(row + ABUF);
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, bhi, acc[mt], 0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, blo, acc[mt], 0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, bhi, acc[mt], 0, 0, 0);
            }
            bhi = nhi;
            blo = nlo;
        }
        const int n = nt * 32 + m;
        const float bn = bias[n];
#pragma unroll
        for (int mt = 0; mt < FMT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = mt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                float v = acc[mt][r] + bn;
                if (RELU) v = fmaxf(v, 0.f);
                if (TO_GLOBAL) {
                    if (row < nrows) out_g[(out_row0 + row) * NOUT + n] = v;
                } else {
                    put_split(out_lds, row, n, v);
                }
            }
    }
}

// Sums of the K members of group r, pixel row i of the patch, into s[c*8 + j] (integers).
// Positions are clamped into the image (they come from the caller for the means entry point).
// A member's row (8C bytes) is read as the 2C + 1 aligned dwords around it and realigned with
// alignbyte; where those dwords would pass the end of the image it is read byte by byte.
template <int C>
__device__ inline void member_row_sums(const uint8_t *img, int64_t stride, int h, int w, const int32_t *grp, int K,
                                       int i, int *s) {
    constexpr int NW = 2 * C;   // dwords of one row of a patch
#pragma unroll
    for (int e = 0; e < 8 * C; ++e) s[e] = 0;
    const uint8_t *img_end = img + (int64_t)(h - 1) * stride + (int64_t)w * C;
    for (int k = 0; k < K; ++k) {
        const int32_t lin = max(grp[k], 0);
        const int y = min(lin / w, h - 8), x = min(lin % w, w - 8);
        const uint8_t *p = img + (int64_t)(y + i) * stride + (int64_t)x * C;
        const uintptr_t pa = reinterpret_cast<uintptr_t>(p);
        const uint32_t *q = reinterpret_cast<const uint32_t *>(pa & ~(uintptr_t)3);
        if (reinterpret_cast<const uint8_t *>(q + NW + 1) <= img_end) {
            const uint32_t off = (uint32_t)(pa & 3);
            uint32_t wv[NW + 1];
#pragma unroll
            for (int t = 0; t <= NW; ++t) wv[t] = q[t];
#pragma unroll
            for (int t = 0; t < NW; ++t) {
                const uint32_t d = __builtin_amdgcn_alignbyte(wv[t + 1], wv[t], off);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int e = 4 * t + b;   // byte e of the row: pixel e / C, channel e % C
                    s[(e % C) * 8 + e / C] += (d >> (8 * b)) & 0xffu;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
                for (int ch = 0; ch < C; ++ch) s[ch * 8 + j] += p[j * C + ch];
        }
    }
}

// Mean patches of the groups, slice-major (c, 8, 8) per group, FP32 (exact for K a power of two).
template <int C>
__global__ __launch_bounds__(256) void means_kernel(const uint8_t *__restrict__ img, int64_t stride, int h, int w,
                                                    const int32_t *__restrict__ idx, int idx_stride, int K,
                                                    int64_t n_ref, float *__restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_ref * 8) return;
    const int64_t r = t >> 3;
    const int i = (int)(t & 7);
    int s[8 * C];
    member_row_sums<C>(img, stride, h, w, idx + r * idx_stride, K, i, s);
    const float inv = 1.f / (float)K;
#pragma unroll
    for (int ch = 0; ch < C; ++ch)
#pragma unroll
        for (int j = 0; j < 8; ++j) out[r * 64 * C + ch * 64 + i * 8 + j] = (float)s[ch * 8 + j] * inv;
}

struct FcnArgs {
    // input: either mean patches (means != nullptr) or groups of an image
    const float *means;
    const uint8_t *img;
    int64_t stride;
    int h, w;
    const int32_t *idx;
    int idx_stride, K;
    int64_t n;
    const v8h *f1, *f2, *f3;
    const float *b1, *b2, *b3;
    float *out;                 // n x P
    // RA flags from the thresholds (groups input only): flag = tau / mult > sigma_min
    const double *tau;
    double inv_mult, sigma_min;
    uint8_t *flags;
};

template <int C>
__global__ __launch_bounds__(FTHREADS) void fcn_fwd_kernel(FcnArgs a) {
    constexpr int P = 64 * C, H = C == 3 ? 256 : 128;
    extern __shared__ __align__(16) _Float16 fcn_smem[];   // two split activation buffers
    _Float16 *bufA = fcn_smem, *bufB = fcn_smem + 2 * ABUF;
    const int64_t r0 = (int64_t)blockIdx.x * FR;
    const int nr = (int)min<int64_t>(FR, a.n - r0);
    const int tid = threadIdx.x;
    // ---- inputs x = (p - 128) / 128 into bufA (rows past the end are zero) ----
    if (a.means) {
        for (int e = tid; e < FR * P; e += FTHREADS) {
            const int m = e / P, q = e % P;
            put_split(bufA, m, q, m < nr ? (a.means[(r0 + m) * P + q] - 128.f) * (1.f / 128.f) : 0.f);
        }
    } else {
        const int m = tid >> 3, i = tid & 7;
        int s[8 * C];
        if (m < nr) {
            member_row_sums<C>(a.img, a.stride, a.h, a.w, a.idx + (r0 + m) * a.idx_stride, a.K, i, s);
        } else {
#pragma unroll
            for (int e = 0; e < 8 * C; ++e) s[e] = 0;
        }
        const float inv = 1.f / (float)a.K;
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                put_split(bufA, m, ch * 64 + i * 8 + j,
                          m < nr ? ((float)s[ch * 8 + j] * inv - 128.f) * (1.f / 128.f) : 0.f);
        if (a.flags && tid < nr) a.flags[r0 + tid] = a.tau[r0 + tid] * a.inv_mult > a.sigma_min ? 1 : 0;
    }
    __syncthreads();
    fcn_layer<P, H, true, false>(bufA, bufB, nullptr, 0, nr, a.f1, a.b1);
    __syncthreads();
    fcn_layer<H, H, true, false>(bufB, bufA, nullptr, 0, nr, a.f2, a.b2);
    __syncthreads();
    fcn_layer<H, P, false, true>(bufA, nullptr, a.out, r0, nr, a.f3, a.b3);
}

// ---------------- training (FP32, vector units) ----------------

// C(m, n) = sum_k A(m, k) B(k, n) (+ bias(n), then ReLU when asked), with A(m, k) at
// A[m * sam + k * sak] and B(k, n) at B[k * sbk + n * sbn]; 64 x 64 tiles, 4 x 4 per thread.
__global__ __launch_bounds__(256) void mm_kernel(const float *__restrict__ A, int64_t sam, int64_t sak,
                                                 const float *__restrict__ B, int64_t sbk, int64_t sbn,
                                                 float *__restrict__ Cm, int M, int N, int Kd,
                                                 const float *__restrict__ bias, int relu) {
    __shared__ float As[16][64 + 1];
    __shared__ float Bs[16][64 + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < Kd; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < M && gk < Kd) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.f;
            const int gn = n0 + mm;
            Bs[kk][mm] = (gn < N && gk < Kd) ? B[(int64_t)gk * sbk + (int64_t)gn * sbn] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gm = m0 + ty * 4 + i, gn = n0 + tx * 4 + j;
            if (gm < M && gn < N) {
                float v = acc[i][j] + (bias ? bias[gn] : 0.f);
                if (relu) v = fmaxf(v, 0.f);
                Cm[(int64_t)gm * N + gn] = v;
            }
        }
}

// x = (p - 128) / 128 for a batch of mean patches.
__global__ void scale_in_kernel(const float *__restrict__ p, float *__restrict__ x, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) x[e] = (p[e] - 128.f) * (1.f / 128.f);
}

// d = 2 (r - (noisy - clean) / 128) / count; per-block partial sums of (r - target)^2.
__global__ void mse_kernel(const float *__restrict__ r, const float *__restrict__ noisy,
                           const float *__restrict__ clean, int64_t count, float *__restrict__ d,
                           double *__restrict__ partial) {
    __shared__ double red[256];
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (e < count) {
        const float t = (noisy[e] - clean[e]) * (1.f / 128.f);
        const float df = r[e] - t;
        d[e] = 2.f * df / (float)count;
        sq = (double)df * df;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dz = dh where the layer's output was positive (h = relu(z) > 0), else 0.
__global__ void relu_back_kernel(float *__restrict__ dz, const float *__restrict__ h, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n && !(h[e] > 0.f)) dz[e] = 0.f;
}

// db(j) = sum over the batch of dz(i, j), in a fixed order.
__global__ void colsum_kernel(const float *__restrict__ dz, int rows, int cols, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += dz[(int64_t)i * cols + j];
    db[j] = s;
}

__global__ void adam_f32_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                                float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t mm(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *Cm, int M,
              int N, int Kd, const float *bias, int relu, hipStream_t st) {
    hipLaunchKernelGGL(mm_kernel, dim3(nblocks(N, 64), nblocks(M, 64)), dim3(256), 0, st, A, sam, sak, B, sbk, sbn,
                       Cm, M, N, Kd, bias, relu);
    return hipGetLastError();
}

}  // namespace

int ra_hidden(int c) { return c == 3 ? 256 : 128; }

int ra_param_count(int c) {
    const int P = 64 * c, H = ra_hidden(c);
    return H * P + H + H * H + H + P * H + P;
}

size_t ra_frag_halves(int c) {
    const int P = 64 * c, H = ra_hidden(c);
    return (size_t)2 * (P * H + H * H + H * P);
}

hipError_t launch_ra_means(const uint8_t *img, int64_t stride, int h, int w, int c, const int32_t *idx,
                           int idx_stride, int K, int64_t n_ref, float *out, hipStream_t st) {
    if (n_ref <= 0) return hipSuccess;
    const unsigned g = nblocks(n_ref * 8, 256);
    if (c == 3)
        hipLaunchKernelGGL(means_kernel<3>, dim3(g), dim3(256), 0, st, img, stride, h, w, idx, idx_stride, K, n_ref,
                           out);
    else
        hipLaunchKernelGGL(means_kernel<1>, dim3(g), dim3(256), 0, st, img, stride, h, w, idx, idx_stride, K, n_ref,
                           out);
    return hipGetLastError();
}

hipError_t launch_ra_forward(int c, const RaWeightsDev &wd, bool folded, const float *means, const uint8_t *img,
                             int64_t stride, int h, int w, const int32_t *idx, int idx_stride, int K, int64_t n,
                             const double *tau, double mult, double sigma_min, uint8_t *flags, float *out,
                             hipStream_t st) {
    if (n <= 0) return hipSuccess;
    FcnArgs a;
    a.means = means;
    a.img = img;
    a.stride = stride;
    a.h = h;
    a.w = w;
    a.idx = idx;
    a.idx_stride = idx_stride;
    a.K = K;
    a.n = n;
    const v8h *fr = reinterpret_cast<const v8h *>(wd.frag);
    const int P = 64 * c, H = ra_hidden(c);
    a.f1 = fr;
    a.f2 = fr + (size_t)P * H * 2 / 8;
    a.f3 = a.f2 + (size_t)H * H * 2 / 8;
    if (folded) a.f3 = reinterpret_cast<const v8h *>(wd.frag3t);
    a.b1 = wd.bias;
    a.b2 = wd.bias + H;
    a.b3 = folded ? wd.bias3t : wd.bias + 2 * H;
    a.out = out;
    a.tau = tau;
    a.inv_mult = mult > 0.0 ? 1.0 / mult : 0.0;
    a.sigma_min = sigma_min;
    a.flags = flags;
    const unsigned g = nblocks(n, FR);
    const int lds = (int)(sizeof(_Float16) * 4 * ABUF);
    const void *kfn = c == 3 ? (const void *)fcn_fwd_kernel<3> : (const void *)fcn_fwd_kernel<1>;
    hipError_t e = prepare_dynamic_lds(kfn, lds, 0);
    if (e != hipSuccess) return e;
    if (c == 3)
        hipLaunchKernelGGL(fcn_fwd_kernel<3>, dim3(g), dim3(FTHREADS), lds, st, a);
    else
        hipLaunchKernelGGL(fcn_fwd_kernel<1>, dim3(g), dim3(FTHREADS), lds, st, a);
    return hipGetLastError();
}

size_t ra_train_ws_floats(int c, int n) {
    const int P = 64 * c, H = ra_hidden(c);
    return (size_t)n * (P + H + H + P) * 2 + (size_t)n * P + 4096;
}

// Loss and gradient of one batch (FP32 master weights w, flattened W1, b1, W2, b2, W3, b3).
hipError_t ra_gradients(int c, const float *w, const float *noisy, const float *clean, int n, float *grad,
                        float *ws, double *partial, int *n_partial, hipStream_t st) {
    const int P = 64 * c, H = ra_hidden(c);
    const float *W1 = w, *b1 = W1 + H * P, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + P * H;
    float *gW1 = grad, *gb1 = gW1 + H * P, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H, *gb3 = gW3 + P * H;
    float *x = ws, *h1 = x + (size_t)n * P, *h2 = h1 + (size_t)n * H, *r = h2 + (size_t)n * H;
    float *dr = r + (size_t)n * P, *dh2 = dr + (size_t)n * P, *dh1 = dh2 + (size_t)n * H;
    hipError_t e;
    hipLaunchKernelGGL(scale_in_kernel, dim3(nblocks((int64_t)n * P, 256)), dim3(256), 0, st, noisy, x, (int64_t)n * P);
    // forward: h1 = relu(x W1^T + b1), h2 = relu(h1 W2^T + b2), r = h2 W3^T + b3
    if ((e = mm(x, P, 1, W1, 1, P, h1, n, H, P, b1, 1, st)) != hipSuccess) return e;
    if ((e = mm(h1, H, 1, W2, 1, H, h2, n, H, H, b2, 1, st)) != hipSuccess) return e;
    if ((e = mm(h2, H, 1, W3, 1, H, r, n, P, H, b3, 0, st)) != hipSuccess) return e;
    const int64_t cnt = (int64_t)n * P;
    *n_partial = (int)nblocks(cnt, 256);
    hipLaunchKernelGGL(mse_kernel, dim3(*n_partial), dim3(256), 0, st, r, noisy, clean, cnt, dr, partial);
    // backward
    if ((e = mm(dr, 1, P, h2, H, 1, gW3, P, H, n, nullptr, 0, st)) != hipSuccess) return e;     // dr^T h2
    hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(P, 256)), dim3(256), 0, st, dr, n, P, gb3);
    if ((e = mm(dr, P, 1, W3, H, 1, dh2, n, H, P, nullptr, 0, st)) != hipSuccess) return e;     // dr W3
    hipLaunchKernelGGL(relu_back_kernel, dim3(nblocks((int64_t)n * H, 256)), dim3(256), 0, st, dh2, h2, (int64_t)n * H);
    if ((e = mm(dh2, 1, H, h1, H, 1, gW2, H, H, n, nullptr, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(H, 256)), dim3(256), 0, st, dh2, n, H, gb2);
    if ((e = mm(dh2, H, 1, W2, H, 1, dh1, n, H, H, nullptr, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(relu_back_kernel, dim3(nblocks((int64_t)n * H, 256)), dim3(256), 0, st, dh1, h1, (int64_t)n * H);
    if ((e = mm(dh1, 1, H, x, P, 1, gW1, H, P, n, nullptr, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(H, 256)), dim3(256), 0, st, dh1, n, H, gb1);
    return hipGetLastError();
}

hipError_t ra_adam(float *w, float *m, float *v, const float *g, int n, float lr, int64_t step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_f32_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace htsvd
