// Learned noise-level network: a 6-layer 3x3 convolutional net that predicts log(sigma)
// for every 8x8 block (the paper's estimator is a CNN, Sec. III-E-1 and Fig. 5; its data
// and weights are not available, so this network is trained here on synthetic crops).
//
//   x0 = (u8 - 128) / 64 (NHWC, C = 1 or 3)
//   L1 3x3 C->32 stride 2 ReLU | L2 32->32 s2 ReLU | L3 32->32 s2 ReLU
//   L4 32->32 s1 ReLU | L5 32->32 s1 ReLU | L6 32->1 s1 (linear) -> z = log(sigma)
//   loss = mean |z - log(sigma_target)|
//
// Storage: activations NHWC bf16 (round to nearest even), weights bf16 for the forward pass
// with FP32 master copies, FP32 accumulation everywhere.  Parameters are one flat array in
// layer order, each layer w[co][ky][kx][ci] then b[co].
//
// Kernels: the 32->32 convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (16 output
// pixels x 16 output channels per instruction, k = the 32 input channels of one tap, 9 taps);
// layer 1 (3 input channels) and layer 6 (1 output channel) run on the vector ALUs.  The
// backward pass (input and weight gradients, FP32) and Adam run on the vector ALUs.
#include <math.h>

#include "common.h"

namespace htsvd {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ __host__ inline uint16_t f2bf(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __host__ inline float bf2f(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

struct ConvShape {
    int N, H, W, Ci;    // input
    int Ho, Wo, Co;     // output
    int s;              // stride
};

// ---- layer 1: u8 image -> 32 channels, vector ALU ----
// One thread per output pixel; the 9 C input taps stay in registers, the weights are uniform
// across the wavefront (scalar loads), the 32 outputs leave as four 16-byte stores.  Image n
// starts at img + n img_batch_stride with row stride img_stride, or, with a table, at
// img_tab[n] with row stride stride_tab[n] (images of one size in separate buffers).
template <int C>
__global__ __launch_bounds__(256) void l1_fwd_kernel(const uint8_t *__restrict__ img, int64_t img_stride,
                                                     int64_t img_batch_stride,
                                                     const uint8_t *const *__restrict__ img_tab,
                                                     const int64_t *__restrict__ stride_tab, ConvShape cs,
                                                     const float *__restrict__ wq, const float *__restrict__ bias,
                                                     uint16_t *__restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)cs.N * cs.Ho * cs.Wo;
    if (p >= total) return;
    const int n = (int)(p / ((int64_t)cs.Ho * cs.Wo));
    const int rem = (int)(p % ((int64_t)cs.Ho * cs.Wo));
    const int yo = rem / cs.Wo, xo = rem % cs.Wo;
    const uint8_t *ibase = img_tab ? img_tab[n] : img + n * img_batch_stride;
    const int64_t rs = img_tab ? stride_tab[n] : img_stride;
    float x[9 * C];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yi = cs.s * yo + t / 3 - 1, xi = cs.s * xo + t % 3 - 1;
        const bool ok = yi >= 0 && yi < cs.H && xi >= 0 && xi < cs.W;
#pragma unroll
        for (int ci = 0; ci < C; ++ci) x[t * C + ci] = 0.f;
        if (ok) {
            const uint8_t *src = ibase + (int64_t)yi * rs + (int64_t)xi * C;
#pragma unroll
            for (int ci = 0; ci < C; ++ci) x[t * C + ci] = ((float)src[ci] - 128.f) * 0.015625f;
        }
    }
    uint32_t packed[16];
#pragma unroll
    for (int co = 0; co < 32; ++co) {
        float acc = bias[co];
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int ci = 0; ci < C; ++ci) acc += wq[(co * 9 + t) * C + ci] * x[t * C + ci];
        const uint32_t h = f2bf(acc > 0.f ? acc : 0.f);
        packed[co >> 1] = (co & 1) ? (packed[co >> 1] | (h << 16)) : h;
    }
    uint4 *o = reinterpret_cast<uint4 *>(out + p * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
}

// ---- 32 -> 32 convolution on the matrix cores ----
// One wavefront computes 16 output pixels x 32 output channels per tile; weights live in
// registers (9 taps x 2 channel tiles of 8 bf16 per lane).
__global__ __launch_bounds__(256) void conv32_fwd_kernel(const uint16_t *__restrict__ in, ConvShape cs,
                                                         const uint16_t *__restrict__ wbf,
                                                         const float *__restrict__ bias,
                                                         uint16_t *__restrict__ out, int relu) {
    const int lane = threadIdx.x & 63;
    const int wave_global = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int n_waves = (gridDim.x * blockDim.x) >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    v8bf bw[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const uint4 raw = *reinterpret_cast<const uint4 *>(wbf + ((16 * nt + i16) * 9 + t) * 32 + 8 * kq);
            bw[t][nt] = __builtin_bit_cast(v8bf, raw);
        }
    const float b0 = bias[i16], b1 = bias[16 + i16];
    const int64_t total = (int64_t)cs.N * cs.Ho * cs.Wo;
    const int64_t n_tiles = (total + 15) / 16;
    for (int64_t tile = wave_global; tile < n_tiles; tile += n_waves) {
        const int64_t p = tile * 16 + i16;
        const bool pv = p < total;
        const int64_t pp = pv ? p : 0;
        const int n = (int)(pp / ((int64_t)cs.Ho * cs.Wo));
        const int rem = (int)(pp % ((int64_t)cs.Ho * cs.Wo));
        const int yo = rem / cs.Wo, xo = rem % cs.Wo;
        v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yi = cs.s * yo + t / 3 - 1, xi = cs.s * xo + t % 3 - 1;
            uint4 raw = {0u, 0u, 0u, 0u};
            if (pv && yi >= 0 && yi < cs.H && xi >= 0 && xi < cs.W)
                raw = *reinterpret_cast<const uint4 *>(in + (((int64_t)n * cs.H + yi) * cs.W + xi) * 32 + 8 * kq);
            const v8bf a = __builtin_bit_cast(v8bf, raw);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t][0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t][1], acc1, 0, 0, 0);
        }
        // lane holds pixels 4*kq + r of the tile, channel i16 (and 16 + i16)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t q = tile * 16 + 4 * kq + r;
            if (q < total) {
                float v0 = acc0[r] + b0, v1 = acc1[r] + b1;
                if (relu) { v0 = v0 > 0.f ? v0 : 0.f; v1 = v1 > 0.f ? v1 : 0.f; }
                out[q * 32 + i16] = f2bf(v0);
                out[q * 32 + 16 + i16] = f2bf(v1);
            }
        }
    }
}

// ---- layer 6: 32 -> 1, vector ALU, FP32 output ----
__global__ void l6_fwd_kernel(const uint16_t *__restrict__ in, ConvShape cs, const float *__restrict__ wq,
                              const float *__restrict__ bias, float *__restrict__ z) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)cs.N * cs.Ho * cs.Wo;
    if (p >= total) return;
    const int n = (int)(p / ((int64_t)cs.Ho * cs.Wo));
    const int rem = (int)(p % ((int64_t)cs.Ho * cs.Wo));
    const int yo = rem / cs.Wo, xo = rem % cs.Wo;
    float acc = bias[0];
    for (int t = 0; t < 9; ++t) {
        const int yi = yo + t / 3 - 1, xi = xo + t % 3 - 1;
        if (yi < 0 || yi >= cs.H || xi < 0 || xi >= cs.W) continue;
        const uint16_t *a = in + (((int64_t)n * cs.H + yi) * cs.W + xi) * 32;
        for (int ci = 0; ci < 32; ++ci) acc += wq[t * 32 + ci] * bf2f(a[ci]);
    }
    z[p] = acc;
}

// ---- loss: mean |z - t|, dz = sign(z - t) / count ----
__global__ void l1loss_kernel(const float *__restrict__ z, const float *__restrict__ t, int64_t count,
                              float *__restrict__ dz, double *__restrict__ loss_sum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < count) {
        const float d = z[i] - t[i];
        dz[i] = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) / (float)count;
        v = fabs((double)d);
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss_sum, v);
}

// dY *= (activation > 0)  (ReLU backward; activations are post-ReLU bf16)
__global__ void relu_mask_kernel(float *__restrict__ dy, const uint16_t *__restrict__ act, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(bf2f(act[i]) > 0.f)) dy[i] = 0.f;
}

// Input of a convolution as FP32: bf16 activations, or the normalised u8 image for layer 1.
struct ConvIn {
    const uint16_t *act;   // NHWC bf16 (Ci channels), or null
    const uint8_t *img;    // NHWC u8, when act is null
    int64_t img_stride, img_batch_stride;
    __device__ inline float at(int n, int y, int x, int ci, const ConvShape &cs) const {
        if (act) return bf2f(act[(((int64_t)n * cs.H + y) * cs.W + x) * cs.Ci + ci]);
        return ((float)img[n * img_batch_stride + (int64_t)y * img_stride + (int64_t)x * cs.Ci + ci] - 128.f) * 0.015625f;
    }
};

// dW[co][tap][ci] += sum_p dY[p][co] * X[in(p, tap)][ci];  db[co] += sum_p dY[p][co].
// grid: (Co, pixel chunks); block: 9*Ci threads, one per (tap, ci).
__global__ void wgrad_kernel(ConvIn xin, ConvShape cs, const float *__restrict__ dy, int64_t chunk,
                             float *__restrict__ dw, float *__restrict__ db) {
    const int co = blockIdx.x;
    const int t = threadIdx.x / cs.Ci, ci = threadIdx.x % cs.Ci;
    if (t >= 9) return;
    const int64_t total = (int64_t)cs.N * cs.Ho * cs.Wo;
    const int64_t p0 = (int64_t)blockIdx.y * chunk, p1 = min(total, p0 + chunk);
    const int ky = t / 3, kx = t % 3;
    float acc = 0.f, accb = 0.f;
    for (int64_t p = p0; p < p1; ++p) {
        const float g = dy[p * cs.Co + co];
        if (g == 0.f) continue;
        const int n = (int)(p / ((int64_t)cs.Ho * cs.Wo));
        const int rem = (int)(p % ((int64_t)cs.Ho * cs.Wo));
        const int yi = cs.s * (rem / cs.Wo) + ky - 1, xi = cs.s * (rem % cs.Wo) + kx - 1;
        accb += g;
        if (yi < 0 || yi >= cs.H || xi < 0 || xi >= cs.W) continue;
        acc += g * xin.at(n, yi, xi, ci, cs);
    }
    atomicAdd(dw + (co * 9 + t) * cs.Ci + ci, acc);
    if (threadIdx.x == 0) atomicAdd(db + co, accb);
}

// dX[q][ci] = sum_{tap, co} dY[out(q, tap)][co] * W[co][tap][ci]; one thread per (q, ci).
__global__ void dgrad_kernel(const float *__restrict__ dy, ConvShape cs, const float *__restrict__ wq,
                             float *__restrict__ dx) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)cs.N * cs.H * cs.W * cs.Ci;
    if (e >= total) return;
    const int ci = (int)(e % cs.Ci);
    const int64_t q = e / cs.Ci;
    const int n = (int)(q / ((int64_t)cs.H * cs.W));
    const int rem = (int)(q % ((int64_t)cs.H * cs.W));
    const int yi = rem / cs.W, xi = rem % cs.W;
    float acc = 0.f;
    for (int t = 0; t < 9; ++t) {
        const int ky = t / 3, kx = t % 3;
        const int ny = yi + 1 - ky, nx = xi + 1 - kx;     // = s * yo
        if (ny < 0 || nx < 0 || ny % cs.s || nx % cs.s) continue;
        const int yo = ny / cs.s, xo = nx / cs.s;
        if (yo >= cs.Ho || xo >= cs.Wo) continue;
        const float *g = dy + (((int64_t)n * cs.Ho + yo) * cs.Wo + xo) * cs.Co;
        for (int co = 0; co < cs.Co; ++co) acc += g[co] * wq[(co * 9 + t) * cs.Ci + ci];
    }
    dx[e] = acc;
}

__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2, float *__restrict__ wq, uint16_t *__restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    const uint16_t hb = f2bf(wi);
    wbf[i] = hb;
    wq[i] = bf2f(hb);
}

__global__ void quantize_kernel(const float *__restrict__ w, int n, float *__restrict__ wq, uint16_t *__restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint16_t hb = f2bf(w[i]);
    wbf[i] = hb;
    wq[i] = bf2f(hb);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// Offsets of each layer's weights and bias in the flat parameter array.
void cnn_layout(int c, int *w_off, int *b_off, int *total) {
    const int ci[6] = {c, 32, 32, 32, 32, 32}, co[6] = {32, 32, 32, 32, 32, 1};
    int off = 0;
    for (int l = 0; l < 6; ++l) {
        w_off[l] = off;
        off += co[l] * 9 * ci[l];
        b_off[l] = off;
        off += co[l];
    }
    *total = off;
}

static ConvShape shape_of(int l, int N, int H, int W, int c) {
    // l = 0..5: the layer; its input size is the output size of the layers before it
    // spatial size entering layer l
    int h = H, w = W;
    const int strides[6] = {2, 2, 2, 1, 1, 1};
    for (int k = 0; k < l; ++k) {
        h = (h + strides[k] - 1) / strides[k];
        w = (w + strides[k] - 1) / strides[k];
    }
    ConvShape cs;
    cs.N = N; cs.H = h; cs.W = w;
    cs.Ci = l == 0 ? c : 32;
    cs.Co = l == 5 ? 1 : 32;
    cs.s = strides[l];
    cs.Ho = (h + cs.s - 1) / cs.s;
    cs.Wo = (w + cs.s - 1) / cs.s;
    return cs;
}

// Activation sizes (elements) for a batch: a[1..5] bf16 (32 channels), z FP32.
size_t cnn_act_elems(int l, int N, int H, int W, int c) {
    ConvShape cs = shape_of(l - 1, N, H, W, c);
    return (size_t)cs.N * cs.Ho * cs.Wo * cs.Co;
}

static hipError_t forward_impl(const CnnBuffers &b, const uint8_t *img, int64_t img_stride,
                               int64_t img_batch_stride, const uint8_t *const *img_tab, const int64_t *stride_tab,
                               int N, int H, int W, int c, hipStream_t st) {
    int wo[6], bo[6], tot;
    cnn_layout(c, wo, bo, &tot);
    ConvShape cs = shape_of(0, N, H, W, c);
    int64_t np = (int64_t)cs.N * cs.Ho * cs.Wo;
    if (c == 3)
        hipLaunchKernelGGL(l1_fwd_kernel<3>, dim3(blocks_for(np, 256)), dim3(256), 0, st, img, img_stride,
                           img_batch_stride, img_tab, stride_tab, cs, b.wq + wo[0], b.wq + bo[0], b.act[1]);
    else if (c == 1)
        hipLaunchKernelGGL(l1_fwd_kernel<1>, dim3(blocks_for(np, 256)), dim3(256), 0, st, img, img_stride,
                           img_batch_stride, img_tab, stride_tab, cs, b.wq + wo[0], b.wq + bo[0], b.act[1]);
    else
        return hipErrorInvalidValue;
    for (int l = 1; l < 5; ++l) {
        cs = shape_of(l, N, H, W, c);
        np = (int64_t)cs.N * cs.Ho * cs.Wo;
        const int64_t tiles = (np + 15) / 16;
        const int64_t want = (tiles + 3) / 4;
        const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
        hipLaunchKernelGGL(conv32_fwd_kernel, dim3(grid), dim3(256), 0, st, b.act[l], cs, b.wbf + wo[l],
                           b.wq + bo[l], b.act[l + 1], 1);
    }
    cs = shape_of(5, N, H, W, c);
    np = (int64_t)cs.N * cs.Ho * cs.Wo;
    hipLaunchKernelGGL(l6_fwd_kernel, dim3(blocks_for(np, 256)), dim3(256), 0, st, b.act[5], cs, b.wq + wo[5],
                       b.wq + bo[5], b.z);
    return hipGetLastError();
}

hipError_t cnn_forward(const CnnBuffers &b, const uint8_t *img, int64_t img_stride, int64_t img_batch_stride,
                       int N, int H, int W, int c, hipStream_t st) {
    return forward_impl(b, img, img_stride, img_batch_stride, nullptr, nullptr, N, H, W, c, st);
}

hipError_t cnn_forward_tab(const CnnBuffers &b, const uint8_t *const *img_tab, const int64_t *stride_tab, int N,
                           int H, int W, int c, hipStream_t st) {
    if (!img_tab || !stride_tab) return hipErrorInvalidValue;
    return forward_impl(b, nullptr, 0, 0, img_tab, stride_tab, N, H, W, c, st);
}

// Backward pass: grads (FP32, zeroed here) of mean |z - target|; d0/d1 are FP32 scratch
// buffers large enough for the largest activation.
hipError_t cnn_backward(const CnnBuffers &b, const uint8_t *img, int64_t img_stride, int64_t img_batch_stride,
                        int N, int H, int W, int c, const float *target, float *grads, float *d0, float *d1,
                        double *loss_sum, hipStream_t st) {
    int wo[6], bo[6], tot;
    cnn_layout(c, wo, bo, &tot);
    hipError_t e = launch_zero(grads, sizeof(float) * tot, st);
    if (e != hipSuccess) return e;
    e = launch_zero(loss_sum, sizeof(double), st);
    if (e != hipSuccess) return e;
    ConvShape cs = shape_of(5, N, H, W, c);
    const int64_t nz = (int64_t)cs.N * cs.Ho * cs.Wo;
    float *dy = d0, *dx = d1;
    hipLaunchKernelGGL(l1loss_kernel, dim3(blocks_for(nz, 256)), dim3(256), 0, st, b.z, target, nz, dy, loss_sum);
    for (int l = 5; l >= 0; --l) {
        cs = shape_of(l, N, H, W, c);
        const int64_t np = (int64_t)cs.N * cs.Ho * cs.Wo;
        if (l < 5) {
            hipLaunchKernelGGL(relu_mask_kernel, dim3(blocks_for(np * cs.Co, 256)), dim3(256), 0, st, dy, b.act[l + 1],
                               np * cs.Co);
        }
        ConvIn xin;
        xin.act = l == 0 ? nullptr : b.act[l];
        xin.img = img;
        xin.img_stride = img_stride;
        xin.img_batch_stride = img_batch_stride;
        const int64_t chunk = 256;
        const int64_t nchunks = (np + chunk - 1) / chunk;
        hipLaunchKernelGGL(wgrad_kernel, dim3(cs.Co, (unsigned)nchunks), dim3(9 * cs.Ci), 0, st, xin, cs, dy, chunk,
                           grads + wo[l], grads + bo[l]);
        if (l > 0) {
            const int64_t nx = (int64_t)cs.N * cs.H * cs.W * cs.Ci;
            hipLaunchKernelGGL(dgrad_kernel, dim3(blocks_for(nx, 256)), dim3(256), 0, st, dy, cs, b.wq + wo[l], dx);
            float *t = dy; dy = dx; dx = t;
        }
    }
    return hipGetLastError();
}

hipError_t cnn_adam(float *w, float *m, float *v, const float *g, int n, float lr, int64_t step, float *wq,
                    uint16_t *wbf, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, c1, c2,
                       wq, wbf);
    return hipGetLastError();
}

hipError_t cnn_quantize(const float *w, int n, float *wq, uint16_t *wbf, hipStream_t st) {
    hipLaunchKernelGGL(quantize_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, w, n, wq, wbf);
    return hipGetLastError();
}

uint16_t host_f2bf(float f) { return f2bf(f); }

}  // namespace htsvd
