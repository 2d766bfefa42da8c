// Collaborative filtering (Eq. 19-21) and aggregation (Algorithm 1) for Haar-tSVD on gfx950.
//
// Per group of K patches:
//   Eq. 19  S = U^T * G * V  x_4  H_K      (t-product via the 3-point DFT along the channel mode:
//                                            slice 0 real, slice 1 complex, slice 2 = conj(slice 1))
//   Eq. 20  keep |S| >= tau, zero the rest
//   Eq. 21  G_est = U * S_trunc * V^T  x_4  H_K^T
//   Algorithm 1: every patch of G_est is added into the image with weight 1, the output is the
//   sum divided by the number of patches that covered the pixel.
//
// Work decomposition.  A workgroup of 4 wavefronts owns a TY x TX tile of references; each
// wavefront filters one group at a time and adds the reconstructed patches into an LDS copy of
// the image region the tile's groups can reach (C sums + 1 count per pixel).  At the end the
// region goes, without atomics, to this tile's slot of a global buffer; the gather kernel then
// sums the (at most a few) regions covering each pixel and divides.  No global float atomics.
//
// Inside a wavefront the group sits in LDS as K x (64 C) floats.  For the separable patch
// transforms a lane owns one output index of an 8-vector (lane & 7) and keeps the matching
// column or row of the basis in registers, while the 8-vector it multiplies is broadcast from
// LDS to the 8 lanes that share it.  The Haar butterflies run in registers with one
// coefficient position (across all K members) per lane.
//
// Threshold guard band: an FP32 coefficient within GUARD of tau is recomputed in FP64 from the
// uint8 group and the FP64 transform matrix by the whole wavefront, and that value decides.
#include "common.h"

namespace htsvd {
namespace {

constexpr float R2F = 0.70710678118654752440f;
constexpr double R2D = 0.70710678118654752440;
constexpr float SQ3_2 = 0.86602540378443864676f;
constexpr float THIRD = 0.33333333333333333333f;
constexpr float SQ3 = 1.73205080756887729353f;
constexpr float GUARD_F = 0.05f;   // >> worst-case FP32 error of a coefficient of 8-bit data
constexpr int NEAR_CAP = 64;
constexpr int NWAVE = 4;

__device__ inline void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

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

// Entry (k, m) of H_n: H_n = 1/sqrt2 [H_{n/2} (x) [1,1]; I_{n/2} (x) [1,-1]], H_1 = [1].
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

// 8*C raw bytes of one patch row (8 pixels) starting at p; aligned dword loads where the
// buffer is known to extend far enough, bytes otherwise.
template <int C>
__device__ inline void load_row(const uint8_t *p, const uint8_t *end, float (&out)[8 * C]) {
    constexpr int NB = 8 * C;
    const uintptr_t a = (uintptr_t)p;
    const uint32_t *base = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
    const int sh = (int)(a & 3);
    constexpr int ND = NB / 4 + 1;
    if ((const uint8_t *)(base + ND) <= end) {
        uint32_t d[ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) d[i] = base[i];
#pragma unroll
        for (int i = 0; i < NB / 4; ++i) {
            const uint32_t v = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh * 1u);
            out[4 * i + 0] = (float)(v & 0xffu);
            out[4 * i + 1] = (float)((v >> 8) & 0xffu);
            out[4 * i + 2] = (float)((v >> 16) & 0xffu);
            out[4 * i + 3] = (float)(v >> 24);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NB; ++i) out[i] = (float)p[i];
    }
}

struct FilterShared {
    int near_k[NWAVE][NEAR_CAP], near_q[NWAVE][NEAR_CAP], near_n[NWAVE];
    int r0, c0;
};

// Filters every group of one reference tile and writes the tile's region (sums, counts).
template <int C, int K>
__device__ __forceinline__ void filter_tile(const ImageGeom &g, const TileGeom &tg, const float *__restrict__ B,
                                            const double *__restrict__ T64, const int32_t *__restrict__ idx,
                                            const double *__restrict__ tau_ref, float *__restrict__ regions,
                                            unsigned long long *__restrict__ guard_count, const int tile,
                                            float *smem, FilterShared &sh, const int idx_stride,
                                            const double tau_mul) {
    constexpr int P = 64 * C;
    constexpr int CH = C + 1;                     // sums + count per pixel
    auto &near_k = sh.near_k;
    auto &near_q = sh.near_q;
    auto &near_n = sh.near_n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ty = tile / tg.tiles_x, tx = tile % tg.tiles_x;

    float *region = smem;                               // [RH][RW][CH]
    float *buf = smem + tg.RH * tg.RW * CH + wave * K * P;
    const int region_elems = tg.RH * tg.RW * CH;
    if (tid == 0) {
        int r0, r1, c0, c1;
        region_rows(g, tg, ty, &r0, &r1);
        region_cols(g, tg, tx, &c0, &c1);
        sh.r0 = r0;
        sh.c0 = c0;
    }
    for (int e = tid; e < region_elems; e += 256) region[e] = 0.f;
    __syncthreads();
    const int r0 = sh.r0, c0 = sh.c0;
    const uint8_t *img_end = g.img + (int64_t)(g.h - 1) * g.stride + (int64_t)g.w * C;

    const float *U0 = B, *V0 = B + 64, *U1r = B + 128, *U1i = B + 192, *V1r = B + 256, *V1i = B + 320;
    const int l8 = lane & 7, sub = lane >> 3;

    const int iy0 = ty * tg.TY, ix0 = tx * tg.TX;
    const int ny_t = min(tg.TY, g.ny - iy0), nx_t = min(tg.TX, g.nx - ix0);
    for (int t = wave; t < ny_t * nx_t; t += NWAVE) {
        const int64_t r = (int64_t)(iy0 + t / nx_t) * g.nx + (ix0 + t % nx_t);
        const double tau = tau_ref[r] * tau_mul;
        const float tauf = (float)tau;
        const bool guard_on = tau > (double)GUARD_F;
        if (lane == 0) near_n[wave] = 0;

        // ---- phase 0: gather rows, channel DFT (slice 0 real, slice 1 = re + i im) ----
        // task = (member m, row a), 8K tasks over 64 lanes
#pragma unroll 1
        for (int task = lane; task < 8 * K; task += 64) {
            const int m = task >> 3, a = task & 7;
            const int32_t lin = idx[r * idx_stride + m];
            const int ym = lin / g.w, xm = lin % g.w;
            float px[8 * C];
            load_row<C>(g.img + (int64_t)(ym + a) * g.stride + (int64_t)xm * C, img_end, px);
            float *row = buf + m * P + a * 8;
            if (C == 3) {
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const float R = px[3 * b], G = px[3 * b + 1], Bc = px[3 * b + 2];
                    row[b] = R + G + Bc;
                    row[64 + b] = R - 0.5f * (G + Bc);
                    row[128 + b] = SQ3_2 * (Bc - G);
                }
            } else {
#pragma unroll
                for (int b = 0; b < 8; ++b) row[b] = px[b];
            }
        }
        wave_lds_sync();

        // ---- phase 1: X = G_hat V_hat (lane: output column j = l8; task: member, row) ----
        {
            float v0[8], vr[8], vi[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                v0[b] = V0[b * 8 + l8];
                if (C == 3) { vr[b] = V1r[b * 8 + l8]; vi[b] = V1i[b * 8 + l8]; }
            }
#pragma unroll 2
            for (int task = sub; task < 8 * K; task += 8) {
                float *row = buf + (task >> 3) * P + (task & 7) * 8;
                float g0[8];
#pragma unroll
                for (int b = 0; b < 8; ++b) g0[b] = row[b];
                float x0 = 0.f;
#pragma unroll
                for (int b = 0; b < 8; ++b) x0 += g0[b] * v0[b];
                if (C == 3) {
                    float gr[8], gi[8];
#pragma unroll
                    for (int b = 0; b < 8; ++b) { gr[b] = row[64 + b]; gi[b] = row[128 + b]; }
                    float xr = 0.f, xi = 0.f;
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        xr += gr[b] * vr[b] - gi[b] * vi[b];
                        xi += gr[b] * vi[b] + gi[b] * vr[b];
                    }
                    row[64 + l8] = xr;
                    row[128 + l8] = xi;
                }
                row[l8] = x0;
            }
        }
        wave_lds_sync();

        // ---- phase 2: S_hat = U_hat^H X, inverse channel DFT (lane: output row i = l8; task: member, column) ----
        {
            float u0[8], ur[8], ui[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                u0[a] = U0[a * 8 + l8];
                if (C == 3) { ur[a] = U1r[a * 8 + l8]; ui[a] = U1i[a * 8 + l8]; }
            }
#pragma unroll 2
            for (int task = sub; task < 8 * K; task += 8) {
                float *col = buf + (task >> 3) * P + (task & 7);
                float x0[8];
#pragma unroll
                for (int a = 0; a < 8; ++a) x0[a] = col[a * 8];
                float s0 = 0.f;
#pragma unroll
                for (int a = 0; a < 8; ++a) s0 += u0[a] * x0[a];
                if (C == 3) {
                    float xr[8], xi[8];
#pragma unroll
                    for (int a = 0; a < 8; ++a) { xr[a] = col[64 + a * 8]; xi[a] = col[128 + a * 8]; }
                    float sr = 0.f, si = 0.f;
#pragma unroll
                    for (int a = 0; a < 8; ++a) {
                        sr += ur[a] * xr[a] + ui[a] * xi[a];
                        si += ur[a] * xi[a] - ui[a] * xr[a];
                    }
                    col[l8 * 8] = (s0 + 2.f * sr) * THIRD;
                    col[64 + l8 * 8] = (s0 - sr - SQ3 * si) * THIRD;
                    col[128 + l8 * 8] = (s0 - sr + SQ3 * si) * THIRD;
                } else {
                    col[l8 * 8] = s0;
                }
            }
        }
        wave_lds_sync();

        // ---- phase 3: Haar along the group, threshold with FP64 guard band, inverse Haar ----
#pragma unroll 1
        for (int q = lane; q < P; q += 64) {
            float v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = buf[k * P + q];
            haar_fwd<K>(v);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float a = fabsf(v[k]);
                if (guard_on && fabsf(a - tauf) < GUARD_F) {
                    const int e = atomicAdd(&near_n[wave], 1);
                    if (e < NEAR_CAP) { near_k[wave][e] = k; near_q[wave][e] = q; }
                    else if (!(a >= tauf)) v[k] = 0.f;
                } else if (!(a >= tauf)) {
                    v[k] = 0.f;
                }
                buf[k * P + q] = v[k];
            }
        }
        wave_lds_sync();
        const int nn = near_n[wave];
        if (nn > 0) {
            if (lane == 0) {
                atomicAdd(guard_count, (unsigned long long)min(nn, NEAR_CAP));
                if (nn > NEAR_CAP) atomicAdd(guard_count + 1, (unsigned long long)(nn - NEAR_CAP));
            }
            for (int e = 0; e < min(nn, NEAR_CAP); ++e) {
                const int k = near_k[wave][e], q = near_q[wave][e];
                double part = 0.0;
                for (int p = lane; p < P; p += 64) {
                    const int ch = p / 64, i = (p / 8) % 8, j = p % 8;
                    double acc = 0.0;
                    for (int mm = 0; mm < K; ++mm) {
                        const double w = haar_weight(k, mm, K);
                        if (w == 0.0) continue;
                        const int32_t l2 = idx[r * idx_stride + mm];
                        const int y2 = l2 / g.w, x2 = l2 % g.w;
                        acc += w * (double)g.img[(int64_t)(y2 + i) * g.stride + (int64_t)(x2 + j) * C + ch];
                    }
                    part += T64[(int64_t)q * P + p] * acc;
                }
                const double s = wave_sum_f64(part);
                if (lane == 0 && !(fabs(s) >= tau)) buf[k * P + q] = 0.f;
            }
            wave_lds_sync();
        }
#pragma unroll 1
        for (int q = lane; q < P; q += 64) {
            float v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = buf[k * P + q];
            haar_inv<K>(v);
#pragma unroll
            for (int k = 0; k < K; ++k) buf[k * P + q] = v[k];
        }
        wave_lds_sync();

        // ---- phase 4: channel DFT of S', Y = U_hat S' (lane: output row a = l8; task: member, column) ----
        {
            float u0[8], ur[8], ui[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                u0[i] = U0[l8 * 8 + i];
                if (C == 3) { ur[i] = U1r[l8 * 8 + i]; ui[i] = U1i[l8 * 8 + i]; }
            }
#pragma unroll 2
            for (int task = sub; task < 8 * K; task += 8) {
                float *col = buf + (task >> 3) * P + (task & 7);
                if (C == 3) {
                    float s0[8], sr[8], si[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const float a = col[i * 8], b = col[64 + i * 8], c = col[128 + i * 8];
                        s0[i] = a + b + c;
                        sr[i] = a - 0.5f * (b + c);
                        si[i] = SQ3_2 * (c - b);
                    }
                    float y0 = 0.f, yr = 0.f, yi = 0.f;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        y0 += u0[i] * s0[i];
                        yr += ur[i] * sr[i] - ui[i] * si[i];
                        yi += ur[i] * si[i] + ui[i] * sr[i];
                    }
                    col[l8 * 8] = y0;
                    col[64 + l8 * 8] = yr;
                    col[128 + l8 * 8] = yi;
                } else {
                    float s0[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) s0[i] = col[i * 8];
                    float y0 = 0.f;
#pragma unroll
                    for (int i = 0; i < 8; ++i) y0 += u0[i] * s0[i];
                    col[l8 * 8] = y0;
                }
            }
        }
        wave_lds_sync();

        // ---- phase 5: P_hat = Y V_hat^H, inverse channel DFT, add into the LDS region ----
        {
            float v0[8], vr[8], vi[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                v0[j] = V0[l8 * 8 + j];
                if (C == 3) { vr[j] = V1r[l8 * 8 + j]; vi[j] = V1i[l8 * 8 + j]; }
            }
#pragma unroll 2
            for (int task = sub; task < 8 * K; task += 8) {
                const int m = task >> 3, a = task & 7;
                const float *row = buf + m * P + a * 8;
                const int32_t lin = idx[r * idx_stride + m];
                const int ym = lin / g.w, xm = lin % g.w;
                float *dst = region + ((ym + a - r0) * tg.RW + (xm + l8 - c0)) * CH;
                float y0[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) y0[j] = row[j];
                float p0 = 0.f;
#pragma unroll
                for (int j = 0; j < 8; ++j) p0 += y0[j] * v0[j];
                if (C == 3) {
                    float yr[8], yi[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) { yr[j] = row[64 + j]; yi[j] = row[128 + j]; }
                    float pr = 0.f, pi = 0.f;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        pr += yr[j] * vr[j] + yi[j] * vi[j];
                        pi += yi[j] * vr[j] - yr[j] * vi[j];
                    }
                    atomicAdd(dst + 0, (p0 + 2.f * pr) * THIRD);
                    atomicAdd(dst + 1, (p0 - pr - SQ3 * pi) * THIRD);
                    atomicAdd(dst + 2, (p0 - pr + SQ3 * pi) * THIRD);
                    atomicAdd(dst + 3, 1.f);
                } else {
                    atomicAdd(dst + 0, p0);
                    atomicAdd(dst + 1, 1.f);
                }
            }
        }
        wave_lds_sync();
    }
    __syncthreads();
    // ---- region -> this tile's slot of the global buffer (plain stores) ----
    float *dst = regions + (int64_t)tile * region_elems;
    for (int e = tid; e < region_elems; e += 256) dst[e] = region[e];
}

template <int C, int K>
__global__ __launch_bounds__(256) void filter_kernel(ImageGeom g, TileGeom tg, const float *__restrict__ B,
                                                     const double *__restrict__ T64, const int32_t *__restrict__ idx,
                                                     const double *__restrict__ tau_ref, float *__restrict__ regions,
                                                     unsigned long long *__restrict__ guard_count) {
    extern __shared__ __align__(16) float smem[];
    __shared__ FilterShared sh;
    const int n_tiles = tg.tiles_y * tg.tiles_x;
    // XCD-aware order: consecutive workgroup ids go round-robin over 8 XCDs; give each XCD a
    // contiguous run of tiles (grid = 8 * ceil(n_tiles / 8), b -> (b%8)*per + b/8 is a bijection).
    const int per = (n_tiles + 7) / 8;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= n_tiles) return;
    filter_tile<C, K>(g, tg, B, T64, idx, tau_ref, regions, guard_count, tile, smem, sh, K, 1.0);
}

// Persistent form over many images: each workgroup pulls (image, tile) units from a queue.
template <int C, int K>
__global__ __launch_bounds__(256) void filter_kernel_batched(const BatchItem *__restrict__ items, int n_items,
                                                             const int *__restrict__ unit_start,
                                                             const float *__restrict__ B,
                                                             const double *__restrict__ T64,
                                                             unsigned long long *__restrict__ guard_count,
                                                             int *__restrict__ queue) {
    extern __shared__ __align__(16) float smem[];
    __shared__ FilterShared sh;
    __shared__ int s_u;
    const int total = unit_start[n_items];
    for (;;) {
        if (threadIdx.x == 0) s_u = atomicAdd(queue, 1);
        __syncthreads();
        const int u = s_u;
        __syncthreads();
        if (u >= total) break;
        const int i = find_unit(unit_start, n_items, u);
        const BatchItem it = items[i];
        if (it.ksel && *it.ksel != K) continue;   // the image took the other group size (uniform per block)
        filter_tile<C, K>(it.g, it.tg, B, T64, it.idx, it.tau, it.regions, guard_count, u - unit_start[i], smem, sh,
                          it.idx_stride, it.tau_mul);
        __syncthreads();
    }
}

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
    const int region_elems = tg.RH * tg.RW * CH;
    for (int ty = ty_lo; ty <= ty_hi; ++ty) {
        int r0, r1;
        region_rows(g, tg, ty, &r0, &r1);
        if (y < r0 || y > r1) continue;
        for (int tx = tx_lo; tx <= tx_hi; ++tx) {
            int c0, c1;
            region_cols(g, tg, tx, &c0, &c1);
            if (x < c0 || x > c1) continue;
            const float *src = regions + (int64_t)(ty * tg.tiles_x + tx) * region_elems +
                               ((y - r0) * tg.RW + (x - c0)) * CH;
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[k] += src[k];
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

// Largest reference tile (<= 16 per side) whose region and group buffers fit in LDS.
TileGeom plan_tiles(const ImageGeom &g, int W, int K, int lds_budget, int max_side = 16) {
    TileGeom tg;
    tg.R = (W - 1) / 2;
    const int CH = g.c + 1;
    const int group_bytes = NWAVE * K * 64 * g.c * 4;
    int T = max(1, min(16, max_side));
    for (; T > 1; --T) {
        const int RH = min((T - 1) * g.s + 2 * tg.R + PS, g.h);
        const int RW = min((T - 1) * g.s + 2 * tg.R + PS, g.w);
        if (RH * RW * CH * 4 + group_bytes <= lds_budget) break;
    }
    tg.TY = tg.TX = T;
    tg.RH = min((T - 1) * g.s + 2 * tg.R + PS, g.h);
    tg.RW = min((T - 1) * g.s + 2 * tg.R + PS, g.w);
    tg.tiles_y = (g.ny + T - 1) / T;
    tg.tiles_x = (g.nx + T - 1) / T;
    return tg;
}

template <int C, int K>
hipError_t launch_filter_t(const ImageGeom &g, const TileGeom &tg, const BasisDev &b, const int32_t *idx,
                           const double *tau_ref, float *regions, unsigned long long *gc, hipStream_t st) {
    const int n_tiles = tg.tiles_y * tg.tiles_x;
    const int lds = (tg.RH * tg.RW * (C + 1) + NWAVE * K * 64 * C) * 4;
    const int static_lds = (2 * NWAVE * NEAR_CAP + NWAVE + 2) * 4;
    hipError_t e = prepare_dynamic_lds((const void *)filter_kernel<C, K>, lds, static_lds);
    if (e != hipSuccess) return e;
    const int per = (n_tiles + 7) / 8;
    hipLaunchKernelGGL((filter_kernel<C, K>), dim3(8 * per), dim3(256), lds, st, g, tg, b.f32, b.T64, idx, tau_ref,
                       regions, gc);
    return hipGetLastError();
}

template <int C, int K>
hipError_t launch_filter_batched_t(const BatchItem *items, int n_items, const int *unit_start, int lds,
                                   const BasisDev &b, unsigned long long *gc, int *queue, int grid, hipStream_t st) {
    const int static_lds = (int)sizeof(FilterShared) + 16;
    hipError_t e = prepare_dynamic_lds((const void *)filter_kernel_batched<C, K>, lds, static_lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((filter_kernel_batched<C, K>), dim3(grid), dim3(256), lds, st, items, n_items, unit_start, b.f32,
                       b.T64, gc, queue);
    return hipGetLastError();
}

}  // namespace

int filter_lds_bytes_for(const TileGeom &tg, int C, int K) { return (tg.RH * tg.RW * (C + 1) + NWAVE * K * 64 * C) * 4; }

TileGeom plan_filter_tiles(const ImageGeom &g, int W, int K, int max_side) {
    return plan_tiles(g, W, K, filter_lds_budget(), max_side > 0 ? max_side : 16);
}

hipError_t launch_filter_batched(int C, int K, const BatchItem *items, int n_items, const int *unit_start, int lds,
                                 const BasisDev &b, unsigned long long *gc, int *queue, int grid, hipStream_t st) {
#define HFB_CASE(CC, KK) \
    if (C == CC && K == KK) return launch_filter_batched_t<CC, KK>(items, n_items, unit_start, lds, b, gc, queue, grid, st);
    HFB_CASE(1, 4) HFB_CASE(1, 8) HFB_CASE(1, 16) HFB_CASE(1, 32)
    HFB_CASE(3, 4) HFB_CASE(3, 8) HFB_CASE(3, 16) HFB_CASE(3, 32)
#undef HFB_CASE
    return hipErrorInvalidValue;
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

int filter_lds_budget() { return 160 * 1024 - (2 * NWAVE * NEAR_CAP + NWAVE + 2) * 4 - 64; }

size_t filter_region_bytes(const ImageGeom &g, int W, int K) {
    TileGeom tg = plan_tiles(g, W, K, filter_lds_budget());
    return (size_t)tg.tiles_y * tg.tiles_x * tg.RH * tg.RW * (g.c + 1) * sizeof(float);
}

hipError_t launch_filter(const ImageGeom &g, int W, int K, const BasisDev &b, const int32_t *idx,
                         const double *tau_ref, float *regions, unsigned long long *gc, float *out, int64_t out_stride,
                         hipStream_t st, bool gather) {
    TileGeom tg = plan_tiles(g, W, K, filter_lds_budget());
    hipError_t e = hipErrorInvalidValue;
    if (!gather) {
#define HF_CASE(CC, KK) \
        if (g.c == CC && K == KK) e = launch_filter_t<CC, KK>(g, tg, b, idx, tau_ref, regions, gc, st);
        HF_CASE(1, 4) HF_CASE(1, 8) HF_CASE(1, 16) HF_CASE(1, 32)
        HF_CASE(3, 4) HF_CASE(3, 8) HF_CASE(3, 16) HF_CASE(3, 32)
#undef HF_CASE
        return e;
    }
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
