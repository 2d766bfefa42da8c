// Hyperspectral tube patches (Sec. IV-D): Haar-tSVD on an h x w x B cube with 8 x 8 x B patches.
//
// Grouping runs on a gray guide, the band mean rounded half up (the block matcher of the other
// paths, Eq. 9 on one channel).  The transform runs in FP64 (so that keep/kill decisions agree
// with an FP64 reference without a guard band).  The t-product S = U^T * P * V (Eq. 19) is taken
// along the band axis through its DFT (Eq. 4-5): the real band DFT of each of the 64 tubes of a
// patch, per frequency f the 8 x 8 complex slice products U_hat_f^H P_hat_f V_hat_f, and the
// inverse band DFT, all in one kernel per direction with the patch spectra in LDS
// (band_tproduct_kernel).  The member coefficients S (member n at S[n*64*B + b*64 + e]) are the
// only patch matrix in HBM: the Haar transform along each group with the hard threshold (Eq. 20)
// works on them in place, and the inverse kernel (Eq. 21, with U_hat_f and V_hat_f^H) adds its
// estimates to uniform aggregation sums (Algorithm 1) in 64-bit fixed point (exact sums, so the
// result does not depend on the order of the additions).
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

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Patches per workgroup and the LDS layout of their spectra: value (i, j) of component c of patch
// p at Z[p*ZP + c*64 + zpos(c, i, j)].  The XOR of j with a function of i, the rotation of the odd
// components by 16 and the patch stride of 16 modulo 32 doubles keep the accesses of the three
// phases free of bank conflicts (64 banks of 4 bytes: a wave's 32-lane halves reach 32 distinct
// double slots).  The inverse kernel reuses a patch's slots for its estimates as Z[p*ZP + e*ES + b]
// (ES = 2 modulo 32), read with the band index fastest.
template <int NB> struct BandTile {
    static constexpr int PP = 2;                       // patches per workgroup (256 threads)
    static constexpr int HALVES = 4 / PP;              // waves sharing one patch in the DFT phases
    static constexpr int CBW = NB / 16 / HALVES;       // 16-row blocks of the DFT outputs per wave
    static constexpr int KS = NB / 4;                  // k-steps of a DFT product
    static constexpr int ES = NB + 2;                  // estimate stride of the inverse kernel
    static constexpr int ZP = ES * 64 + 16;            // doubles per patch
    static constexpr int ROWB = ((8 * NB + 15) / 16 + 1) * 16;   // staged bytes per patch row
};

__device__ inline int zpos(int c, int i, int j) {
    return (8 * i + (j ^ (((i >> 2) << 1) ^ (((i >> 1) & 1) << 2))) + 16 * (c & 1)) & 63;
}

// One direction of the t-product along the bands for PP patches per workgroup (Eq. 4-5, 19, 21),
// every product on v_mfma_f64_16x16x4f64 (lanes: A(m, k) in m + 16 (k mod 4), B(k, n) in
// n + 16 (k mod 4), result (m, n) in register m / 4 of lane n + 16 (m mod 4)):
//   1. band DFT  Z(c, e) = sum_b D(c, b) x(b, e): D as the A operand, held in registers across
//      the phase, the patch's values at the 64 positions e as the B operand (forward: the
//      8 B contiguous bytes of each patch row first staged in LDS with aligned 16-byte loads);
//   2. per frequency f (one wave) and pair of patches, the slice products T = L * P_f and
//      Y_f = T * R, with complex 8 x 8 matrices in their real 16 x 16 embeddings:
//        L on the left,  [[Lr, -Li], [Li, Lr]] times P stacked as [Pr; Pi] (columns: 2 patches x 8);
//        R on the right, T laid out as [Tr | Ti] (rows: 2 patches x 8) times [[Rr, Ri], [-Ri, Rr]];
//      T goes back to the LDS slots of P_f and Y_f to the same slots (the slots of f belong to
//      one wave, and its LDS accesses execute in order);
//   3. inverse band DFT  y(b, e) = sum_c Dinv(b, c) Z(c, e), Dinv in registers.
// Forward (INV = false): x from the cube through the group indices, L = U_hat_f^H, R = V_hat_f,
// y stored to S[(n*B + b)*64 + e].  Inverse (INV = true): x from S, L = U_hat_f, R = V_hat_f^H,
// y clamped and added in fixed point to the uniform aggregation sums (Algorithm 1).
template <int NB, bool INV>
__global__ __launch_bounds__(256) void band_tproduct_kernel(const uint8_t *__restrict__ cube,
                                                            const uint8_t *__restrict__ cube_end, int64_t stride, int w,
                                                            int B, const int32_t *__restrict__ idx, int64_t n_patch,
                                                            const double *__restrict__ D,
                                                            const double *__restrict__ Dinv,
                                                            const double *__restrict__ frag, double *__restrict__ S,
                                                            unsigned long long *__restrict__ acc,
                                                            int *__restrict__ cnt) {
    using T = BandTile<NB>;
    constexpr int PP = T::PP, ZP = T::ZP, ES = T::ES, CBW = T::CBW, KS = T::KS, ROWB = T::ROWB;
    __shared__ double Z[PP * ZP];
    __shared__ __align__(16) uint8_t stg[INV ? 16 : PP * 8 * ROWB];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int q = lane >> 4, col = lane & 15;
    const int64_t n0 = (int64_t)blockIdx.x * PP;
    // wave -> (patch, half of the 16-row output blocks) in the DFT phases
    const int p = wave % PP, half = wave / PP;
    const int64_t n = n0 + p;
    const bool valid = n < n_patch;

    // 1. band DFT
    {
        double a[CBW][KS];
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
            for (int s = 0; s < KS; ++s) a[cb][s] = D[(16 * (half * CBW + cb) + col) * NB + 4 * s + q];
        // forward: rows of the workgroup's patches into LDS, 16-byte chunks from the aligned
        // address below each row; a chunk not wholly inside the cube is copied byte by byte
        uintptr_t rbase = 0;   // address of the patch's first row: row i starts (rbase + i stride) mod 16 into its slot
        if (!INV) {
            constexpr int CH = ROWB / 16;
            for (int t = tid; t < PP * 8 * CH; t += 256) {
                const int pp = t / (8 * CH), i = (t / CH) % 8, k = t % CH;
                if (n0 + pp >= n_patch) continue;
                const int32_t lin = idx[n0 + pp];
                const uint8_t *seg = cube + (int64_t)(lin / w + i) * stride + (int64_t)(lin % w) * B;
                const uint8_t *seg_end = seg + 8 * B;
                const uint8_t *ck = (const uint8_t *)((uintptr_t)seg & ~(uintptr_t)15) + 16 * k;
                if (ck >= seg_end) continue;
                uint8_t *dst = stg + (pp * 8 + i) * ROWB + 16 * k;
                if (ck >= cube && ck + 16 <= cube_end) {
                    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(ck);
                } else {
                    for (int j = 0; j < 16; ++j)
                        if (ck + j >= seg && ck + j < seg_end) dst[j] = ck[j];
                }
            }
            if (valid) {
                const int32_t lin = idx[n];
                rbase = (uintptr_t)(cube + (int64_t)(lin / w) * stride + (int64_t)(lin % w) * B);
            }
            __syncthreads();
        }
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            const int e = 16 * blk + col;
            double x[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int b = 4 * s + q;
                if (INV)
                    x[s] = (valid && b < B) ? S[(n * B + b) * 64 + e] : 0.0;
                else
                    x[s] = (valid && b < B) ? (double)stg[(p * 8 + (e >> 3)) * ROWB +
                                                          (int)((rbase + (uintptr_t)((e >> 3) * stride)) & 15) +
                                                          (e & 7) * B + b]
                                            : 0.0;
            }
#pragma unroll
            for (int cb = 0; cb < CBW; ++cb) {
                dbl4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < KS; ++s) t = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cb][s], x[s], t, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 16 * (half * CBW + cb) + q + 4 * r;
                    if (c < B) Z[p * ZP + c * 64 + zpos(c, e >> 3, e & 7)] = t[r];
                }
            }
        }
    }
    __syncthreads();

    // 2. slice products on the matrix cores: wave -> frequencies f = wave (mod 4), each for every
    //    pair of patches (the operands of f are loaded once, those of the next f ahead of use)
    {
        constexpr int NPAIR = PP / 2;
        const int NF = B / 2 + 1;
        double fr[8], nx[8];
        if (wave < NF) {
#pragma unroll
            for (int v = 0; v < 8; ++v) nx[v] = frag[(size_t)wave * 512 + v * 64 + lane];
        }
        for (int f = wave; f < NF; f += 4) {
#pragma unroll
            for (int v = 0; v < 8; ++v) fr[v] = nx[v];
            if (f + 4 < NF) {
#pragma unroll
                for (int v = 0; v < 8; ++v) nx[v] = frag[(size_t)(f + 4) * 512 + v * 64 + lane];
            }
            const bool real = f == 0 || 2 * f == B;
            const int cre = f == 0 ? 0 : (2 * f == B ? B - 1 : 2 * f - 1), cim = 2 * f;
            dbl4 t[NPAIR];
            // T = L * [Pr; Pi]: B operand rows k = 4s + q = (ri, i), columns col = (p, j)
#pragma unroll
            for (int pr = 0; pr < NPAIR; ++pr) {
                const double *zb = Z + (2 * pr) * ZP;
                double v[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int ri = s >> 1, i = 4 * (s & 1) + q, c = ri ? cim : cre;
                    v[s] = (ri && real) ? 0.0 : zb[(col >> 3) * ZP + c * 64 + zpos(c, i, col & 7)];
                }
                t[pr] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < 4; ++s) t[pr] = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[s], v[s], t[pr], 0, 0, 0);
            }
            // result rows q + 4r = (ri', i'), columns (p, j)
#pragma unroll
            for (int pr = 0; pr < NPAIR; ++pr) {
                double *zb = Z + (2 * pr) * ZP;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ri = r >> 1, i = q + 4 * (r & 1), c = ri ? cim : cre;
                    if (!(ri && real)) zb[(col >> 3) * ZP + c * 64 + zpos(c, i, col & 7)] = t[pr][r];
                }
            }
            // Y = [Tr | Ti] * R: A operand rows col = (p, i'), columns k = 4s + q = (ri, j)
#pragma unroll
            for (int pr = 0; pr < NPAIR; ++pr) {
                const double *zb = Z + (2 * pr) * ZP;
                double v[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int ri = s >> 1, j = 4 * (s & 1) + q, c = ri ? cim : cre;
                    v[s] = (ri && real) ? 0.0 : zb[(col >> 3) * ZP + c * 64 + zpos(c, col & 7, j)];
                }
                t[pr] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < 4; ++s) t[pr] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[s], fr[4 + s], t[pr], 0, 0, 0);
            }
            // result rows q + 4r = (p, i'), columns col = (ri', j')
#pragma unroll
            for (int pr = 0; pr < NPAIR; ++pr) {
                double *zb = Z + (2 * pr) * ZP;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pp = r >> 1, i = q + 4 * (r & 1), ri = col >> 3, c = ri ? cim : cre;
                    if (!(ri && real)) zb[pp * ZP + c * 64 + zpos(c, i, col & 7)] = t[pr][r];
                }
            }
        }
    }
    __syncthreads();

    // 3. inverse band DFT
    double y[4][CBW][4];
    {
        double a[CBW][KS];
#pragma unroll
        for (int bb = 0; bb < CBW; ++bb)
#pragma unroll
            for (int s = 0; s < KS; ++s) a[bb][s] = Dinv[(16 * (half * CBW + bb) + col) * NB + 4 * s + q];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            const int e = 16 * blk + col;
            double z[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int c = 4 * s + q;
                z[s] = c < B ? Z[p * ZP + c * 64 + zpos(c, e >> 3, e & 7)] : 0.0;
            }
#pragma unroll
            for (int bb = 0; bb < CBW; ++bb) {
                dbl4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < KS; ++s) t = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bb][s], z[s], t, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) y[blk][bb][r] = t[r];
            }
        }
    }
    if (!INV) {
        if (valid) {
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int bb = 0; bb < CBW; ++bb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int b = 16 * (half * CBW + bb) + q + 4 * r;
                        if (b < B) S[(n * B + b) * 64 + 16 * blk + col] = y[blk][bb][r];
                    }
        }
        return;
    }
    __syncthreads();   // every spectrum read before the estimates replace it
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int bb = 0; bb < CBW; ++bb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = 16 * (half * CBW + bb) + q + 4 * r;
                if (b < B) Z[p * ZP + (16 * blk + col) * ES + b] = y[blk][bb][r];
            }
    __syncthreads();
    // aggregation with the band index fastest, so that a wave's atomics cover contiguous words
    const int np = (int)std::min<int64_t>(PP, n_patch - n0);
    for (int t = tid; t < np * 64 * B; t += 256) {
        const int b = t % B, pe = t / B, pp = pe >> 6, ee = pe & 63;
        const int32_t lin = idx[n0 + pp];
        const int64_t pix = (int64_t)(lin / w + (ee >> 3)) * w + (lin % w + (ee & 7));
        const double v = fmin(fmax(Z[pp * ZP + ee * ES + b], -1024.0), 1024.0);
        const long long qv = __double2ll_rn(v * (double)(1 << BFS));
        atomicAdd(acc + pix * B + b, (unsigned long long)qv);
        if (b == 0) atomicAdd(cnt + pix, 1);
    }
}

// Haar transform along each group (orthonormal butterflies), hard threshold |s| >= tau, inverse.
// One thread per (group, position q of the 64 x B values of a patch); member k of group g holds
// position q at S[(g*K + k)*64*B + q].
template <int K>
__global__ void haar_threshold_kernel(double *__restrict__ S, int64_t n_group, int B, double tau) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride_k = (int64_t)64 * B;
    if (t >= n_group * stride_k) return;
    const int64_t g = t / stride_k, q = t % stride_k;
    double v[K];
    double *base = S + g * K * stride_k + q;
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

template <int NB>
hipError_t launch_tproduct(const BandMaps &bm, bool inverse, const uint8_t *cube, int64_t stride, int h, int w,
                           int B, const int32_t *idx, int64_t n_patch, double *S, unsigned long long *acc, int *cnt,
                           hipStream_t st) {
    const unsigned grid = nb(n_patch, BandTile<NB>::PP);
    const uint8_t *cube_end = cube + (int64_t)(h - 1) * stride + (int64_t)w * B;   // one past the last pixel
    if (inverse)
        hipLaunchKernelGGL((band_tproduct_kernel<NB, true>), dim3(grid), dim3(256), 0, st, cube, cube_end, stride, w,
                           B, idx, n_patch, bm.D, bm.Dinv, bm.frag_inv, S, acc, cnt);
    else
        hipLaunchKernelGGL((band_tproduct_kernel<NB, false>), dim3(grid), dim3(256), 0, st, cube, cube_end, stride, w,
                           B, idx, n_patch, bm.D, bm.Dinv, bm.frag_fwd, S, acc, cnt);
    return hipGetLastError();
}

hipError_t tproduct(const BandMaps &bm, bool inverse, const uint8_t *cube, int64_t stride, int h, int w, int B,
                    const int32_t *idx, int64_t n_patch, double *S, unsigned long long *acc, int *cnt,
                    hipStream_t st) {
    if (bm.nb != band_nb(B)) return hipErrorInvalidValue;
    return B <= 32 ? launch_tproduct<32>(bm, inverse, cube, stride, h, w, B, idx, n_patch, S, acc, cnt, st)
                   : launch_tproduct<64>(bm, inverse, cube, stride, h, w, B, idx, n_patch, S, acc, cnt, st);
}

}  // namespace

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

// Groups per pass of the filter: the FP64 patch matrix S stays below cap bytes.
int64_t band_chunk_groups(int B, int K, int64_t n_group, int64_t cap) {
    const int64_t per = (int64_t)K * 64 * B * (int64_t)sizeof(double);
    return std::max<int64_t>(1, std::min<int64_t>(n_group, cap / per));
}

size_t band_ws_bytes(int h, int w, int B, int K, int64_t n_group, int64_t cap) {
    const int64_t n_patch = band_chunk_groups(B, K, n_group, cap) * K;
    const size_t mat = sizeof(double) * (size_t)n_patch * 64 * B;
    return ((mat + 255) & ~(size_t)255) + (((size_t)h * w * B * 8 + 255) & ~(size_t)255) +
           (((size_t)h * w * 4 + 255) & ~(size_t)255);
}

// Per pass: the forward t-product of every member into S, the Haar transform with the hard
// threshold along each group, and the inverse t-product with aggregation; then normalisation.
hipError_t launch_band_filter(const BandMaps &bm, const uint8_t *cube, int64_t stride, int h, int w, int B,
                              const int32_t *idx, int64_t n_group, int K, double tau, int64_t cap, void *ws,
                              float *out, int64_t out_stride, hipStream_t st) {
    const int64_t chunk = band_chunk_groups(B, K, n_group, cap);
    const size_t mat = ((sizeof(double) * (size_t)(chunk * K) * 64 * B) + 255) & ~(size_t)255;
    double *S = (double *)ws;
    unsigned long long *acc = (unsigned long long *)((char *)ws + mat);
    int *cnt = (int *)((char *)acc + (((size_t)h * w * B * 8 + 255) & ~(size_t)255));
    hipError_t e;
    if ((e = launch_zero(acc, (size_t)h * w * B * 8, st)) != hipSuccess) return e;
    if ((e = launch_zero(cnt, (size_t)h * w * 4, st)) != hipSuccess) return e;
    for (int64_t g0 = 0; g0 < n_group; g0 += chunk) {
        const int64_t ng = std::min<int64_t>(chunk, n_group - g0), n_patch = ng * K;
        const int32_t *ix = idx + g0 * K;
        if ((e = tproduct(bm, false, cube, stride, h, w, B, ix, n_patch, S, acc, cnt, st)) != hipSuccess) return e;
        const int64_t nt = ng * 64 * B;
        switch (K) {
            case 4: hipLaunchKernelGGL(haar_threshold_kernel<4>, dim3(nb(nt, 256)), dim3(256), 0, st, S, ng, B, tau); break;
            case 8: hipLaunchKernelGGL(haar_threshold_kernel<8>, dim3(nb(nt, 256)), dim3(256), 0, st, S, ng, B, tau); break;
            case 16: hipLaunchKernelGGL(haar_threshold_kernel<16>, dim3(nb(nt, 256)), dim3(256), 0, st, S, ng, B, tau); break;
            case 32: hipLaunchKernelGGL(haar_threshold_kernel<32>, dim3(nb(nt, 256)), dim3(256), 0, st, S, ng, B, tau); break;
            default: return hipErrorInvalidValue;
        }
        if ((e = tproduct(bm, true, cube, stride, h, w, B, ix, n_patch, S, acc, cnt, st)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(normalize_kernel, dim3(nb((int64_t)h * w * B, 256)), dim3(256), 0, st, acc, cnt, cube, stride, h,
                       w, B, out, out_stride);
    return hipGetLastError();
}

}  // namespace htsvd
