// Collaborative filtering (Eq. 19-21) and aggregation (Algorithm 1) on the matrix cores of gfx950.
//
// The per-patch transform S = U^T * G * V is linear in the patch, and with the 3-point DFT along
// the channel mode (Eq. 4-5) it splits into a real 64 x 64 map on the channel sum and a real
// 128 x 128 map on the (real, imaginary) pair of the first Fourier slice; the third slice is the
// conjugate of the second.  Thirty-two patches at a time are contracted against these matrices
// with v_mfma_f32_32x32x16_f16:
//
//   forward   [s0'; re'; im'] (32 patches x 192) = [a0, ar, ai] (32 x 192) . F^T
//             a0 = R+G+B, ar = 2R-G-B, ai = B-G are integers, exact in fp16; F is split into
//             fp16 hi + lo (two products, ~22-bit matrix); accumulation in fp32.
//             S0 = s0' + 2 re', S1 = s0' - re' - im', S2 = s0' - re' + im'  (1/3 and sqrt3 folded into F)
//   Haar      along the group (Eq. 7-8), in registers: the result layout of the MFMA puts 16
//             patches of one coefficient column in one lane, the other 16 in lane + 32.
//             Unnormalised butterflies; the threshold of a coefficient produced by l butterflies
//             is tau * 2^(l/2), and the inverse scales kept values by 2^-l (exact).
//   threshold keep |s| >= tau (Eq. 20); values within 0.05 of tau are re-decided in FP64 from the
//             uint8 group and the FP64 transform.
//   inverse   the kept coefficients, recombined as s0 = S0+S1+S2, sr = 2S0-S1-S2, d = S2-S1,
//             are split into fp16 hi (nearest) + lo, transposed through LDS into the A-operand
//             layout and multiplied by the inverse matrix with three products
//             (hi.hi + hi.lo + lo.hi); R, G, B follow as above.
//   Algorithm 1: every reconstructed patch is added (sums and a count) into an LDS copy of the
//             image region the tile's groups reach; the region goes to the tile's slot of a
//             global buffer and the gather kernel divides.  Groups whose members lie anywhere
//             (the spatio-temporal groups of a video) add into global 64-bit fixed-point sums
//             instead, with a histogram of patch positions for the counts.
//
// c = 1 uses the single 64 x 64 map and no channel DFT.
#include "common.h"

namespace htsvd {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

namespace {

constexpr int MW = 8;          // wavefronts per workgroup (two per SIMD)
constexpr int MNEAR = 64;      // near-threshold list capacity per wavefront
constexpr float MGUARD = 0.05f;
constexpr int XS = 33;         // words per row of the per-wave transpose buffer (32 + 1 pad)
constexpr int XWORDS = 32 * XS;

struct MfmaShared {
    int r0, c0;
    int near_n[MW];
    int near_a[MW][MNEAR];     // lane | tile << 6 | reg << 9 | group << 13
    int near_b[MW][MNEAR];     // haar row k | coefficient q << 8
    int near_kill[MW][MNEAR];
};

// Number of pairs of fragment tables: c = 3: forward/inverse x hi/lo x 40 (tile, k-step) blocks.
template <int C>
struct Frag {
    static constexpr int NPAIR = C == 3 ? 40 : 8;
};

// Pair index of (output tile t, k-step s) in the block-diagonal fragment table.
template <int C>
__device__ __host__ constexpr int pair_of(int t, int s) {
    return (C == 1 || t < 2) ? t * 4 + s : 8 + (t - 2) * 8 + (s - 4);
}

__device__ inline v8h ldfrag(const v8h *__restrict__ base, int dir, int term, int pair, int npair, int lane) {
    return base[((dir * 2 + term) * npair + pair) * 64 + lane];
}

// 8*C bytes of one patch row starting at p (dword loads + byte alignment when in bounds).
template <int C>
__device__ inline void load_row_u8(const uint8_t *p, const uint8_t *end, uint32_t (&out)[2 * C]) {
    constexpr int ND = 2 * C + 1;
    const uintptr_t a = (uintptr_t)p;
    const uint32_t *base = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
    const int sh = (int)(a & 3);
    if ((const uint8_t *)(base + ND) <= end) {
        uint32_t d[ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) d[i] = base[i];
#pragma unroll
        for (int i = 0; i < 2 * C; ++i) out[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh * 1u);
    } else {
#pragma unroll
        for (int i = 0; i < 2 * C; ++i)
            out[i] = (uint32_t)p[4 * i] | ((uint32_t)p[4 * i + 1] << 8) | ((uint32_t)p[4 * i + 2] << 16) |
                     ((uint32_t)p[4 * i + 3] << 24);
    }
}

__device__ inline int byte_of(const uint32_t *w, int i) { return (int)((w[i >> 2] >> (8 * (i & 3))) & 0xffu); }

// Byte i of the words as a float (one byte-to-float conversion).
__device__ inline float byte_f(const uint32_t *w, int i) { return (float)((w[i >> 2] >> (8 * (i & 3))) & 0xffu); }

// Two floats as a packed pair of fp16 (round toward zero), low half first.
__device__ inline uint32_t pack_rtz(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(lo, hi));
}

// Entry (k, m) of the orthonormal Haar matrix H_n of Eq. 8.
__device__ inline double haar_w(int k, int m, int n) {
    const double r2 = 0.70710678118654752440;
    double w = 1.0;
    while (n > 1) {
        if (k < n / 2) {
            w *= r2;
            m >>= 1;
            n >>= 1;
        } else {
            const int i = k - n / 2;
            return m == 2 * i ? w * r2 : (m == 2 * i + 1 ? -w * r2 : 0.0);
        }
    }
    return w;
}

__device__ inline void wave_lds_fence() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Value of the same register in lane l ^ 32.
__device__ inline float swap_half(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(threadIdx.x & 32 ? r[0] : r[1]);
}

// Butterfly count l of the coefficient left in register r (group size K, 16 registers per lane).
template <int K>
__device__ __host__ constexpr int haar_level(int r) {
    constexpr int KL = K < 16 ? K : 16;
    constexpr int LK = K == 32 ? 5 : (K == 16 ? 4 : (K == 8 ? 3 : 2));
    const int i = r % KL;
    if (i == 0) return LK;
    int l = 1;
    while (!((i >> (l - 1)) & 1)) ++l;
    return l;
}

// Haar row k (Eq. 8 order) of the coefficient in register r of lane half h.
template <int K>
__device__ inline int haar_row(int r, int h) {
    constexpr int KL = K < 16 ? K : 16;
    const int i = r % KL;
    if (i == 0) return K == 32 ? h : 0;
    const int l = haar_level<K>(r);
    const int mu0 = (K == 32 ? 16 * h : 0) + i - (1 << (l - 1));
    return (K >> l) + (mu0 >> l);
}

// Contribution in fixed point (round to nearest even); |v| is clamped to 1024 (four times the
// 8-bit range) so that no region sum can overflow (see the accumulation shift of the tiling).
// The scale 2^FS (FS <= 12) is applied here, after the fp16 products, whose range it would
// exceed.  |v| scale <= 2^22, so v scale + 1.5 * 2^23 lies in [2^23, 2^24], where floats are
// the integers: one fused multiply-add rounds to nearest even and the bits give the integer.
__device__ inline int to_fixed(float v, float scale) {
    constexpr float MAGIC = 12582912.0f;   // 1.5 * 2^23
    const float t = fmaf(fminf(fmaxf(v, -1024.f), 1024.f), scale, MAGIC);
    return __float_as_int(t) - __float_as_int(MAGIC);
}

// Fixed-point shift of the global aggregation.  Its 64-bit sums cannot overflow; the int32 slot
// regions of a tile receive at most TY TX K contributions per pixel (one per member of each of
// the tile's groups), each of |v| <= 1024, so a tiling uses the largest shift <= GA_FS that
// keeps TY TX K 1024 2^FS below 2^31, and only tilings with a shift of at least GA_MIN_FS.
constexpr int GA_FS = 12;
constexpr int GA_MIN_FS = 9;
constexpr int GA_MAX_TILE = 8;   // largest tile side of the slot regions

// Geometry of a video for the global aggregation: frames of h_frame rows stacked vertically,
// ny_frame reference rows each; with slot regions (GA == 2) a tile's references lie in one
// frame t and its LDS region holds, per channel, the frames f_lo .. f_lo + nslot - 1 (f_lo =
// max(0, t - radius)) as nslot blocks of RH x RP int32 (columns RW used).
struct VideoTiling {
    int T = 1, h_frame = 0, ny_frame = 0, radius = 0, nslot = 1;
    int RH = 0, RW = 0, RP = 0;
};

// 2^e for a small integer exponent (exact).
__device__ inline float exp2i(int e) { return __int_as_float((e + 127) << 23); }

// Fragments of the slice-0 pairs (pair < 8: the 64 x 64 map) of both directions and terms,
// kept in LDS: [dir][term][pair][lane].
constexpr int F0_PAIRS = 8;
constexpr int F0_BYTES = 2 * 2 * F0_PAIRS * 64 * 16;

__device__ inline v8h ldfrag0(const v8h *FL0, int dir, int term, int pair, int lane) {
    return FL0[((dir * 2 + term) * F0_PAIRS + pair) * 64 + lane];
}

// One reference tile: every group of the tile, 32 patches (32/K groups) per wavefront step.
//   FL0: LDS copy of the slice-0 fragments (the 64 x 64 map, both directions); FG: the whole
//   tables (forward at dir 0, inverse at dir 1), read through the caches for the other slices.
//   The eight wavefronts of a workgroup share both and the tile's LDS region.
//   GA: global aggregation into gacc[pix*C + ch] (units of 2^-tg.FS) and ghist[pix] (patches by
//   top-left pixel).  GA == 1: every contribution goes to gacc, the tile only schedules
//   references and region is unused; GA == 2: the tile (references of one frame) adds into its
//   LDS slot region, which then goes to the tile's slot of a global region buffer (at gacc,
//   C * plane int32 per tile) for ga_gather_kernel.
template <int C, int K, bool RA = false, int GA = 0>
__device__ __forceinline__ void filter_tile_mfma(const ImageGeom &g, const TileGeom &tg, const v8h *FL0,
                                                 const v8h *__restrict__ FG, const double *__restrict__ T64,
                                                 const int32_t *__restrict__ idx, const int idx_stride,
                                                 const double *__restrict__ tau_ref, const double tau_mul,
                                                 float *__restrict__ regions,
                                                 unsigned long long *__restrict__ guard_count, const int tile,
                                                 float *region, uint32_t *xbuf_all, MfmaShared &sh,
                                                 const float *__restrict__ ra_d = nullptr,
                                                 const uint8_t *__restrict__ ra_flag = nullptr,
                                                 unsigned long long *__restrict__ gacc = nullptr,
                                                 int *__restrict__ ghist = nullptr,
                                                 const VideoTiling &vt = VideoTiling{}) {
    constexpr int P = 64 * C;
    constexpr int CH = C + 1;
    constexpr int NT = 2 * C;            // 32-column tiles of the 64C coefficients
    constexpr int NPAIR = Frag<C>::NPAIR;
    constexpr int G = 32 / K;            // groups per step
    constexpr int KL = K < 16 ? K : 16;  // group members per lane-half block
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c32 = lane & 31, h = lane >> 5;
    const int ty = tile / tg.tiles_x, tx = tile % tg.tiles_x;
    uint32_t *xbuf = xbuf_all + wave * XWORDS;
    const int plane = region_plane(tg), relems = region_elems(tg, C);
    // LDS accumulation in int32 (float atomics in LDS are far slower than integer ones):
    // channel sums in units of 2^-FS, then patches by top-left pixel, which become the count.
    int *iregion = reinterpret_cast<int *>(region);
    int *hist = iregion + C * plane;
    const float fscale = (float)(1 << tg.FS);
    // references of the tile: rows iy0 .. iy0 + ny_t - 1 of the grid; with slot regions the
    // tiles are cut per frame (frame t_v, its reference rows from iyl0)
    int iy0 = ty * tg.TY, ny_t = min(tg.TY, g.ny - iy0);
    int t_v = 0, f_lo = 0;
    if constexpr (GA == 2) {
        const int tyf = (vt.ny_frame + tg.TY - 1) / tg.TY;
        t_v = ty / tyf;
        const int iyl0 = (ty - t_v * tyf) * tg.TY;
        iy0 = t_v * vt.ny_frame + iyl0;
        ny_t = min(tg.TY, vt.ny_frame - iyl0);
        f_lo = max(0, t_v - vt.radius);
        if (tid == 0) {
            sh.r0 = max(0, ref_pos(iyl0, vt.ny_frame, vt.h_frame, g.s) - tg.R);
            sh.c0 = max(0, ref_pos(tx * tg.TX, g.nx, g.w, g.s) - tg.R);
        }
        for (int e = tid; e < C * plane; e += MW * 64) iregion[e] = 0;
    }
    if constexpr (!GA) {
        if (tid == 0) {
            int r0, r1, c0, c1;
            region_rows(g, tg, ty, &r0, &r1);
            region_cols(g, tg, tx, &c0, &c1);
            sh.r0 = r0;
            sh.c0 = c0;
        }
        for (int e = tid; e < relems; e += MW * 64) iregion[e] = 0;
    }
    __syncthreads();
    const int r0 = sh.r0, c0 = sh.c0;
    const uint8_t *img_end = g.img + (int64_t)(g.h - 1) * g.stride + (int64_t)g.w * C;
    const int ix0 = tx * tg.TX;
    const int nx_t = min(tg.TX, g.nx - ix0);
    const int nref = ny_t * nx_t;

    // pixel of patch position 32 tq + c held by this lane in the output layout
    const int rp = GA == 1 ? g.w : tg.RP;   // row pitch of the aggregation target
    const int lane_off[2] = {(c32 >> 3) * rp + (c32 & 7), (4 + (c32 >> 3)) * rp + (c32 & 7)};
    // MFMA row rho = lane % 32 holds group member mu_in of this step's 32 patches
    const int rho = c32;
    const int mu_in = 16 * ((rho >> 2) & 1) + 4 * (rho >> 3) + (rho & 3);

    for (int base = wave * G; base < nref; base += MW * G) {
        const bool full = base + G <= nref;
        auto ref_of = [&](int gi) -> int64_t {
            const int t = min(base + gi, nref - 1);
            return (int64_t)(iy0 + t / nx_t) * g.nx + (ix0 + t % nx_t);
        };
        // ---- this lane's patch: A operands of the forward products (pixel rows 2 sp + h) ----
        uint32_t raw[4][2 * C];   // pixel rows 2 sp + h of this lane's patch (8 C bytes each)
        int off_in;   // region offset of the patch (for the aggregation, shared by lane shuffles)
        {
            const int64_t r_in = ref_of(mu_in / K);
            const int32_t lin_in = idx[r_in * idx_stride + (mu_in % K)];
            const int yin = lin_in / g.w, xin = lin_in % g.w;
            if constexpr (GA == 1) {
                off_in = lin_in;
                if (h == 0 && (full || base + mu_in / K < nref)) atomicAdd(ghist + lin_in, 1);
            } else if constexpr (GA == 2) {
                const int f = yin / vt.h_frame;   // stacked row -> frame, slot and row in the frame
                off_in = ((f - f_lo) * vt.RH + (yin - f * vt.h_frame - r0)) * tg.RP + (xin - c0);
                if (h == 0 && (full || base + mu_in / K < nref)) atomicAdd(ghist + lin_in, 1);
            } else {
                off_in = (yin - r0) * tg.RP + (xin - c0);
                if (h == 0 && (full || base + mu_in / K < nref)) atomicAdd(hist + off_in, 1);
            }
            const uint8_t *pin = g.img + (int64_t)yin * g.stride + (int64_t)xin * C;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) load_row_u8<C>(pin + (int64_t)(2 * sp + h) * g.stride, img_end, raw[sp]);
        }
        // ---- thresholds of the groups this lane half holds ----
        // per (group slot, butterfly count l): keep-or-undecided above lo, undecided below hi
        // (the guard band (tau - g, tau + g) scaled by 2^(l/2)); without a guard band lo is the
        // float just below the threshold and hi = lo (empty band)
        constexpr int NS = 16 / KL;
        constexpr int LK = K == 32 ? 5 : (K == 16 ? 4 : (K == 8 ? 3 : 2));
        float tau_l[NS], lo_t[NS][LK + 1], hi_t[NS][LK + 1];
#pragma unroll
        for (int gs = 0; gs < NS; ++gs) {
            const int gi = K == 32 ? 0 : (16 * h + gs * KL) / K;
            const bool valid = base + gi < nref;
            const double tau = tau_ref[ref_of(gi)] * tau_mul;
            tau_l[gs] = valid ? (float)tau : __builtin_inff();
            const bool guard = valid && tau > (double)MGUARD;
#pragma unroll
            for (int l = 1; l <= LK; ++l) {
                const float sc = l == 1 ? 1.41421356237309505f : (l == 2 ? 2.f : (l == 3 ? 2.82842712474619010f
                                 : (l == 4 ? 4.f : 5.65685424949238019f)));
                const float tl = tau_l[gs] * sc;
                // a >= tl  <=>  a > (the float just below tl); tl = 0 keeps everything
                const float below = tl > 0.f ? __int_as_float(__float_as_int(tl) - 1) : -1.f;
                lo_t[gs][l] = guard ? tl - MGUARD * sc : below;
                hi_t[gs][l] = guard ? tl + MGUARD * sc : lo_t[gs][l];
            }
        }
        // RA-Haar-tSVD: the forward products of every member of a refined group start from
        // -ra_d(q) (in the accumulators' (s0', re', im') form) instead of 0.  The Haar rows past
        // the first sum to zero over the group, so only the first row changes, to
        // sum - K ra_d(q) = K (T p_est)(q); ramask marks the registers that hold it, which are
        // kept without threshold.
        uint32_t ramask = 0, raflag = 0;
        int64_t ra_row[NS];
        if constexpr (RA) {
#pragma unroll
            for (int gs = 0; gs < NS; ++gs) {
                const int gi = K == 32 ? 0 : (16 * h + gs * KL) / K;
                ra_row[gs] = ref_of(gi) * P;
                if (base + gi < nref && ra_flag[ref_of(gi)]) {
                    raflag |= 1u << gs;
                    if (K < 32 || h == 0) ramask |= 1u << (gs * KL);
                }
            }
        }

        v16f out[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) out[t] = (v16f){};

        // two passes over the coefficient positions 32 tp + c (tp = 0, 1)
#pragma unroll 1
        for (int tp = 0; tp < 2; ++tp) {
            // the raw bytes are converted again in each pass (keeps the converted operands short-lived)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int i = 0; i < 2 * C; ++i) asm volatile("" : "+v"(raw[sp][i]));
            // ---- forward products for the tiles (slice, tp) ----
            v16f acc[C];
#pragma unroll
            for (int sl = 0; sl < C; ++sl) acc[sl] = (v16f){};
            if constexpr (RA) {
#pragma unroll
                for (int gs = 0; gs < NS; ++gs)
                    if ((raflag >> gs) & 1u) {
                        float d[C], a[C];
#pragma unroll
                        for (int sl = 0; sl < C; ++sl) d[sl] = ra_d[ra_row[gs] + 64 * sl + 32 * tp + c32];
                        if (C == 3) {   // inverse of S0 = s0' + 2re', S1 = s0' - re' - im', S2 = s0' - re' + im'
                            a[0] = -(d[0] + d[1] + d[2]) * (1.f / 3.f);
                            a[1] = -(2.f * d[0] - d[1] - d[2]) * (1.f / 6.f);
                            a[2] = -(d[2] - d[1]) * 0.5f;
                        } else {
                            a[0] = -d[0];
                        }
#pragma unroll
                        for (int sl = 0; sl < C; ++sl)
#pragma unroll
                            for (int r = gs * KL; r < gs * KL + KL; ++r) acc[sl][r] = a[sl];
                    }
            }
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                // bytes straight to float, the channel DFT in float, pairs packed to fp16 with
                // round-toward-zero (all values are integers below 2^11, exact either way)
                uint32_t w0[4], wr[4], wi[4];
#pragma unroll
                for (int b = 0; b < 8; b += 2) {
                    if (C == 3) {
                        const float R0 = byte_f(raw[sp], 3 * b), G0 = byte_f(raw[sp], 3 * b + 1), B0 = byte_f(raw[sp], 3 * b + 2);
                        const float R1 = byte_f(raw[sp], 3 * b + 3), G1 = byte_f(raw[sp], 3 * b + 4), B1 = byte_f(raw[sp], 3 * b + 5);
                        const float t0 = G0 + B0, t1 = G1 + B1;
                        w0[b / 2] = pack_rtz(R0 + t0, R1 + t1);
                        wr[b / 2] = pack_rtz(fmaf(2.f, R0, -t0), fmaf(2.f, R1, -t1));
                        wi[b / 2] = pack_rtz(B0 - G0, B1 - G1);
                    } else {
                        w0[b / 2] = pack_rtz(byte_f(raw[sp], b), byte_f(raw[sp], b + 1));
                    }
                }
                const v8h a0 = __builtin_bit_cast(v8h, make_uint4(w0[0], w0[1], w0[2], w0[3]));
                const v8h ar = C == 3 ? __builtin_bit_cast(v8h, make_uint4(wr[0], wr[1], wr[2], wr[3])) : a0;
                const v8h ai = C == 3 ? __builtin_bit_cast(v8h, make_uint4(wi[0], wi[1], wi[2], wi[3])) : a0;
                const int p0 = pair_of<C>(tp, sp);
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, ldfrag0(FL0, 0, 0, p0, lane), acc[0], 0, 0, 0);
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, ldfrag0(FL0, 0, 1, p0, lane), acc[0], 0, 0, 0);
                if (C == 3) {
#pragma unroll
                    for (int sl = 1; sl < C; ++sl) {
                        const int t = 2 * sl + tp;
                        const int pr = pair_of<C>(t, 4 + sp), pi = pair_of<C>(t, 8 + sp);
                        acc[sl] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ar, ldfrag(FG, 0, 0, pr, NPAIR, lane), acc[sl], 0, 0, 0);
                        acc[sl] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ar, ldfrag(FG, 0, 1, pr, NPAIR, lane), acc[sl], 0, 0, 0);
                        acc[sl] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ai, ldfrag(FG, 0, 0, pi, NPAIR, lane), acc[sl], 0, 0, 0);
                        acc[sl] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ai, ldfrag(FG, 0, 1, pi, NPAIR, lane), acc[sl], 0, 0, 0);
                    }
                }
            }
            // ---- inverse channel DFT: (s0', re', im') -> S0, S1, S2 ----
            if (C == 3) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float s0 = acc[0][r], re = acc[1][r], im = acc[2][r];
                    const float t0 = s0 - re;
                    acc[0][r] = s0 + 2.f * re;
                    acc[1][r] = t0 - im;
                    acc[2][r] = t0 + im;
                }
            }

            // ---- Haar along the group; threshold; guard-band values kept for now ----
            bool any_near = false;
#pragma unroll
            for (int sl = 0; sl < C; ++sl) {
                float v[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = acc[sl][r];
#pragma unroll
                for (int st = 1; st < KL; st <<= 1)
#pragma unroll
                    for (int i = 0; i < 16; i += 2 * st) {
                        const float a = v[i], b = v[i + st];
                        v[i] = a + b;
                        v[i + st] = a - b;
                    }
                if (K == 32) {
                    const float o = swap_half(v[0]);
                    v[0] = h ? o - v[0] : v[0] + o;
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int l = haar_level<K>(r);
                    const int gs = r / KL;
                    const float a = fabsf(v[r]);
                    bool keep = a > lo_t[gs][l];
                    bool near = keep && a < hi_t[gs][l];
                    if constexpr (RA) {
                        if (r % KL == 0 && ((ramask >> r) & 1u)) {
                            keep = true;
                            near = false;
                        }
                    }
                    any_near |= near;
                    v[r] = keep ? v[r] * exp2i(-l) : 0.f;   // kept values scaled by 2^-l (inverse Haar)
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[sl][r] = v[r];
            }

            // ---- FP64 re-decision of the coefficients inside the guard band (rare) ----
            if (__ballot(any_near)) {
                // rebuild the band membership from the kept (scaled) values
                uint32_t nearbits[C];
#pragma unroll
                for (int sl = 0; sl < C; ++sl) {
                    uint32_t nb = 0;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int l = haar_level<K>(r);
                        const int gs = r / KL;
                        const float a = fabsf(acc[sl][r]) * exp2i(l);
                        nb |= (uint32_t)(a > lo_t[gs][l] && a < hi_t[gs][l]) << r;
                    }
                    nearbits[sl] = RA ? nb & ~ramask : nb;
                }
                if (lane == 0) sh.near_n[wave] = 0;
                wave_lds_fence();
                uint32_t kill[C];
#pragma unroll
                for (int sl = 0; sl < C; ++sl) {
                    kill[sl] = 0;
                    uint32_t bits = nearbits[sl];
                    while (bits) {
                        const int r = __builtin_ctz(bits);
                        bits &= bits - 1;
                        const int e = atomicAdd(&sh.near_n[wave], 1);
                        const int gi = K == 32 ? 0 : (16 * h + r) / K;
                        if (e < MNEAR) {
                            sh.near_a[wave][e] = lane | (sl << 6) | (r << 9) | (gi << 13);
                            sh.near_b[wave][e] = haar_row<K>(r, h) | ((32 * (2 * sl + tp) + c32) << 8);
                        } else {   // list full: the FP32 value decides
                            const int l = haar_level<K>(r);
                            const float sc = l == 1 ? 1.41421356237309505f : (l == 2 ? 2.f : (l == 3 ? 2.82842712474619010f
                                             : (l == 4 ? 4.f : 5.65685424949238019f)));
                            float vr = 0.f;
#pragma unroll
                            for (int rr = 0; rr < 16; ++rr) vr = rr == r ? acc[sl][rr] : vr;
                            float tauv = tau_l[0];
#pragma unroll
                            for (int gs = 0; gs < NS; ++gs) tauv = gs == r / KL ? tau_l[gs] : tauv;
                            if (!(fabsf(vr) * exp2i(l) >= tauv * sc)) kill[sl] |= 1u << r;
                        }
                    }
                }
                wave_lds_fence();
                const int n_all = sh.near_n[wave];
                const int nn = min(n_all, MNEAR);
                if (lane == 0) {
                    atomicAdd(guard_count, (unsigned long long)nn);
                    if (n_all > nn) atomicAdd(guard_count + 1, (unsigned long long)(n_all - nn));
                }
                for (int e = 0; e < nn; ++e) {
                    const int ia = sh.near_a[wave][e], ib = sh.near_b[wave][e];
                    const int gi = (ia >> 13) & 7, k = ib & 255, q = ib >> 8;
                    const int64_t rr = ref_of(gi);
                    double part = 0.0;
                    for (int p = lane; p < P; p += 64) {
                        const int ch = p / 64, i = (p / 8) % 8, j = p % 8;
                        double accp = 0.0;
                        for (int m = 0; m < K; ++m) {
                            const double w = haar_w(k, m, K);
                            if (w == 0.0) continue;
                            const int32_t l2 = idx[rr * idx_stride + m];
                            accp += w * (double)g.img[(int64_t)(l2 / g.w + i) * g.stride + (int64_t)(l2 % g.w + j) * C + ch];
                        }
                        part += T64[(int64_t)q * P + p] * accp;
                    }
                    const double sv = wave_sum64(part);
                    const double tau = tau_ref[rr] * tau_mul;
                    if (lane == 0) sh.near_kill[wave][e] = !(fabs(sv) >= tau);
                }
                wave_lds_fence();
                for (int e = 0; e < nn; ++e) {
                    const int ia = sh.near_a[wave][e];
                    if ((ia & 63) == lane && sh.near_kill[wave][e]) {
                        const int sl = (ia >> 6) & 7, r = (ia >> 9) & 15;
#pragma unroll
                        for (int ss = 0; ss < C; ++ss)
                            if (ss == sl) kill[ss] |= 1u << r;
                    }
                }
#pragma unroll
                for (int sl = 0; sl < C; ++sl)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if ((kill[sl] >> r) & 1u) acc[sl][r] = 0.f;
            }

            // ---- inverse Haar (transposed butterfly network) ----
#pragma unroll
            for (int sl = 0; sl < C; ++sl) {
                float v[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = acc[sl][r];
                if (K == 32) {
                    const float o = swap_half(v[0]);
                    v[0] = h ? o - v[0] : v[0] + o;
                }
#pragma unroll
                for (int st = KL / 2; st >= 1; st >>= 1)
#pragma unroll
                    for (int i = 0; i < 16; i += 2 * st) {
                        const float a = v[i], b = v[i + st];
                        v[i] = a + b;
                        v[i + st] = a - b;
                    }
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[sl][r] = v[r];
            }
            // ---- channel DFT of the kept coefficients: s0, 2 re, d ----
            if (C == 3) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float a = acc[0][r], b = acc[1][r], cc = acc[2][r];
                    const float u = b + cc;
                    acc[0][r] = a + u;
                    acc[1][r] = 2.f * a - u;
                    acc[2][r] = cc - b;
                }
            }

            // ---- inverse products: each 32-coefficient tile is transposed through LDS ----
#pragma unroll
            for (int sl = 0; sl < C; ++sl) {
                const int j = 2 * sl + tp;   // tile of the k dimension
                constexpr int NTMAX = C == 3 ? 4 : 2;
                const int tlo = sl == 0 ? 0 : 2, ntile = sl == 0 ? 2 : 4;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    // hi = v rounded to fp16 (nearest), lo = the rest (toward zero), one word.
                    // Rounding keeps |lo| <= 2^-11 |v|; a hi cut toward zero (one AND) doubles the
                    // residual and missed the pixel bar on the large refined rows of RA-Haar-tSVD.
                    const float v = acc[sl][r];
                    const float hf = (float)(_Float16)v;
                    xbuf[(16 * h + r) * XS + c32] = pack_rtz(hf, v - hf);
                }
                wave_lds_fence();
#pragma unroll
                for (int ss = 0; ss < 2; ++ss) {
                    v8h ahi, alo;
                    uint32_t any = 0;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const uint32_t wd = xbuf[mu_in * XS + 16 * ss + 8 * h + jj];
                        any |= wd;
                        ahi[jj] = __builtin_bit_cast(_Float16, (uint16_t)(wd & 0xffffu));
                        alo[jj] = __builtin_bit_cast(_Float16, (uint16_t)(wd >> 16));
                    }
                    // a block of 16 coefficient positions that thresholding killed in all 32 patches
                    // adds nothing: its products are skipped (wave-uniform; the sums are unchanged)
                    if (!__builtin_amdgcn_ballot_w64(any != 0u)) continue;
#pragma unroll
                    for (int tt = 0; tt < ntile; ++tt) {
                        const int t = tlo + tt;
                        const int pr = pair_of<C>(t, 2 * j + ss);
                        const v8h fbh = sl == 0 ? ldfrag0(FL0, 1, 0, pr, lane) : ldfrag(FG, 1, 0, pr, NPAIR, lane);
                        const v8h fbl = sl == 0 ? ldfrag0(FL0, 1, 1, pr, lane) : ldfrag(FG, 1, 1, pr, NPAIR, lane);
                        out[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, fbh, out[t], 0, 0, 0);
                        out[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, fbl, out[t], 0, 0, 0);
                        out[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, fbh, out[t], 0, 0, 0);
                    }
                }
                wave_lds_fence();
            }
        }

        // ---- aggregation into the LDS region ----
        // patch offsets of the MFMA rows 8(r/4) + 4h + r%4 through the (now free) transpose
        // buffer: one store per lane, four 16-byte reads
        xbuf[lane] = (uint32_t)off_in;
        wave_lds_fence();
        int offs[16];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const uint4 o4 = *reinterpret_cast<const uint4 *>(xbuf + 8 * q4 + 4 * h);
            offs[4 * q4] = (int)o4.x;
            offs[4 * q4 + 1] = (int)o4.y;
            offs[4 * q4 + 2] = (int)o4.z;
            offs[4 * q4 + 3] = (int)o4.w;
        }
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int mu = 16 * h + r;
            const int gi = mu / K;
            const int off = offs[r];
            if (!full && base + gi >= nref) continue;
#pragma unroll
            for (int tq = 0; tq < 2; ++tq) {
                if constexpr (GA == 1) {
                    unsigned long long *dst = gacc + (int64_t)(off + lane_off[tq]) * C;
                    auto add = [&](int ch, float v) {
                        atomicAdd(dst + ch, (unsigned long long)(long long)to_fixed(v, fscale));
                    };
                    if (C == 3) {
                        const float p0 = out[tq][r], pr = out[2 + tq][r], pi = out[4 + tq][r];
                        const float t0 = p0 - pr;
                        add(0, p0 + 2.f * pr);
                        add(1, t0 - pi);
                        add(2, t0 + pi);
                    } else {
                        add(0, out[tq][r]);
                    }
                    continue;
                }
                int *dst = iregion + off + lane_off[tq];
                if (C == 3) {
                    const float p0 = out[tq][r], pr = out[2 + tq][r], pi = out[4 + tq][r];
                    const float t0 = p0 - pr;
                    atomicAdd(dst, to_fixed(p0 + 2.f * pr, fscale));
                    atomicAdd(dst + plane, to_fixed(t0 - pi, fscale));
                    atomicAdd(dst + 2 * plane, to_fixed(t0 + pi, fscale));
                } else {
                    atomicAdd(dst, to_fixed(out[tq][r], fscale));
                }
            }
        }
    }
    if constexpr (GA == 1) return;   // the caller's barrier follows
    if constexpr (GA == 2) {
        // the slot region to the tile's own slot of the global region buffer (plain stores; the
        // gather kernel sums the regions covering each pixel)
        __syncthreads();
        int4 *dst = reinterpret_cast<int4 *>(reinterpret_cast<int *>(gacc) + (int64_t)tile * C * plane);
        const int4 *src = reinterpret_cast<const int4 *>(iregion);
        for (int e = tid; e < C * plane / 4; e += MW * 64) dst[e] = src[e];
        return;   // the caller's barrier follows
    }
    __syncthreads();
    // coverage count of every pixel: 8 x 8 box sum of the patch histogram (separable, in place,
    // one row then one column per thread; prev[] holds the histogram values leaving the window)
    for (int y = tid; y < tg.RH; y += MW * 64) {
        int *row = hist + y * tg.RP;
        int prev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int run = 0;
        for (int x0 = 0; x0 < tg.RW; x0 += 8) {
            int cur[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) cur[i] = x0 + i < tg.RW ? row[x0 + i] : 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                run += cur[i] - prev[i];
                if (x0 + i < tg.RW) row[x0 + i] = run;
                prev[i] = cur[i];
            }
        }
    }
    __syncthreads();
    for (int x = tid; x < tg.RW; x += MW * 64) {
        int prev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int run = 0;
        for (int y0 = 0; y0 < tg.RH; y0 += 8) {
            int cur[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) cur[i] = y0 + i < tg.RH ? hist[(y0 + i) * tg.RP + x] : 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                run += cur[i] - prev[i];
                if (y0 + i < tg.RH) hist[(y0 + i) * tg.RP + x] = run;
                prev[i] = cur[i];
            }
        }
    }
    __syncthreads();
    float *dst = regions + (int64_t)tile * relems;
    const float unscale = 1.f / fscale;
    for (int e = tid; e < relems; e += MW * 64) dst[e] = (float)iregion[e] * (e < C * plane ? unscale : 1.f);
}

// Persistent over the tiles of one image: workgroup b takes tiles b, b + grid, ... in an
// XCD-aware order (consecutive ids go round-robin over the 8 XCDs; with grid a multiple of 8
// each workgroup stays in one class, whose tiles form a contiguous run).
template <int C, int K, bool RA>
__global__ __launch_bounds__(MW * 64) void filter_mfma_kernel(ImageGeom g, TileGeom tg, const v8h *__restrict__ F,
                                                             const double *__restrict__ T64,
                                                             const int32_t *__restrict__ idx,
                                                             const double *__restrict__ tau_ref,
                                                             float *__restrict__ regions,
                                                             unsigned long long *__restrict__ guard_count,
                                                             const float *__restrict__ ra_d,
                                                             const uint8_t *__restrict__ ra_flag) {
    extern __shared__ __align__(16) float smem[];
    __shared__ MfmaShared sh;
    v8h *FL0 = reinterpret_cast<v8h *>(smem);
    for (int e = threadIdx.x; e < F0_BYTES / 16; e += MW * 64) {
        const int dt = e / (F0_PAIRS * 64), pl = e % (F0_PAIRS * 64);
        FL0[e] = F[(dt * Frag<C>::NPAIR) * 64 + pl];
    }
    __syncthreads();
    float *region = smem + F0_BYTES / 4;
    uint32_t *xb = reinterpret_cast<uint32_t *>(region + region_elems(tg, C));
    const int n_tiles = tg.tiles_y * tg.tiles_x;
    const int per = (n_tiles + 7) / 8;
    for (int v = blockIdx.x; v < 8 * per; v += gridDim.x) {
        const int tile = (v & 7) * per + (v >> 3);
        if (tile >= n_tiles) continue;
        filter_tile_mfma<C, K, RA>(g, tg, FL0, F, T64, idx, K, tau_ref, 1.0, regions, guard_count, tile, region, xb,
                                   sh, ra_d, ra_flag);
        __syncthreads();
    }
}

// Groups anywhere in the image (video), global aggregation: GA == 1 the tiles only schedule the
// work (LDS: the slice-0 fragments and the transpose buffers); GA == 2 each tile also has its
// slot region after them.
template <int C, int K, bool RA, int GA>
__global__ __launch_bounds__(MW * 64) void filter_mfma_ga_kernel(ImageGeom g, TileGeom tg, VideoTiling vt,
                                                                const v8h *__restrict__ F,
                                                                const double *__restrict__ T64,
                                                                const int32_t *__restrict__ idx,
                                                                const double *__restrict__ tau_ref,
                                                                unsigned long long *__restrict__ gacc,
                                                                int *__restrict__ ghist,
                                                                unsigned long long *__restrict__ guard_count,
                                                                const float *__restrict__ ra_d,
                                                                const uint8_t *__restrict__ ra_flag) {
    extern __shared__ __align__(16) float smem[];
    __shared__ MfmaShared sh;
    v8h *FL0 = reinterpret_cast<v8h *>(smem);
    for (int e = threadIdx.x; e < F0_BYTES / 16; e += MW * 64) {
        const int dt = e / (F0_PAIRS * 64), pl = e % (F0_PAIRS * 64);
        FL0[e] = F[(dt * Frag<C>::NPAIR) * 64 + pl];
    }
    __syncthreads();
    uint32_t *xb = reinterpret_cast<uint32_t *>(smem + F0_BYTES / 4);
    float *region = GA == 2 ? reinterpret_cast<float *>(xb + MW * XWORDS) : nullptr;
    const int n_tiles = tg.tiles_y * tg.tiles_x;
    const int per = (n_tiles + 7) / 8;   // XCD-aware order, as in filter_mfma_kernel
    for (int v = blockIdx.x; v < 8 * per; v += gridDim.x) {
        const int tile = (v & 7) * per + (v >> 3);
        if (tile >= n_tiles) continue;
        filter_tile_mfma<C, K, RA, GA>(g, tg, FL0, F, T64, idx, K, tau_ref, 1.0, nullptr, guard_count, tile,
                                       region, xb, sh, ra_d, ra_flag, gacc, ghist, vt);
        __syncthreads();
    }
}

// out = sum / (count 2^fs), count = 8 x 8 box sum of the patch histogram; the noisy value
// where no patch landed.
template <int C>
__global__ void ga_normalize_kernel(const unsigned long long *__restrict__ gacc, const int *__restrict__ ghist,
                                    const uint8_t *__restrict__ img, int64_t stride, int h, int w, int fs,
                                    float *__restrict__ out, int64_t out_stride) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)h * w) return;
    const int y = (int)(e / w), x = (int)(e % w);
    int n = 0;
    for (int dy = 0; dy < PS && dy <= y; ++dy)
        for (int dx = 0; dx < PS && dx <= x; ++dx) n += ghist[(int64_t)(y - dy) * w + (x - dx)];
    float *o = out + (int64_t)y * out_stride + (int64_t)x * C;
    const uint8_t *px = img + (int64_t)y * stride + (int64_t)x * C;
    const double inv = n > 0 ? 1.0 / ((double)n * (double)(1 << fs)) : 0.0;
#pragma unroll
    for (int ch = 0; ch < C; ++ch)
        o[ch] = n > 0 ? (float)((double)(long long)gacc[e * C + ch] * inv) : (float)px[ch];
}

// Slot regions (GA == 2): pixel (f, y, x) of the stacked frames sums, over the frames t within
// the radius of f, the regions of frame t's tiles that cover (y, x) at f's slot; the count is
// the 8 x 8 box sum of the patch histogram.  out = sum / (count 2^fs), or the noisy value.
template <int C>
__global__ void ga_gather_kernel(const int *__restrict__ regions, TileGeom tg, VideoTiling vt, int s, int nx,
                                 const int *__restrict__ ghist, const uint8_t *__restrict__ img, int64_t stride,
                                 int w, float *__restrict__ out, int64_t out_stride) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int hh = vt.T * vt.h_frame;
    if (e >= (int64_t)hh * w) return;
    const int Y = (int)(e / w), x = (int)(e % w);
    const int f = Y / vt.h_frame, y = Y - f * vt.h_frame;
    int n = 0;
    for (int dy = 0; dy < PS && dy <= Y; ++dy)
        for (int dx = 0; dx < PS && dx <= x; ++dx) n += ghist[(int64_t)(Y - dy) * w + (x - dx)];
    float *o = out + (int64_t)Y * out_stride + (int64_t)x * C;
    const uint8_t *px = img + (int64_t)Y * stride + (int64_t)x * C;
    if (n == 0) {
#pragma unroll
        for (int ch = 0; ch < C; ++ch) o[ch] = (float)px[ch];
        return;
    }
    const int plane = tg.RH * tg.RP;
    const int tyf = (vt.ny_frame + tg.TY - 1) / tg.TY;
    const int span_y = tg.TY * s, span_x = tg.TX * s;
    // tiles whose region rows r0 .. r0 + RH - 1 can hold y: r0 = max(0, first reference row - R)
    const int ty_hi = min(tyf - 1, (y + tg.R) / span_y + 1), ty_lo = max(0, (y + tg.R - vt.RH) / span_y - 1);
    const int tx_hi = min(tg.tiles_x - 1, (x + tg.R) / span_x + 1), tx_lo = max(0, (x + tg.R - vt.RW) / span_x - 1);
    long long acc[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] = 0;
    for (int t = max(0, f - vt.radius); t <= min(vt.T - 1, f + vt.radius); ++t) {
        const int slot = f - max(0, t - vt.radius);
        for (int tyl = ty_lo; tyl <= ty_hi; ++tyl) {
            const int r0 = max(0, ref_pos(tyl * tg.TY, vt.ny_frame, vt.h_frame, s) - tg.R);
            if (y < r0 || y >= r0 + vt.RH) continue;
            for (int tx = tx_lo; tx <= tx_hi; ++tx) {
                const int c0 = max(0, ref_pos(tx * tg.TX, nx, w, s) - tg.R);
                if (x < c0 || x >= c0 + vt.RW) continue;
                const int *src = regions + ((int64_t)(t * tyf + tyl) * tg.tiles_x + tx) * C * plane +
                                 (slot * vt.RH + (y - r0)) * tg.RP + (x - c0);
#pragma unroll
                for (int ch = 0; ch < C; ++ch) acc[ch] += src[ch * plane];
            }
        }
    }
    const double inv = 1.0 / ((double)n * (double)(1 << tg.FS));
#pragma unroll
    for (int ch = 0; ch < C; ++ch) o[ch] = (float)((double)acc[ch] * inv);
}

template <int C, int K>
__global__ __launch_bounds__(MW * 64) void filter_mfma_kernel_batched(const BatchItem *__restrict__ items,
                                                                     int n_items, const int *__restrict__ unit_start,
                                                                     const v8h *__restrict__ F,
                                                                     const double *__restrict__ T64,
                                                                     unsigned long long *__restrict__ guard_count,
                                                                     int *__restrict__ queue) {
    extern __shared__ __align__(16) float smem[];
    __shared__ MfmaShared sh;
    __shared__ int s_u;
    v8h *FL0 = reinterpret_cast<v8h *>(smem);
    for (int e = threadIdx.x; e < F0_BYTES / 16; e += MW * 64) {
        const int dt = e / (F0_PAIRS * 64), pl = e % (F0_PAIRS * 64);
        FL0[e] = F[(dt * Frag<C>::NPAIR) * 64 + pl];
    }
    __syncthreads();
    float *region = smem + F0_BYTES / 4;
    const int total = unit_start[n_items];
    for (;;) {
        // thread 0 claims the next unit of an image filtered with this group size; units of an
        // image that took the other size are skipped by moving the queue past the image's end
        // (every value below the end that the queue then skips is one of its units).  The skip
        // loop holds no barrier, so the block's barriers below stay on uniform paths.
        if (threadIdx.x == 0) {
            int c;
            for (;;) {
                c = atomicAdd(queue, 1);
                if (c >= total) break;
                const int ic = find_unit(unit_start, n_items, c);
                const int *ks = items[ic].ksel;
                if (!ks || *ks == K) break;
                atomicMax(queue, unit_start[ic + 1]);
            }
            s_u = c;
        }
        __syncthreads();
        const int u = s_u;
        __syncthreads();
        if (u >= total) break;
        const int i = find_unit(unit_start, n_items, u);
        const BatchItem it = items[i];
        uint32_t *xb = reinterpret_cast<uint32_t *>(region + region_elems(it.tg, C));
        filter_tile_mfma<C, K>(it.g, it.tg, FL0, F, T64, it.idx, it.idx_stride, it.tau, it.tau_mul, it.regions,
                               guard_count, u - unit_start[i], region, xb, sh);
        __syncthreads();
    }
}

}  // namespace

int filter_mfma_lds_bytes(const TileGeom &tg, int C) {
    return F0_BYTES + region_elems(tg, C) * 4 + MW * XWORDS * 4;
}

int filter_mfma_group_bytes(int C) {
    (void)C;
    return F0_BYTES + MW * XWORDS * 4;
}

int filter_mfma_static_bytes() { return (int)sizeof(MfmaShared) + 16; }

template <int C, int K, bool RA>
static hipError_t launch_mfma_t(const ImageGeom &g, const TileGeom &tg, const BasisDev &b, const int32_t *idx,
                                const double *tau_ref, float *regions, unsigned long long *gc, const float *ra_d,
                                const uint8_t *ra_flag, hipStream_t st) {
    const int n_tiles = tg.tiles_y * tg.tiles_x;
    const int lds = filter_mfma_lds_bytes(tg, C);
    hipError_t e = prepare_dynamic_lds((const void *)filter_mfma_kernel<C, K, RA>, lds, (int)sizeof(MfmaShared));
    if (e != hipSuccess) return e;
    int dev = 0, n_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (n_cu < 8) n_cu = 8;
    const int per = (n_tiles + 7) / 8;
    const int grid = min(8 * per, (n_cu / 8) * 8);
    hipLaunchKernelGGL((filter_mfma_kernel<C, K, RA>), dim3(grid), dim3(MW * 64), lds, st, g, tg, (const v8h *)b.frag,
                       b.T64, idx, tau_ref, regions, gc, ra_d, ra_flag);
    return hipGetLastError();
}

hipError_t launch_filter_mfma(const ImageGeom &g, const TileGeom &tg, int K, const BasisDev &b, const int32_t *idx,
                              const double *tau_ref, float *regions, unsigned long long *gc, hipStream_t st,
                              const float *ra_d, const uint8_t *ra_flag) {
    if (!b.frag) return hipErrorInvalidValue;
#define HM_CASE(CC, KK)                                                                                          \
    if (g.c == CC && K == KK)                                                                                    \
        return ra_d ? launch_mfma_t<CC, KK, true>(g, tg, b, idx, tau_ref, regions, gc, ra_d, ra_flag, st)         \
                    : launch_mfma_t<CC, KK, false>(g, tg, b, idx, tau_ref, regions, gc, nullptr, nullptr, st);
    HM_CASE(1, 4) HM_CASE(1, 8) HM_CASE(1, 16) HM_CASE(1, 32)
    HM_CASE(3, 4) HM_CASE(3, 8) HM_CASE(3, 16) HM_CASE(3, 32)
#undef HM_CASE
    return hipErrorInvalidValue;
}

template <int C, int K, bool RA, int GA>
static hipError_t launch_mfma_ga_t(const ImageGeom &g, const TileGeom &tg, const VideoTiling &vt, int lds,
                                   const BasisDev &b, const int32_t *idx, const double *tau_ref,
                                   unsigned long long *gacc, int *ghist, unsigned long long *gc, const float *ra_d,
                                   const uint8_t *ra_flag, hipStream_t st) {
    const int n_tiles = tg.tiles_y * tg.tiles_x;
    hipError_t e = prepare_dynamic_lds((const void *)filter_mfma_ga_kernel<C, K, RA, GA>, lds, (int)sizeof(MfmaShared));
    if (e != hipSuccess) return e;
    int dev = 0, n_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (n_cu < 8) n_cu = 8;
    const int per = (n_tiles + 7) / 8;
    const int grid = min(8 * per, (n_cu / 8) * 8);
    hipLaunchKernelGGL((filter_mfma_ga_kernel<C, K, RA, GA>), dim3(grid), dim3(MW * 64), lds, st, g, tg, vt,
                       (const v8h *)b.frag, b.T64, idx, tau_ref, gacc, ghist, gc, ra_d, ra_flag);
    return hipGetLastError();
}

// Largest fixed-point shift (<= GA_FS) for slot regions of side x side references of K members.
static int ga_shift(int side, int K) {
    int fs = GA_FS;
    while (fs > 0 && (double)side * side * K * 1024.0 * (double)(1 << fs) >= 2147483647.0) --fs;
    return fs;
}

// Tiling of the video filter: the largest tile side (<= GA_MAX_TILE) whose fixed-point shift is
// at least GA_MIN_FS and whose slot region fits in LDS beside the fragments and transpose
// buffers; 0 when none does (direct global aggregation).
static int video_tile_side(int C, int K, int h_frame, int w, int s, int W, int nslot, VideoTiling *vt) {
    const int R = (W - 1) / 2;
    for (int side = GA_MAX_TILE; side >= 1; --side) {
        if (ga_shift(side, K) < GA_MIN_FS) continue;
        const int RH = min((side - 1) * s + 2 * R + PS, h_frame), RW = min((side - 1) * s + 2 * R + PS, w);
        const int RP = RW + ((8 - RW % 16) + 16) % 16;   // pitch % 16 == 8, as for the image regions
        const int bytes = filter_mfma_group_bytes(C) + C * nslot * RH * RP * 4;
        if (bytes <= filter_lds_budget()) {
            vt->RH = RH;
            vt->RW = RW;
            vt->RP = RP;
            return side;
        }
    }
    return 0;
}

// Plan of the video filter: frame-aligned tiles with slot regions (side > 0), or the direct
// global sums (side 0).
static int plan_video(const ImageGeom &g, int T, int radius, int W, int K, bool force_direct, VideoTiling *vt,
                      TileGeom *tg) {
    vt->T = T;
    vt->h_frame = g.h / T;
    vt->ny_frame = g.ny / T;
    vt->radius = radius;
    vt->nslot = min(2 * radius + 1, T);
    const int side = force_direct ? 0 : video_tile_side(g.c, K, vt->h_frame, g.w, g.s, W, vt->nslot, vt);
    *tg = TileGeom{};
    tg->R = (W - 1) / 2;
    tg->FS = side > 0 ? ga_shift(side, K) : GA_FS;
    if (side > 0) {   // frame-aligned tiles with slot regions
        tg->TY = tg->TX = side;
        tg->tiles_y = T * ((vt->ny_frame + side - 1) / side);
        tg->tiles_x = (g.nx + side - 1) / side;
        tg->RH = vt->nslot * vt->RH;   // one plane per channel: the slots stacked
        tg->RW = vt->RW;
        tg->RP = vt->RP;
    } else {          // direct: 8 x 8 references of the stacked grid per scheduling unit
        tg->TY = tg->TX = 8;
        tg->tiles_y = (g.ny + tg->TY - 1) / tg->TY;
        tg->tiles_x = (g.nx + tg->TX - 1) / tg->TX;
    }
    return side;
}

// Bytes of the accumulation buffer of launch_filter_mfma_global: the tiles' slot regions, or
// the 64-bit global sums.
size_t filter_mfma_global_bytes(const ImageGeom &g, int T, int radius, int W, int K, bool force_direct) {
    if (T < 1 || g.h % T || g.ny % T) return 0;
    VideoTiling vt;
    TileGeom tg;
    const int side = plan_video(g, T, radius, W, K, force_direct, &vt, &tg);
    if (side > 0) return (size_t)tg.tiles_y * tg.tiles_x * g.c * region_plane(tg) * sizeof(int);
    return (size_t)g.h * g.w * g.c * sizeof(unsigned long long);
}

// Filtering of groups whose members lie anywhere in the frames of a video (T frames of g.h / T
// rows stacked vertically, reference grid T*ny x nx frame-major, members within `radius` frames
// of their reference's), then the normalisation.  accum: filter_mfma_global_bytes of scratch;
// ghist (h*w int32) must be zero on entry.  force_direct skips the slot regions.
hipError_t launch_filter_mfma_global(const ImageGeom &g, int T, int radius, int W, int K, const BasisDev &b,
                                     const int32_t *idx, const double *tau_ref, void *accum, int *ghist,
                                     unsigned long long *gc, float *out, int64_t out_stride, hipStream_t st,
                                     const float *ra_d, const uint8_t *ra_flag, bool force_direct) {
    if (!b.frag || T < 1 || g.h % T || g.ny % T) return hipErrorInvalidValue;
    VideoTiling vt;
    TileGeom tg;
    const int side = plan_video(g, T, radius, W, K, force_direct, &vt, &tg);
    int lds = filter_mfma_group_bytes(g.c);
    unsigned long long *gacc = (unsigned long long *)accum;
    hipError_t e;
    if (side > 0) {
        lds += g.c * region_plane(tg) * 4;
    } else if ((e = launch_zero(accum, (size_t)g.h * g.w * g.c * sizeof(unsigned long long), st)) != hipSuccess) {
        return e;
    }
    e = hipErrorInvalidValue;
#define HG_CASE(CC, KK)                                                                                          \
    if (g.c == CC && K == KK) {                                                                                  \
        if (side > 0)                                                                                            \
            e = ra_d ? launch_mfma_ga_t<CC, KK, true, 2>(g, tg, vt, lds, b, idx, tau_ref, gacc, ghist, gc, ra_d,  \
                                                          ra_flag, st)                                           \
                     : launch_mfma_ga_t<CC, KK, false, 2>(g, tg, vt, lds, b, idx, tau_ref, gacc, ghist, gc,       \
                                                           nullptr, nullptr, st);                                \
        else                                                                                                     \
            e = ra_d ? launch_mfma_ga_t<CC, KK, true, 1>(g, tg, vt, lds, b, idx, tau_ref, gacc, ghist, gc, ra_d,  \
                                                          ra_flag, st)                                           \
                     : launch_mfma_ga_t<CC, KK, false, 1>(g, tg, vt, lds, b, idx, tau_ref, gacc, ghist, gc,       \
                                                           nullptr, nullptr, st);                                \
    }
    HG_CASE(1, 4) HG_CASE(1, 8) HG_CASE(1, 16) HG_CASE(1, 32)
    HG_CASE(3, 4) HG_CASE(3, 8) HG_CASE(3, 16) HG_CASE(3, 32)
#undef HG_CASE
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)g.h * g.w;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (side > 0) {
        if (g.c == 3)
            hipLaunchKernelGGL(ga_gather_kernel<3>, dim3(grid), dim3(256), 0, st, (const int *)accum, tg, vt, g.s, g.nx,
                               ghist, g.img, g.stride, g.w, out, out_stride);
        else
            hipLaunchKernelGGL(ga_gather_kernel<1>, dim3(grid), dim3(256), 0, st, (const int *)accum, tg, vt, g.s, g.nx,
                               ghist, g.img, g.stride, g.w, out, out_stride);
    } else if (g.c == 3) {
        hipLaunchKernelGGL(ga_normalize_kernel<3>, dim3(grid), dim3(256), 0, st, gacc, ghist, g.img, g.stride, g.h,
                           g.w, tg.FS, out, out_stride);
    } else {
        hipLaunchKernelGGL(ga_normalize_kernel<1>, dim3(grid), dim3(256), 0, st, gacc, ghist, g.img, g.stride, g.h,
                           g.w, tg.FS, out, out_stride);
    }
    return hipGetLastError();
}

template <int C, int K>
static hipError_t launch_mfma_batched_t(const BatchItem *items, int n_items, const int *unit_start, int lds,
                                        const BasisDev &b, unsigned long long *gc, int *queue, int grid,
                                        hipStream_t st) {
    hipError_t e = prepare_dynamic_lds((const void *)filter_mfma_kernel_batched<C, K>, lds,
                                       (int)sizeof(MfmaShared) + 16);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((filter_mfma_kernel_batched<C, K>), dim3(grid), dim3(MW * 64), lds, st, items, n_items,
                       unit_start, (const v8h *)b.frag, b.T64, gc, queue);
    return hipGetLastError();
}

hipError_t launch_filter_mfma_batched(int C, int K, const BatchItem *items, int n_items, const int *unit_start,
                                      int lds, const BasisDev &b, unsigned long long *gc, int *queue, int grid,
                                      hipStream_t st) {
    if (!b.frag) return hipErrorInvalidValue;
#define HMB_CASE(CC, KK) \
    if (C == CC && K == KK) return launch_mfma_batched_t<CC, KK>(items, n_items, unit_start, lds, b, gc, queue, grid, st);
    HMB_CASE(1, 4) HMB_CASE(1, 8) HMB_CASE(1, 16) HMB_CASE(1, 32)
    HMB_CASE(3, 4) HMB_CASE(3, 8) HMB_CASE(3, 16) HMB_CASE(3, 32)
#undef HMB_CASE
    return hipErrorInvalidValue;
}

}  // namespace htsvd
