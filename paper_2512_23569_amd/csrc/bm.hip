// Block matching (grouping) for Haar-tSVD on gfx950.
//
// Sec. III-A, Eq. 9: the distance between the reference patch and a candidate is the
// green-channel distance when gamma^2 ||G_ref||^2 >= max(||R_ref||^2, ||B_ref||^2), and the
// distance of the channel averages otherwise (here the channel sum: same order and ties).
// Distances are squared Euclidean and exact.  Algorithm 1 "Grouping" keeps the K
// smallest, ordered by (distance, row, column).
//
// Mapping.  One workgroup (16 waves, four per SIMD) owns a 4x4 tile of references.  The union of their
// search windows (at most 64x64 candidate positions) is staged in LDS as
//   - the shifted green (or gray) plane x-128 in int8, in 4 byte-shifted copies so any
//     8-pixel row segment is a 4-byte-aligned pair of dwords, and
//   - the shifted channel-sum plane R+G+B-384 in fp16 (exact: |v| <= 384), in 2 copies.
// ||a-b||^2 = ||a||^2 + ||b||^2 - 2 a.b, where a.b for 16 references x 16 candidates is one
// v_mfma_i32_16x16x64_i8 (one 8x8 patch = the whole k = 64 contraction), or two
// v_mfma_f32_16x16x32_f16 for the sum plane (all partial sums are integers < 2^24, so the
// fp32 accumulation is exact).  Distances of each reference land in an LDS table indexed
// by the raster position inside its clipped window, so (distance, position) orders like
// (distance, row, column).  Each wave then selects the K smallest keys of one reference:
// the K-th smallest of the 64 lane minima bounds the answer from above, the keys under
// that bound are compacted and sorted with a wave bitonic network.
//
// Video (Sec. IV-C): the frames are stacked vertically, and a reference's candidates are the
// positions of its clipped window in every frame within a temporal radius.  The workgroup keeps
// the reference patches of its own frame in registers, stages one frame after another, and
// merges each frame's K best (distance, frame slot, position) keys into a running list in LDS.
#include "common.h"

namespace htsvd {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

constexpr int NREF = REF_TILE * REF_TILE;  // 16
constexpr int BMW = 16;                    // wavefronts per workgroup (four per SIMD)
constexpr int BMT = BMW * 64;
constexpr int SEL_CAP = 512;               // >= K * ceil(MAX_CAND / 64) for K <= 32
// Words per reference row of the distance table: 964 = 4 (mod 64), so the four references a
// quarter-wave writes for 16 consecutive candidates land on disjoint LDS banks.
constexpr int TAB_STRIDE = 964;
static_assert(TAB_STRIDE >= MAX_CAND, "table rows hold a whole window");
constexpr int RUN_K = 32;                  // running list per reference of the video search

// Frames of a video search: g.img is frame 0 of T frames of g.h rows each, frame_bytes apart.
struct VideoArgs {
    int T, radius;
    int64_t frame_bytes;
};

struct TileInfo {
    int ry[NREF], rx[NREF];        // reference position, ry = -1 if the slot is empty
    int wy0[NREF], wx0[NREF];      // clipped window origin (candidate positions)
    int wh[NREF], ww[NREF];        // clipped window size
    int green[NREF];               // Eq. 9 branch: 1 green/gray distance, 0 channel-sum distance
    int any_sum;                   // some reference uses the channel-sum distance
};

// Byte layout of the dynamic LDS for one launch.
struct BmLds {
    int pitch8;     // bytes per row of one int8 plane copy
    int pitch16;    // halves per row of one fp16 plane copy
    int rows;       // plane rows (union rows + 7)
    int plane8;     // bytes between the int8 plane copies (a row multiple plus a bank offset)
    int off_p8, off_p16, off_n8, off_n16, off_tab, off_sel, total;   // video: running lists last
};

__device__ inline uint32_t lds_u32(const unsigned char *base, int byte_off) {
    return *reinterpret_cast<const uint32_t *>(base + byte_off);
}

__device__ inline void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline uint64_t readlane_u64(uint64_t v, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending sort of one u64 per lane across the 64 lanes of a wave.
__device__ inline uint64_t wave_sort64(uint64_t v, int lane) { return wave_sort_asc<uint64_t>(v, lane); }

__device__ inline int wave_excl_scan(int v, int lane, int *total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63);
    return x - v;
}

// Ascending bitonic sort of P (power of two <= SEL_CAP) keys in LDS by one wave.
template <typename T>
__device__ void lds_sort(T *a, int P, int lane) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < P / 2; t += 64) {
                int i = 2 * t - (t & (j - 1));
                int m = i + j;
                T x = a[i], y = a[m];
                bool up = (i & k) == 0;
                if ((x > y) == up) {
                    a[i] = y;
                    a[m] = x;
                }
            }
            wave_lds_sync();
        }
    }
}

// Groups of the 16 references of tile b (VIDEO: tile b of the frames' tiles, frame-major).
template <bool VIDEO>
__device__ __forceinline__ void bm_tile(const ImageGeom &g0, const MethodParams &mp, const int tiles_x, const int b_in,
                                        const BmLds &L, int32_t *__restrict__ idx_out,
                                        int32_t *__restrict__ dist_out, unsigned char *smem, TileInfo &ti,
                                        const VideoArgs &va) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int b = b_in, t = 0, f_lo = 0, nf = 1;
    ImageGeom g = g0;   // the reference's frame
    if constexpr (VIDEO) {
        const int tiles_frame = ((g0.ny + REF_TILE - 1) / REF_TILE) * tiles_x;
        t = b_in / tiles_frame;
        b = b_in - t * tiles_frame;
        g.img = g0.img + (int64_t)t * va.frame_bytes;
        f_lo = max(0, t - va.radius);
        nf = min(va.T - 1, t + va.radius) - f_lo + 1;
    }
    const int tyi = b / tiles_x, txi = b % tiles_x;
    const int R = (mp.W - 1) / 2;

    // ---- tile geometry ----
    // The union of the 16 windows in closed form (positions increase along each side), so every
    // thread has it at once and the staging loads need not wait for the per-reference table.
    const int iya = tyi * REF_TILE, iyb = min(iya + REF_TILE, g.ny) - 1;
    const int ixa = txi * REF_TILE, ixb = min(ixa + REF_TILE, g.nx) - 1;
    const int uy0 = max(0, ref_pos(iya, g.ny, g.h, g.s) - R);
    const int ux0 = max(0, ref_pos(ixa, g.nx, g.w, g.s) - R);
    const int uh = min(g.h - PS, ref_pos(iyb, g.ny, g.h, g.s) + R) - uy0 + 1;
    const int uw = min(g.w - PS, ref_pos(ixb, g.nx, g.w, g.s) + R) - ux0 + 1;
    if (tid < NREF) {
        const int iy = tyi * REF_TILE + tid / REF_TILE, ix = txi * REF_TILE + tid % REF_TILE;
        if (iy < g.ny && ix < g.nx) {
            const int y = ref_pos(iy, g.ny, g.h, g.s), x = ref_pos(ix, g.nx, g.w, g.s);
            const int y0 = max(0, y - R), y1 = min(g.h - PS, y + R);
            const int x0 = max(0, x - R), x1 = min(g.w - PS, x + R);
            ti.ry[tid] = y; ti.rx[tid] = x;
            ti.wy0[tid] = y0; ti.wx0[tid] = x0;
            ti.wh[tid] = y1 - y0 + 1; ti.ww[tid] = x1 - x0 + 1;
        } else {
            ti.ry[tid] = -1; ti.rx[tid] = -1;
            ti.wy0[tid] = 0; ti.wx0[tid] = 0; ti.wh[tid] = 0; ti.ww[tid] = 0;
        }
    }
    // Eq. 9 branch per reference from the raw channel norms (16 threads per reference; the
    // reference position is recomputed here, so these loads overlap with the staging below).
    if (g.c == 3) {
        const int i = tid >> 4, sub = tid & 15;   // 16 threads per reference (the first 256 threads)
        int nr = 0, ng = 0, nb = 0;
        const int iy = iya + i / REF_TILE, ix = ixa + i % REF_TILE;
        if (i < NREF && iy < g.ny && ix < g.nx) {
            const int ry = ref_pos(iy, g.ny, g.h, g.s), rx = ref_pos(ix, g.nx, g.w, g.s);
            for (int p = sub; p < PS * PS; p += 16) {
                const uint8_t *px = g.img + (int64_t)(ry + p / PS) * g.stride + (int64_t)(rx + p % PS) * 3;
                nr += px[0] * px[0]; ng += px[1] * px[1]; nb += px[2] * px[2];
            }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            nr += __shfl_xor(nr, o); ng += __shfl_xor(ng, o); nb += __shfl_xor(nb, o);
        }
        if (sub == 0 && i < NREF) {
            const int64_t mx = nr > nb ? nr : nb;
            ti.green[i] = (int64_t)mp.gnum * mp.gnum * ng >= (int64_t)mp.gden * mp.gden * mx ? 1 : 0;
        }
    } else if (tid < NREF) {
        ti.green[tid] = 1;
    }
    const int prow = uh + PS - 1, pcol = uw + PS - 1;

    unsigned char *p8 = smem + L.off_p8;
    _Float16 *p16 = reinterpret_cast<_Float16 *>(smem + L.off_p16);
    int32_t *n8 = reinterpret_cast<int32_t *>(smem + L.off_n8);
    int32_t *n16 = reinterpret_cast<int32_t *>(smem + L.off_n16);
    uint32_t *tab = reinterpret_cast<uint32_t *>(smem + L.off_tab);
    const int plane8 = L.plane8;
    const int plane16 = L.rows * L.pitch16;

    // Per-lane state of the distance phase, kept across the frames of a video search: the A
    // fragments of reference i16 and the window and norm of the 4 references of this lane's
    // accumulators.
    const int i16 = lane & 15, q = lane >> 4;
    v4i a8;
    v8h a16a = {}, a16b = {};
    bool any_sum = false;
    int rwy0[4], rwx0[4], rwh[4], rww[4], rgreen[4], rn[4];
    uint64_t *run = reinterpret_cast<uint64_t *>(smem + L.total - NREF * RUN_K * 8);
    const int K = mp.K;

    for (int fi = 0; fi < nf; ++fi) {
        int slot = 0;
        const uint8_t *fimg = g.img;
        if constexpr (VIDEO) {
            // the reference's own frame first (its patches become the A fragments), then the others
            const int f = fi == 0 ? t : f_lo + fi - 1 + (f_lo + fi - 1 >= t ? 1 : 0);
            slot = f - f_lo;
            fimg = g0.img + (int64_t)f * va.frame_bytes;
            if (fi > 0) __syncthreads();   // the last frame's table and selection scratch are reused
        }

        // ---- stage the shifted planes: one thread per (row, group of 4 columns) ----
        // Dword w of int8 copy k holds the row's pixels 4w + k .. 4w + k + 3, and halves 4w .. 4w + 3
        // of fp16 copy k hold the pixels 4w + k .. 4w + k + 3, so a thread needs pixels 4w .. 4w + 6.
        // Bytes at or beyond the staged width pcol are never read (candidates end at pcol - 1).
        {
            const int nw = (pcol + 3) >> 2;
            const uint8_t *img_end = fimg + (int64_t)(g.h - 1) * g.stride + (int64_t)g.w * g.c;
            uint32_t *p8w = reinterpret_cast<uint32_t *>(p8);
            uint32_t *p16w = reinterpret_cast<uint32_t *>(p16);
            for (int e = tid; e < prow * nw; e += BMT) {
                const int r = e / nw, w4 = 4 * (e - r * nw);
                const int npx = min(7, pcol - w4);
                const uint8_t *a = fimg + (int64_t)(uy0 + r) * g.stride + (int64_t)(ux0 + w4) * g.c;
                uint32_t raw[6];   // bytes 0 .. 23 from a
                const uintptr_t ai = (uintptr_t)a;
                const uint32_t *ab = reinterpret_cast<const uint32_t *>(ai & ~(uintptr_t)3);
                if (npx == 7 && (const uint8_t *)(ab + 7) <= img_end) {
                    const uint32_t sh = (uint32_t)(ai & 3);
                    uint32_t d[7];
#pragma unroll
                    for (int i = 0; i < 7; ++i) d[i] = ab[i];
#pragma unroll
                    for (int i = 0; i < 6; ++i) raw[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
                } else {   // row end: only the pixels that exist, byte by byte
#pragma unroll
                    for (int i = 0; i < 6; ++i) raw[i] = 0u;
                    const int nb = npx * g.c;
                    for (int b = 0; b < nb; ++b) raw[b >> 2] |= (uint32_t)a[b] << (8 * (b & 3));
                }
                auto byte_at = [&](int i) { return (int)((raw[i >> 2] >> (8 * (i & 3))) & 0xffu); };
                int v8[7], vs[7];
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    if (g.c == 3) {
                        const int R = byte_at(3 * q), G = byte_at(3 * q + 1), B = byte_at(3 * q + 2);
                        v8[q] = G - 128;
                        vs[q] = R + G + B - 384;
                    } else {
                        v8[q] = byte_at(q) - 128;
                        vs[q] = 0;
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    p8w[(k * plane8 + r * L.pitch8 + w4) >> 2] =
                        (uint32_t)(uint8_t)v8[k] | ((uint32_t)(uint8_t)v8[k + 1] << 8) |
                        ((uint32_t)(uint8_t)v8[k + 2] << 16) | ((uint32_t)(uint8_t)v8[k + 3] << 24);
                if (g.c == 3) {
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            const uint32_t lo = __builtin_bit_cast(uint16_t, (_Float16)vs[2 * hh + k]);
                            const uint32_t hi = __builtin_bit_cast(uint16_t, (_Float16)vs[2 * hh + k + 1]);
                            p16w[(k * plane16 + r * L.pitch16 + w4 + 2 * hh) >> 1] = lo | (hi << 16);
                        }
                }
            }
        }
        __syncthreads();
        if (fi == 0 && tid == 0) {   // read after the norm phase's barriers
            int any = 0;
            for (int i = 0; i < NREF; ++i) any |= (ti.ry[i] >= 0 && !ti.green[i]);
            ti.any_sum = any;
        }

        // ---- squared norms at every candidate position (horizontal then vertical 8-sums) ----
        // Four consecutive outputs per thread from one window of 11 values, sliding (exact integers).
        // Reads past the last valid output stay inside the staged planes and the table; the
        // outputs they feed are not stored.
        {
            int32_t *rs8 = reinterpret_cast<int32_t *>(tab);          // prow x uw, tab is free now
            int32_t *rs16 = rs8 + prow * uw;
            const int ng = (uw + 3) >> 2;
            for (int e = tid; e < prow * ng; e += BMT) {
                const int r = e / ng, c0 = 4 * (e - r * ng);
                int q8[11], q16[11];
                {
                    const uint32_t *w8 = reinterpret_cast<const uint32_t *>(p8 + r * L.pitch8 + c0);
                    const uint32_t b[3] = {w8[0], w8[1], w8[2]};
#pragma unroll
                    for (int j = 0; j < 11; ++j) {
                        const int v = (int)(int8_t)(b[j >> 2] >> (8 * (j & 3)));
                        q8[j] = v * v;
                    }
                }
                if (g.c == 3) {
                    const uint32_t *w16 = reinterpret_cast<const uint32_t *>(p16 + r * L.pitch16 + c0);
                    uint32_t b[6];
#pragma unroll
                    for (int i = 0; i < 6; ++i) b[i] = w16[i];
#pragma unroll
                    for (int j = 0; j < 11; ++j) {
                        const int t = (int)__builtin_bit_cast(_Float16, (uint16_t)(b[j >> 1] >> (16 * (j & 1))));
                        q16[j] = t * t;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 11; ++j) q16[j] = 0;
                }
                int a = 0, t = 0;
#pragma unroll
                for (int j = 0; j < PS; ++j) {
                    a += q8[j];
                    t += q16[j];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (c0 + k < uw) {
                        rs8[r * uw + c0 + k] = a;
                        rs16[r * uw + c0 + k] = t;
                    }
                    if (k < 3) {
                        a += q8[k + PS] - q8[k];
                        t += q16[k + PS] - q16[k];
                    }
                }
            }
            __syncthreads();
            const int nr4 = (uh + 3) >> 2;
            for (int e = tid; e < nr4 * uw; e += BMT) {
                const int r4 = 4 * (e / uw), col = e - (r4 >> 2) * uw;
                int c8[11], c16[11];
#pragma unroll
                for (int i = 0; i < 11; ++i) {
                    c8[i] = rs8[(r4 + i) * uw + col];
                    c16[i] = rs16[(r4 + i) * uw + col];
                }
                int a = 0, t = 0;
#pragma unroll
                for (int i = 0; i < PS; ++i) {
                    a += c8[i];
                    t += c16[i];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (r4 + k < uh) {
                        n8[(r4 + k) * uw + col] = a;
                        n16[(r4 + k) * uw + col] = t;
                    }
                    if (k < 3) {
                        a += c8[k + PS] - c8[k];
                        t += c16[k + PS] - c16[k];
                    }
                }
            }
            __syncthreads();
        }

        // ---- distances on the matrix cores ----
        {
            if (fi == 0) {
                // A fragments: reference i16, rows 2q, 2q+1 (int8) and rows q, q+4 (fp16).
                int ar = ti.ry[i16] >= 0 ? ti.ry[i16] - uy0 : 0;
                int ac = ti.ry[i16] >= 0 ? ti.rx[i16] - ux0 : 0;
                {
                    const int k = ac & 3;
                    const unsigned char *base = p8 + k * plane8;
                    const int o0 = (ar + 2 * q) * L.pitch8 + ac - k, o1 = o0 + L.pitch8;
                    a8[0] = (int)lds_u32(base, o0); a8[1] = (int)lds_u32(base, o0 + 4);
                    a8[2] = (int)lds_u32(base, o1); a8[3] = (int)lds_u32(base, o1 + 4);
                }
                any_sum = ti.any_sum != 0;
                if (any_sum) {
                    const int k = ac & 1;
                    const _Float16 *base = p16 + k * plane16;
                    const _Float16 *ra = base + (ar + q) * L.pitch16 + ac - k;
                    const _Float16 *rb = base + (ar + q + 4) * L.pitch16 + ac - k;
#pragma unroll
                    for (int t = 0; t < 8; ++t) { a16a[t] = ra[t]; a16b[t] = rb[t]; }
                }
                // Per-lane info of the 4 references this lane's accumulators belong to.
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ii = 4 * q + r;
                    rwy0[r] = ti.wy0[ii]; rwx0[r] = ti.wx0[ii];
                    rwh[r] = ti.wh[ii]; rww[r] = ti.ww[ii];
                    rgreen[r] = ti.green[ii];
                    if (ti.ry[ii] >= 0) {
                        const int pe = (ti.ry[ii] - uy0) * uw + (ti.rx[ii] - ux0);
                        rn[r] = rgreen[r] ? n8[pe] : n16[pe];
                    } else {
                        rn[r] = 0;
                        rwh[r] = 0;
                    }
                }
            }
            if constexpr (VIDEO) {
                // reloaded for every frame: only the norms and the A fragments stay live across frames
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ii = 4 * q + r;
                    rwy0[r] = ti.wy0[ii]; rwx0[r] = ti.wx0[ii];
                    rwh[r] = ti.ry[ii] >= 0 ? ti.wh[ii] : 0; rww[r] = ti.ww[ii];
                    rgreen[r] = ti.green[ii];
                }
            }
            const int nU = uh * uw;
            const int nchunks = (nU + 15) >> 4;
            // candidate j = 16 chunk + i16 at (row, column) = (j / uw, j % uw), stepped by 16 BMW
            constexpr int JSTEP = 16 * BMW;
            const int step_r = JSTEP / uw, step_c = JSTEP % uw;
            int jr = (16 * wave + i16) / uw, jc = (16 * wave + i16) % uw;
            for (int chunk = wave; chunk < nchunks; chunk += BMW) {
                const int j = chunk * 16 + i16;
                const int cr = j < nU ? jr : 0, cc = j < nU ? jc : 0;
                jr += step_r;
                jc += step_c;
                if (jc >= uw) {
                    jc -= uw;
                    ++jr;
                }
                v4i b8;
                {
                    const int k = cc & 3;
                    const unsigned char *base = p8 + k * plane8;
                    const int o0 = (cr + 2 * q) * L.pitch8 + cc - k, o1 = o0 + L.pitch8;
                    b8[0] = (int)lds_u32(base, o0); b8[1] = (int)lds_u32(base, o0 + 4);
                    b8[2] = (int)lds_u32(base, o1); b8[3] = (int)lds_u32(base, o1 + 4);
                }
                v4i acc8 = {0, 0, 0, 0};
                acc8 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a8, b8, acc8, 0, 0, 0);
                v4f acc16 = {0.f, 0.f, 0.f, 0.f};
                if (any_sum) {
                    // 8 halves from the copy in which they start on a dword (pitch and offsets even)
                    const int k = cc & 1;
                    const _Float16 *base = p16 + k * plane16;
                    const uint32_t *ra = reinterpret_cast<const uint32_t *>(base + (cr + q) * L.pitch16 + cc - k);
                    const uint32_t *rb = reinterpret_cast<const uint32_t *>(base + (cr + q + 4) * L.pitch16 + cc - k);
                    const v8h b16a = __builtin_bit_cast(v8h, make_uint4(ra[0], ra[1], ra[2], ra[3]));
                    const v8h b16b = __builtin_bit_cast(v8h, make_uint4(rb[0], rb[1], rb[2], rb[3]));
                    acc16 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a16a, b16a, acc16, 0, 0, 0);
                    acc16 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a16b, b16b, acc16, 0, 0, 0);
                }
                if (j < nU) {
                    const int cy = uy0 + cr, cx = ux0 + cc;
                    const int nb8 = n8[j], nb16 = n16[j];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int dy = cy - rwy0[r], dx = cx - rwx0[r];
                        if ((unsigned)dy < (unsigned)rwh[r] && (unsigned)dx < (unsigned)rww[r]) {
                            const int d = rgreen[r] ? rn[r] + nb8 - 2 * acc8[r] : rn[r] + nb16 - 2 * (int)acc16[r];
                            tab[(4 * q + r) * TAB_STRIDE + dy * rww[r] + dx] = (uint32_t)d;
                        }
                    }
                }
            }
        }
        __syncthreads();

        // ---- top-K per reference ----
        uint64_t *sel = reinterpret_cast<uint64_t *>(smem + L.off_sel) + wave * SEL_CAP;
        for (int ii = wave; ii < NREF; ii += BMW) {
            if (ti.ry[ii] < 0) continue;
            const int n = ti.wh[ii] * ti.ww[ii];
            const uint32_t *row = tab + ii * TAB_STRIDE;
            // this lane's candidates p = lane + 64 i, read once; key = (distance, position)
            constexpr int NPL = (MAX_CAND + 63) / 64;
            uint32_t dv[NPL];
            uint32_t dmin = 0xFFFFFFFFu;   // valid distances are below 2^26
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int p = lane + 64 * i;
                dv[i] = p < n ? row[p] : 0xFFFFFFFFu;
                dmin = min(dmin, dv[i]);
            }
            if constexpr (VIDEO) {
                if (fi > 0) {
                    // Only keys below the running K-th can enter the list.  When at most 64 - K of
                    // this frame's candidates are, one sort of them with the list is the merge.
                    const uint64_t th = run[ii * RUN_K + K - 1];
                    const uint64_t sk = (uint64_t)slot << 10;
                    int cnt = 0;
#pragma unroll
                    for (int i = 0; i < NPL; ++i) {
                        const int p = lane + 64 * i;
                        cnt += (p < n && (((uint64_t)dv[i] << 16) | sk | (uint64_t)p) < th);
                    }
                    int total;
                    int off = wave_excl_scan(cnt, lane, &total);
                    if (total <= 64 - K) {
#pragma unroll
                        for (int i = 0; i < NPL; ++i) {
                            const int p = lane + 64 * i;
                            const uint64_t key = ((uint64_t)dv[i] << 16) | sk | (uint64_t)p;
                            if (p < n && key < th) sel[off++] = key;
                        }
                        wave_lds_sync();
                        uint64_t v = lane < total ? sel[lane]
                                                  : (lane < total + K ? run[ii * RUN_K + lane - total] : ~0ull);
                        v = wave_sort64(v, lane);
                        if (lane < K) run[ii * RUN_K + lane] = v;
                        wave_lds_sync();
                        continue;
                    }
                }
            }
            // the lane's smallest key: its smallest distance at the first (smallest) position
            int pmin = 0;
#pragma unroll
            for (int i = NPL - 1; i >= 0; --i) pmin = dv[i] == dmin ? lane + 64 * i : pmin;
            if (!VIDEO && ti.green[ii]) {
                // green or gray distances are below 2^22 (64 * 255^2) and positions below 1024, so
                // the key (distance, position) fits 32 bits and stays below the empty key ~0
                const uint32_t lmin32 = dmin == 0xFFFFFFFFu ? ~0u : ((dmin << 10) | (uint32_t)pmin);
                const uint32_t sorted32 = wave_sort_asc<uint32_t>(lmin32, lane);
                const uint32_t theta32 = __builtin_amdgcn_readlane(sorted32, K - 1);
                int cnt32 = 0;
#pragma unroll
                for (int i = 0; i < NPL; ++i) {
                    const int p = lane + 64 * i;
                    cnt32 += (p < n && ((dv[i] << 10) | (uint32_t)p) <= theta32);
                }
                int total32;
                int off32 = wave_excl_scan(cnt32, lane, &total32);
                uint32_t *sel32 = reinterpret_cast<uint32_t *>(sel);
#pragma unroll
                for (int i = 0; i < NPL; ++i) {
                    const int p = lane + 64 * i;
                    const uint32_t key = (dv[i] << 10) | (uint32_t)p;
                    if (p < n && key <= theta32) sel32[off32++] = key;
                }
                wave_lds_sync();
                uint32_t mine32;
                if (total32 <= 64) {
                    mine32 = wave_sort_asc<uint32_t>(lane < total32 ? sel32[lane] : ~0u, lane);
                } else {
                    int P = 64;
                    while (P < total32) P <<= 1;
                    for (int t = total32 + lane; t < P; t += 64) sel32[t] = ~0u;
                    wave_lds_sync();
                    lds_sort(sel32, P, lane);
                    mine32 = lane < K ? sel32[lane] : ~0u;
                }
                if (lane < K) {
                    const int p = (int)(mine32 & 1023u);
                    const int y = ti.wy0[ii] + p / ti.ww[ii], x = ti.wx0[ii] + p % ti.ww[ii];
                    const int iy = tyi * REF_TILE + ii / REF_TILE, ix = txi * REF_TILE + ii % REF_TILE;
                    const int64_t r = (int64_t)iy * g.nx + ix;
                    idx_out[r * K + lane] = y * g.w + x;
                    if (dist_out) dist_out[r * K + lane] = (int32_t)(mine32 >> 10);
                }
                wave_lds_sync();
                continue;
            }
            const uint64_t lmin = dmin == 0xFFFFFFFFu ? ~0ull : (((uint64_t)dmin << 10) | (uint64_t)pmin);
            const uint64_t sorted = wave_sort64(lmin, lane);
            const uint64_t theta = readlane_u64(sorted, K - 1);
            int cnt = 0;
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int p = lane + 64 * i;
                cnt += (p < n && (((uint64_t)dv[i] << 10) | (uint64_t)p) <= theta);
            }
            int total;
            int off = wave_excl_scan(cnt, lane, &total);
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int p = lane + 64 * i;
                const uint64_t key = ((uint64_t)dv[i] << 10) | (uint64_t)p;
                if (p < n && key <= theta) sel[off++] = key;
            }
            wave_lds_sync();
            uint64_t mine;
            if (total <= 64) {
                uint64_t v = lane < total ? sel[lane] : ~0ull;
                mine = wave_sort64(v, lane);
            } else {
                int P = 64;
                while (P < total) P <<= 1;
                for (int t = total + lane; t < P; t += 64) sel[t] = ~0ull;
                wave_lds_sync();
                lds_sort(sel, P, lane);
                mine = lane < K ? sel[lane] : ~0ull;
            }
            if constexpr (VIDEO) {
                // merge into the running list: keys (distance, frame slot, position); only this wave
                // touches reference ii's list
                uint64_t v = lane < K ? (((mine >> 10) << 16) | ((uint64_t)slot << 10) | (mine & 1023u)) : ~0ull;
                if (fi > 0) {
                    if (lane >= K && lane < 2 * K) v = run[ii * RUN_K + lane - K];
                    v = wave_sort64(v, lane);
                }
                if (lane < K) run[ii * RUN_K + lane] = v;
            } else if (lane < K) {
                const int p = (int)(mine & 1023u);
                const int y = ti.wy0[ii] + p / ti.ww[ii], x = ti.wx0[ii] + p % ti.ww[ii];
                const int iy = tyi * REF_TILE + ii / REF_TILE, ix = txi * REF_TILE + ii % REF_TILE;
                const int64_t r = (int64_t)iy * g.nx + ix;
                idx_out[r * K + lane] = y * g.w + x;
                if (dist_out) dist_out[r * K + lane] = (int32_t)(mine >> 10);
            }
            wave_lds_sync();
        }
    }   // frames

    if constexpr (VIDEO) {
        for (int ii = wave; ii < NREF; ii += BMW) {
            if (ti.ry[ii] < 0 || lane >= K) continue;
            const uint64_t key = run[ii * RUN_K + lane];
            const int p = (int)(key & 1023u), f = f_lo + (int)((key >> 10) & 63u);
            const int y = ti.wy0[ii] + p / ti.ww[ii], x = ti.wx0[ii] + p % ti.ww[ii];
            const int iy = tyi * REF_TILE + ii / REF_TILE, ix = txi * REF_TILE + ii % REF_TILE;
            const int64_t r = ((int64_t)t * g.ny + iy) * g.nx + ix;
            idx_out[r * K + lane] = (f * g.h + y) * g.w + x;
            if (dist_out) dist_out[r * K + lane] = (int32_t)(key >> 16);
        }
    }
}

__global__ __launch_bounds__(BMT) void bm_kernel(ImageGeom g, MethodParams mp, int tiles_x, int n_tiles,
                                                 BmLds L, int32_t *__restrict__ idx_out,
                                                 int32_t *__restrict__ dist_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ TileInfo ti;
    // XCD-aware order: consecutive workgroups are dealt round-robin over the 8 XCDs; give
    // each XCD a contiguous run of tiles so neighbouring tiles share its L2.
    // The grid has 8*ceil(n_tiles/8) workgroups; b -> (b%8)*per + b/8 is a bijection on it.
    const int per = (n_tiles + 7) / 8;
    const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= n_tiles) return;
    bm_tile<false>(g, mp, tiles_x, b, L, idx_out, dist_out, smem, ti, VideoArgs{});
}

// Spatio-temporal form: n_tiles covers the tiles of all frames.
__global__ __launch_bounds__(BMT) void bm_video_kernel(ImageGeom g, MethodParams mp, int tiles_x, int n_tiles,
                                                       VideoArgs va, BmLds L, int32_t *__restrict__ idx_out,
                                                       int32_t *__restrict__ dist_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ TileInfo ti;
    const int per = (n_tiles + 7) / 8;
    const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= n_tiles) return;
    bm_tile<true>(g, mp, tiles_x, b, L, idx_out, dist_out, smem, ti, va);
}

// Persistent form over many images: each workgroup pulls (image, tile) units from a queue.
__global__ __launch_bounds__(BMT) void bm_kernel_batched(const BatchItem *__restrict__ items, int n_items,
                                                         const int *__restrict__ unit_start, BmLds L,
                                                         int *__restrict__ queue) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ TileInfo ti;
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
        bm_tile<false>(it.g, it.mp, it.bm_tiles_x, u - unit_start[i], L, it.idx, nullptr, smem, ti, VideoArgs{});
        __syncthreads();
    }
}

BmLds bm_lds_layout(int uh_max, int uw_max, bool video = false) {
    BmLds L;
    L.rows = uh_max + PS - 1;
    // The int8 planes: rows of 96 bytes (enough for a union of 64 columns plus the patch and the
    // dword reads past it) and copies 16 bytes past a row multiple apart.  With these offsets the
    // 64 lanes' dword reads of a distance step (16 consecutive candidates x 4 row pairs, each
    // candidate in the copy where it starts on a dword) spread over the LDS banks (at most 1.5
    // reads per bank against 2 to 4 for tightly packed rows, whether 32 or 64 banks serve a
    // half or a whole wave).
    const int pitch_min = ((uw_max + PS + 3) / 4) * 4 + 4;
    L.pitch8 = pitch_min > 96 ? pitch_min : 96;
    L.plane8 = L.rows * L.pitch8 + 16;
    L.pitch16 = ((uw_max + PS + 1) / 2) * 2 + 2;
    int off = 0;
    L.off_p8 = off;  off += 4 * L.plane8;
    off = (off + 15) & ~15;
    L.off_p16 = off; off += 2 * L.rows * L.pitch16 * 2;
    off = (off + 15) & ~15;
    L.off_n8 = off;  off += uh_max * uw_max * 4;
    L.off_n16 = off; off += uh_max * uw_max * 4;
    off = (off + 15) & ~15;
    // the selection scratch reuses the plane/norm region once the distances are in the table
    const int sel_bytes = BMW * SEL_CAP * 8;
    int region = off;
    L.off_sel = 0;
    if (region < sel_bytes) region = sel_bytes;
    off = (region + 15) & ~15;
    L.off_tab = off;
    int tab_bytes = NREF * TAB_STRIDE * 4;
    const int rs_bytes = 2 * L.rows * uw_max * 4;  // row sums of the norm pass live in the table
    if (tab_bytes < rs_bytes) tab_bytes = rs_bytes;
    off += tab_bytes;
    if (video) off += NREF * RUN_K * 8;   // the running lists of the video search
    L.total = off;
    return L;
}

}  // namespace

hipError_t launch_block_match(const ImageGeom &g, const MethodParams &mp, int32_t *idx, int32_t *dist,
                              hipStream_t st) {
    const int tiles_y = (g.ny + REF_TILE - 1) / REF_TILE, tiles_x = (g.nx + REF_TILE - 1) / REF_TILE;
    const int n_tiles = tiles_y * tiles_x;
    // largest union of windows over a tile: 3 grid steps plus the window, capped by the image
    const int span = (REF_TILE - 1) * g.s + mp.W;
    const int uh = span < g.h - PS + 1 ? span : g.h - PS + 1;
    const int uw = span < g.w - PS + 1 ? span : g.w - PS + 1;
    BmLds L = bm_lds_layout(uh, uw);
    hipError_t e = prepare_dynamic_lds((const void *)bm_kernel, L.total, (int)sizeof(TileInfo));
    if (e != hipSuccess) return e;
    // round the grid up to a multiple of 8 so the XCD remap is a bijection onto [0, 8*per)
    const int per = (n_tiles + 7) / 8;
    hipLaunchKernelGGL(bm_kernel, dim3(8 * per), dim3(BMT), L.total, st, g, mp, tiles_x, n_tiles, L, idx, dist);
    return hipGetLastError();
}

// Spatio-temporal block matching of T frames of g.h rows stacked from g.img (Sec. IV-C): the
// candidates of a reference in frame t are its clipped window in frames t - radius .. t + radius
// (within [0, T)).  idx/dist: T * ny * nx references, frame-major; idx = (f*h + y)*w + x.
hipError_t launch_block_match_video(const ImageGeom &g, const MethodParams &mp, int T, int radius, int32_t *idx,
                                    int32_t *dist, hipStream_t st) {
    const int tiles_y = (g.ny + REF_TILE - 1) / REF_TILE, tiles_x = (g.nx + REF_TILE - 1) / REF_TILE;
    const int64_t n_tiles64 = (int64_t)tiles_y * tiles_x * T;
    if (T < 1 || radius < 0 || radius > 31 || mp.K > RUN_K || n_tiles64 > (int64_t)1 << 30)
        return hipErrorInvalidValue;
    const int n_tiles = (int)n_tiles64;
    const int span = (REF_TILE - 1) * g.s + mp.W;
    const int uh = span < g.h - PS + 1 ? span : g.h - PS + 1;
    const int uw = span < g.w - PS + 1 ? span : g.w - PS + 1;
    BmLds L = bm_lds_layout(uh, uw, true);
    hipError_t e = prepare_dynamic_lds((const void *)bm_video_kernel, L.total, (int)sizeof(TileInfo));
    if (e != hipSuccess) return e;
    VideoArgs va{T, radius, (int64_t)g.h * g.stride};
    const int per = (n_tiles + 7) / 8;
    hipLaunchKernelGGL(bm_video_kernel, dim3(8 * per), dim3(BMT), L.total, st, g, mp, tiles_x, n_tiles, va, L, idx,
                       dist);
    return hipGetLastError();
}

// Batched block matching: one persistent launch over the tiles of all images; the LDS layout
// is the largest any image of the batch needs.
hipError_t launch_block_match_batched(const BatchItem *items, int n_items, const int *unit_start, int max_s,
                                      int max_W, int max_h, int max_w, int *queue, int grid, hipStream_t st) {
    const int span = (REF_TILE - 1) * max_s + max_W;
    const int uh = span < max_h - PS + 1 ? span : max_h - PS + 1;
    const int uw = span < max_w - PS + 1 ? span : max_w - PS + 1;
    BmLds L = bm_lds_layout(uh, uw);
    hipError_t e = prepare_dynamic_lds((const void *)bm_kernel_batched, L.total, (int)sizeof(TileInfo) + 16);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bm_kernel_batched, dim3(grid), dim3(BMT), L.total, st, items, n_items, unit_start, L, queue);
    return hipGetLastError();
}

int bm_lds_bytes(int s, int W, int h, int w) {
    const int span = (REF_TILE - 1) * s + W;
    const int uh = span < h - PS + 1 ? span : h - PS + 1;
    const int uw = span < w - PS + 1 ? span : w - PS + 1;
    return bm_lds_layout(uh, uw).total;
}

hipError_t prepare_dynamic_lds(const void *kernel, int bytes, int static_bytes) {
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (bytes + static_bytes > max_lds) return hipErrorInvalidValue;
    if (bytes > 64 * 1024) {
        // opt-in for large dynamic LDS where the runtime asks for it; a runtime that does not
        // need the opt-in may reject the attribute, which is harmless
        if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
            (void)hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace htsvd
