// Channel Gram sums of all reference patches of one image: the device half of learning the
// t-SVD basis pair from the image itself (Sec. III-B, Eq. 10-11).
//
// Over the reference grid (rows ys, columns xs, Algorithm 1) the row sums
//   G_row[a][b][i][k] = sum_{y in ys, x in xs} sum_j X(y+i, x+j, a) X(y+k, x+j, b)
// regroup by image column: for a fixed y the pair (x, j) only enters through col = x + j, so
//   G_row = sum_{y in ys} sum_col m(col) v v^T,   v = X(y..y+7, col, :),
// with m(col) the number of reference columns whose patch covers col.  The column sums are the
// same with the roles of rows and columns swapped (horizontal 8-vectors at the reference
// columns, weighted by the number of reference rows covering the pixel row).  Every entry is an
// exact integer (below 2^50 for any image the library accepts), accumulated in 32-bit per staged
// chunk and in 64-bit across chunks.
#include "common.h"

namespace htsvd {

namespace {

constexpr int GR_THREADS = 256;
constexpr int GR_CHUNK = 256;    // vectors staged per step, one per thread
constexpr int GR_MAX_BLOCKS = 1024;

// Reference positions along a side of n pixels (n_ref of them) whose patch covers pixel pos:
// regular positions i*s for i <= n_ref - 2, plus the last one at n - 8.
__device__ inline int cover_count(int pos, int n, int n_ref, int s) {
    int cnt = 0;
    if (n_ref >= 2) {
        const int lo = pos >= PS - 1 ? (pos - (PS - 1) + s - 1) / s : 0;
        const int hi = min(n_ref - 2, pos / s);
        cnt = max(0, hi - lo + 1);
    }
    return cnt + (pos >= n - PS ? 1 : 0);
}

// Thread tasks: an entry row r = ch*8 + i (A = 8c of them) times a block of 4 entry columns
// starting at 4*bb, for bb >= r/4 (the other blocks follow by symmetry).  T = 4c(2c+1) tasks.
template <int C>
__global__ __launch_bounds__(GR_THREADS) void gram_kernel(const uint8_t *__restrict__ img, int64_t stride, int h,
                                                          int w, int s, int ny, int nx,
                                                          unsigned long long *__restrict__ out) {
    constexpr int A = 8 * C, NBB = 2 * C, T = 4 * C * (2 * C + 1), GRP = GR_THREADS / T;
    __shared__ __align__(16) uint32_t sv[GR_CHUNK * A];    // the staged vectors
    __shared__ __align__(16) uint32_t smv[GR_CHUNK * A];   // the same, times their weight
    __shared__ unsigned long long sred[GRP * T * 4];
    const int g = blockIdx.y;   // 0: row sums, 1: column sums
    const int64_t n_vec = g == 0 ? (int64_t)ny * w : (int64_t)nx * h;
    const int64_t n_chunks = (n_vec + GR_CHUNK - 1) / GR_CHUNK;
    const int tid = threadIdx.x;
    const int grp = tid / T, task = tid % T;
    const bool active = grp < GRP;
    int r = 0, bb = 0;
    {
        int rem = task;
        while (rem >= NBB - r / 4) {
            rem -= NBB - r / 4;
            ++r;
        }
        bb = r / 4 + rem;
    }
    unsigned long long tot0 = 0, tot1 = 0, tot2 = 0, tot3 = 0;
    for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
        const int64_t q0 = ch * GR_CHUNK;
        const int nv = (int)min<int64_t>(GR_CHUNK, n_vec - q0);
        if (tid < nv) {
            const int64_t q = q0 + tid;
            const uint8_t *p;
            int64_t step;
            uint32_t m;
            if (g == 0) {
                const int iy = (int)(q / w), col = (int)(q % w);
                p = img + (int64_t)ref_pos(iy, ny, h, s) * stride + (int64_t)col * C;
                step = stride;
                m = cover_count(col, w, nx, s);
            } else {
                const int row = (int)(q / nx), ix = (int)(q % nx);
                p = img + (int64_t)row * stride + (int64_t)ref_pos(ix, nx, w, s) * C;
                step = C;
                m = cover_count(row, h, ny, s);
            }
#pragma unroll
            for (int i = 0; i < PS; ++i)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const uint32_t v = p[i * step + c];
                    sv[tid * A + c * PS + i] = v;
                    smv[tid * A + c * PS + i] = __umul24(m, v);
                }
        }
        __syncthreads();
        if (active) {
            // At most 256/GRP vectors of weight <= 9 per chunk: every partial sum stays below 2^32.
            // Factors below 2^24 (weighted value <= 9 * 255, value <= 255): 24-bit multiply-adds.
            uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
            int v = grp;
            for (; v + 3 * GRP < nv; v += 4 * GRP) {
                uint32_t x[4];
                uint4 y[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    x[u] = smv[(v + u * GRP) * A + r];
                    y[u] = *reinterpret_cast<const uint4 *>(&sv[(v + u * GRP) * A + 4 * bb]);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a0 = __umul24(x[u], y[u].x) + a0;
                    a1 = __umul24(x[u], y[u].y) + a1;
                    a2 = __umul24(x[u], y[u].z) + a2;
                    a3 = __umul24(x[u], y[u].w) + a3;
                }
            }
            for (; v < nv; v += GRP) {
                const uint32_t x = smv[v * A + r];
                const uint4 y = *reinterpret_cast<const uint4 *>(&sv[v * A + 4 * bb]);
                a0 = __umul24(x, y.x) + a0;
                a1 = __umul24(x, y.y) + a1;
                a2 = __umul24(x, y.z) + a2;
                a3 = __umul24(x, y.w) + a3;
            }
            tot0 += a0;
            tot1 += a1;
            tot2 += a2;
            tot3 += a3;
        }
        __syncthreads();
    }
    if (active) {
        unsigned long long *d = sred + (grp * T + task) * 4;
        d[0] = tot0;
        d[1] = tot1;
        d[2] = tot2;
        d[3] = tot3;
    }
    __syncthreads();
    // One atomic per entry and block; the mirrored entry (b, r) is added too where no task of
    // its own covers it (column block below its row's block).
    for (int e = tid; e < T * 4; e += GR_THREADS) {
        unsigned long long sum = 0;
        for (int k = 0; k < GRP; ++k) sum += sred[k * T * 4 + e];
        if (sum == 0) continue;
        int rr = 0, rem = e / 4;
        while (rem >= NBB - rr / 4) {
            rem -= NBB - rr / 4;
            ++rr;
        }
        const int b = 4 * (rr / 4 + rem) + (e & 3);
        // entry (rr, b) = (ch1*8 + i, ch2*8 + k) -> out[g][ch1][ch2][i][k]
        unsigned long long *og = out + (size_t)g * C * C * 64;
        atomicAdd(og + ((rr / PS) * C + b / PS) * 64 + (rr % PS) * PS + b % PS, sum);
        if (b / 4 != rr / 4) atomicAdd(og + ((b / PS) * C + rr / PS) * 64 + (b % PS) * PS + rr % PS, sum);
    }
}

// The same sums for a runtime channel count C (hyperspectral bands, up to 64), taken before the
// regrouping by column: the row sums over the vectors v = X(y..y+7, x+j, :) of every reference
// (y, x) and offset j, the column sums over X(y+i, x..x+7, :), without weights.  A block owns a
// 64 x 64 tile pair (ta <= tb) of the A x A matrix (A = 8C) and a slice of the vectors; it stages
// 64 vectors at a time in LDS, the bytes of 4 consecutive vectors packed in one word per entry
// (P[group][entry]), and each thread adds a 4 x 4 block of entries with v_dot4_u32_u8 (four
// byte products per instruction).  Per chunk the 32-bit partial is at most 64 * 255^2; the
// blocks add 64-bit totals with integer atomics (exact, so in any order).
constexpr int GB_VEC = 64;            // vectors per staged chunk
constexpr int GB_GROUPS = GB_VEC / 4;

__global__ __launch_bounds__(256) void gram_bands_kernel(const uint8_t *__restrict__ img, int64_t stride, int h,
                                                         int w, int C, int s, int ny, int nx,
                                                         unsigned long long *__restrict__ out) {
    __shared__ uint32_t P[2][GB_GROUPS][64];
    const int A = 8 * C;
    const int g = blockIdx.y;
    // tile pair (ta, tb), ta <= tb, row-major over the upper triangle of the tile grid
    const int nt = (A + 63) / 64;
    int ta = 0, rem = blockIdx.x;
    while (rem >= nt - ta) {
        rem -= nt - ta;
        ++ta;
    }
    const int tb = ta + rem;
    const int64_t n_vec = (int64_t)ny * nx * 8;
    const int64_t n_chunks = (n_vec + GB_VEC - 1) / GB_VEC;
    const int64_t c_begin = n_chunks * blockIdx.z / gridDim.z, c_end = n_chunks * (blockIdx.z + 1) / gridDim.z;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    unsigned long long tot[4][4] = {};
    for (int64_t ck = c_begin; ck < c_end; ++ck) {
        // staging: 2 x 16 x 64 words, one per (tile side, 4-vector group, entry)
        for (int t = threadIdx.x; t < 2 * GB_GROUPS * 64; t += 256) {
            const int side = t / (GB_GROUPS * 64), k = (t / 64) % GB_GROUPS, ai = t % 64;
            const int a = (side ? tb : ta) * 64 + ai;
            const int64_t q = ck * GB_VEC + 4 * k;   // first of 4 vectors with the same reference
            uint32_t word = 0;
            if (a < A && q < n_vec) {
                const int iy = (int)(q / ((int64_t)nx * 8)), rm = (int)(q % ((int64_t)nx * 8));
                const int ix = rm / 8, off = rm % 8, ch = a / 8, e = a % 8;
                const int y = ref_pos(iy, ny, h, s), x = ref_pos(ix, nx, w, s);
                // g = 0: entry e is the row offset, the 4 vectors are columns x+off..x+off+3;
                // g = 1: entry e is the column offset, the 4 vectors are rows y+off..y+off+3
                const uint8_t *px = g == 0 ? img + (int64_t)(y + e) * stride + (int64_t)(x + off) * C + ch
                                           : img + (int64_t)(y + off) * stride + (int64_t)(x + e) * C + ch;
                const int64_t step = g == 0 ? C : stride;
                word = (uint32_t)px[0] | ((uint32_t)px[step] << 8) | ((uint32_t)px[2 * step] << 16) |
                       ((uint32_t)px[3 * step] << 24);
            }
            P[side][k][ai] = word;
        }
        __syncthreads();
        uint32_t acc[4][4] = {};
#pragma unroll 4
        for (int k = 0; k < GB_GROUPS; ++k) {
            const uint4 pa = *reinterpret_cast<const uint4 *>(&P[0][k][ty * 4]);
            const uint4 pb = *reinterpret_cast<const uint4 *>(&P[1][k][tx * 4]);
            const uint32_t va[4] = {pa.x, pa.y, pa.z, pa.w}, vb[4] = {pb.x, pb.y, pb.z, pb.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_udot4(va[i], vb[j], acc[i][j], false);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) tot[i][j] += acc[i][j];
        __syncthreads();
    }
    unsigned long long *og = out + (size_t)g * C * C * 64;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = ta * 64 + ty * 4 + i, b = tb * 64 + tx * 4 + j;
            if (a >= A || b >= A || tot[i][j] == 0) continue;
            atomicAdd(og + ((a / 8) * C + b / 8) * 64 + (a % 8) * 8 + b % 8, tot[i][j]);
            if (ta != tb) atomicAdd(og + ((b / 8) * C + a / 8) * 64 + (b % 8) * 8 + a % 8, tot[i][j]);
        }
}

}  // namespace

hipError_t launch_gram(const uint8_t *img, int64_t stride, int h, int w, int c, int s, int64_t *out, hipStream_t st) {
    const int ny = ref_count(h, s), nx = ref_count(w, s);
    hipError_t e = launch_zero(out, sizeof(int64_t) * 2 * c * c * 64, st);
    if (e != hipSuccess) return e;
    if (c != 1 && c != 3) {
        const int nt = (8 * c + 63) / 64, n_tp = nt * (nt + 1) / 2;
        // vector slices for about 1024 workgroups, each with at least 8 chunks
        const int64_t n_chunks = ((int64_t)ny * nx * 8 + GB_VEC - 1) / GB_VEC;
        const int64_t zs = std::max<int64_t>(1, std::min<int64_t>((1024 + 2 * n_tp - 1) / (2 * n_tp), n_chunks / 8));
        hipLaunchKernelGGL(gram_bands_kernel, dim3((unsigned)n_tp, 2, (unsigned)zs), dim3(256), 0, st, img, stride, h,
                           w, c, s, ny, nx, reinterpret_cast<unsigned long long *>(out));
        return hipGetLastError();
    }
    const int64_t n_vec = std::max<int64_t>((int64_t)ny * w, (int64_t)nx * h);
    const int nb = (int)std::min<int64_t>(GR_MAX_BLOCKS, (n_vec + GR_CHUNK - 1) / GR_CHUNK);
    unsigned long long *o = reinterpret_cast<unsigned long long *>(out);
    if (c == 3)
        hipLaunchKernelGGL(gram_kernel<3>, dim3(nb, 2), dim3(GR_THREADS), 0, st, img, stride, h, w, s, ny, nx, o);
    else
        hipLaunchKernelGGL(gram_kernel<1>, dim3(nb, 2), dim3(GR_THREADS), 0, st, img, stride, h, w, s, ny, nx, o);
    return hipGetLastError();
}

}  // namespace htsvd
