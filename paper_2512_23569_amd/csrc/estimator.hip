// Plain noise-level estimation and the adaptive adjustment of Sec. III-E-1.
//
// sigma_est per sub-image (the paper's estimator is a CNN trained on data that is not
// available; this library's plain estimator follows the rationale of Eq. 12 -- the noisy
// patch correlation is the clean one plus sigma^2 I): the covariance of every 8x8 patch
// whose top-left pixel lies in the sub-image, its eigenvalues, and the noise-only tail
// chosen by the rule of Chen, Zhu and Heng (ICCV 2015): the first tail (eigenvalues in
// descending order) with as many members above its mean as below it; sigma^2 is that mean.
// Channels combine as sigma_est = sqrt(mean_c sigma_c^2).
//
//   - The patch second moments are a contraction over patches: S = X^T X with X the
//     n x 64 matrix of shifted patches (x - 128, int8).  One workgroup per (sub-image,
//     channel) runs it on v_mfma_i32_16x16x64_i8 with 64 patches per k-step; the row sums
//     come from the same instruction with an all-ones operand.  int32 partials are exact.
//   - The 64x64 FP64 covariance is diagonalised in LDS by cyclic Jacobi rotations with the
//     round-robin pairing (32 disjoint rotations per step).
//
// Eq. 22-23 vote: for a few groups per sub-image the rank a of the alternating eigenvalue
// lambda_hat = |sum_m (-1)^m p_m|^2 among the K eigenvalues of circ(G) circ(G)^T, whose
// closed-form spectrum is lambda_k = sum_d c_d cos(2 pi k d / K) with the exact integer
// autocorrelations c_d = sum_m p_m . p_{(m+d) mod K}; a group votes "adjust" if a <= gamma
// and a majority sets sigma_hat = sigma_est / beta.
#include <math.h>

#include "common.h"

namespace htsvd {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int COV_MAX_SIDE = 128 + PS - 1;   // staged pixels per side for a 128 sub-image
constexpr int COV_PITCH = 140;                 // bytes per staged row (>= 135 + 4, multiple of 4)

struct CovLds {
    int tile;   // sub-image side
};

__device__ inline void tile_bounds(const ImageGeom &g, int T, int t, int *y0, int *y1, int *x0, int *x1) {
    const int ntx = (g.w + T - 1) / T;
    const int ty = t / ntx, tx = t % ntx;
    *y0 = min(ty * T, g.h - PS);
    *y1 = min(ty * T + T - 1, g.h - PS);
    *x0 = min(tx * T, g.w - PS);
    *x1 = min(tx * T + T - 1, g.w - PS);
}

// 16 consecutive shifted pixels of staged row r starting at column col (any alignment),
// read from the byte-shifted copies; bytes at or beyond `valid` are zeroed.
__device__ inline v4i frag16(const unsigned char *lds, int plane, int r, int col, int valid) {
    const int k = col & 3;
    const uint32_t *p = reinterpret_cast<const uint32_t *>(lds + k * plane + r * COV_PITCH + col - k);
    v4i f;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        uint32_t v = p[d];
        const int lo = 4 * d;
        if (valid <= lo) v = 0u;
        else if (valid < lo + 4) v &= (1u << (8 * (valid - lo))) - 1u;
        f[d] = (int)v;
    }
    return f;
}

__global__ __launch_bounds__(256) void cov_eig_kernel(ImageGeom g, int T, double *__restrict__ sigma2) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_y0, s_y1, s_x0, s_x1;
    __shared__ int s_stop;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t = blockIdx.x / g.c, ch = blockIdx.x % g.c;
    if (tid == 0) {
        int y0, y1, x0, x1;
        tile_bounds(g, T, t, &y0, &y1, &x0, &x1);
        s_y0 = y0; s_y1 = y1; s_x0 = x0; s_x1 = x1;
    }
    __syncthreads();
    const int y0 = s_y0, y1 = s_y1, x0 = s_x0, x1 = s_x1;
    const int ny = y1 - y0 + 1, nx = x1 - x0 + 1;   // patch positions
    const int prow = ny + PS - 1, pcol = nx + PS - 1;
    const int plane = COV_MAX_SIDE * COV_PITCH;

    // stage x - 128 of this channel in 4 byte-shifted copies
    for (int e = tid; e < prow * pcol; e += 256) {
        const int r = e / pcol, col = e % pcol;
        const int v = (int)g.img[(int64_t)(y0 + r) * g.stride + (int64_t)(x0 + col) * g.c + ch] - 128;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (col >= k) smem[k * plane + r * COV_PITCH + col - k] = (unsigned char)(int8_t)v;
    }
    // zero the padding columns a fragment may read past pcol (masked anyway, keep defined)
    __syncthreads();

    // ---- second moments on the matrix cores ----
    // k-step = 64 consecutive patch positions of one row; lane (i = l%16, kq = l/16) holds
    // patch-vector entry 16*blk + i for patches 16*kq .. 16*kq+15 of the step.
    v4i acc[10];
    v4i acc1[4];
#pragma unroll
    for (int i = 0; i < 10; ++i) acc[i] = (v4i){0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) acc1[i] = (v4i){0, 0, 0, 0};
    const v4i ones = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
    const int i16 = lane & 15, kq = lane >> 4;
    const int xsteps = (nx + 63) / 64;
    for (int stp = wave; stp < ny * xsteps; stp += 4) {
        const int py = stp / xsteps, pxs = (stp % xsteps) * 64;
        const int k0 = pxs + 16 * kq;                 // first patch column of this lane
        const int valid = min(16, max(0, nx - k0));
        v4i f[4];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            const int e = 16 * blk + i16;             // patch-vector entry (a, b) = (e/8, e%8)
            f[blk] = frag16(smem, plane, py + e / 8, k0 + e % 8, valid);
        }
        int a = 0;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
#pragma unroll
            for (int jb = ib; jb < 4; ++jb) {
                acc[a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[ib], f[jb], acc[a], 0, 0, 0);
                ++a;
            }
            acc1[ib] = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[ib], ones, acc1[ib], 0, 0, 0);
        }
    }
    __syncthreads();  // staging no longer needed: reuse LDS

    // per-wave partials -> LDS, summed in int64
    int32_t *part = reinterpret_cast<int32_t *>(smem);          // [4 waves][64][64]
    int32_t *part1 = part + 4 * 64 * 64;                        // [4 waves][64]
    {
        int a = 0;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
#pragma unroll
            for (int jb = ib; jb < 4; ++jb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ib + 4 * kq + r, col = 16 * jb + i16;
                    part[(wave * 64 + row) * 64 + col] = acc[a][r];
                }
                ++a;
            }
            if (i16 == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) part1[wave * 64 + 16 * ib + 4 * kq + r] = acc1[ib][r];
            }
        }
    }
    __syncthreads();
    double *A = reinterpret_cast<double *>(smem + (4 * 64 * 64 + 4 * 64) * 4);   // 64 x 64
    double *S1 = A + 64 * 64;
    const double n = (double)ny * (double)nx;
    if (tid < 64) {
        int64_t s = 0;
        for (int w = 0; w < 4; ++w) s += part1[w * 64 + tid];
        S1[tid] = (double)s;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
        const int i = e / 64, j = e % 64;
        const int ii = min(i, j), jj = max(i, j);   // only blocks ib <= jb were computed
        int64_t s = 0;
        if ((ii / 16) <= (jj / 16)) {
            for (int w = 0; w < 4; ++w) s += part[(w * 64 + ii) * 64 + jj];
        }
        A[e] = (double)s / n - (S1[i] / n) * (S1[j] / n);
    }
    __syncthreads();

    // ---- cyclic Jacobi, round-robin pairs ----
    __shared__ double rc[32], rs[32];
    __shared__ int rp[32], rq[32];
    for (int sweep = 0; sweep < 20; ++sweep) {
        for (int rnd = 0; rnd < 63; ++rnd) {
            if (tid < 32) {
                int p, q;
                if (tid == 0) { p = rnd; q = 63; }
                else { p = (rnd + tid) % 63; q = (rnd - tid + 63) % 63; }
                if (p > q) { int x = p; p = q; q = x; }
                const double apq = A[p * 64 + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double app = A[p * 64 + p], aqq = A[q * 64 + q];
                    const double theta = (aqq - app) / (2.0 * apq);
                    double tt = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                    if (theta < 0.0) tt = -tt;
                    c = 1.0 / sqrt(tt * tt + 1.0);
                    s = tt * c;
                }
                rc[tid] = c; rs[tid] = s; rp[tid] = p; rq[tid] = q;
            }
            __syncthreads();
            // rows p, q <- J^T A
            for (int e = tid; e < 32 * 64; e += 256) {
                const int k = e / 64, j = e % 64;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double ap = A[p * 64 + j], aq = A[q * 64 + j];
                A[p * 64 + j] = c * ap - s * aq;
                A[q * 64 + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns p, q <- A J
            for (int e = tid; e < 32 * 64; e += 256) {
                const int k = e / 64, i = e % 64;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double ap = A[i * 64 + p], aq = A[i * 64 + q];
                A[i * 64 + p] = c * ap - s * aq;
                A[i * 64 + q] = s * ap + c * aq;
            }
            __syncthreads();
        }
        // convergence: off-diagonal mass relative to the diagonal
        if (tid < 64) {
            double off = 0.0, dg = 0.0;
            for (int j = 0; j < 64; ++j) {
                const double v = A[tid * 64 + j];
                if (j == tid) dg += v * v; else off += v * v;
            }
            S1[tid] = off;
            S1[64 + tid] = dg;  // S1 has room: it is followed by unused LDS (see layout)
        }
        __syncthreads();
        if (tid == 0) {
            double off = 0.0, dg = 0.0;
            for (int j = 0; j < 64; ++j) { off += S1[j]; dg += S1[64 + j]; }
            s_stop = off <= 1e-30 * dg;
        }
        __syncthreads();
        if (s_stop) break;
    }
    // ---- eigenvalues descending, tail rule ----
    if (tid == 0) {
        double ev[64];
        for (int i = 0; i < 64; ++i) ev[i] = A[i * 64 + i];
        for (int i = 1; i < 64; ++i) {          // insertion sort, descending
            const double v = ev[i];
            int j = i - 1;
            while (j >= 0 && ev[j] < v) { ev[j + 1] = ev[j]; --j; }
            ev[j + 1] = v;
        }
        double res = ev[63];
        for (int i = 0; i < 64; ++i) {
            double sum = 0.0;
            for (int j = i; j < 64; ++j) sum += ev[j];
            const double tau = sum / (double)(64 - i);
            int above = 0, below = 0;
            for (int j = i; j < 64; ++j) { above += ev[j] > tau; below += ev[j] < tau; }
            if (above == below) { res = tau; break; }
        }
        sigma2[t * g.c + ch] = res;
    }
}

__global__ void combine_sigma_kernel(const double *sigma2, int c, int n_tiles, double *sigma_est) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    double s = 0.0;
    for (int ch = 0; ch < c; ++ch) s += sigma2[t * c + ch];
    s /= (double)c;
    sigma_est[t] = s > 0.0 ? sqrt(s) : 0.0;
}

__global__ void fill_const_kernel(double *p, int n, double v) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// SplitMix64 output for the given state (after its increment), Steele, Lea & Flood 2014.
__device__ inline uint64_t splitmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// First and last reference index along one side whose position lies in [lo, hi].
__device__ inline void ref_range(int n_ref, int n, int s, int lo, int hi, int *first, int *last) {
    int f = -1, l = -2;
    for (int i = 0; i < n_ref; ++i) {
        const int p = ref_pos(i, n_ref, n, s);
        if (p >= lo && p <= hi) {
            if (f < 0) f = i;
            l = i;
        }
    }
    *first = f;
    *last = l;
}

// One wavefront per sub-image: up to n_vote sampled groups, rank of lambda_hat, majority.
template <int K>
__global__ __launch_bounds__(64) void vote_kernel(ImageGeom g, const int32_t *__restrict__ idx, int T, int n_vote,
                                                  uint64_t seed, int gamma_rank, double beta,
                                                  const double *__restrict__ sigma_est, double *__restrict__ sigma_hat,
                                                  int32_t *__restrict__ votes) {
    const int t = blockIdx.x, lane = threadIdx.x;
    const int ntx = (g.w + T - 1) / T;
    const int ty = t / ntx, tx = t % ntx;
    __shared__ int s_iy0, s_iy1, s_ix0, s_ix1;
    if (lane == 0) {
        ref_range(g.ny, g.h, g.s, ty * T, ty * T + T - 1, &s_iy0, &s_iy1);
        ref_range(g.nx, g.w, g.s, tx * T, tx * T + T - 1, &s_ix0, &s_ix1);
    }
    __syncthreads();
    const int nyr = s_iy1 - s_iy0 + 1, nxr = s_ix1 - s_ix0 + 1;
    const int64_t n_t = (s_iy0 < 0 || s_ix0 < 0) ? 0 : (int64_t)nyr * nxr;
    const double se = sigma_est[t];
    if (n_t == 0) {
        if (lane == 0) { sigma_hat[t] = se; if (votes) votes[t] = 0; }
        return;
    }
    const int nv = n_t <= n_vote ? (int)n_t : n_vote;
    const int P = 64 * g.c;
    int yes = 0;
    for (int i = 0; i < nv; ++i) {
        int64_t j;
        if (n_t <= n_vote) {
            j = i;
        } else {
            const uint64_t ctr = (uint64_t)t * (uint64_t)n_vote + (uint64_t)i + 1ull;
            j = (int64_t)(splitmix64(seed + ctr * 0x9E3779B97F4A7C15ull) % (uint64_t)n_t);
        }
        const int64_t r = (int64_t)(s_iy0 + j / nxr) * g.nx + (s_ix0 + j % nxr);
        // c_d for d = 0..K/2 (c_d = c_{K-d}), exact integers
        int64_t cd[K / 2 + 1];
#pragma unroll
        for (int d = 0; d <= K / 2; ++d) cd[d] = 0;
        for (int e = lane; e < P; e += 64) {
            const int ch = e / 64, a = (e / 8) % 8, b = e % 8;
            int v[K];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const int32_t lin = idx[r * K + m];
                const int y = lin / g.w, x = lin % g.w;
                v[m] = g.img[(int64_t)(y + a) * g.stride + (int64_t)(x + b) * g.c + ch];
            }
#pragma unroll
            for (int d = 0; d <= K / 2; ++d) {
                int s = 0;
#pragma unroll
                for (int m = 0; m < K; ++m) s += v[m] * v[(m + d) % K];
                cd[d] += s;
            }
        }
#pragma unroll
        for (int d = 0; d <= K / 2; ++d) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) cd[d] += __shfl_xor(cd[d], o);
        }
        if (lane == 0) {
            double lam[K / 2 + 1];
            for (int k = 0; k <= K / 2; ++k) {
                double acc = 0.0;
                for (int d = 0; d < K; ++d) {
                    const int dd = d <= K / 2 ? d : K - d;
                    acc += (double)cd[dd] * cos(2.0 * M_PI * (double)((k * d) % K) / (double)K);
                }
                lam[k] = acc;
            }
            const double lhat = lam[K / 2];
            const double tol = 1e-10 * (double)K * (double)cd[0];
            int a = 1;
            if (lam[0] < lhat - tol) a += 1;
            for (int k = 1; k < K / 2; ++k)
                if (lam[k] < lhat - tol) a += 2;
            if (a <= gamma_rank) ++yes;
        }
    }
    if (lane == 0) {
        sigma_hat[t] = 2 * yes > nv ? se / beta : se;
        if (votes) votes[t] = yes;
    }
}

}  // namespace

int cov_lds_bytes() {
    const int stage = 4 * COV_MAX_SIDE * COV_PITCH;
    const int red = (4 * 64 * 64 + 4 * 64) * 4 + (64 * 64 + 128) * 8;
    return stage > red ? stage : red;
}

hipError_t launch_sigma_est(const ImageGeom &g, int tile, double *work, double *sigma_est, hipStream_t st) {
    if (tile != 128) return hipErrorInvalidValue;
    const int n_tiles = ((g.h + tile - 1) / tile) * ((g.w + tile - 1) / tile);
    const int lds = cov_lds_bytes();
    hipError_t e0 = prepare_dynamic_lds((const void *)cov_eig_kernel, lds, 1024);
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(cov_eig_kernel, dim3(n_tiles * g.c), dim3(256), lds, st, g, tile, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(combine_sigma_kernel, dim3((n_tiles + 255) / 256), dim3(256), 0, st, work, g.c, n_tiles,
                       sigma_est);
    return hipGetLastError();
}

hipError_t launch_fill_const(double *p, int n, double v, hipStream_t st) {
    hipLaunchKernelGGL(fill_const_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_vote(const ImageGeom &g, const MethodParams &mp, const int32_t *idx, int tile, int n_vote,
                       uint64_t seed, int gamma_rank, double beta, const double *sigma_est, double *sigma_hat,
                       int32_t *votes, hipStream_t st) {
    const int n_tiles = ((g.h + tile - 1) / tile) * ((g.w + tile - 1) / tile);
#define HV_CASE(KK)                                                                                              \
    if (mp.K == KK) {                                                                                            \
        hipLaunchKernelGGL(vote_kernel<KK>, dim3(n_tiles), dim3(64), 0, st, g, idx, tile, n_vote, seed, gamma_rank, \
                           beta, sigma_est, sigma_hat, votes);                                                   \
        return hipGetLastError();                                                                                \
    }
    HV_CASE(4) HV_CASE(8) HV_CASE(16) HV_CASE(32)
#undef HV_CASE
    return hipErrorInvalidValue;
}

}  // namespace htsvd
