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
//     come from the same instruction with an all-ones operand.  int32 partials are exact and
//     go to a scratch buffer (mom_kernel).
//   - The eigenvalues of the 64x64 FP64 covariance take one wavefront per (sub-image,
//     channel) (eig_kernel): Householder reduction to tridiagonal form with lane i holding
//     row i in registers, then Sturm-count bisection with lane i finding the i-th smallest
//     eigenvalue.  Keeping this stage apart from the moments lets every SIMD run two such
//     wavefronts, whose serial dependency chains would otherwise leave the CU idle.
//
// Eq. 22-23 vote: for a few groups per sub-image the rank a of the alternating eigenvalue
// lambda_hat = |sum_m (-1)^m p_m|^2 among the K eigenvalues of circ(G) circ(G)^T, whose
// closed-form spectrum is lambda_k = sum_d c_d cos(2 pi k d / K) with the exact integer
// autocorrelations c_d = sum_m p_m . p_{(m+d) mod K}; a group votes "adjust" if a <= gamma
// and a majority sets sigma_hat = sigma_est / beta.
#include <math.h>

#include "common.h"
#include "sigma_dev.h"

namespace htsvd {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int COV_PITCH = 140;                 // bytes per staged row (>= 135 + 4, multiple of 4)

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

// 1/q: the hardware estimate refined by two Newton steps (each squares the relative error).
__device__ inline double recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    double e = fma(-q, r, 1.0);
    r = fma(r, e, r);
    e = fma(-q, r, 1.0);
    return fma(r, e, r);
}

// Sum over the 64 lanes of a wavefront (every lane gets the total; partners exchange by DPP
// and row swaps, offsets 32, 16, ..., 1).
__device__ __forceinline__ double wave_sum_d(double v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = xor_lane((uint32_t)b, o, lane), hi = xor_lane((uint32_t)(b >> 32), o, lane);
        v += __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    }
    return v;
}

// LDS layout of mom_kernel (bytes)
constexpr int COV_BAND = 16;                               // patch rows per staged band
constexpr int COV_STAGE_ROWS = COV_BAND + PS - 1;          // 23 pixel rows per band
constexpr int COV_PLANE = COV_STAGE_ROWS * COV_PITCH;      // one byte-shifted copy
constexpr int S2_PITCH = 65;                               // int32 row pitch of the second moments
constexpr int COV_OFF_S2 = 0;                              // int32 [64][65] second moments
constexpr int COV_OFF_S1 = COV_OFF_S2 + 64 * S2_PITCH * 4; // int32 [64] first moments
constexpr int COV_OFF_STAGE = COV_OFF_S1 + 64 * 4;         // 4 copies of the band
constexpr int COV_LDS = COV_OFF_STAGE + 4 * COV_PLANE;

// Moments of one (sub-image, channel) in global memory: the full symmetric 64 x 64 second
// moments (row-major), then the 64 first moments, int32 (exact).
constexpr int MOM_INTS = 64 * 64 + 64;

// Moments of one (sub-image, channel), one workgroup of 4 waves: exact integer second moments
// of the shifted patches on the matrix cores, the sub-image staged band by band; written to
// mom (MOM_INTS int32).
__device__ __forceinline__ void mom_tile(unsigned char *smem, const ImageGeom g, int T, int t, int ch,
                                int32_t *__restrict__ mom) {
    int32_t *S2 = reinterpret_cast<int32_t *>(smem + COV_OFF_S2);
    int32_t *S1 = reinterpret_cast<int32_t *>(smem + COV_OFF_S1);
    unsigned char *stage = smem + COV_OFF_STAGE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int y0, y1, x0, x1;
    tile_bounds(g, T, t, &y0, &y1, &x0, &x1);
    const int ny = y1 - y0 + 1, nx = x1 - x0 + 1;   // patch positions
    const int pcol = nx + PS - 1;
    for (int e = tid; e < 64 * S2_PITCH + 64; e += 256) S2[e] = 0;   // S1 follows S2

    // ---- phase 1: second moments on the matrix cores ----
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
    for (int b0 = 0; b0 < ny; b0 += COV_BAND) {
        const int nb = min(COV_BAND, ny - b0);
        const int prow = nb + PS - 1;
        __syncthreads();   // previous band consumed
        for (int e = tid; e < prow * pcol; e += 256) {
            const int r = e / pcol, col = e % pcol;
            const int v = (int)g.img[(int64_t)(y0 + b0 + r) * g.stride + (int64_t)(x0 + col) * g.c + ch] - 128;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (col >= k) stage[k * COV_PLANE + r * COV_PITCH + col - k] = (unsigned char)(int8_t)v;
        }
        __syncthreads();
        for (int stp = wave; stp < nb * xsteps; stp += 4) {
            const int py = stp / xsteps, pxs = (stp % xsteps) * 64;
            const int k0 = pxs + 16 * kq;                 // first patch column of this lane
            const int valid = min(16, max(0, nx - k0));
            v4i f[4];
#pragma unroll
            for (int blk = 0; blk < 4; ++blk) {
                const int e = 16 * blk + i16;             // patch-vector entry (a, b) = (e/8, e%8)
                f[blk] = frag16(stage, COV_PLANE, py + e / 8, k0 + e % 8, valid);
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
    }
    // wave partials -> LDS (integer adds: exact, order free; totals < 2^28)
    {
        int a = 0;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
#pragma unroll
            for (int jb = ib; jb < 4; ++jb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) atomicAdd(&S2[(16 * ib + 4 * kq + r) * S2_PITCH + 16 * jb + i16], acc[a][r]);
                ++a;
            }
            if (i16 == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) atomicAdd(&S1[16 * ib + 4 * kq + r], acc1[ib][r]);
            }
        }
    }
    __syncthreads();
    // only the blocks ib <= jb were accumulated: entry (r, c) of the full matrix is S2[min][max]
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        mom[e] = S2[min(r, c) * S2_PITCH + max(r, c)];
    }
    if (tid < 64) mom[64 * 64 + tid] = S1[tid];
}

// Householder steps k = 8B .. min(8B + 8, 62) - 1 on the rows held one per lane (lane i: row i).
// The reflector vector v is zero at indices <= k, so for a step of this block the products and
// updates of the columns below 8B are exact zeros for every entry read later (the tridiagonal
// entries of the reduced rows, and v, w, p): those columns are left out.
template <int B>
__device__ __forceinline__ void hh_block(double (&row)[64], int i) {
    constexpr int J0 = 8 * B;
    constexpr int KEND = J0 + 8 < 62 ? J0 + 8 : 62;
    for (int k = J0; k < KEND; ++k) {
        double xk = 0.0;
#pragma unroll
        for (int j = J0; j < J0 + 8; ++j) xk = (j == k) ? row[j] : xk;   // lane i: A[i][k]
        const double tail = wave_sum_d(i > k + 1 ? xk * xk : 0.0);
        const double x0 = readlane_f64(xk, k + 1);
        if (tail == 0.0) continue;                       // column already reduced (uniform)
        const double nrm = sqrt(x0 * x0 + tail);
        const double alpha = x0 > 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double beta = 2.0 / (v0 * v0 + tail);
        const double vi = i == k + 1 ? v0 : (i > k + 1 ? xk : 0.0);
        // v and w are broadcast lane by lane as scalar operands (no LDS round trip)
        double pi = 0.0;
#pragma unroll
        for (int j = J0 + 1; j < 64; ++j) pi += row[j] * readlane_f64(vi, j);
        pi *= beta;
        const double Kc = 0.5 * beta * wave_sum_d(pi * vi);
        const double wi = pi - Kc * vi;
#pragma unroll
        for (int j = J0; j < 64; ++j) row[j] -= vi * readlane_f64(wi, j) + wi * readlane_f64(vi, j);
    }
}

// Eigenvalue stage of one (sub-image, channel), one wavefront: covariance rows in registers
// (lane i holds row i), Householder reduction to tridiagonal form, eigenvalues by Sturm-count
// bisection (lane i finds the i-th smallest), tail rule.  vec: 3 x 64 doubles of LDS for this
// wave.  Writes sigma_c^2 to *out (lane 0).
__device__ __forceinline__ void eig_tile(double *vec, const int32_t *__restrict__ mom, double n, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    // ---- phase 2: covariance row i = lane, in registers ----
    const int i = lane;
    const int32_t *S1 = mom + 64 * 64;
    const double s1i = (double)S1[i] / n;
    double row[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) row[j] = (double)mom[i * 64 + j] / n - s1i * ((double)S1[j] / n);
    // Householder: step k annihilates column k below the subdiagonal; steps run in blocks of 8.
    hh_block<0>(row, i);
    hh_block<1>(row, i);
    hh_block<2>(row, i);
    hh_block<3>(row, i);
    hh_block<4>(row, i);
    hh_block<5>(row, i);
    hh_block<6>(row, i);
    hh_block<7>(row, i);
    // tridiagonal: d_i = A[i][i], e_{i-1} = A[i][i-1]
    double di = 0.0, sub = 0.0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        di = (j == i) ? row[j] : di;
        sub = (j == i - 1) ? row[j] : sub;
    }
    double *dd = vec, *e2 = vec + 64, *ev = vec + 128;
    __builtin_amdgcn_wave_barrier();
    dd[i] = di;
    e2[i] = i > 0 ? sub * sub : 0.0;    // e2[i] = e_{i-1}^2
    // Gershgorin interval
    const double se = fabs(sub) + fabs(__shfl(sub, (i + 1) & 63) * (i < 63 ? 1.0 : 0.0));
    double lo = di - se, hi = di + se;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
    }
    __builtin_amdgcn_wave_barrier();
    // The i-th smallest eigenvalue by quadrisection: count(x) = #eigenvalues < x (Sturm sequence
    // of the LDL^T pivots); three interior points per step, evaluated as three interleaved
    // chains, so 30 steps narrow the interval by 2^60 like 60 bisection steps.
    const double span = fmax(hi - lo, 1e-300);
    lo -= 1e-12 * span;
    hi += 1e-12 * span;
    for (int it = 0; it < 30; ++it) {
        const double qw = 0.25 * (hi - lo);
        const double x1 = lo + qw, x2 = lo + 2.0 * qw, x3 = lo + 3.0 * qw;
        double q1 = dd[0] - x1, q2 = dd[0] - x2, q3 = dd[0] - x3;
        int c1 = q1 < 0.0, c2 = q2 < 0.0, c3 = q3 < 0.0;
        for (int j = 1; j < 64; ++j) {
            const double dj = dd[j], ej = e2[j];
            q1 = (dj - x1) - ej * recip(q1 == 0.0 ? 1e-300 : q1);
            q2 = (dj - x2) - ej * recip(q2 == 0.0 ? 1e-300 : q2);
            q3 = (dj - x3) - ej * recip(q3 == 0.0 ? 1e-300 : q3);
            c1 += q1 < 0.0;
            c2 += q2 < 0.0;
            c3 += q3 < 0.0;
        }
        if (c1 > i) {
            hi = x1;
        } else if (c2 > i) {
            lo = x1;
            hi = x2;
        } else if (c3 > i) {
            lo = x2;
            hi = x3;
        } else {
            lo = x3;
        }
    }
    const double lam = 0.5 * (lo + hi);   // ascending: lane i holds the i-th smallest
    ev[i] = lam;
    __builtin_amdgcn_wave_barrier();
    // tail rule on the descending order: tail m = the 64 - m smallest values (lane m)
    const int m = lane, len = 64 - m;
    double sum = 0.0;
    for (int j = len - 1; j >= 0; --j) sum += ev[j];   // largest of the tail first
    const double tau = sum / (double)len;
    int above = 0, below = 0;
    for (int j = 0; j < len; ++j) {
        above += ev[j] > tau;
        below += ev[j] < tau;
    }
    const uint64_t hit = __ballot(above == below);
    // cross-lane read with every lane active; the smallest eigenvalue when no tail qualifies
    const double tau_first = __shfl(tau, hit ? __ffsll((unsigned long long)hit) - 1 : 0);
    if (lane == 0) *out = hit ? tau_first : ev[0];
}

// Number of patch positions of sub-image t.
__device__ inline double tile_patches(const ImageGeom &g, int T, int t) {
    int y0, y1, x0, x1;
    tile_bounds(g, T, t, &y0, &y1, &x0, &x1);
    return (double)(y1 - y0 + 1) * (double)(x1 - x0 + 1);
}

// One workgroup per (sub-image, channel): unit u = t * c + ch = unit0 + block.
__global__ __launch_bounds__(256) void mom_kernel(ImageGeom g, int T, int unit0, int32_t *__restrict__ mom) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int u = unit0 + (int)blockIdx.x;
    mom_tile(smem, g, T, u / g.c, u % g.c, mom + (int64_t)blockIdx.x * MOM_INTS);
}

// One wavefront per (sub-image, channel), EIG_WAVES per workgroup.
constexpr int EIG_WAVES = 4;

// Units unit0 .. unit0 + n_units - 1; mom and sigma2 indexed from unit0.
__global__ __launch_bounds__(64 * EIG_WAVES, 2) void eig_kernel(ImageGeom g, int T, int unit0, int n_units,
                                                             const int32_t *__restrict__ mom,
                                                             double *__restrict__ sigma2) {
    __shared__ double vec[EIG_WAVES][3 * 64];
    const int wave = threadIdx.x >> 6;
    const int u = blockIdx.x * EIG_WAVES + wave;
    if (u >= n_units) return;
    eig_tile(vec[wave], mom + (int64_t)u * MOM_INTS, tile_patches(g, T, (unit0 + u) / g.c), sigma2 + u);
}

// Batched: units (item, sub-image, channel) of the list; mom is indexed by the global unit.
__global__ __launch_bounds__(256) void mom_kernel_batched(const SigmaItem *__restrict__ items,
                                                          const int *__restrict__ sel, const int *__restrict__ start,
                                                          int n, int T, int32_t *__restrict__ mom) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int j = find_unit(start, n, blockIdx.x);
    const ImageGeom g = items[sel[j]].g;
    const int u = blockIdx.x - start[j];
    mom_tile(smem, g, T, u / g.c, u % g.c, mom + (int64_t)blockIdx.x * MOM_INTS);
}

__global__ __launch_bounds__(64 * EIG_WAVES, 2) void eig_kernel_batched(const SigmaItem *__restrict__ items,
                                                                     const int *__restrict__ sel,
                                                                     const int *__restrict__ start, int n, int total,
                                                                     int T, const int32_t *__restrict__ mom) {
    __shared__ double vec[EIG_WAVES][3 * 64];
    const int wave = threadIdx.x >> 6;
    const int gu = blockIdx.x * EIG_WAVES + wave;
    if (gu >= total) return;
    const int j = find_unit(start, n, gu);
    const SigmaItem &it = items[sel[j]];
    const ImageGeom g = it.g;
    const int u = gu - start[j];
    eig_tile(vec[wave], mom + (int64_t)gu * MOM_INTS, tile_patches(g, T, u / g.c), it.cov + u);
}

__global__ void combine_sigma_kernel(const double *sigma2, int c, int n_tiles, double *sigma_est) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    sigma_est[t] = combine_sigma_tile(sigma2, c, t);
}

// Batched per-sub-image stage: sigma_est from a known sigma, the plain estimate, or the learned
// map judged by the plain estimate; sigma_hat = sigma_est until the vote (if on) replaces it.
__global__ void sigma_tiles_batched_kernel(const SigmaItem *__restrict__ items, const int *__restrict__ sel,
                                           const int *__restrict__ start, int n, int total, int T,
                                           double bound) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= total) return;
    const int j = find_unit(start, n, u);
    const SigmaItem &it = items[sel[j]];
    const int t = u - start[j];
    double se;
    if (it.mode == SIGMA_KNOWN) {
        se = it.sigma;
    } else {
        const double sp = combine_sigma_tile(it.cov, it.g.c, t);
        if (it.mode == SIGMA_PLAIN) {
            se = sp;
        } else {
            it.sig_plain[t] = sp;
            se = judge_tile(it.g, T, t, it.zmap, sp, bound, it.use_plain + t);
        }
    }
    it.sig_est[t] = se;
    it.sig_hat[t] = se;   // the level before the vote (the vote, when on, replaces it)
    if (!it.adaptive) it.votes[t] = 0;
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

// First and last reference index along one side whose position lies in [lo, hi] (lo >= 0),
// or first > last.  Positions increase strictly: i s for i < n_ref - 1, then n - PS.
__device__ inline void ref_range(int n_ref, int n, int s, int lo, int hi, int *first, int *last) {
    const int reg = n_ref - 1;          // references on the regular grid: 0 .. reg - 1
    const int pl = n - PS;              // position of the last reference
    int f = (lo + s - 1) / s;           // smallest regular i with i s >= lo
    if (f >= reg) f = pl >= lo ? reg : n_ref;
    int l;
    if (pl <= hi) {
        l = reg;
    } else {
        l = min(hi / s, reg - 1);       // largest regular i with i s <= hi
    }
    if (f > l) {
        f = -1;
        l = -2;
    }
    *first = f;
    *last = l;
}

// One workgroup (4 wavefronts) per sub-image: the sampled groups are spread over the waves;
// per group the exact autocorrelations c_d, then lambda_k = sum_d c_d cos(2 pi k d / K) with
// lane k computing lambda_k (same summation order for every k), the rank of lambda_hat, and
// the majority over the groups.
template <int K>
struct VoteShared {
    int iy0, iy1, ix0, ix1, yes;
    double cos_tab[K];
};

template <int K>
__device__ __forceinline__ void vote_tile(VoteShared<K> &sh, const ImageGeom g, const int32_t *__restrict__ idx,
                                 int idx_stride, int T, int t, int n_vote, uint64_t seed, int gamma_rank, double beta,
                                 const double *__restrict__ sigma_est, double *__restrict__ sigma_hat,
                                 int32_t *__restrict__ votes) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntx = (g.w + T - 1) / T;
    const int ty = t / ntx, tx = t % ntx;
    int &s_iy0 = sh.iy0, &s_iy1 = sh.iy1, &s_ix0 = sh.ix0, &s_ix1 = sh.ix1, &s_yes = sh.yes;
    double *cos_tab = sh.cos_tab;
    if (tid == 0) {
        ref_range(g.ny, g.h, g.s, ty * T, ty * T + T - 1, &s_iy0, &s_iy1);
        ref_range(g.nx, g.w, g.s, tx * T, tx * T + T - 1, &s_ix0, &s_ix1);
        s_yes = 0;
    }
    if (tid < K) cos_tab[tid] = cos(2.0 * M_PI * (double)tid / (double)K);
    __syncthreads();
    const int nyr = s_iy1 - s_iy0 + 1, nxr = s_ix1 - s_ix0 + 1;
    const int64_t n_t = (s_iy0 < 0 || s_ix0 < 0) ? 0 : (int64_t)nyr * nxr;
    const double se = sigma_est[t];
    if (n_t == 0) {
        if (tid == 0) { sigma_hat[t] = se; if (votes) votes[t] = 0; }
        return;
    }
    const int nv = n_t <= n_vote ? (int)n_t : n_vote;
    const int P = 64 * g.c;
    int yes = 0;
    for (int i = wave; i < nv; i += 4) {
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
                const int32_t lin = idx[r * idx_stride + m];
                const int y = lin / g.w, x = lin % g.w;
                v[m] = g.img[(int64_t)(y + a) * g.stride + (int64_t)(x + b) * g.c + ch];
            }
#pragma unroll
            for (int d = 0; d <= K / 2; ++d) {
                int sacc = 0;
#pragma unroll
                for (int m = 0; m < K; ++m) sacc += v[m] * v[(m + d) % K];
                cd[d] += sacc;
            }
        }
#pragma unroll
        for (int d = 0; d <= K / 2; ++d) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) cd[d] += __shfl_xor(cd[d], o);
        }
        // lane k <= K/2: lambda_k
        const int k = lane <= K / 2 ? lane : 0;
        double lam = 0.0;
#pragma unroll
        for (int d = 0; d < K; ++d) {
            const int dd = d <= K / 2 ? d : K - d;
            lam += (double)cd[dd] * cos_tab[(k * d) % K];
        }
        const double lhat = __shfl(lam, K / 2);
        const double tol = 1e-10 * (double)K * (double)cd[0];
        const bool below = lam < lhat - tol;
        const uint64_t inner = __ballot(below && lane >= 1 && lane < K / 2);
        const uint64_t first = __ballot(below && lane == 0);
        const int a = 1 + (first ? 1 : 0) + 2 * __popcll(inner);
        if (lane == 0 && a <= gamma_rank) ++yes;
    }
    if (lane == 0 && yes) atomicAdd(&s_yes, yes);
    __syncthreads();
    if (tid == 0) {
        sigma_hat[t] = 2 * s_yes > nv ? se / beta : se;
        if (votes) votes[t] = s_yes;
    }
}

template <int K>
__global__ __launch_bounds__(256) void vote_kernel(ImageGeom g, const int32_t *__restrict__ idx, int T, int n_vote,
                                                   uint64_t seed, int gamma_rank, double beta,
                                                   const double *__restrict__ sigma_est, double *__restrict__ sigma_hat,
                                                   int32_t *__restrict__ votes) {
    __shared__ VoteShared<K> sh;
    vote_tile<K>(sh, g, idx, K, T, blockIdx.x, n_vote, seed, gamma_rank, beta, sigma_est, sigma_hat, votes);
}

template <int K>
__global__ __launch_bounds__(256) void vote_kernel_batched(const SigmaItem *__restrict__ items,
                                                           const int *__restrict__ sel,
                                                           const int *__restrict__ start, int n, int T, int n_vote,
                                                           uint64_t seed, int gamma_rank, double beta) {
    __shared__ VoteShared<K> sh;
    const int j = find_unit(start, n, blockIdx.x);
    const SigmaItem &it = items[sel[j]];
    // an image whose group size is chosen on the device is listed for both sizes; the launch of
    // the other size leaves it (the condition is uniform over the workgroup)
    if (it.ksel && *it.ksel != K) return;
    vote_tile<K>(sh, it.g, it.idx, it.K, T, blockIdx.x - start[j], n_vote, seed, gamma_rank, beta, it.sig_est,
                 it.sig_hat, it.votes);
}

}  // namespace

int cov_lds_bytes() { return COV_LDS; }
int sigma_mom_ints() { return MOM_INTS; }

hipError_t launch_sigma2_units(const ImageGeom &g, int tile, int unit0, int n_units, int32_t *mom, double *sigma2,
                               hipStream_t st) {
    if (tile != 128) return hipErrorInvalidValue;
    if (n_units <= 0) return hipSuccess;
    const int lds = cov_lds_bytes();
    hipError_t e = prepare_dynamic_lds((const void *)mom_kernel, lds, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mom_kernel, dim3(n_units), dim3(256), lds, st, g, tile, unit0, mom);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(eig_kernel, dim3((n_units + EIG_WAVES - 1) / EIG_WAVES), dim3(64 * EIG_WAVES), 0, st, g, tile,
                       unit0, n_units, (const int32_t *)mom, sigma2);
    return hipGetLastError();
}

hipError_t launch_sigma_est(const ImageGeom &g, int tile, int32_t *mom, double *work, double *sigma_est,
                            hipStream_t st) {
    if (tile != 128) return hipErrorInvalidValue;
    const int n_tiles = ((g.h + tile - 1) / tile) * ((g.w + tile - 1) / tile);
    hipError_t e = launch_sigma2_units(g, tile, 0, n_tiles * g.c, mom, work, st);
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
        hipLaunchKernelGGL(vote_kernel<KK>, dim3(n_tiles), dim3(256), 0, st, g, idx, tile, n_vote, seed, gamma_rank, \
                           beta, sigma_est, sigma_hat, votes);                                                   \
        return hipGetLastError();                                                                                \
    }
    HV_CASE(4) HV_CASE(8) HV_CASE(16) HV_CASE(32)
#undef HV_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sigma_est_batched(const SigmaItem *items, const int *sel, const int *start, int n, int total,
                                    int tile, int32_t *mom, hipStream_t st) {
    if (tile != 128) return hipErrorInvalidValue;
    if (n <= 0 || total <= 0) return hipSuccess;
    const int lds = cov_lds_bytes();
    hipError_t e = prepare_dynamic_lds((const void *)mom_kernel_batched, lds, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mom_kernel_batched, dim3(total), dim3(256), lds, st, items, sel, start, n, tile, mom);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(eig_kernel_batched, dim3((total + EIG_WAVES - 1) / EIG_WAVES), dim3(64 * EIG_WAVES), 0, st,
                       items, sel, start, n, total, tile, (const int32_t *)mom);
    return hipGetLastError();
}

hipError_t launch_sigma_tiles_batched(const SigmaItem *items, const int *sel, const int *start, int n, int total,
                                      int tile, double ratio_bound, hipStream_t st) {
    if (n <= 0 || total <= 0) return hipSuccess;
    hipLaunchKernelGGL(sigma_tiles_batched_kernel, dim3((total + 255) / 256), dim3(256), 0, st, items, sel, start, n,
                       total, tile, ratio_bound);
    return hipGetLastError();
}

hipError_t launch_vote_batched(int K, const SigmaItem *items, const int *sel, const int *start, int n, int total,
                               int tile, int n_vote, uint64_t seed, int gamma_rank, double beta, hipStream_t st) {
    if (n <= 0 || total <= 0) return hipSuccess;
#define HVB_CASE(KK)                                                                                             \
    if (K == KK) {                                                                                               \
        hipLaunchKernelGGL(vote_kernel_batched<KK>, dim3(total), dim3(256), 0, st, items, sel, start, n, tile,      \
                           n_vote, seed, gamma_rank, beta);                                                     \
        return hipGetLastError();                                                                                \
    }
    HVB_CASE(4) HVB_CASE(8) HVB_CASE(16) HVB_CASE(32)
#undef HVB_CASE
    return hipErrorInvalidValue;
}

}  // namespace htsvd
