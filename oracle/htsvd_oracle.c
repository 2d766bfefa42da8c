/*
 * Haar-tSVD FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow reference that the GPU path is checked
 * against.  It shares no code with the HIP library (no headers, no helpers,
 * no tables) and may only be loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  The product never calls it.
 *
 * What it computes (paper: "Image Denoising Using Global and Local Circulant
 * Representation", Kong, Yang, Zhang):
 *   - Algorithm 1 (Haar-tSVD): for every reference patch, grouping by the
 *     green-channel-prior distance (Sec. III-A, Eq. 9), one-step filtering
 *     by the unified t-SVD + Haar transform (Sec. III-D, Eq. 19-21) and
 *     uniform ("average") aggregation.
 *   - The t-product through its literal block-circulant definition
 *     (Sec. II-C, Eq. 2-3): bcirc(A*B) = bcirc(A) bcirc(B), and
 *     bcirc(A^T) = bcirc(A)^T.
 *   - The Haar matrix by the recursion of Sec. II-D (Eq. 7-8), built as an
 *     explicit K x K matrix and applied as a dense matrix product.
 *   - Spatio-temporal grouping of a video (Sec. IV-C): the same distance
 *     over the reference's window in the frames within a temporal radius.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - reference grid: {0, s, 2s, ...} <= n-ps, plus n-ps when missing;
 *   - search window W is an odd side, centred on the reference, clipped at
 *     the image border; candidates move with stride 1 and include the
 *     reference itself;
 *   - Eq. 9 is evaluated with squared norms and gamma as a rational
 *     gnum/gden (6/5), so the branch test is exact in integers; the
 *     "average" channel is replaced by the channel sum (same order, same
 *     ties); distances are squared Euclidean (same order);
 *   - ties between equal distances go to the smaller (row, column); in a
 *     video to the smaller (frame, row, column), and a reference's window is
 *     clipped inside its frame and searched at the same place in the others;
 *   - hard threshold keeps |s| >= tau (Eq. 20), no coefficient is exempt;
 *   - aggregation weights are uniform; pixels no patch covers keep the
 *     noisy value; the output is FP64 and unclipped.
 *
 * Layouts: the image is uint8, row-major, channels interleaved:
 * img[y*stride + x*c + ch].  A patch or basis tensor of size ps x ps x c is
 * stored slice-major: T[(k*ps + i)*ps + j] = T(i, j, k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESHAPE (-2)
#define ORC_ENOMEM (-3)

/* ---- reference grid ---------------------------------------------------- */

/* Positions {0, s, 2s, ...} <= n-ps, plus n-ps if it is not already there. */
int orc_ref_grid(int n, int ps, int s, int *out)
{
    if (n < ps || s < 1) return 0;
    int cnt = 0;
    for (int v = 0; v <= n - ps; v += s) out[cnt++] = v;
    if (out[cnt - 1] != n - ps) out[cnt++] = n - ps;
    return cnt;
}

/* ---- Haar matrix, Sec. II-D, Eq. 7-8 ----------------------------------- */

/* H_1 = [1];  H_2N = 1/sqrt(2) [ H_N (x) [1, 1] ; I_N (x) [1, -1] ].
 * H is K x K, row-major.  K must be a power of two. */
int orc_haar(int K, double *H)
{
    if (K < 1 || (K & (K - 1))) return ORC_EINVAL;
    double *cur = (double *)malloc(sizeof(double) * K * K);
    double *nxt = (double *)malloc(sizeof(double) * K * K);
    if (!cur || !nxt) { free(cur); free(nxt); return ORC_ENOMEM; }
    cur[0] = 1.0;
    const double r = 1.0 / sqrt(2.0);
    for (int N = 1; N < K; N *= 2) {
        int M = 2 * N;
        memset(nxt, 0, sizeof(double) * M * M);
        /* top half: H_N kron [1, 1] */
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                nxt[i * M + 2 * j] = r * cur[i * N + j];
                nxt[i * M + 2 * j + 1] = r * cur[i * N + j];
            }
        /* bottom half: I_N kron [1, -1] */
        for (int i = 0; i < N; ++i) {
            nxt[(N + i) * M + 2 * i] = r;
            nxt[(N + i) * M + 2 * i + 1] = -r;
        }
        double *t = cur; cur = nxt; nxt = t;
    }
    memcpy(H, cur, sizeof(double) * K * K);
    free(cur);
    free(nxt);
    return ORC_OK;
}

/* ---- block circulant representation, Sec. II-C, Eq. 2 ------------------ */

/* bcirc(A) for A of size n x n x c: an (n c) x (n c) matrix whose block
 * (bi, bj) is the frontal slice A^((bi - bj) mod c). */
void orc_bcirc(const double *A, int n, int c, double *B)
{
    const int N = n * c;
    for (int bi = 0; bi < c; ++bi)
        for (int bj = 0; bj < c; ++bj) {
            const double *slice = A + (size_t)(((bi - bj) % c + c) % c) * n * n;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    B[(size_t)(bi * n + i) * N + bj * n + j] = slice[i * n + j];
        }
}

/* C (m x p) = A (m x k) * B (k x p), all row-major, plain triple loop. */
static void matmul(const double *A, const double *B, double *C, int m, int k, int p)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < p; ++j) {
            double acc = 0.0;
            for (int t = 0; t < k; ++t) acc += A[(size_t)i * k + t] * B[(size_t)t * p + j];
            C[(size_t)i * p + j] = acc;
        }
}

static void transpose(const double *A, double *At, int m, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) At[(size_t)j * m + i] = A[(size_t)i * n + j];
}

/* The frontal slices of a tensor X (ps x ps x c) are the first block column
 * of bcirc(X): X^(k) = block (k, 0). */
static void first_block_column_to_tensor(const double *Bcol /* N x ps */, int ps, int c, double *X)
{
    for (int k = 0; k < c; ++k)
        for (int i = 0; i < ps; ++i)
            for (int j = 0; j < ps; ++j) X[(k * ps + i) * ps + j] = Bcol[(size_t)(k * ps + i) * ps + j];
}

/* Precomputed block-circulant forms of a basis pair (U, V). */
typedef struct {
    int ps, c, N;
    double *bU;   /* bcirc(U),   N x N */
    double *bUt;  /* bcirc(U)^T, N x N */
    double *bV0;  /* first block column of bcirc(V),   N x ps */
    double *bVt0; /* first block column of bcirc(V)^T, N x ps */
} basis_t;

static int basis_init(basis_t *b, const double *U, const double *V, int ps, int c)
{
    const int N = ps * c;
    b->ps = ps; b->c = c; b->N = N;
    b->bU = (double *)malloc(sizeof(double) * N * N);
    b->bUt = (double *)malloc(sizeof(double) * N * N);
    b->bV0 = (double *)malloc(sizeof(double) * N * ps);
    b->bVt0 = (double *)malloc(sizeof(double) * N * ps);
    double *bV = (double *)malloc(sizeof(double) * N * N);
    double *bVt = (double *)malloc(sizeof(double) * N * N);
    if (!b->bU || !b->bUt || !b->bV0 || !b->bVt0 || !bV || !bVt) {
        free(bV); free(bVt);
        free(b->bU); free(b->bUt); free(b->bV0); free(b->bVt0);
        b->bU = b->bUt = b->bV0 = b->bVt0 = NULL;
        return ORC_ENOMEM;
    }
    orc_bcirc(U, ps, c, b->bU);
    transpose(b->bU, b->bUt, N, N);
    orc_bcirc(V, ps, c, bV);
    transpose(bV, bVt, N, N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < ps; ++j) {
            b->bV0[(size_t)i * ps + j] = bV[(size_t)i * N + j];
            b->bVt0[(size_t)i * ps + j] = bVt[(size_t)i * N + j];
        }
    free(bV);
    free(bVt);
    return ORC_OK;
}

static void basis_free(basis_t *b)
{
    free(b->bU); free(b->bUt); free(b->bV0); free(b->bVt0);
}

/* S = U^T * G * V  (Eq. 19 without the mode-4 Haar product):
 * bcirc(S) = bcirc(U)^T bcirc(G) bcirc(V); only its first block column is
 * needed.  work must hold N*N + 2*N*ps doubles. */
static void patch_forward(const basis_t *b, const double *G, double *S, double *work)
{
    const int N = b->N, ps = b->ps;
    double *bG = work, *T1 = work + (size_t)N * N, *T2 = T1 + (size_t)N * ps;
    orc_bcirc(G, ps, b->c, bG);
    matmul(bG, b->bV0, T1, N, N, ps);      /* first block column of bcirc(G)bcirc(V) */
    matmul(b->bUt, T1, T2, N, N, ps);      /* first block column of bcirc(U)^T(...)  */
    first_block_column_to_tensor(T2, ps, b->c, S);
}

/* G = U * S * V^T  (Eq. 21 without the Haar inverse). */
static void patch_inverse(const basis_t *b, const double *S, double *G, double *work)
{
    const int N = b->N, ps = b->ps;
    double *bS = work, *T1 = work + (size_t)N * N, *T2 = T1 + (size_t)N * ps;
    orc_bcirc(S, ps, b->c, bS);
    matmul(bS, b->bVt0, T1, N, N, ps);
    matmul(b->bU, T1, T2, N, N, ps);
    first_block_column_to_tensor(T2, ps, b->c, G);
}

/* Exported single-patch transforms (used by the tests). */
int orc_patch_forward(const double *U, const double *V, int ps, int c, const double *G, double *S)
{
    basis_t b;
    if (basis_init(&b, U, V, ps, c)) return ORC_ENOMEM;
    double *work = (double *)malloc(sizeof(double) * (b.N * b.N + 2 * b.N * ps));
    if (!work) { basis_free(&b); return ORC_ENOMEM; }
    patch_forward(&b, G, S, work);
    free(work);
    basis_free(&b);
    return ORC_OK;
}

int orc_patch_inverse(const double *U, const double *V, int ps, int c, const double *S, double *G)
{
    basis_t b;
    if (basis_init(&b, U, V, ps, c)) return ORC_ENOMEM;
    double *work = (double *)malloc(sizeof(double) * (b.N * b.N + 2 * b.N * ps));
    if (!work) { basis_free(&b); return ORC_ENOMEM; }
    patch_inverse(&b, S, G, work);
    free(work);
    basis_free(&b);
    return ORC_OK;
}

/* ---- grouping: Sec. III-A, Eq. 9; Algorithm 1 step "Grouping" ---------- */

typedef struct {
    int64_t d;
    int32_t y, x;
} cand_t;

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    return 0;
}

typedef struct {
    const uint8_t *img;
    int h, w, c;
    int64_t stride;
    int ps, W, K, gnum, gden;
} bm_ctx_t;

static inline int px(const bm_ctx_t *m, int y, int x, int ch)
{
    return m->img[(int64_t)y * m->stride + (int64_t)x * m->c + ch];
}

/* Which distance Eq. 9 uses for the reference at (y, x): 1 = green channel,
 * 0 = channel average (here the channel sum).  gamma^2 ||G||^2 >=
 * max(||R||^2, ||B||^2) with gamma = gnum/gden, in exact integers. */
int orc_gcp_green(const uint8_t *img, int64_t stride, int c, int ps, int y, int x, int gnum, int gden)
{
    if (c != 3) return 1;
    int64_t n[3] = {0, 0, 0};
    for (int i = 0; i < ps; ++i)
        for (int j = 0; j < ps; ++j)
            for (int ch = 0; ch < 3; ++ch) {
                int64_t v = img[(int64_t)(y + i) * stride + (int64_t)(x + j) * 3 + ch];
                n[ch] += v * v;
            }
    int64_t mx = n[0] > n[2] ? n[0] : n[2];
    return (int64_t)gnum * gnum * n[1] >= (int64_t)gden * gden * mx;
}

/* Squared distance between the patches at (yr, xr) and (yc, xc). */
static int64_t patch_dist(const bm_ctx_t *m, int green, int yr, int xr, int yc, int xc)
{
    int64_t d = 0;
    for (int i = 0; i < m->ps; ++i)
        for (int j = 0; j < m->ps; ++j) {
            int64_t a, b;
            if (m->c == 1) {
                a = px(m, yr + i, xr + j, 0);
                b = px(m, yc + i, xc + j, 0);
            } else if (green) {
                a = px(m, yr + i, xr + j, 1);
                b = px(m, yc + i, xc + j, 1);
            } else {
                a = px(m, yr + i, xr + j, 0) + px(m, yr + i, xr + j, 1) + px(m, yr + i, xr + j, 2);
                b = px(m, yc + i, xc + j, 0) + px(m, yc + i, xc + j, 1) + px(m, yc + i, xc + j, 2);
            }
            d += (a - b) * (a - b);
        }
    return d;
}

/* The K most similar patches to the reference at (y, x), in (d, y, x)
 * order.  cand must hold W*W entries.  Returns ORC_ESHAPE if the clipped
 * window holds fewer than K candidates. */
static int group_one(const bm_ctx_t *m, int y, int x, cand_t *cand, int32_t *oy, int32_t *ox, int64_t *od)
{
    const int R = (m->W - 1) / 2;
    const int green = orc_gcp_green(m->img, m->stride, m->c, m->ps, y, x, m->gnum, m->gden);
    const int ylo = y - R < 0 ? 0 : y - R, yhi = y + R > m->h - m->ps ? m->h - m->ps : y + R;
    const int xlo = x - R < 0 ? 0 : x - R, xhi = x + R > m->w - m->ps ? m->w - m->ps : x + R;
    int n = 0;
    for (int yc = ylo; yc <= yhi; ++yc)
        for (int xc = xlo; xc <= xhi; ++xc) {
            cand[n].d = patch_dist(m, green, y, x, yc, xc);
            cand[n].y = yc;
            cand[n].x = xc;
            ++n;
        }
    if (n < m->K) return ORC_ESHAPE;
    qsort(cand, n, sizeof(cand_t), cand_cmp);
    for (int k = 0; k < m->K; ++k) {
        oy[k] = cand[k].y;
        ox[k] = cand[k].x;
        if (od) od[k] = cand[k].d;
    }
    return ORC_OK;
}

static int check_common(int h, int w, int c, int64_t stride, int ps, int s, int W, int K)
{
    if (c != 1 && c != 3) return ORC_EINVAL;
    if (ps < 1 || s < 1 || W < 1 || (W & 1) == 0) return ORC_EINVAL;
    if (K < 1 || (K & (K - 1))) return ORC_EINVAL;
    if (h < ps || w < ps || stride < (int64_t)w * c) return ORC_ESHAPE;
    return ORC_OK;
}

/* Groups of every reference on the grid, reference r = iy*nx + ix.
 * idx[r*K + k] = y*w + x of the k-th member, dist[r*K + k] its distance. */
int orc_block_match(const uint8_t *img, int h, int w, int c, int64_t stride, int ps, int s, int W, int K,
                    int gnum, int gden, int32_t *idx, int64_t *dist, int nthreads)
{
    int err = check_common(h, w, c, stride, ps, s, W, K);
    if (err) return err;
    int *ys = (int *)malloc(sizeof(int) * (h / s + 2));
    int *xs = (int *)malloc(sizeof(int) * (w / s + 2));
    const int ny = orc_ref_grid(h, ps, s, ys), nx = orc_ref_grid(w, ps, s, xs);
    bm_ctx_t m = {img, h, w, c, stride, ps, W, K, gnum, gden};
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * W * W);
        int32_t *gy = (int32_t *)malloc(sizeof(int32_t) * K), *gx = (int32_t *)malloc(sizeof(int32_t) * K);
        int64_t *gd = (int64_t *)malloc(sizeof(int64_t) * K);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int r = 0; r < ny * nx; ++r) {
            int e = group_one(&m, ys[r / nx], xs[r % nx], cand, gy, gx, gd);
            if (e) {
                #pragma omp atomic write
                status = e;
                continue;
            }
            for (int k = 0; k < K; ++k) {
                idx[(int64_t)r * K + k] = gy[k] * w + gx[k];
                if (dist) dist[(int64_t)r * K + k] = gd[k];
            }
        }
        free(cand); free(gy); free(gx); free(gd);
    }
    free(ys);
    free(xs);
    return status;
}

/* Groups of the listed references only (raster indices into the reference grid); row i of
 * idx/dist belongs to refs[i].  Same grouping as orc_block_match. */
int orc_block_match_list(const uint8_t *img, int h, int w, int c, int64_t stride, int ps, int s, int W, int K,
                         int gnum, int gden, const int64_t *refs, int64_t n, int32_t *idx, int64_t *dist,
                         int nthreads)
{
    int err = check_common(h, w, c, stride, ps, s, W, K);
    if (err) return err;
    int *ys = (int *)malloc(sizeof(int) * (h / s + 2));
    int *xs = (int *)malloc(sizeof(int) * (w / s + 2));
    const int ny = orc_ref_grid(h, ps, s, ys), nx = orc_ref_grid(w, ps, s, xs);
    bm_ctx_t m = {img, h, w, c, stride, ps, W, K, gnum, gden};
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * W * W);
        int32_t *gy = (int32_t *)malloc(sizeof(int32_t) * K), *gx = (int32_t *)malloc(sizeof(int32_t) * K);
        int64_t *gd = (int64_t *)malloc(sizeof(int64_t) * K);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t i = 0; i < n; ++i) {
            const int64_t r = refs[i];
            if (r < 0 || r >= (int64_t)ny * nx) {
                #pragma omp atomic write
                status = ORC_EINVAL;
                continue;
            }
            int e = group_one(&m, ys[r / nx], xs[r % nx], cand, gy, gx, gd);
            if (e) {
                #pragma omp atomic write
                status = e;
                continue;
            }
            for (int k = 0; k < K; ++k) {
                idx[i * K + k] = gy[k] * w + gx[k];
                if (dist) dist[i * K + k] = gd[k];
            }
        }
        free(cand); free(gy); free(gx); free(gd);
    }
    free(ys);
    free(xs);
    return status;
}

/* ---- Haar-tSVD denoising, Algorithm 1 ---------------------------------- */

/* Denoises the image with per-reference thresholds tau_ref[r] (r = iy*nx+ix).
 * U, V: basis tensors (ps x ps x c, slice-major).  out: h*w*c FP64.
 * guard > 0 and n_near != NULL: counts coefficients with ||s| - tau| < guard.
 * Only references with r in [r_begin, r_end) are processed (r_end < 0 means
 * all); the output then averages only their contributions.
 * pest (n_ref x P, patch layout as the group, may be NULL) and ra_on (n_ref flags): refined
 * group means of RA-Haar-tSVD for the references whose flag is set. */
int orc_denoise(const uint8_t *img, int h, int w, int c, int64_t stride, int ps, int s, int W, int K,
                int gnum, int gden, const double *tau_ref, const double *U, const double *V, double *out,
                double guard, int64_t *n_near, int nthreads, int64_t r_begin, int64_t r_end,
                const double *pest, const uint8_t *ra_on)
{
    int err = check_common(h, w, c, stride, ps, s, W, K);
    if (err) return err;
    int *ys = (int *)malloc(sizeof(int) * (h / s + 2));
    int *xs = (int *)malloc(sizeof(int) * (w / s + 2));
    double *H = (double *)malloc(sizeof(double) * K * K);
    basis_t basis;
    if (!ys || !xs || !H || basis_init(&basis, U, V, ps, c)) {
        free(ys); free(xs); free(H);
        return ORC_ENOMEM;
    }
    const int ny = orc_ref_grid(h, ps, s, ys), nx = orc_ref_grid(w, ps, s, xs);
    const int64_t n_ref = (int64_t)ny * nx;
    if (r_end < 0 || r_end > n_ref) r_end = n_ref;
    if (r_begin < 0) r_begin = 0;
    const int R = (W - 1) / 2;
    const int P = ps * ps * c; /* values per patch */
    orc_haar(K, H);
    bm_ctx_t m = {img, h, w, c, stride, ps, W, K, gnum, gden};

    double *num = (double *)calloc((size_t)h * w * c, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)h * w, sizeof(int64_t));
    int status = ORC_OK;
    int64_t near_total = 0;
    int nt = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    nt = omp_get_max_threads();
#endif
    /* Each thread owns a contiguous run of references and accumulates into a
     * private band of rows; the bands are summed in thread order afterwards. */
    double **bnum = (double **)calloc(nt, sizeof(double *));
    int64_t **bcnt = (int64_t **)calloc(nt, sizeof(int64_t *));
    int *brow0 = (int *)calloc(nt, sizeof(int)), *brows = (int *)calloc(nt, sizeof(int));
#ifdef _OPENMP
#pragma omp parallel num_threads(nt) reduction(+ : near_total)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        const int64_t span = r_end - r_begin;
        const int64_t rb = r_begin + span * tid / nt, re = r_begin + span * (tid + 1) / nt;
        if (re > rb) {
            int y_first = ys[rb / nx], y_last = ys[(re - 1) / nx];
            int row0 = y_first - R < 0 ? 0 : y_first - R;
            int row1 = y_last + R + ps > h ? h : y_last + R + ps;
            brow0[tid] = row0;
            brows[tid] = row1 - row0;
            double *ln = (double *)calloc((size_t)(row1 - row0) * w * c, sizeof(double));
            int64_t *lc = (int64_t *)calloc((size_t)(row1 - row0) * w, sizeof(int64_t));
            bnum[tid] = ln;
            bcnt[tid] = lc;
            cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * W * W);
            int32_t *gy = (int32_t *)malloc(sizeof(int32_t) * K), *gx = (int32_t *)malloc(sizeof(int32_t) * K);
            double *G = (double *)malloc(sizeof(double) * K * P);   /* group, member-major */
            double *S = (double *)malloc(sizeof(double) * K * P);   /* patch coefficients */
            double *Sh = (double *)malloc(sizeof(double) * K * P);  /* after the Haar product */
            double *work = (double *)malloc(sizeof(double) * (basis.N * basis.N + 2 * basis.N * ps));
            for (int64_t r = rb; r < re; ++r) {
                const int y = ys[r / nx], x = xs[r % nx];
                int e = group_one(&m, y, x, cand, gy, gx, NULL);
                if (e) {
                    #pragma omp atomic write
                    status = e;
                    continue;
                }
                /* gather: G_m = P_{j_m} as FP64 integers 0..255 */
                for (int k = 0; k < K; ++k)
                    for (int ch = 0; ch < c; ++ch)
                        for (int i = 0; i < ps; ++i)
                            for (int j = 0; j < ps; ++j)
                                G[(size_t)k * P + (ch * ps + i) * ps + j] = px(&m, gy[k] + i, gx[k] + j, ch);
                /* Eq. 19: S = U^T * G * V  x_4  H_K */
                for (int k = 0; k < K; ++k) patch_forward(&basis, G + (size_t)k * P, S + (size_t)k * P, work);
                for (int a = 0; a < K; ++a)
                    for (int q = 0; q < P; ++q) {
                        double acc = 0.0;
                        for (int k = 0; k < K; ++k) acc += H[a * K + k] * S[(size_t)k * P + q];
                        Sh[(size_t)a * P + q] = acc;
                    }
                /* RA-Haar-tSVD (Eq. 24-25): the first Haar row is sqrt(K) times the transformed
                 * group mean; with a refined mean p_est it becomes sqrt(K) U^T * p_est * V and is
                 * kept as it is (no threshold); the other rows are thresholded as usual. */
                int64_t q_first = 0;
                if (pest && ra_on && ra_on[r]) {
                    patch_forward(&basis, pest + (size_t)r * P, S, work);
                    for (int q = 0; q < P; ++q) Sh[q] = sqrt((double)K) * S[q];
                    q_first = P;
                }
                /* Eq. 20: hard threshold */
                const double tau = tau_ref[r];
                for (int64_t q = q_first; q < (int64_t)K * P; ++q) {
                    double v = fabs(Sh[q]);
                    if (guard > 0 && fabs(v - tau) < guard) near_total += 1;
                    if (!(v >= tau)) Sh[q] = 0.0;
                }
                /* Eq. 21: G_est = U * S_trunc * V^T  x_4  H_K^{-1}  (H_K^{-1} = H_K^T) */
                for (int k = 0; k < K; ++k)
                    for (int q = 0; q < P; ++q) {
                        double acc = 0.0;
                        for (int a = 0; a < K; ++a) acc += H[a * K + k] * Sh[(size_t)a * P + q];
                        S[(size_t)k * P + q] = acc;
                    }
                for (int k = 0; k < K; ++k) patch_inverse(&basis, S + (size_t)k * P, G + (size_t)k * P, work);
                /* Algorithm 1, aggregation: uniform weights */
                for (int k = 0; k < K; ++k)
                    for (int i = 0; i < ps; ++i)
                        for (int j = 0; j < ps; ++j) {
                            const int yy = gy[k] + i - row0, xx = gx[k] + j;
                            for (int ch = 0; ch < c; ++ch)
                                ln[((size_t)yy * w + xx) * c + ch] += G[(size_t)k * P + (ch * ps + i) * ps + j];
                            lc[(size_t)yy * w + xx] += 1;
                        }
            }
            free(cand); free(gy); free(gx); free(G); free(S); free(Sh); free(work);
        }
    }
    for (int t = 0; t < nt; ++t) {
        if (!bnum[t]) continue;
        for (int64_t yy = 0; yy < brows[t]; ++yy)
            for (int64_t xx = 0; xx < w; ++xx) {
                const int64_t g = (yy + brow0[t]) * w + xx;
                cnt[g] += bcnt[t][yy * w + xx];
                for (int ch = 0; ch < c; ++ch) num[g * c + ch] += bnum[t][(yy * w + xx) * c + ch];
            }
        free(bnum[t]);
        free(bcnt[t]);
    }
    for (int64_t yy = 0; yy < h; ++yy)
        for (int64_t xx = 0; xx < w; ++xx) {
            const int64_t g = yy * w + xx;
            for (int ch = 0; ch < c; ++ch)
                out[g * c + ch] = cnt[g] > 0 ? num[g * c + ch] / (double)cnt[g]
                                             : (double)img[yy * stride + xx * c + ch];
        }
    if (n_near) *n_near = near_total;
    free(bnum); free(bcnt); free(brow0); free(brows);
    free(num); free(cnt); free(H); free(ys); free(xs);
    basis_free(&basis);
    return status;
}

/* Spatio-temporal grouping of a video (Sec. IV-C): T frames of h x w x c stacked vertically
 * (frame t occupies rows t*h .. t*h + h - 1 of the stacked image).  The reference at (y, x) of
 * frame t takes its candidates from the clipped window around (y, x) in every frame f with
 * |f - t| <= radius; the distance follows Eq. 9 as decided by the reference; the K nearest are
 * ordered by (distance, frame, row, column).  References: frame-major, then the grid of each
 * frame (Algorithm 1).  idx[r*K + k] = (f*h + y)*w + x in the stacked image, dist (may be NULL). */
int orc_block_match_video(const uint8_t *frames, int T, int h, int w, int c, int64_t stride, int ps, int s, int W,
                          int K, int radius, int gnum, int gden, int32_t *idx, int64_t *dist, int nthreads)
{
    int err = check_common(h, w, c, stride, ps, s, W, K);
    if (err) return err;
    if (T < 1 || radius < 0) return ORC_EINVAL;
    int *ys = (int *)malloc(sizeof(int) * (h / s + 2));
    int *xs = (int *)malloc(sizeof(int) * (w / s + 2));
    const int ny = orc_ref_grid(h, ps, s, ys), nx = orc_ref_grid(w, ps, s, xs);
    const int64_t per = (int64_t)ny * nx, n_ref = per * T;
    bm_ctx_t m = {frames, h * T, w, c, stride, ps, W, K, gnum, gden};
    const int R = (W - 1) / 2;
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * W * W * (2 * radius + 1));
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t r = 0; r < n_ref; ++r) {
            const int t = (int)(r / per);
            const int y = ys[(r % per) / nx], x = xs[(r % per) % nx];
            const int yr = t * h + y;
            const int green = orc_gcp_green(frames, stride, c, ps, yr, x, gnum, gden);
            const int ylo = y - R < 0 ? 0 : y - R, yhi = y + R > h - ps ? h - ps : y + R;
            const int xlo = x - R < 0 ? 0 : x - R, xhi = x + R > w - ps ? w - ps : x + R;
            int n = 0;
            for (int f = t - radius; f <= t + radius; ++f) {
                if (f < 0 || f >= T) continue;
                for (int yc = ylo; yc <= yhi; ++yc)
                    for (int xc = xlo; xc <= xhi; ++xc) {
                        cand[n].d = patch_dist(&m, green, yr, x, f * h + yc, xc);
                        cand[n].y = f * h + yc;   /* stacked rows order as (frame, row) */
                        cand[n].x = xc;
                        ++n;
                    }
            }
            if (n < K) {
                #pragma omp atomic write
                status = ORC_ESHAPE;
                continue;
            }
            qsort(cand, n, sizeof(cand_t), cand_cmp);
            for (int k = 0; k < K; ++k) {
                idx[r * K + k] = cand[k].y * w + cand[k].x;
                if (dist) dist[r * K + k] = cand[k].d;
            }
        }
        free(cand);
    }
    free(ys);
    free(xs);
    return status;
}

/* Collaborative filtering (Eq. 19-21) and uniform aggregation (Algorithm 1) of given groups,
 * for any channel count c (hyperspectral tube patches: c = bands, Sec. IV-D): group r has
 * the K members idx[r*K + k] = y*w + x.  The transform is the bcirc t-product above; the
 * threshold of group r is tau_ref[r].  out: h*w*c FP64 (pixels no patch covers keep their
 * input value). */
int orc_filter_groups(const uint8_t *img, int h, int w, int c, int64_t stride, int ps, int K, int64_t n_ref,
                      const int32_t *idx, const double *tau_ref, const double *U, const double *V, double *out,
                      int nthreads, const double *pest, const uint8_t *ra_on)
{
    if (c < 1 || ps < 1 || K < 1 || (K & (K - 1)) || h < ps || w < ps || stride < (int64_t)w * c) return ORC_EINVAL;
    for (int64_t q = 0; q < n_ref * K; ++q) {
        const int y = idx[q] / w, x = idx[q] % w;
        if (idx[q] < 0 || y > h - ps || x > w - ps) return ORC_EINVAL;
    }
    const int P = ps * ps * c;
    double *H = (double *)malloc(sizeof(double) * K * K);
    basis_t basis;
    if (!H || basis_init(&basis, U, V, ps, c)) {
        free(H);
        return ORC_ENOMEM;
    }
    orc_haar(K, H);
    double *num = (double *)calloc((size_t)h * w * c, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)h * w, sizeof(int64_t));
    int nt = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    nt = omp_get_max_threads();
#endif
    /* Each thread filters a contiguous run of groups into private sums, added in thread order. */
    double **tnum = (double **)calloc(nt, sizeof(double *));
    int64_t **tcnt = (int64_t **)calloc(nt, sizeof(int64_t *));
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        const int64_t rb = n_ref * tid / nt, re = n_ref * (tid + 1) / nt;
        double *ln = (double *)calloc((size_t)h * w * c, sizeof(double));
        int64_t *lc = (int64_t *)calloc((size_t)h * w, sizeof(int64_t));
        tnum[tid] = ln;
        tcnt[tid] = lc;
        double *G = (double *)malloc(sizeof(double) * K * P);
        double *S = (double *)malloc(sizeof(double) * K * P);
        double *Sh = (double *)malloc(sizeof(double) * K * P);
        double *work = (double *)malloc(sizeof(double) * (basis.N * basis.N + 2 * basis.N * ps));
        for (int64_t r = rb; r < re; ++r) {
            const int32_t *g = idx + r * K;
            for (int k = 0; k < K; ++k)
                for (int ch = 0; ch < c; ++ch)
                    for (int i = 0; i < ps; ++i)
                        for (int j = 0; j < ps; ++j)
                            G[(size_t)k * P + (ch * ps + i) * ps + j] =
                                img[(int64_t)(g[k] / w + i) * stride + (int64_t)(g[k] % w + j) * c + ch];
            for (int k = 0; k < K; ++k) patch_forward(&basis, G + (size_t)k * P, S + (size_t)k * P, work);
            for (int a = 0; a < K; ++a)
                for (int q = 0; q < P; ++q) {
                    double acc = 0.0;
                    for (int k = 0; k < K; ++k) acc += H[a * K + k] * S[(size_t)k * P + q];
                    Sh[(size_t)a * P + q] = acc;
                }
            /* RA-Haar-tSVD (Eq. 24-25), as in orc_denoise: a refined mean p_est gives the first
             * Haar row sqrt(K) U^T * p_est * V, kept without threshold. */
            int64_t q_first = 0;
            if (pest && ra_on && ra_on[r]) {
                patch_forward(&basis, pest + (size_t)r * P, S, work);
                for (int q = 0; q < P; ++q) Sh[q] = sqrt((double)K) * S[q];
                q_first = P;
            }
            for (int64_t q = q_first; q < (int64_t)K * P; ++q)
                if (!(fabs(Sh[q]) >= tau_ref[r])) Sh[q] = 0.0;
            for (int k = 0; k < K; ++k)
                for (int q = 0; q < P; ++q) {
                    double acc = 0.0;
                    for (int a = 0; a < K; ++a) acc += H[a * K + k] * Sh[(size_t)a * P + q];
                    S[(size_t)k * P + q] = acc;
                }
            for (int k = 0; k < K; ++k) patch_inverse(&basis, S + (size_t)k * P, G + (size_t)k * P, work);
            for (int k = 0; k < K; ++k)
                for (int i = 0; i < ps; ++i)
                    for (int j = 0; j < ps; ++j) {
                        const int64_t pix = (int64_t)(g[k] / w + i) * w + (g[k] % w + j);
                        for (int ch = 0; ch < c; ++ch) ln[pix * c + ch] += G[(size_t)k * P + (ch * ps + i) * ps + j];
                        lc[pix] += 1;
                    }
        }
        free(G); free(S); free(Sh); free(work);
    }
    for (int t = 0; t < nt; ++t) {
        for (int64_t q = 0; q < (int64_t)h * w; ++q) {
            cnt[q] += tcnt[t][q];
            for (int ch = 0; ch < c; ++ch) num[q * c + ch] += tnum[t][q * c + ch];
        }
        free(tnum[t]);
        free(tcnt[t]);
    }
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            const int64_t q = y * w + x;
            for (int ch = 0; ch < c; ++ch)
                out[q * c + ch] = cnt[q] > 0 ? num[q * c + ch] / (double)cnt[q] : (double)img[y * stride + x * c + ch];
        }
    free(tnum); free(tcnt); free(num); free(cnt); free(H);
    basis_free(&basis);
    return ORC_OK;
}

/* Number of reference positions along a side (for sizing outputs). */
int orc_ref_count(int n, int ps, int s)
{
    if (n < ps || s < 1) return 0;
    int c = (n - ps) / s + 1;
    if ((n - ps) % s) c += 1;
    return c;
}
