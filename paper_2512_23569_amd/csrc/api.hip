// Host runtime behind the C ABI of include/htsvd.h: argument validation, the context's
// workspace and basis constants, and the stream-ordered launch sequence of one call.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/htsvd.h"
#include "common.h"
#include "hevd.h"

namespace htsvd {
hipError_t launch_filter(const ImageGeom &g, int W, int K, const BasisDev &b, const int32_t *idx,
                         const double *tau_ref, float *regions, unsigned long long *gc, float *out, int64_t out_stride,
                         hipStream_t st, bool gather, const float *ra_d = nullptr, const uint8_t *ra_flag = nullptr);
size_t filter_region_bytes(const ImageGeom &g, int W, int K);
hipError_t launch_fill_const(double *p, int n, double v, hipStream_t st);
int bm_lds_bytes(int s, int W, int h, int w);
}  // namespace htsvd

using namespace htsvd;

// Scratch of htsvd_denoise_noalloc: a fixed device array, one copy per GPU, held until the
// process ends.  Host code never uses the array's name as an address (on the host it names a
// stand-in, not device memory): htsvd_create looks up each device's address once, with that
// device current, and the entry point passes that address to the kernels.
static __device__ __align__(256) unsigned char scratch[HTSVD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
void *g_scratch_addr[SCRATCH_MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on `device` (looked up by htsvd_create), or nullptr.
void *scratch_ptr(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_addr[device];
}

// Records the address on the current device `device`; false if the lookup failed.
bool lookup_scratch(int device, hipError_t *err) {
    *err = hipSuccess;
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return false;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_addr[device]) return true;
    void *ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess || !ptr) return false;
    g_scratch_addr[device] = ptr;
    return true;
}
}  // namespace

// RA-Haar-tSVD refinement network: FP32 master weights with Adam state, and the fp16 hi/lo
// operand tables the inference kernel reads (plain, and with the last layer folded with the
// patch transform), rebuilt on the host when the weights or the basis change.
struct RaState {
    int n = 0;   // parameters (0: no network)
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *frag = nullptr, *frag3t = nullptr;
    float *bias = nullptr, *bias3t = nullptr;
    int64_t step = 0;
    uint64_t wgen = 1, frag_wgen = 0, fold_wgen = 0, fold_bgen = 0;
    float *train_ws = nullptr;
    size_t train_ws_floats = 0;
    double *partial = nullptr;
    int partial_cap = 0;
};

// Learned noise-level network state (device buffers) and its activation workspace.
struct CnnState {
    int c = 0, n = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *wq = nullptr, *grad = nullptr;
    uint16_t *wbf = nullptr;
    int64_t step = 0;
    void *ws = nullptr;
    size_t ws_size = 0;
    double *d_loss = nullptr;
};

// A planned (and possibly captured) batch: device-side descriptors and the graph replaying it.
struct BatchCache {
    uint64_t sig = 0;
    bool valid = false;
    void *dev = nullptr;           // items, unit tables, sigma/mult arrays, queues
    size_t dev_size = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // per image of the caller's array: group size as planned, whether it is chosen on the device,
    // its reference count, and its thresholds and device choice (workspace / descriptor block)
    std::vector<int> k_plan, auto_k;
    std::vector<int64_t> n_ref;
    std::vector<const double *> tau;
    std::vector<const int *> ksel;
    double mul_alt = 1.0;   // threshold factor of an auto image filtered with K = 16
};

struct htsvd_ctx {
    int device = 0;
    BasisDev basis[2] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};  // [0]: c=1, [1]: c=3
    bool has_basis[2] = {false, false};
    void *ws = nullptr;
    size_t ws_size = 0;
    unsigned long long *d_guard = nullptr;  // [0] re-decided in FP64, [1] past the per-group list
    int64_t *d_gram = nullptr;              // channel Gram sums of the basis learning pass
    size_t d_gram_n = 0;                    // its capacity (int64 values)
    std::vector<double> T64h[2];            // host copies of the FP64 patch transforms
    uint64_t basis_gen[2] = {0, 0};         // bumped by every basis install
    RaState ra[2];                          // RA-Haar-tSVD networks, [0]: c=1, [1]: c=3
    int bands = 0;                          // band count of the hyperspectral basis (0: none)
    double *d_band_maps = nullptr;          // its D, Dinv and slice maps (FP64)
    int64_t band_cap = (int64_t)4 << 30;    // bytes per patch matrix of one pass of the band filter
    // Optional per-stage timing with HIP events recorded on the call's stream.
    bool timing = false;
    hipEvent_t ev[2 * HTSVD_N_STAGES] = {};
    bool ev_pending[HTSVD_N_STAGES] = {};
    double stage_ms[HTSVD_N_STAGES] = {};
    int64_t stage_calls[HTSVD_N_STAGES] = {};
    CnnState cnn;
    BatchCache batch;
    hipStream_t cap_stream = nullptr;   // stream used only to capture batch graphs
};

namespace {

thread_local std::string g_err;

htsvd_status fail(htsvd_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

htsvd_status hip_fail(hipError_t e, const char *what) {
    return fail(HTSVD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Validates image geometry and method parameters; fills geometry and parameters.
htsvd_status validate(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c, int64_t in_stride,
                      const htsvd_params *p, ImageGeom *g, MethodParams *mp, bool need_basis) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (!d_in) return fail(HTSVD_EINVAL, "null input image");
    if (!p) return fail(HTSVD_EINVAL, "null params");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    if (p->ps != PS) return fail(HTSVD_ENOTSUP, "only ps = 8 is supported");
    if (p->window < 3 || p->window > MAX_WINDOW || (p->window & 1) == 0)
        return fail(HTSVD_EINVAL, "window must be odd and in [3, 31]");
    if (!(p->K == 4 || p->K == 8 || p->K == 16 || p->K == 32))
        return fail(HTSVD_ENOTSUP, "K must be 4, 8, 16 or 32");
    if (p->stride < 1) return fail(HTSVD_EINVAL, "stride must be >= 1");
    if ((REF_TILE - 1) * p->stride + p->window > MAX_UNION)
        return fail(HTSVD_ENOTSUP, "3*stride + window must not exceed 64");
    if (p->gcp_num < 1 || p->gcp_den < 1 || p->gcp_num > 1000 || p->gcp_den > 1000)
        return fail(HTSVD_EINVAL, "gcp_num/gcp_den must be in [1, 1000]");
    if (h < PS || w < PS) return fail(HTSVD_ESHAPE, "image smaller than one patch");
    if (in_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "in_stride < w*c");
    if ((int64_t)h * w > (int64_t)1 << 30) return fail(HTSVD_ENOTSUP, "image larger than 2^30 pixels");
    const int R = (p->window - 1) / 2;
    const int mh = (R < h - PS ? R : h - PS) + 1, mw = (R < w - PS ? R : w - PS) + 1;
    if (mh * mw < p->K) return fail(HTSVD_ESHAPE, "a clipped search window holds fewer than K candidates");
    if (need_basis && !ctx->has_basis[c == 3]) return fail(HTSVD_ESTATE, "no basis set for this channel count");
    if (p->subimage != 128) return fail(HTSVD_ENOTSUP, "subimage must be 128");
    if (p->ra != 0 && p->ra != 1) return fail(HTSVD_EINVAL, "ra must be 0 or 1");
    if (p->ra && !(p->ra_sigma >= 0.0)) return fail(HTSVD_EINVAL, "ra_sigma must be >= 0");

    if (p->adaptive) {
        if (p->n_vote < 1 || p->n_vote > 1024) return fail(HTSVD_EINVAL, "n_vote must be in [1, 1024]");
        if (!(p->beta > 0.0)) return fail(HTSVD_EINVAL, "beta must be > 0");
    }
    g->img = d_in;
    g->stride = in_stride;
    g->h = h;
    g->w = w;
    g->c = c;
    g->s = p->stride;
    g->ny = ref_count(h, p->stride);
    g->nx = ref_count(w, p->stride);
    mp->W = p->window;
    mp->K = p->K;
    mp->gnum = p->gcp_num;
    mp->gden = p->gcp_den;
    return HTSVD_OK;
}

// Grows the context workspace to at least `bytes` (synchronises the device before freeing).
htsvd_status ensure_ws(htsvd_ctx *ctx, size_t bytes) {
    if (ctx->ws_size >= bytes) return HTSVD_OK;
    hipError_t e;
    if (ctx->ws) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "synchronise before workspace growth");
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    ctx->batch.valid = false;   // a captured batch graph points into the old workspace
    ctx->batch.k_plan.clear();
    size_t sz = bytes + (bytes >> 3);
    e = hipMalloc(&ctx->ws, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HTSVD_ENOMEM, "workspace allocation failed");
    }
    ctx->ws_size = sz;
    return HTSVD_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// fp16 bits of x (through FP32), rounded to nearest even, with subnormals.
uint16_t host_f16(double x) {
    const float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    const uint32_t sgn = (u >> 16) & 0x8000u;
    const float af = std::fabs(f);
    if (af >= 65520.f) return (uint16_t)(sgn | 0x7c00u);
    if (af < 6.103515625e-05f) {   // subnormal: multiples of 2^-24
        const float q = std::nearbyint(af * 16777216.f);
        return (uint16_t)(sgn | (uint32_t)q);
    }
    uint32_t e = ((u >> 23) & 0xffu) - 127 + 15, m = u & 0x7fffffu;
    uint32_t hm = m >> 13, rem = m & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (hm & 1u))) {
        if (++hm == 0x400u) {
            hm = 0;
            ++e;
        }
    }
    return (uint16_t)(sgn | (e << 10) | hm);
}

double host_f16_value(uint16_t hbits) {
    const uint32_t e = (hbits >> 10) & 31u, m = hbits & 1023u;
    const double v = e == 0 ? std::ldexp((double)m, -24) : std::ldexp(1.0 + m / 1024.0, (int)e - 15);
    return (hbits & 0x8000u) ? -v : v;
}

// Largest ratio between the learned and the plain sigma of a sub-image at which the learned map
// is trusted there.
constexpr double JUDGE_RATIO = 1.5;

double default_mult(int c, int K) { return sqrt(2.0 * log((double)c * K * PS * PS)); }

// Workspace carve-up for one denoise call.
struct Ws {
    int32_t *idx;
    float *regions;
    double *tau;
    double *sig_est;
    double *sig_hat;
    int32_t *votes;
    double *cov;
    int32_t *use_plain;
    double *sig_plain;
    int32_t *mom;      // per (sub-image, channel) moments of the plain estimator
    size_t total;
};

Ws plan_ws(void *base, const ImageGeom &g, int W, int K, int tile) {
    Ws w;
    const int64_t n_ref = (int64_t)g.ny * g.nx;
    const int64_t n_tiles = (int64_t)((g.h + tile - 1) / tile) * ((g.w + tile - 1) / tile);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return (char *)base + o;
    };
    w.idx = (int32_t *)take(sizeof(int32_t) * n_ref * K);
    w.regions = (float *)take(filter_region_bytes(g, W, K));
    w.tau = (double *)take(sizeof(double) * n_ref);
    w.sig_est = (double *)take(sizeof(double) * n_tiles);
    w.sig_hat = (double *)take(sizeof(double) * n_tiles);
    w.votes = (int32_t *)take(sizeof(int32_t) * n_tiles);
    w.cov = (double *)take(sizeof(double) * n_tiles * g.c);  // per-channel tail variances
    w.use_plain = (int32_t *)take(sizeof(int32_t) * n_tiles);
    w.sig_plain = (double *)take(sizeof(double) * n_tiles);
    w.mom = (int32_t *)take(sizeof(int32_t) * sigma_mom_ints() * n_tiles * g.c);
    w.total = off;
    return w;
}

// Stage timing: an event pair per stage; the elapsed time of the previous pair is
// harvested (after it completed) when the stage is recorded again or on request.
void harvest(htsvd_ctx *ctx, int s) {
    if (!ctx->ev_pending[s]) return;
    float ms = 0.f;
    if (hipEventSynchronize(ctx->ev[2 * s + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, ctx->ev[2 * s], ctx->ev[2 * s + 1]) == hipSuccess) {
        ctx->stage_ms[s] += ms;
        ctx->stage_calls[s] += 1;
    }
    ctx->ev_pending[s] = false;
}

struct StageScope {
    htsvd_ctx *ctx;
    int s;
    hipStream_t st;
    StageScope(htsvd_ctx *c, int stage, hipStream_t stream) : ctx(c), s(stage), st(stream) {
        if (!ctx->timing) return;
        harvest(ctx, s);
        (void)hipEventRecord(ctx->ev[2 * s], st);
    }
    ~StageScope() {
        if (!ctx->timing) return;
        (void)hipEventRecord(ctx->ev[2 * s + 1], st);
        ctx->ev_pending[s] = true;
    }
};

// The denoising sequence after tau is known: grouping, filtering, aggregation, normalisation.
// ---- learned network helpers ----
struct CnnWs {
    uint16_t *act[6];
    float *z, *d0, *d1;
    size_t total;
};

CnnWs plan_cnn_ws(void *base, int N, int H, int W, int c, bool train) {
    CnnWs w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return (char *)base + o;
    };
    w.act[0] = nullptr;
    for (int l = 1; l <= 5; ++l) w.act[l] = (uint16_t *)take(sizeof(uint16_t) * cnn_act_elems(l, N, H, W, c));
    w.z = (float *)take(sizeof(float) * cnn_act_elems(6, N, H, W, c));
    const size_t dbig = train ? cnn_act_elems(1, N, H, W, c) : 0;
    w.d0 = (float *)take(sizeof(float) * dbig);
    w.d1 = (float *)take(sizeof(float) * dbig);
    w.total = off;
    return w;
}

htsvd_status ensure_cnn_ws(htsvd_ctx *ctx, size_t bytes) {
    CnnState &cs = ctx->cnn;
    if (cs.ws_size >= bytes) return HTSVD_OK;
    hipError_t e;
    ctx->batch.valid = false;
    ctx->batch.k_plan.clear();
    if (cs.ws) {
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise before workspace growth");
        (void)hipFree(cs.ws);
        cs.ws = nullptr;
        cs.ws_size = 0;
    }
    const size_t sz = bytes + (bytes >> 3);
    if (hipMalloc(&cs.ws, sz) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HTSVD_ENOMEM, "network workspace allocation failed");
    }
    cs.ws_size = sz;
    return HTSVD_OK;
}

CnnBuffers cnn_buffers(const CnnState &cs, const CnnWs &w) {
    CnnBuffers b;
    b.wq = cs.wq;
    b.wbf = cs.wbf;
    for (int l = 0; l < 6; ++l) b.act[l] = w.act[l];
    b.z = w.z;
    return b;
}

void cnn_free(CnnState &cs) {
    float *fs[5] = {cs.w, cs.m, cs.v, cs.wq, cs.grad};
    for (float *f : fs)
        if (f) (void)hipFree(f);
    if (cs.wbf) (void)hipFree(cs.wbf);
    if (cs.ws) (void)hipFree(cs.ws);
    if (cs.d_loss) (void)hipFree(cs.d_loss);
    cs = CnnState();
}

// Allocates the parameter buffers for c channels (keeps them when the size already matches).
htsvd_status cnn_alloc(htsvd_ctx *ctx, int c) {
    CnnState &cs = ctx->cnn;
    int wo[6], bo[6], n;
    cnn_layout(c, wo, bo, &n);
    if (cs.w && cs.c == c) return HTSVD_OK;
    if ((hipSetDevice(ctx->device)) != hipSuccess) return fail(HTSVD_EDEVICE, "hipSetDevice");
    (void)hipDeviceSynchronize();
    void *ws = cs.ws;
    size_t ws_size = cs.ws_size;
    cs.ws = nullptr;
    cnn_free(cs);
    cs.ws = ws;
    cs.ws_size = ws_size;
    cs.c = c;
    cs.n = n;
    float **fs[5] = {&cs.w, &cs.m, &cs.v, &cs.wq, &cs.grad};
    for (float **f : fs)
        if (hipMalloc(f, sizeof(float) * n) != hipSuccess) return fail(HTSVD_ENOMEM, "network allocation");
    if (hipMalloc(&cs.wbf, sizeof(uint16_t) * n) != hipSuccess) return fail(HTSVD_ENOMEM, "network allocation");
    if (hipMalloc(&cs.d_loss, sizeof(double)) != hipSuccess) return fail(HTSVD_ENOMEM, "network allocation");
    return HTSVD_OK;
}

// Uploads master weights, clears Adam state, refreshes the bf16 copies (synchronous).
htsvd_status cnn_upload(htsvd_ctx *ctx, const float *h, int n) {
    CnnState &cs = ctx->cnn;
    hipError_t e;
    if ((e = hipMemcpy(cs.w, h, sizeof(float) * n, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "upload");
    if ((e = hipMemset(cs.m, 0, sizeof(float) * n)) != hipSuccess) return hip_fail(e, "clear");
    if ((e = hipMemset(cs.v, 0, sizeof(float) * n)) != hipSuccess) return hip_fail(e, "clear");
    if ((e = cnn_quantize(cs.w, n, cs.wq, cs.wbf, nullptr)) != hipSuccess) return hip_fail(e, "quantise");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "upload");
    cs.step = 0;
    return HTSVD_OK;
}

// One draw of a standard normal from the counter-based SplitMix64 stream (Box-Muller).
double counter_normal(uint64_t seed, uint64_t i) {
    auto mix = [](uint64_t z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    const uint64_t a = mix(seed + (2 * i + 1) * 0x9E3779B97F4A7C15ull);
    const uint64_t b = mix(seed + (2 * i + 2) * 0x9E3779B97F4A7C15ull);
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

htsvd_status validate_crops(htsvd_ctx *ctx, const uint8_t *d, int32_t n, int32_t h, int32_t w, int32_t c) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (!d) return fail(HTSVD_EINVAL, "null input");
    if (!ctx->cnn.w) return fail(HTSVD_ESTATE, "network weights not set");
    if (c != ctx->cnn.c) return fail(HTSVD_EINVAL, "channel count differs from the network's");
    if (n < 1 || h < 1 || w < 1) return fail(HTSVD_ESHAPE, "empty batch");
    if ((int64_t)n * h * w > (int64_t)1 << 31) return fail(HTSVD_ENOTSUP, "batch too large");
    return HTSVD_OK;
}

// Learned log-sigma map of one image into the network workspace; returns its device pointer.
htsvd_status run_cnn_map(htsvd_ctx *ctx, const ImageGeom &g, hipStream_t st, const float **zmap) {
    CnnState &cs = ctx->cnn;
    if (!cs.w) return fail(HTSVD_ESTATE, "learned estimator requested but no network weights are set");
    if (cs.c != g.c) return fail(HTSVD_EINVAL, "network channel count differs from the image's");
    CnnWs w0 = plan_cnn_ws(nullptr, 1, g.h, g.w, g.c, false);
    htsvd_status s = ensure_cnn_ws(ctx, w0.total);
    if (s != HTSVD_OK) return s;
    CnnWs w = plan_cnn_ws(cs.ws, 1, g.h, g.w, g.c, false);
    StageScope sc(ctx, HTSVD_STAGE_SIGMA, st);
    hipError_t e = cnn_forward(cnn_buffers(cs, w), g.img, g.stride, 0, 1, g.h, g.w, g.c, st);
    if (e != hipSuccess) return hip_fail(e, "network forward");
    *zmap = w.z;
    return HTSVD_OK;
}

htsvd_status run_bm(htsvd_ctx *ctx, const ImageGeom &g, const MethodParams &mp, const Ws &w, hipStream_t st) {
    StageScope sc(ctx, HTSVD_STAGE_BM, st);
    hipError_t e = launch_block_match(g, mp, w.idx, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "block matching");
    return HTSVD_OK;
}

// Noise level per sub-image: sigma_est (known or plain estimator), then the Eq. 23 vote.
// Needs the groups (w.idx) when p->adaptive is set.  Leaves sigma_hat in w.sig_hat.
htsvd_status run_sigma(htsvd_ctx *ctx, const ImageGeom &g, const MethodParams &mp, const htsvd_params *p,
                       float sigma, const Ws &w, const float *zmap, hipStream_t st) {
    StageScope sc(ctx, HTSVD_STAGE_SIGMA, st);
    const int T = p->subimage;
    const int n_tiles = ((g.h + T - 1) / T) * ((g.w + T - 1) / T);
    hipError_t e;
    if (sigma > 0.f) {
        if ((e = launch_fill_const(w.sig_est, n_tiles, (double)sigma, st)) != hipSuccess) return hip_fail(e, "sigma");
    } else if (p->estimator == 1) {
        // learned map (already in zmap) judged per tile by the plain estimate
        if ((e = launch_sigma_est(g, T, w.mom, w.cov, w.sig_plain, st)) != hipSuccess) return hip_fail(e, "sigma estimation");
        if ((e = launch_learned_judge(g, T, zmap, w.sig_plain, JUDGE_RATIO, w.use_plain, w.sig_est, st)) != hipSuccess)
            return hip_fail(e, "sigma judge");
    } else {
        if ((e = launch_sigma_est(g, T, w.mom, w.cov, w.sig_est, st)) != hipSuccess) return hip_fail(e, "sigma estimation");
    }
    if (p->adaptive) {
        if ((e = launch_vote(g, mp, w.idx, T, p->n_vote, p->vote_seed, p->gamma_rank, p->beta, w.sig_est,
                             w.sig_hat, w.votes, st)) != hipSuccess)
            return hip_fail(e, "vote");
    } else {
        if ((e = hipMemcpyAsync(w.sig_hat, w.sig_est, sizeof(double) * n_tiles, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return hip_fail(e, "sigma copy");
        if ((e = launch_zero(w.votes, sizeof(int32_t) * n_tiles, st)) != hipSuccess) return hip_fail(e, "votes");
    }
    return HTSVD_OK;
}

htsvd_status run_filter(htsvd_ctx *ctx, const ImageGeom &g, const MethodParams &mp, const Ws &w,
                        const double *tau, float *d_out, int64_t out_stride, hipStream_t st,
                        const float *ra_d = nullptr, const uint8_t *ra_flag = nullptr) {
    hipError_t e;
    {
        StageScope sc(ctx, HTSVD_STAGE_CLEAR, st);
        if ((e = launch_zero(ctx->d_guard, 2 * sizeof(unsigned long long), st)) != hipSuccess)
            return hip_fail(e, "zero counters");
    }
    {
        StageScope sc(ctx, HTSVD_STAGE_FILTER, st);
        if ((e = launch_filter(g, mp.W, mp.K, ctx->basis[g.c == 3], w.idx, tau, w.regions, ctx->d_guard, d_out,
                               out_stride, st, false, ra_d, ra_flag)) != hipSuccess)
            return hip_fail(e, "filtering");
    }
    {
        StageScope sc(ctx, HTSVD_STAGE_NORMALIZE, st);
        if ((e = launch_filter(g, mp.W, mp.K, ctx->basis[g.c == 3], w.idx, tau, w.regions, ctx->d_guard, d_out,
                               out_stride, st, true)) != hipSuccess)
            return hip_fail(e, "aggregation");
    }
    return HTSVD_OK;
}

// Maps of the t-product along B channels (Eq. 4-5) for the FP64 filter of arbitrary groups: the
// channel DFT, its inverse and the per-frequency slice maps, after an orthogonality check of
// every slice.
htsvd_status build_band_maps(int B, const double *h_U, const double *h_V, std::vector<double> &maps) {
    typedef std::complex<double> cd;
    const int NF = B / 2 + 1;
    std::vector<cd> Uh((size_t)NF * 64), Vh((size_t)NF * 64);
    for (int f = 0; f < NF; ++f)
        for (int e = 0; e < 64; ++e) {
            cd u = 0, v = 0;
            for (int k = 0; k < B; ++k) {
                const cd tw = std::polar(1.0, -2.0 * M_PI * (double)((f * k) % B) / B);
                u += h_U[k * 64 + e] * tw;
                v += h_V[k * 64 + e] * tw;
            }
            Uh[(size_t)f * 64 + e] = u;
            Vh[(size_t)f * 64 + e] = v;
        }
    for (int f = 0; f < NF; ++f)
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
                cd su = 0, sv = 0;
                for (int a = 0; a < 8; ++a) {
                    su += std::conj(Uh[(size_t)f * 64 + a * 8 + i]) * Uh[(size_t)f * 64 + a * 8 + j];
                    sv += std::conj(Vh[(size_t)f * 64 + a * 8 + i]) * Vh[(size_t)f * 64 + a * 8 + j];
                }
                const double t = i == j ? 1.0 : 0.0;
                if (std::abs(su - t) > 1e-9 || std::abs(sv - t) > 1e-9)
                    return fail(HTSVD_EINVAL, "basis tensors are not orthogonal");
            }
    const int NB = band_nb(B);
    maps.assign((size_t)2 * NB * NB + (size_t)2 * NF * 512, 0.0);
    double *D = maps.data(), *Dinv = D + NB * NB, *frag = Dinv + NB * NB;
    for (int b = 0; b < B; ++b) {
        D[0 * NB + b] = 1.0;
        Dinv[b * NB + 0] = 1.0 / B;
        for (int f = 1; f < NF; ++f) {
            const double a = 2.0 * M_PI * (double)((f * b) % B) / B;
            if (2 * f == B) {   // the real slice of an even band count
                D[(B - 1) * NB + b] = std::cos(a);
                Dinv[b * NB + B - 1] = std::cos(a) / B;
            } else {
                D[(2 * f - 1) * NB + b] = std::cos(a);
                D[(2 * f) * NB + b] = -std::sin(a);
                Dinv[b * NB + 2 * f - 1] = 2.0 * std::cos(a) / B;
                Dinv[b * NB + 2 * f] = -2.0 * std::sin(a) / B;
            }
        }
    }
    // Slice products of frequency f: forward T = L P with L(a, b) = conj(U(b, a)), then Y = T R with
    // R = V; inverse L = U, R(a, b) = conj(V(b, a)).  Real embeddings: L as [[Lr, -Li], [Li, Lr]]
    // acting on [Pr; Pi], R as [[Rr, Ri], [-Ri, Rr]] acting on [Tr | Ti] from the right.  Operand
    // lanes of v_mfma_f64_16x16x4f64: A(m, k) in lane m + 16 (k mod 4), B(k, n) in lane n + 16 (k mod 4).
    for (int dir = 0; dir < 2; ++dir)
        for (int f = 0; f < NF; ++f) {
            const cd *U = Uh.data() + (size_t)f * 64, *V = Vh.data() + (size_t)f * 64;
            auto L = [&](int a, int b) { return dir == 0 ? std::conj(U[b * 8 + a]) : U[a * 8 + b]; };
            auto R = [&](int a, int b) { return dir == 0 ? V[a * 8 + b] : std::conj(V[b * 8 + a]); };
            double *fr = frag + ((size_t)dir * NF + f) * 512;
            for (int st = 0; st < 4; ++st)
                for (int lane = 0; lane < 64; ++lane) {
                    const int m = lane & 15, k = 4 * st + (lane >> 4);
                    // left factor: row m = (ri', a), column k = (ri, b)
                    const cd l = L(m & 7, k & 7);
                    const int rm = m >> 3, rk = k >> 3;
                    fr[st * 64 + lane] = rm == rk ? l.real() : (rm == 0 ? -l.imag() : l.imag());
                    // right factor: row k = (ri, a), column m = (ri', b)
                    const cd r = R(k & 7, m & 7);
                    fr[(4 + st) * 64 + lane] = rk == rm ? r.real() : (rk == 0 ? r.imag() : -r.imag());
                }
        }
    return HTSVD_OK;
}

// Uploads maps into *d (replacing what it held).  Synchronises the device first.
htsvd_status upload_maps(htsvd_ctx *ctx, const std::vector<double> &maps, double **d) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise before basis upload");
    if (*d) (void)hipFree(*d);
    *d = nullptr;
    if (hipMalloc(d, sizeof(double) * maps.size()) != hipSuccess) {
        *d = nullptr;
        (void)hipGetLastError();
        return fail(HTSVD_ENOMEM, "basis allocation");
    }
    if ((e = hipMemcpy(*d, maps.data(), sizeof(double) * maps.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "basis upload");
    return HTSVD_OK;
}

// Basis of the hyperspectral path (B bands).
htsvd_status set_basis_bands(htsvd_ctx *ctx, int B, const double *h_U, const double *h_V) {
    std::vector<double> maps;
    htsvd_status s = build_band_maps(B, h_U, h_V, maps);
    if (s != HTSVD_OK) return s;
    ctx->bands = 0;
    if ((s = upload_maps(ctx, maps, &ctx->d_band_maps)) != HTSVD_OK) return s;
    ctx->bands = B;
    return HTSVD_OK;
}

// Rebuilds the network's operand tables from the master weights when they changed (and the
// folded last layer when the weights or the basis changed).  Host work; synchronises the device.
htsvd_status ra_prepare(htsvd_ctx *ctx, int c, bool folded) {
    RaState &r = ctx->ra[c == 3];
    const int slot = c == 3;
    if (r.n == 0) return fail(HTSVD_ESTATE, "no RA network set for this channel count");
    const bool need_plain = r.frag_wgen != r.wgen;
    const bool need_fold = folded && (r.fold_wgen != r.wgen || r.fold_bgen != ctx->basis_gen[slot]);
    if (!need_plain && !need_fold) return HTSVD_OK;
    if (folded && !ctx->has_basis[slot]) return fail(HTSVD_ESTATE, "no basis set for this channel count");
    const int P = 64 * c, H = ra_hidden(c);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise before network upload");
    std::vector<float> w(r.n);
    if ((e = hipMemcpy(w.data(), r.w, sizeof(float) * r.n, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "network download");
    const float *W1 = w.data(), *b1 = W1 + H * P, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + P * H;
    // operand fragments of a NOUT x KIN row-major matrix: W(nt*32 + l%32, ks*16 + 8*(l/32) + e)
    auto build = [](const double *M, int NOUT, int KIN, uint16_t *dst) {
        const int KS = KIN / 16, NT = NOUT / 32;
        for (int nt = 0; nt < NT; ++nt)
            for (int ks = 0; ks < KS; ++ks)
                for (int l = 0; l < 64; ++l)
                    for (int el = 0; el < 8; ++el) {
                        const double v = M[(size_t)(nt * 32 + l % 32) * KIN + ks * 16 + 8 * (l / 32) + el];
                        const uint16_t hi = host_f16(v), lo = host_f16(v - host_f16_value(hi));
                        dst[((size_t)((nt * KS + ks) * 2 + 0) * 64 + l) * 8 + el] = hi;
                        dst[((size_t)((nt * KS + ks) * 2 + 1) * 64 + l) * 8 + el] = lo;
                    }
    };
    if (need_plain) {
        std::vector<uint16_t> fr(ra_frag_halves(c));
        const std::vector<double> d1(W1, W1 + H * P), d2(W2, W2 + H * H), d3(W3, W3 + P * H);
        build(d1.data(), H, P, fr.data());
        build(d2.data(), H, H, fr.data() + (size_t)2 * H * P);
        build(d3.data(), P, H, fr.data() + (size_t)2 * H * P + (size_t)2 * H * H);
        std::vector<float> bias(2 * H + P);
        std::copy(b1, b1 + H, bias.begin());
        std::copy(b2, b2 + H, bias.begin() + H);
        std::copy(b3, b3 + P, bias.begin() + 2 * H);
        if ((e = hipMemcpy(r.frag, fr.data(), sizeof(uint16_t) * fr.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(r.bias, bias.data(), sizeof(float) * bias.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "network upload");
        r.frag_wgen = r.wgen;
    }
    if (need_fold) {
        // 128 T W3 and 128 T b3: the network's change of the first Haar row, per coefficient
        const std::vector<double> &T = ctx->T64h[slot];
        std::vector<double> W3t((size_t)P * H, 0.0);
        std::vector<float> b3t(P);
        for (int q = 0; q < P; ++q) {
            double bq = 0.0;
            for (int pp = 0; pp < P; ++pp) {
                const double t = T[(size_t)q * P + pp];
                if (t == 0.0) continue;
                for (int u = 0; u < H; ++u) W3t[(size_t)q * H + u] += t * W3[(size_t)pp * H + u];
                bq += t * b3[pp];
            }
            b3t[q] = (float)(128.0 * bq);
        }
        for (double &x : W3t) x *= 128.0;
        std::vector<uint16_t> fr((size_t)2 * P * H);
        build(W3t.data(), P, H, fr.data());
        if ((e = hipMemcpy(r.frag3t, fr.data(), sizeof(uint16_t) * fr.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(r.bias3t, b3t.data(), sizeof(float) * P, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "network upload");
        r.fold_wgen = r.wgen;
        r.fold_bgen = ctx->basis_gen[slot];
    }
    return HTSVD_OK;
}

RaWeightsDev ra_dev(const RaState &r) {
    RaWeightsDev d;
    d.frag = r.frag;
    d.frag3t = r.frag3t;
    d.bias = r.bias;
    d.bias3t = r.bias3t;
    return d;
}

// Workspace of the RA step: the first-Haar-row corrections (n_ref x P floats), then the flags.
size_t ra_ws_bytes(const ImageGeom &g) {
    const int64_t n_ref = (int64_t)g.ny * g.nx;
    return align256(sizeof(float) * n_ref * 64 * g.c) + align256((size_t)n_ref);
}

// Mean patches of the groups and the network's corrections of their first Haar rows, with the
// flags of the groups it applies to (tau / mult > sigma_min).
htsvd_status run_ra(htsvd_ctx *ctx, const ImageGeom &g, const MethodParams &mp, const Ws &w, const double *tau,
                    void *base, double mult, double sigma_min, hipStream_t st, const float **d_out,
                    const uint8_t **f_out) {
    htsvd_status s = ra_prepare(ctx, g.c, true);
    if (s != HTSVD_OK) return s;
    const int64_t n_ref = (int64_t)g.ny * g.nx;
    float *D = (float *)base;
    uint8_t *F = (uint8_t *)base + align256(sizeof(float) * n_ref * 64 * g.c);
    hipError_t e = launch_ra_forward(g.c, ra_dev(ctx->ra[g.c == 3]), true, nullptr, g.img, g.stride, g.h, g.w, w.idx,
                                     mp.K, mp.K, n_ref, tau, mult, sigma_min, F, D, st);
    if (e != hipSuccess) return hip_fail(e, "refinement network");
    *d_out = D;
    *f_out = F;
    return HTSVD_OK;
}

htsvd_status ra_grad_impl(htsvd_ctx *ctx, int c, const float *d_noisy, const float *d_clean, int n, float *d_grad,
                          double *h_loss, hipStream_t st) {
    if (!ctx || !d_noisy || !d_clean || !d_grad) return fail(HTSVD_EINVAL, "null argument");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    if (n < 1 || n > (1 << 20)) return fail(HTSVD_EINVAL, "batch must hold 1 .. 2^20 pairs");
    RaState &r = ctx->ra[c == 3];
    if (r.n == 0) return fail(HTSVD_ESTATE, "no RA network set for this channel count");
    hipError_t e;
    const size_t need = ra_train_ws_floats(c, n);
    const int np = (int)(((int64_t)n * 64 * c + 255) / 256);
    if (r.train_ws_floats < need || r.partial_cap < np) {
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise before workspace growth");
        if (r.train_ws) (void)hipFree(r.train_ws);
        if (r.partial) (void)hipFree(r.partial);
        r.train_ws = nullptr;
        r.partial = nullptr;
        r.train_ws_floats = 0;
        r.partial_cap = 0;
        if (hipMalloc(&r.train_ws, sizeof(float) * need) != hipSuccess ||
            hipMalloc(&r.partial, sizeof(double) * np) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HTSVD_ENOMEM, "training workspace");
        }
        r.train_ws_floats = need;
        r.partial_cap = np;
    }
    int n_partial = 0;
    if ((e = ra_gradients(c, r.w, d_noisy, d_clean, n, d_grad, r.train_ws, r.partial, &n_partial, st)) != hipSuccess)
        return hip_fail(e, "network gradients");
    if (h_loss) {
        std::vector<double> part(n_partial);
        if ((e = hipMemcpyAsync(part.data(), r.partial, sizeof(double) * n_partial, hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "loss download");
        double sum = 0.0;
        for (double v : part) sum += v;
        *h_loss = sum / ((double)n * 64 * c);
    }
    return HTSVD_OK;
}

}  // namespace

extern "C" {

htsvd_status htsvd_create(htsvd_ctx **out, int device) {
    if (!out) return fail(HTSVD_EINVAL, "null output pointer");
    *out = nullptr;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipError_t se;
    if (!lookup_scratch(device, &se))
        return se != hipSuccess ? hip_fail(se, "scratch address") : fail(HTSVD_ENOTSUP, "device index too large");
    htsvd_ctx *ctx = new htsvd_ctx();
    ctx->device = device;
    e = hipMalloc(&ctx->d_guard, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(e, "counter allocation");
    }
    *out = ctx;
    return HTSVD_OK;
}

void htsvd_destroy(htsvd_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 2 * HTSVD_N_STAGES; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    for (int i = 0; i < 2; ++i) {
        if (ctx->basis[i].f32) (void)hipFree(ctx->basis[i].f32);
        if (ctx->basis[i].T64) (void)hipFree(ctx->basis[i].T64);
        if (ctx->basis[i].frag) (void)hipFree(const_cast<void *>(ctx->basis[i].frag));
    }
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->d_guard) (void)hipFree(ctx->d_guard);
    if (ctx->d_gram) (void)hipFree(ctx->d_gram);
    if (ctx->d_band_maps) (void)hipFree(ctx->d_band_maps);
    for (int i = 0; i < 2; ++i) {
        RaState &r = ctx->ra[i];
        for (void *q : {(void *)r.w, (void *)r.m, (void *)r.v, (void *)r.grad, (void *)r.frag, (void *)r.frag3t,
                        (void *)r.bias, (void *)r.bias3t, (void *)r.train_ws, (void *)r.partial})
            if (q) (void)hipFree(q);
    }
    cnn_free(ctx->cnn);
    if (ctx->batch.exec) (void)hipGraphExecDestroy(ctx->batch.exec);
    if (ctx->batch.graph) (void)hipGraphDestroy(ctx->batch.graph);
    if (ctx->batch.dev) (void)hipFree(ctx->batch.dev);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

htsvd_status htsvd_default_params(int32_t c, htsvd_params *out) {
    if (!out) return fail(HTSVD_EINVAL, "null output pointer");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    memset(out, 0, sizeof(*out));
    out->ps = PS;
    out->stride = 4;
    out->window = c == 3 ? 31 : 21;
    out->K = c == 3 ? 32 : 16;
    out->tau_mult = 0.0;
    out->adaptive = 0;
    out->beta = 1.2;
    out->gamma_rank = 13;
    out->gcp_num = 6;
    out->gcp_den = 5;
    out->estimator = 0;
    out->subimage = 128;
    out->n_vote = 15;
    out->vote_seed = 0;
    out->ra = 0;
    out->ra_sigma = 30.0;
    return HTSVD_OK;
}

int32_t htsvd_ref_count(int32_t n, int32_t ps, int32_t stride) {
    if (ps != PS) return 0;
    return ref_count(n, stride);
}

htsvd_status htsvd_set_basis(htsvd_ctx *ctx, int32_t ps, int32_t c, const double *h_U, const double *h_V) {
    typedef std::complex<double> cd;
    if (!ctx || !h_U || !h_V) return fail(HTSVD_EINVAL, "null argument");
    if (ps != PS) return fail(HTSVD_ENOTSUP, "only ps = 8 is supported");
    if (c == 2 || (c > 3 && c <= MAX_BANDS)) return set_basis_bands(ctx, c, h_U, h_V);
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3, or 2 .. 64 bands");
    // Fourier-domain slices (DFT along the channel mode, Eq. 5): X_hat^(f) = sum_k X^(k) w^(f k).
    const cd wv = std::polar(1.0, -2.0 * M_PI / c);
    cd twp[3], twm[3];   // w^m and w^-m
    for (int m = 0; m < c; ++m) {
        twp[m] = std::pow(wv, (double)m);
        twm[m] = std::pow(wv, -(double)m);
    }
    cd Uh[3][64], Vh[3][64];
    for (int f = 0; f < c; ++f)
        for (int e = 0; e < 64; ++e) {
            cd u = 0, v = 0;
            for (int k = 0; k < c; ++k) {
                const cd tw = twp[(f * k) % c];
                u += h_U[k * 64 + e] * tw;
                v += h_V[k * 64 + e] * tw;
            }
            Uh[f][e] = u;
            Vh[f][e] = v;
        }
    // Orthogonality: U_hat^(f)^H U_hat^(f) = I for every slice.
    for (int f = 0; f < c; ++f)
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
                cd su = 0, sv = 0;
                for (int a = 0; a < 8; ++a) {
                    su += std::conj(Uh[f][a * 8 + i]) * Uh[f][a * 8 + j];
                    sv += std::conj(Vh[f][a * 8 + i]) * Vh[f][a * 8 + j];
                }
                const double t = i == j ? 1.0 : 0.0;
                if (std::abs(su - t) > 1e-9 || std::abs(sv - t) > 1e-9)
                    return fail(HTSVD_EINVAL, "basis tensors are not orthogonal");
            }
    std::vector<float> f32(6 * 64, 0.f);
    for (int e = 0; e < 64; ++e) {
        f32[e] = (float)Uh[0][e].real();
        f32[64 + e] = (float)Vh[0][e].real();
        if (c == 3) {
            f32[128 + e] = (float)Uh[1][e].real();
            f32[192 + e] = (float)Uh[1][e].imag();
            f32[256 + e] = (float)Vh[1][e].real();
            f32[320 + e] = (float)Vh[1][e].imag();
        }
    }
    // FP64 matrix of the forward patch transform S = U^T * G * V on slice-major vectors,
    // built column by column from unit patches (Eq. 4: slice products in the Fourier domain).
    const int P = 64 * c;
    std::vector<double> T((size_t)P * P);
    for (int p = 0; p < P; ++p) {
        // The unit patch p has a single nonzero per Fourier slice, w^(f kin) at (a0, b0), so
        // S_hat^(f)(i, j) = conj(U_hat^(f)(a0, i)) w^(f kin) V_hat^(f)(b0, j).
        const int kin = p / 64, a0 = (p % 64) / 8, b0 = p % 8;
        cd Sh[3][64];
        for (int f = 0; f < c; ++f) {
            const cd g = twp[(f * kin) % c];
            for (int i = 0; i < 8; ++i)
                for (int j = 0; j < 8; ++j) Sh[f][i * 8 + j] = std::conj(Uh[f][a0 * 8 + i]) * g * Vh[f][b0 * 8 + j];
        }
        for (int k = 0; k < c; ++k)
            for (int e = 0; e < 64; ++e) {
                cd acc = 0;
                for (int f = 0; f < c; ++f) acc += Sh[f][e] * twm[(f * k) % c];
                T[(size_t)(k * 64 + e) * P + p] = acc.real() / c;
            }
    }
    // MFMA operand fragments of the block-diagonal per-slice maps (see the filter's header):
    //   forward F = L_S^-1 T L_x^-1, inverse Finv = L_S^-1 T^T L_x^-1, with L_x the per-position
    //   channel map (R,G,B) -> (R+G+B, 2R-G-B, B-G) and S = L_S (s0', re', im') the recombination
    //   S0 = s0' + 2re', S1 = s0' - re' - im', S2 = s0' - re' + im'  (c = 1: identities).
    std::vector<uint16_t> frag;
    {
        const int NP = c == 3 ? 40 : 8;
        std::vector<double> Lxi((size_t)P * P, 0.0), LSi((size_t)P * P, 0.0);
        if (c == 3) {
            // inverses of [[1,1,1],[2,-1,-1],[0,-1,1]] and [[1,2,0],[1,-1,-1],[1,-1,1]]
            const double lxi[3][3] = {{1.0 / 3, 1.0 / 3, 0.0}, {1.0 / 3, -1.0 / 6, -0.5}, {1.0 / 3, -1.0 / 6, 0.5}};
            const double lsi[3][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {1.0 / 3, -1.0 / 6, -1.0 / 6}, {0.0, -0.5, 0.5}};
            for (int e2 = 0; e2 < 64; ++e2)
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        Lxi[(size_t)(a * 64 + e2) * P + b * 64 + e2] = lxi[a][b];
                        LSi[(size_t)(a * 64 + e2) * P + b * 64 + e2] = lsi[a][b];
                    }
        } else {
            for (int e2 = 0; e2 < 64; ++e2) Lxi[(size_t)e2 * P + e2] = LSi[(size_t)e2 * P + e2] = 1.0;
        }
        // A B (or A B^T) over the nonzeros of both factors (the channel maps are sparse).
        auto mul = [&](const std::vector<double> &A, const std::vector<double> &B, bool bt) {
            std::vector<std::vector<std::pair<int, double>>> nz(P);
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j) {
                    const double b = bt ? B[(size_t)j * P + k] : B[(size_t)k * P + j];
                    if (b != 0.0) nz[k].emplace_back(j, b);
                }
            std::vector<double> Cm((size_t)P * P, 0.0);
            for (int i = 0; i < P; ++i)
                for (int k = 0; k < P; ++k) {
                    const double a = A[(size_t)i * P + k];
                    if (a == 0.0) continue;
                    for (const auto &jb : nz[k]) Cm[(size_t)i * P + jb.first] += a * jb.second;
                }
            return Cm;
        };
        const std::vector<double> Ff = mul(mul(LSi, T, false), Lxi, false);
        const std::vector<double> Fi = mul(mul(LSi, T, true), Lxi, false);
        for (int n = 0; n < P; ++n)
            for (int k = 0; k < P; ++k)
                if ((n < 64) != (k < 64) && (std::fabs(Ff[(size_t)n * P + k]) > 1e-12 || std::fabs(Fi[(size_t)n * P + k]) > 1e-12))
                    return fail(HTSVD_EINVAL, "per-slice transform is not block diagonal");
        auto f16 = host_f16;
        auto f16v = host_f16_value;
        frag.assign((size_t)2 * 2 * NP * 64 * 8, 0);
        for (int dir = 0; dir < 2; ++dir) {
            const std::vector<double> &M = dir == 0 ? Ff : Fi;
            int pr = 0;
            for (int t = 0; t < 2 * c; ++t)
                for (int st = 0; st < 4 * c; ++st) {
                    const bool blk0 = t < 2, kin0 = st < 4;
                    if (blk0 != kin0) continue;   // zero blocks are skipped
                    for (int l = 0; l < 64; ++l)
                        for (int jj = 0; jj < 8; ++jj) {
                            const int k = 16 * st + 8 * (l / 32) + jj, n = 32 * t + (l % 32);
                            const double v = M[(size_t)n * P + k];
                            const uint16_t hi = f16(v), lo = f16(v - f16v(hi));
                            frag[((size_t)((dir * 2 + 0) * NP + pr) * 64 + l) * 8 + jj] = hi;
                            frag[((size_t)((dir * 2 + 1) * NP + pr) * 64 + l) * 8 + jj] = lo;
                        }
                    ++pr;
                }
            if (pr != NP) return fail(HTSVD_EINVAL, "internal: fragment table size");
        }
    }
    const int slot = c == 3;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (!ctx->basis[slot].f32) {
        if ((e = hipMalloc(&ctx->basis[slot].f32, sizeof(float) * 6 * 64)) != hipSuccess)
            return fail(HTSVD_ENOMEM, "basis allocation");
        if ((e = hipMalloc(&ctx->basis[slot].T64, sizeof(double) * 192 * 192)) != hipSuccess)
            return fail(HTSVD_ENOMEM, "basis allocation");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise before basis upload");
    if ((e = hipMemcpy(ctx->basis[slot].f32, f32.data(), sizeof(float) * 6 * 64, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "basis upload");
    if ((e = hipMemcpy(ctx->basis[slot].T64, T.data(), sizeof(double) * P * P, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "basis upload");
    if (!ctx->basis[slot].frag) {
        void *fp = nullptr;
        if ((e = hipMalloc(&fp, sizeof(uint16_t) * 2 * 2 * 40 * 64 * 8)) != hipSuccess)
            return fail(HTSVD_ENOMEM, "basis allocation");
        ctx->basis[slot].frag = fp;
    }
    if ((e = hipMemcpy(const_cast<void *>(ctx->basis[slot].frag), frag.data(), sizeof(uint16_t) * frag.size(),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "basis upload");
    ctx->has_basis[slot] = true;
    ctx->T64h[slot] = T;
    ++ctx->basis_gen[slot];
    return HTSVD_OK;
}

namespace {

htsvd_status check_gram_args(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                             int64_t in_stride, int32_t ps, int32_t stride) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (!d_in) return fail(HTSVD_EINVAL, "null input image");
    if (c < 1 || c > MAX_BANDS) return fail(HTSVD_EINVAL, "c must be 1 .. 64");
    if (ps != PS) return fail(HTSVD_ENOTSUP, "only ps = 8 is supported");
    if (stride < 1) return fail(HTSVD_EINVAL, "stride must be >= 1");
    if (h < PS || w < PS) return fail(HTSVD_ESHAPE, "image smaller than one patch");
    if (in_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "in_stride < w*c");
    if ((int64_t)h * w > (int64_t)1 << 30) return fail(HTSVD_ENOTSUP, "image larger than 2^30 pixels");
    return HTSVD_OK;
}

}  // namespace

htsvd_status htsvd_basis_gram(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                              int64_t in_stride, int32_t ps, int32_t stride, int64_t *d_gram, void *stream) {
    htsvd_status s = check_gram_args(ctx, d_in, h, w, c, in_stride, ps, stride);
    if (s != HTSVD_OK) return s;
    if (!d_gram) return fail(HTSVD_EINVAL, "null output");
    hipError_t e = launch_gram(d_in, in_stride, h, w, c, stride, d_gram, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "Gram sums");
    return HTSVD_OK;
}

htsvd_status htsvd_learn_basis(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, int32_t ps, int32_t stride, double *h_U, double *h_V,
                               void *stream) {
    htsvd_status s = check_gram_args(ctx, d_in, h, w, c, in_stride, ps, stride);
    if (s != HTSVD_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t gram_n = (size_t)2 * c * c * 64;
    if (ctx->d_gram_n < gram_n) {
        if (ctx->d_gram) {
            (void)hipDeviceSynchronize();
            (void)hipFree(ctx->d_gram);
        }
        ctx->d_gram = nullptr;
        ctx->d_gram_n = 0;
        if ((e = hipMalloc(&ctx->d_gram, sizeof(int64_t) * std::max<size_t>(gram_n, 2 * 9 * 64))) != hipSuccess) {
            ctx->d_gram = nullptr;
            (void)hipGetLastError();
            return fail(HTSVD_ENOMEM, "Gram buffer allocation");
        }
        ctx->d_gram_n = std::max<size_t>(gram_n, 2 * 9 * 64);
    }
    hipStream_t st = (hipStream_t)stream;
    if ((e = launch_gram(d_in, in_stride, h, w, c, stride, ctx->d_gram, st)) != hipSuccess)
        return hip_fail(e, "Gram sums");
    std::vector<int64_t> gram((size_t)2 * c * c * 64);
    if ((e = hipMemcpyAsync(gram.data(), ctx->d_gram, sizeof(int64_t) * gram.size(), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return hip_fail(e, "Gram download");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "Gram download");
    std::vector<double> U((size_t)64 * c), V((size_t)64 * c);
    basis_from_gram(c, gram.data(), U.data(), V.data(), nullptr, nullptr);
    if ((s = htsvd_set_basis(ctx, ps, c, U.data(), V.data())) != HTSVD_OK) return s;
    if (h_U) memcpy(h_U, U.data(), sizeof(double) * U.size());
    if (h_V) memcpy(h_V, V.data(), sizeof(double) * V.size());
    return HTSVD_OK;
}

htsvd_status htsvd_block_match(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, const htsvd_params *p, int32_t *d_idx, int32_t *d_dist,
                               void *stream) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate(ctx, d_in, h, w, c, in_stride, p, &g, &mp, false);
    if (s != HTSVD_OK) return s;
    if (!d_idx) return fail(HTSVD_EINVAL, "null index output");
    hipError_t e = launch_block_match(g, mp, d_idx, d_dist, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "block matching");
    return HTSVD_OK;
}

htsvd_status htsvd_denoise_tau(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, const double *d_tau_ref, const htsvd_params *p, float *d_out,
                               int64_t out_stride, void *stream) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate(ctx, d_in, h, w, c, in_stride, p, &g, &mp, true);
    if (s != HTSVD_OK) return s;
    if (!d_tau_ref || !d_out) return fail(HTSVD_EINVAL, "null tau or output");
    if (out_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "out_stride < w*c");
    const int tile = p->subimage > 0 ? p->subimage : 128;
    Ws w0 = plan_ws(nullptr, g, mp.W, mp.K, tile);
    const size_t off_ra = align256(w0.total);
    if ((s = ensure_ws(ctx, off_ra + (p->ra ? ra_ws_bytes(g) : 0))) != HTSVD_OK) return s;
    Ws wk = plan_ws(ctx->ws, g, mp.W, mp.K, tile);
    hipStream_t st = (hipStream_t)stream;
    if ((s = run_bm(ctx, g, mp, wk, st)) != HTSVD_OK) return s;
    const float *ra_d = nullptr;
    const uint8_t *ra_f = nullptr;
    if (p->ra) {
        const double mult = p->tau_mult > 0.0 ? p->tau_mult : default_mult(c, mp.K);
        if ((s = run_ra(ctx, g, mp, wk, d_tau_ref, (char *)ctx->ws + off_ra, mult, p->ra_sigma, st, &ra_d, &ra_f)) !=
            HTSVD_OK)
            return s;
    }
    return run_filter(ctx, g, mp, wk, d_tau_ref, d_out, out_stride, st, ra_d, ra_f);
}

}  // extern "C"

namespace {

// htsvd_denoise on the context's workspace (fixed_ws == nullptr, grown on demand), or on a
// caller-fixed block of fixed_cap bytes that is never grown (the no-allocation entry point:
// plain or known sigma, no RA, so that no other buffer is needed).
htsvd_status denoise_impl(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c, int64_t in_stride,
                          float sigma, const htsvd_params *p, float *d_out, int64_t out_stride, void *stream,
                          void *fixed_ws, size_t fixed_cap) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate(ctx, d_in, h, w, c, in_stride, p, &g, &mp, true);
    if (s != HTSVD_OK) return s;
    if (!d_out) return fail(HTSVD_EINVAL, "null output");
    if (out_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "out_stride < w*c");
    if (!(sigma > 0.f) && sigma != HTSVD_SIGMA_AUTO) return fail(HTSVD_EINVAL, "sigma must be > 0 or AUTO");
    if (p->estimator != 0 && p->estimator != 1) return fail(HTSVD_EINVAL, "estimator must be 0 or 1");
    const bool learned = sigma == HTSVD_SIGMA_AUTO && p->estimator == 1;
    const int tile = p->subimage;
    Ws w0 = plan_ws(nullptr, g, mp.W, mp.K, tile);
    const size_t off_ra = align256(w0.total);
    void *base = fixed_ws;
    if (fixed_ws) {
        if (learned) return fail(HTSVD_ENOTSUP, "the no-allocation call takes the plain estimator or a known sigma");
        if (p->ra) return fail(HTSVD_ENOTSUP, "the no-allocation call does not run RA-Haar-tSVD");
        if (w0.total > fixed_cap)
            return fail(HTSVD_ENOMEM, "the image needs " + std::to_string(w0.total) + " bytes of scratch; the "
                                      "fixed array holds " + std::to_string(fixed_cap));
    } else {
        if ((s = ensure_ws(ctx, off_ra + (p->ra ? ra_ws_bytes(g) : 0))) != HTSVD_OK) return s;
        base = ctx->ws;
    }
    Ws wk = plan_ws(base, g, mp.W, mp.K, tile);
    const double mult = p->tau_mult > 0.0 ? p->tau_mult : default_mult(c, mp.K);
    hipStream_t st = (hipStream_t)stream;
    const float *zmap = nullptr;
    if (learned && (s = run_cnn_map(ctx, g, st, &zmap)) != HTSVD_OK) return s;
    if ((s = run_bm(ctx, g, mp, wk, st)) != HTSVD_OK) return s;
    hipError_t e;
    if (sigma > 0.f && !p->adaptive) {
        e = launch_fill_tau(wk.tau, (int64_t)g.ny * g.nx, nullptr, (double)sigma, mult, g, tile, st);
    } else {
        if ((s = run_sigma(ctx, g, mp, p, sigma, wk, zmap, st)) != HTSVD_OK) return s;
        if (learned)
            e = launch_fill_tau_learned(wk.tau, g, tile, zmap, wk.use_plain, wk.sig_est, wk.sig_hat, mult, st);
        else
            e = launch_fill_tau(wk.tau, (int64_t)g.ny * g.nx, wk.sig_hat, 0.0, mult, g, tile, st);
    }
    if (e != hipSuccess) return hip_fail(e, "tau");
    const float *ra_d = nullptr;
    const uint8_t *ra_f = nullptr;
    if (p->ra && (s = run_ra(ctx, g, mp, wk, wk.tau, (char *)ctx->ws + off_ra, mult, p->ra_sigma, st, &ra_d, &ra_f)) !=
                     HTSVD_OK)
        return s;
    return run_filter(ctx, g, mp, wk, wk.tau, d_out, out_stride, st, ra_d, ra_f);
}

}  // namespace

extern "C" {

htsvd_status htsvd_denoise(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                           int64_t in_stride, float sigma, const htsvd_params *p, float *d_out,
                           int64_t out_stride, void *stream) {
    return denoise_impl(ctx, d_in, h, w, c, in_stride, sigma, p, d_out, out_stride, stream, nullptr, 0);
}

htsvd_status htsvd_denoise_noalloc(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                                   int64_t in_stride, float sigma, const htsvd_params *p, float *d_out,
                                   int64_t out_stride, void *stream) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    void *ptr = scratch_ptr(ctx->device);
    if (!ptr) return fail(HTSVD_ESTATE, "no scratch address for this device");
    return denoise_impl(ctx, d_in, h, w, c, in_stride, sigma, p, d_out, out_stride, stream, ptr,
                        (size_t)HTSVD_NOALLOC_SCRATCH_BYTES);
}

htsvd_status htsvd_denoise_sweep(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                                 int64_t in_stride, int32_t n, const htsvd_sweep_item *items,
                                 const htsvd_params *p, void *stream) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate(ctx, d_in, h, w, c, in_stride, p, &g, &mp, true);
    if (s != HTSVD_OK) return s;
    if (n < 1 || !items) return fail(HTSVD_EINVAL, "a sweep needs at least one setting");
    if (p->adaptive) return fail(HTSVD_ENOTSUP, "sweeps take known sigma without the vote (adaptive = 0)");
    if (p->ra) return fail(HTSVD_ENOTSUP, "RA-Haar-tSVD runs in htsvd_denoise and htsvd_denoise_tau");
    bool need_prefix = false;
    size_t region_max = 0;
    for (int i = 0; i < n; ++i) {
        const htsvd_sweep_item &it = items[i];
        if (!(it.sigma > 0.f) || !std::isfinite(it.sigma)) return fail(HTSVD_EINVAL, "sweep sigma must be > 0");
        if (!(it.K == 4 || it.K == 8 || it.K == 16 || it.K == 32) || it.K > mp.K)
            return fail(HTSVD_EINVAL, "sweep K must be 4, 8, 16 or 32 and at most params K");
        if (!it.d_out) return fail(HTSVD_EINVAL, "null sweep output");
        if (it.out_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "out_stride < w*c");
        need_prefix |= it.K < mp.K;
        region_max = std::max(region_max, filter_region_bytes(g, mp.W, it.K));
    }
    const int tile = p->subimage;
    const int64_t n_ref = (int64_t)g.ny * g.nx;
    // Workspace: the single-call layout for p->K, then the prefix groups and a region buffer
    // sized for the largest tiling among the settings.
    const Ws w0 = plan_ws(nullptr, g, mp.W, mp.K, tile);
    const size_t off_pre = align256(w0.total);
    const size_t off_reg = off_pre + align256(need_prefix ? sizeof(int32_t) * n_ref * (mp.K / 2) : 0);
    if ((s = ensure_ws(ctx, off_reg + region_max)) != HTSVD_OK) return s;
    const Ws wk = plan_ws(ctx->ws, g, mp.W, mp.K, tile);
    int32_t *idx_pre = (int32_t *)((char *)ctx->ws + off_pre);
    float *regions = (float *)((char *)ctx->ws + off_reg);
    hipStream_t st = (hipStream_t)stream;
    if ((s = run_bm(ctx, g, mp, wk, st)) != HTSVD_OK) return s;
    int pre_k = 0;   // group size currently held in idx_pre
    hipError_t e;
    for (int i = 0; i < n; ++i) {
        const htsvd_sweep_item &it = items[i];
        MethodParams mpi = mp;
        mpi.K = it.K;
        Ws wi = wk;
        wi.regions = regions;
        if (it.K < mp.K) {
            if (pre_k != it.K) {
                if ((e = launch_idx_prefix(wk.idx, mp.K, idx_pre, it.K, n_ref, st)) != hipSuccess)
                    return hip_fail(e, "group prefix");
                pre_k = it.K;
            }
            wi.idx = idx_pre;
        }
        const double mult = p->tau_mult > 0.0 ? p->tau_mult : default_mult(c, it.K);
        if ((e = launch_fill_tau(wk.tau, n_ref, nullptr, (double)it.sigma, mult, g, tile, st)) != hipSuccess)
            return hip_fail(e, "tau");
        if ((s = run_filter(ctx, g, mpi, wi, wk.tau, it.d_out, it.out_stride, st)) != HTSVD_OK) return s;
    }
    return HTSVD_OK;
}

htsvd_status htsvd_estimate_sigma(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                                  int64_t in_stride, float sigma, const htsvd_params *p, double *d_sigma_est,
                                  double *d_sigma_hat, int32_t *d_votes, double *d_sigma_map, void *stream) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate(ctx, d_in, h, w, c, in_stride, p, &g, &mp, false);
    if (s != HTSVD_OK) return s;
    if (!(sigma > 0.f) && sigma != HTSVD_SIGMA_AUTO) return fail(HTSVD_EINVAL, "sigma must be > 0 or AUTO");
    if (p->estimator != 0 && p->estimator != 1) return fail(HTSVD_EINVAL, "estimator must be 0 or 1");
    const bool learned = sigma == HTSVD_SIGMA_AUTO && p->estimator == 1;
    const int tile = p->subimage;
    Ws w0 = plan_ws(nullptr, g, mp.W, mp.K, tile);
    if ((s = ensure_ws(ctx, w0.total)) != HTSVD_OK) return s;
    Ws wk = plan_ws(ctx->ws, g, mp.W, mp.K, tile);
    hipStream_t st = (hipStream_t)stream;
    const float *zmap = nullptr;
    if (learned && (s = run_cnn_map(ctx, g, st, &zmap)) != HTSVD_OK) return s;
    if (p->adaptive && (s = run_bm(ctx, g, mp, wk, st)) != HTSVD_OK) return s;
    if ((s = run_sigma(ctx, g, mp, p, sigma, wk, zmap, st)) != HTSVD_OK) return s;
    const int n_tiles = ((h + tile - 1) / tile) * ((w + tile - 1) / tile);
    hipError_t e;
    if (d_sigma_est &&
        (e = hipMemcpyAsync(d_sigma_est, wk.sig_est, sizeof(double) * n_tiles, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(e, "copy sigma_est");
    if (d_sigma_hat &&
        (e = hipMemcpyAsync(d_sigma_hat, wk.sig_hat, sizeof(double) * n_tiles, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(e, "copy sigma_hat");
    if (d_votes &&
        (e = hipMemcpyAsync(d_votes, wk.votes, sizeof(int32_t) * n_tiles, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(e, "copy votes");
    if (d_sigma_map && (e = launch_sigma_map(d_sigma_map, g, tile, learned ? zmap : nullptr, wk.use_plain, wk.sig_est,
                                             wk.sig_hat, st)) != hipSuccess)
        return hip_fail(e, "sigma map");
    return HTSVD_OK;
}

int32_t htsvd_cnn_param_count(int32_t c) {
    if (c != 1 && c != 3) return 0;
    int wo[6], bo[6], n;
    cnn_layout(c, wo, bo, &n);
    return n;
}

htsvd_status htsvd_cnn_init(htsvd_ctx *ctx, int32_t c, uint64_t seed) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    int wo[6], bo[6], n;
    cnn_layout(c, wo, bo, &n);
    std::vector<float> h(n, 0.f);
    const int ci[6] = {c, 32, 32, 32, 32, 32}, co[6] = {32, 32, 32, 32, 32, 1};
    uint64_t ctr = 0;
    for (int l = 0; l < 6; ++l) {
        const double sd = sqrt(2.0 / (9.0 * ci[l])) * (l == 5 ? 0.1 : 1.0);
        for (int k = 0; k < co[l] * 9 * ci[l]; ++k) h[wo[l] + k] = (float)(sd * counter_normal(seed, ctr++));
    }
    h[bo[5]] = (float)log(20.0);
    htsvd_status s = cnn_alloc(ctx, c);
    if (s != HTSVD_OK) return s;
    return cnn_upload(ctx, h.data(), n);
}

htsvd_status htsvd_cnn_set_weights(htsvd_ctx *ctx, int32_t c, const float *h_params, int64_t n) {
    if (!ctx || !h_params) return fail(HTSVD_EINVAL, "null argument");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    if (n != htsvd_cnn_param_count(c)) return fail(HTSVD_EINVAL, "wrong parameter count");
    htsvd_status s = cnn_alloc(ctx, c);
    if (s != HTSVD_OK) return s;
    return cnn_upload(ctx, h_params, (int)n);
}

htsvd_status htsvd_cnn_get_weights(htsvd_ctx *ctx, float *h_params, int64_t n) {
    if (!ctx || !h_params) return fail(HTSVD_EINVAL, "null argument");
    if (!ctx->cnn.w) return fail(HTSVD_ESTATE, "network weights not set");
    if (n != ctx->cnn.n) return fail(HTSVD_EINVAL, "wrong parameter count");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise");
    if ((e = hipMemcpy(h_params, ctx->cnn.w, sizeof(float) * n, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "download");
    return HTSVD_OK;
}

htsvd_status htsvd_cnn_forward(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                               int64_t in_stride, float *d_log_sigma, void *stream) {
    htsvd_status s = validate_crops(ctx, d_in, 1, h, w, c);
    if (s != HTSVD_OK) return s;
    if (!d_log_sigma) return fail(HTSVD_EINVAL, "null output");
    if (in_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "in_stride < w*c");
    CnnState &cs = ctx->cnn;
    CnnWs w0 = plan_cnn_ws(nullptr, 1, h, w, c, false);
    if ((s = ensure_cnn_ws(ctx, w0.total)) != HTSVD_OK) return s;
    CnnWs wk = plan_cnn_ws(cs.ws, 1, h, w, c, false);
    CnnBuffers b = cnn_buffers(cs, wk);
    b.z = d_log_sigma;
    hipError_t e = cnn_forward(b, d_in, in_stride, 0, 1, h, w, c, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "network forward");
    return HTSVD_OK;
}

htsvd_status cnn_grad_impl(htsvd_ctx *ctx, const uint8_t *d_crops, int32_t n, int32_t h, int32_t w, int32_t c,
                           const float *d_target, float *d_grad, double *h_loss, hipStream_t st) {
    htsvd_status s = validate_crops(ctx, d_crops, n, h, w, c);
    if (s != HTSVD_OK) return s;
    if (!d_target || !d_grad) return fail(HTSVD_EINVAL, "null target or gradient");
    CnnState &cs = ctx->cnn;
    CnnWs w0 = plan_cnn_ws(nullptr, n, h, w, c, true);
    if ((s = ensure_cnn_ws(ctx, w0.total)) != HTSVD_OK) return s;
    CnnWs wk = plan_cnn_ws(cs.ws, n, h, w, c, true);
    CnnBuffers b = cnn_buffers(cs, wk);
    const int64_t sb = (int64_t)w * c, bb = (int64_t)h * w * c;
    hipError_t e = cnn_forward(b, d_crops, sb, bb, n, h, w, c, st);
    if (e != hipSuccess) return hip_fail(e, "network forward");
    e = cnn_backward(b, d_crops, sb, bb, n, h, w, c, d_target, d_grad, wk.d0, wk.d1, cs.d_loss, st);
    if (e != hipSuccess) return hip_fail(e, "network backward");
    if (h_loss) {
        double v = 0.0;
        if ((e = hipMemcpyAsync(&v, cs.d_loss, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return hip_fail(e, "loss copy");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronise");
        *h_loss = v / (double)cnn_act_elems(6, n, h, w, c);
    }
    return HTSVD_OK;
}

htsvd_status htsvd_cnn_gradients(htsvd_ctx *ctx, const uint8_t *d_crops, int32_t n, int32_t h, int32_t w,
                                 int32_t c, const float *d_target_log, float *d_grad, double *h_loss, void *stream) {
    return cnn_grad_impl(ctx, d_crops, n, h, w, c, d_target_log, d_grad, h_loss, (hipStream_t)stream);
}

htsvd_status htsvd_cnn_train_step(htsvd_ctx *ctx, const uint8_t *d_crops, int32_t n, int32_t h, int32_t w,
                                  int32_t c, const float *d_target_log, float lr, double *h_loss, void *stream) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (!(lr > 0.f)) return fail(HTSVD_EINVAL, "lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    htsvd_status s = cnn_grad_impl(ctx, d_crops, n, h, w, c, d_target_log, ctx->cnn.grad, h_loss, st);
    if (s != HTSVD_OK) return s;
    CnnState &cs = ctx->cnn;
    cs.step += 1;
    hipError_t e = cnn_adam(cs.w, cs.m, cs.v, cs.grad, cs.n, lr, cs.step, cs.wq, cs.wbf, st);
    if (e != hipSuccess) return hip_fail(e, "adam");
    return HTSVD_OK;
}

// Checkpoint file: "HTCN", version 1, c, n, step, then w, m, v (FP32, n each).
htsvd_status htsvd_cnn_save(htsvd_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(HTSVD_EINVAL, "null argument");
    CnnState &cs = ctx->cnn;
    if (!cs.w) return fail(HTSVD_ESTATE, "network weights not set");
    std::vector<float> buf((size_t)3 * cs.n);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise");
    float *src[3] = {cs.w, cs.m, cs.v};
    for (int i = 0; i < 3; ++i)
        if ((e = hipMemcpy(buf.data() + (size_t)i * cs.n, src[i], sizeof(float) * cs.n, hipMemcpyDeviceToHost)) !=
            hipSuccess)
            return hip_fail(e, "download");
    FILE *f = fopen(path, "wb");
    if (!f) return fail(HTSVD_EINVAL, std::string("cannot open ") + path);
    const int32_t hdr[4] = {0x4E435448 /* "HTCN" */, 1, cs.c, cs.n};
    bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(&cs.step, sizeof(cs.step), 1, f) == 1 &&
              fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(HTSVD_EINVAL, std::string("cannot write ") + path);
    return HTSVD_OK;
}

htsvd_status htsvd_cnn_load(htsvd_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(HTSVD_EINVAL, "null argument");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(HTSVD_EINVAL, std::string("cannot open ") + path);
    int32_t hdr[4];
    int64_t step = 0;
    bool ok = fread(hdr, sizeof(hdr), 1, f) == 1 && fread(&step, sizeof(step), 1, f) == 1;
    if (!ok || hdr[0] != 0x4E435448 || hdr[1] != 1 || (hdr[2] != 1 && hdr[2] != 3) ||
        hdr[3] != htsvd_cnn_param_count(hdr[2])) {
        fclose(f);
        return fail(HTSVD_EINVAL, std::string("not a network checkpoint: ") + path);
    }
    const int n = hdr[3];
    std::vector<float> buf((size_t)3 * n);
    ok = fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return fail(HTSVD_EINVAL, std::string("truncated checkpoint: ") + path);
    htsvd_status s = cnn_alloc(ctx, hdr[2]);
    if (s != HTSVD_OK) return s;
    if ((s = cnn_upload(ctx, buf.data(), n)) != HTSVD_OK) return s;
    CnnState &cs = ctx->cnn;
    hipError_t e;
    if ((e = hipMemcpy(cs.m, buf.data() + n, sizeof(float) * n, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "upload");
    if ((e = hipMemcpy(cs.v, buf.data() + 2 * (size_t)n, sizeof(float) * n, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "upload");
    cs.step = step;
    return HTSVD_OK;
}

}  // extern "C"

namespace {

uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

struct BatchImage {
    int src;                 // index in the caller's array
    ImageGeom g;
    MethodParams mp;
    TileGeom tg, tg_alt;        // tiling for mp.K, and for K = 16 (auto images)
    bool auto_k;
    int bm_tiles_x, bm_tiles;
    int64_t n_ref, n_tiles_sigma;
    size_t off_idx, off_tau, off_reg, off_sig;   // byte offsets in the workspace
    size_t off_z;                                 // learned log-sigma map (learned images)
    bool learned;
    float *out;
    int64_t out_stride;
    float sigma;
};

// Learned images of one size: one network run over all of them, their maps contiguous.
struct CnnClass {
    int h, w;
    std::vector<int> members;   // indices into BatchPlan::im
    size_t ws_bytes;            // network workspace for the class
};

// Host plan of a batch: workspace layout, unit tables, per-class descriptor lists.
struct BatchPlan {
    std::vector<BatchImage> im;
    std::vector<int> classes;                     // distinct K values
    size_t ws_total = 0;
    size_t off_mom = 0;                           // plain-estimator moments of all estimated images
    std::vector<CnnClass> cnn;                    // learned images grouped by size
    size_t cnn_ws = 0;                            // largest network workspace of a class
    int max_s = 1, max_W = 3, max_h = 8, max_w = 8;
    bool any_auto = false;
};

htsvd_status plan_batch(htsvd_ctx *ctx, int32_t n, const htsvd_image *imgs, const htsvd_params *p, int tile_side,
                        BatchPlan *bp) {
    BatchPlan &P = *bp;
    const int T = p->subimage;
    for (int i = 0; i < n; ++i) {
        const htsvd_image &x = imgs[i];
        htsvd_params pi = *p;
        BatchImage b;
        b.auto_k = x.K == HTSVD_K_AUTO;
        if (b.auto_k) pi.K = 32;
        else if (x.K) pi.K = x.K;
        htsvd_status s = validate(ctx, x.d_in, x.h, x.w, x.c, x.in_stride, &pi, &b.g, &b.mp, true);
        if (s != HTSVD_OK) return fail(s, std::string("image ") + std::to_string(i) + ": " + htsvd_last_error());
        if (!x.d_out || x.out_stride < (int64_t)x.w * x.c) return fail(HTSVD_EINVAL, "bad output of image " + std::to_string(i));
        if (!(x.sigma > 0.f) && x.sigma != HTSVD_SIGMA_AUTO) return fail(HTSVD_EINVAL, "bad sigma of image " + std::to_string(i));
        if (i > 0 && x.c != imgs[0].c) return fail(HTSVD_ENOTSUP, "all images of a batch must have the same channel count");
        b.src = i;
        b.sigma = x.sigma;
        b.out = x.d_out;
        b.out_stride = x.out_stride;
        b.bm_tiles_x = (b.g.nx + REF_TILE - 1) / REF_TILE;
        b.bm_tiles = ((b.g.ny + REF_TILE - 1) / REF_TILE) * b.bm_tiles_x;
        b.tg = plan_filter_tiles(b.g, b.mp.W, b.mp.K, tile_side);
        b.tg_alt = plan_filter_tiles(b.g, b.mp.W, 16, tile_side);
        b.n_ref = (int64_t)b.g.ny * b.g.nx;
        b.n_tiles_sigma = (int64_t)((b.g.h + T - 1) / T) * ((b.g.w + T - 1) / T);
        b.learned = x.sigma == HTSVD_SIGMA_AUTO && p->estimator == 1;
        b.off_z = 0;
        P.any_auto |= (x.sigma == HTSVD_SIGMA_AUTO) || p->adaptive;
        P.im.push_back(b);
    }
    // largest images first: their units enter the work queues first and the tail is short
    std::stable_sort(P.im.begin(), P.im.end(), [](const BatchImage &a, const BatchImage &b) {
        return (int64_t)a.g.h * a.g.w > (int64_t)b.g.h * b.g.w;
    });
    size_t off = 0;
    for (BatchImage &b : P.im) {
        b.off_idx = off; off = align256(off + sizeof(int32_t) * b.n_ref * b.mp.K);
        b.off_tau = off; off = align256(off + sizeof(double) * b.n_ref);
        b.off_reg = off;
        size_t reg = (size_t)b.tg.tiles_y * b.tg.tiles_x * region_elems(b.tg, b.g.c) * sizeof(float);
        if (b.auto_k)
            reg = std::max(reg, (size_t)b.tg_alt.tiles_y * b.tg_alt.tiles_x * region_elems(b.tg_alt, b.g.c) *
                                    sizeof(float));
        off = align256(off + reg);
        b.off_sig = off;  // sig_est, sig_hat, votes, cov (c per tile), use_plain, sig_plain
        off = align256(off + b.n_tiles_sigma * (sizeof(double) * (3 + b.g.c) + 2 * sizeof(int32_t)));
        P.max_s = std::max(P.max_s, b.g.s);
        P.max_W = std::max(P.max_W, b.mp.W);
        P.max_h = std::max(P.max_h, b.g.h);
        P.max_w = std::max(P.max_w, b.g.w);
        if (std::find(P.classes.begin(), P.classes.end(), b.mp.K) == P.classes.end()) P.classes.push_back(b.mp.K);
        if (b.auto_k && std::find(P.classes.begin(), P.classes.end(), 16) == P.classes.end()) P.classes.push_back(16);
    }
    // learned maps: one contiguous block per size class (the network writes a class at once)
    for (size_t i = 0; i < P.im.size(); ++i) {
        const BatchImage &b = P.im[i];
        if (!b.learned) continue;
        size_t k = 0;
        while (k < P.cnn.size() && !(P.cnn[k].h == b.g.h && P.cnn[k].w == b.g.w)) ++k;
        if (k == P.cnn.size()) P.cnn.push_back(CnnClass{b.g.h, b.g.w, {}, 0});
        P.cnn[k].members.push_back((int)i);
    }
    for (CnnClass &cc : P.cnn) {
        const int c = P.im[cc.members[0]].g.c;
        const size_t zone = sizeof(float) * cnn_act_elems(6, 1, cc.h, cc.w, c);
        for (size_t n = 0; n < cc.members.size(); ++n) P.im[cc.members[n]].off_z = off + n * zone;
        off = align256(off + zone * cc.members.size());
        cc.ws_bytes = plan_cnn_ws(nullptr, (int)cc.members.size(), cc.h, cc.w, c, false).total;
        P.cnn_ws = std::max(P.cnn_ws, cc.ws_bytes);
    }
    int64_t mom_units = 0;
    for (const BatchImage &b : P.im)
        if (b.sigma == HTSVD_SIGMA_AUTO) mom_units += b.n_tiles_sigma * b.g.c;
    P.off_mom = off;
    off = align256(off + sizeof(int32_t) * sigma_mom_ints() * mom_units);
    int64_t px = 0, refs = 0, bm = 0;
    for (const BatchImage &b : P.im) {
        px += (int64_t)b.g.h * b.g.w;
        refs += b.n_ref;
        bm += b.bm_tiles;
    }
    if (px >= ((int64_t)1 << 31) || refs >= ((int64_t)1 << 31) || bm >= ((int64_t)1 << 31))
        return fail(HTSVD_ENOTSUP, "batch too large (2^31 pixels at most)");
    P.ws_total = off;
    return HTSVD_OK;
}

// Per-image workspace view (the layout the single-image helpers expect).
Ws image_ws(void *base, const BatchImage &b) {
    Ws w;
    char *c = (char *)base;
    w.idx = (int32_t *)(c + b.off_idx);
    w.tau = (double *)(c + b.off_tau);
    w.regions = (float *)(c + b.off_reg);
    double *sig = (double *)(c + b.off_sig);
    w.sig_est = sig;
    w.sig_hat = sig + b.n_tiles_sigma;
    w.cov = sig + 2 * b.n_tiles_sigma;
    w.sig_plain = sig + (2 + b.g.c) * b.n_tiles_sigma;
    w.votes = (int32_t *)(sig + (3 + b.g.c) * b.n_tiles_sigma);
    w.use_plain = w.votes + b.n_tiles_sigma;
    w.mom = nullptr;   // batched estimation uses the batch's shared moments buffer
    w.total = 0;
    return w;
}

}  // namespace

extern "C" {

htsvd_status htsvd_denoise_batch(htsvd_ctx *ctx, int32_t n, const htsvd_image *imgs, const htsvd_params *p,
                                 const htsvd_batch_opts *opts, void *stream) {
    if (!ctx || !imgs || !p) return fail(HTSVD_EINVAL, "null argument");
    if (n < 1) return fail(HTSVD_EINVAL, "empty batch");
    if (p->ra) return fail(HTSVD_ENOTSUP, "RA-Haar-tSVD runs in htsvd_denoise and htsvd_denoise_tau");
    htsvd_batch_opts o = {1, 1, 0.f, 0};
    if (opts) o = *opts;
    if (o.blocks_per_cu < 1) o.blocks_per_cu = 1;
    if (o.blocks_per_cu > 8) return fail(HTSVD_EINVAL, "blocks_per_cu must be in [1, 8]");
    if (!(o.k_sigma_cutoff >= 0.f)) return fail(HTSVD_EINVAL, "k_sigma_cutoff must be >= 0");
    if (o.tile_side < 0 || o.tile_side > 16) return fail(HTSVD_EINVAL, "tile_side must be in [0, 16]");
    hipStream_t st = (hipStream_t)stream;

    // signature of the batch, field by field (struct padding is not hashed)
    uint64_t sig = 0xcbf29ce484222325ull;
    for (int i = 0; i < n; ++i) {
        const htsvd_image &x = imgs[i];
        sig = fnv1a(sig, &x.d_in, sizeof(x.d_in));
        sig = fnv1a(sig, &x.h, sizeof(x.h));
        sig = fnv1a(sig, &x.w, sizeof(x.w));
        sig = fnv1a(sig, &x.c, sizeof(x.c));
        sig = fnv1a(sig, &x.in_stride, sizeof(x.in_stride));
        sig = fnv1a(sig, &x.sigma, sizeof(x.sigma));
        sig = fnv1a(sig, &x.K, sizeof(x.K));
        sig = fnv1a(sig, &x.d_out, sizeof(x.d_out));
        sig = fnv1a(sig, &x.out_stride, sizeof(x.out_stride));
    }
    const int32_t pi32[] = {p->ps, p->stride, p->window, p->K, p->adaptive, p->gamma_rank, p->gcp_num,
                            p->gcp_den, p->estimator, p->subimage, p->n_vote};
    sig = fnv1a(sig, pi32, sizeof(pi32));
    sig = fnv1a(sig, &p->tau_mult, sizeof(p->tau_mult));
    sig = fnv1a(sig, &p->beta, sizeof(p->beta));
    sig = fnv1a(sig, &p->vote_seed, sizeof(p->vote_seed));
    sig = fnv1a(sig, &o, sizeof(o));
    sig = fnv1a(sig, &ctx->cnn.w, sizeof(ctx->cnn.w));
    sig = fnv1a(sig, &ctx->cnn.c, sizeof(ctx->cnn.c));
    if (o.use_graph && ctx->batch.valid && ctx->batch.sig == sig) {
        hipError_t e = hipGraphLaunch(ctx->batch.exec, st);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
        return HTSVD_OK;
    }

    ctx->batch.k_plan.clear();   // valid again once this batch is planned
    BatchPlan P;
    htsvd_status s = plan_batch(ctx, n, imgs, p, o.tile_side, &P);
    if (s != HTSVD_OK) return s;
    const int ni = (int)P.im.size();
    const int C = P.im[0].g.c;
    const bool learned_any = p->estimator == 1;
    (void)learned_any;
    if (!P.cnn.empty()) {
        if (!ctx->cnn.w) return fail(HTSVD_ESTATE, "learned estimator requested but no network weights are set");
        if (ctx->cnn.c != C) return fail(HTSVD_EINVAL, "network channel count differs from the images'");
        if ((s = ensure_cnn_ws(ctx, P.cnn_ws)) != HTSVD_OK) return s;
    }
    if ((s = ensure_ws(ctx, P.ws_total)) != HTSVD_OK) return s;

    // descriptor tables (host), then one upload
    std::vector<BatchItem> items(ni);
    std::vector<int> bm_start(ni + 1, 0), ref_start(ni + 1, 0), pix_start(ni + 1, 0);
    std::vector<double> sigma_h(ni), mult_h(ni);
    std::vector<int> ksel_h(ni), auto_list;
    for (int i = 0; i < ni; ++i) {
        const BatchImage &b = P.im[i];
        Ws w = image_ws(ctx->ws, b);
        BatchItem &it = items[i];
        it.g = b.g;
        it.mp = b.mp;
        it.tg = b.tg;
        it.bm_tiles_x = b.bm_tiles_x;
        it.idx = w.idx;
        it.tau = w.tau;
        it.regions = w.regions;
        it.out = b.out;
        it.out_stride = b.out_stride;
        it.idx_stride = b.mp.K;
        it.tau_mul = 1.0;
        it.ksel = nullptr;       // set to the device table below for auto images
        it.k_alt = 16;
        it.tg_alt = b.tg_alt;
        ksel_h[i] = b.mp.K;
        if (b.auto_k) auto_list.push_back(i);
        bm_start[i + 1] = bm_start[i] + b.bm_tiles;
        ref_start[i + 1] = ref_start[i] + (int)b.n_ref;
        pix_start[i + 1] = pix_start[i] + b.g.h * b.g.w;
        sigma_h[i] = b.sigma > 0.f ? (double)b.sigma : 0.0;
        mult_h[i] = p->tau_mult > 0.0 ? p->tau_mult : default_mult(C, b.mp.K);
    }
    // device layout: items | class items... | bm_start | ref_start | pix_start | class starts... | sigma | mult |
    // ksel | auto list | queues
    size_t off = 0;
    auto reserve = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_items = reserve(sizeof(BatchItem) * ni);
    const size_t o_ksel = reserve(sizeof(int) * ni), o_auto = reserve(sizeof(int) * std::max<size_t>(1, auto_list.size()));
    // per-class (K) filter tables: items of the class and their tile prefix sums.  An auto image
    // appears in the class 32 list and, with its K = 16 tiling and threshold factor, in class 16.
    std::vector<std::vector<BatchItem>> cls_items(P.classes.size());
    std::vector<std::vector<int>> cls_start(P.classes.size()), cls_src(P.classes.size());
    std::vector<int> cls_lds(P.classes.size(), 0);
    for (size_t k = 0; k < P.classes.size(); ++k) {
        const int K = P.classes[k];
        cls_start[k].push_back(0);
        for (int i = 0; i < ni; ++i) {
            BatchItem it = items[i];
            if (it.mp.K != K) {
                if (!(P.im[i].auto_k && K == 16)) continue;
                it.mp.K = 16;
                it.tg = P.im[i].tg_alt;
                it.tau_mul = p->tau_mult > 0.0 ? 1.0 : default_mult(C, 16) / default_mult(C, 32);
            }
            cls_items[k].push_back(it);
            cls_src[k].push_back(i);
            cls_start[k].push_back(cls_start[k].back() + it.tg.tiles_y * it.tg.tiles_x);
            cls_lds[k] = std::max(cls_lds[k], filter_lds_bytes_for(it.tg, C, K));
        }
    }
    std::vector<size_t> o_citems(P.classes.size()), o_cstart(P.classes.size());
    for (size_t k = 0; k < P.classes.size(); ++k) o_citems[k] = reserve(sizeof(BatchItem) * cls_items[k].size());
    const size_t o_bm = reserve(sizeof(int) * (ni + 1)), o_ref = reserve(sizeof(int) * (ni + 1)),
                 o_pix = reserve(sizeof(int) * (ni + 1));
    for (size_t k = 0; k < P.classes.size(); ++k) o_cstart[k] = reserve(sizeof(int) * cls_start[k].size());
    const size_t o_sig = reserve(sizeof(double) * ni), o_mult = reserve(sizeof(double) * ni);
    const size_t o_q = reserve(sizeof(int) * (1 + P.classes.size()));
    // noise-level stage tables over the images whose sigma is estimated or adjusted
    std::vector<SigmaItem> sitems;
    std::vector<int> sitem_img;   // image (index into P.im) of each item
    std::vector<int> cov_sel, tile_sel, ref_sel, cov_st{0}, tile_st{0}, ref_st{0};
    std::vector<int> aref_sel, aref_st{0};   // auto-K images among them (level before the vote)
    constexpr int NVK = 4;
    const int vK[NVK] = {4, 8, 16, 32};
    std::vector<int> vote_sel[NVK], vote_st[NVK];
    for (int v = 0; v < NVK; ++v) vote_st[v].push_back(0);
    for (int i = 0; i < ni; ++i) {
        const BatchImage &b = P.im[i];
        if (!(b.sigma == HTSVD_SIGMA_AUTO || p->adaptive)) continue;
        const Ws w = image_ws(ctx->ws, b);
        SigmaItem si;
        si.g = b.g;
        si.K = b.mp.K;
        si.mode = b.sigma > 0.f ? SIGMA_KNOWN : (b.learned ? SIGMA_LEARNED : SIGMA_PLAIN);
        si.adaptive = p->adaptive ? 1 : 0;
        si.n_tiles = (int)b.n_tiles_sigma;
        si.sigma = b.sigma > 0.f ? (double)b.sigma : 0.0;
        si.mult = mult_h[i];
        si.idx = w.idx;
        si.tau = w.tau;
        si.sig_est = w.sig_est;
        si.sig_hat = w.sig_hat;
        si.cov = w.cov;
        si.sig_plain = w.sig_plain;
        si.votes = w.votes;
        si.use_plain = w.use_plain;
        si.zmap = b.learned ? (const float *)((char *)ctx->ws + b.off_z) : nullptr;
        si.ksel = nullptr;   // set to the device choice below for auto images
        const int k = (int)sitems.size();
        sitems.push_back(si);
        sitem_img.push_back(i);
        if (si.mode != SIGMA_KNOWN) {
            cov_sel.push_back(k);
            cov_st.push_back(cov_st.back() + si.n_tiles * b.g.c);
        }
        tile_sel.push_back(k);
        tile_st.push_back(tile_st.back() + si.n_tiles);
        if (si.adaptive) {
            // an auto image votes with the groups of the size chosen for it (16 or 32): it is listed
            // for both, and the vote launch of the other size skips it
            for (int v = 0; v < NVK; ++v) {
                if (!(vK[v] == si.K || (b.auto_k && vK[v] == 16))) continue;
                vote_sel[v].push_back(k);
                vote_st[v].push_back(vote_st[v].back() + si.n_tiles);
            }
            if (std::find(vK, vK + NVK, si.K) == vK + NVK) return fail(HTSVD_ENOTSUP, "group size without a vote kernel");
        }
        ref_sel.push_back(k);
        ref_st.push_back(ref_st.back() + (int)b.n_ref);
        if (b.auto_k) {
            aref_sel.push_back(k);
            aref_st.push_back(aref_st.back() + (int)b.n_ref);
        }
    }
    const size_t o_sitems = reserve(sizeof(SigmaItem) * std::max<size_t>(1, sitems.size()));
    // per size class of learned images: their input pointers and row strides
    std::vector<size_t> o_ctab(P.cnn.size()), o_cstr(P.cnn.size());
    for (size_t k = 0; k < P.cnn.size(); ++k) {
        o_ctab[k] = reserve(sizeof(const uint8_t *) * P.cnn[k].members.size());
        o_cstr[k] = reserve(sizeof(int64_t) * P.cnn[k].members.size());
    }
    auto reserve_ints = [&](const std::vector<int> &v) { return reserve(sizeof(int) * std::max<size_t>(1, v.size())); };
    const size_t o_cov_sel = reserve_ints(cov_sel), o_cov_st = reserve_ints(cov_st);
    const size_t o_tile_sel = reserve_ints(tile_sel), o_tile_st = reserve_ints(tile_st);
    const size_t o_ref_sel = reserve_ints(ref_sel), o_ref_st = reserve_ints(ref_st);
    const size_t o_aref_sel = reserve_ints(aref_sel), o_aref_st = reserve_ints(aref_st);
    size_t o_vote_sel[NVK], o_vote_st[NVK];
    for (int v = 0; v < NVK; ++v) {
        o_vote_sel[v] = reserve_ints(vote_sel[v]);
        o_vote_st[v] = reserve_ints(vote_st[v]);
    }
    int64_t auto_refs = 1;
    for (int i : auto_list) auto_refs = std::max(auto_refs, P.im[i].n_ref);
    const int k_chunks = select_k_chunks(auto_refs);
    const size_t o_kpart = reserve(sizeof(double) * k_chunks * std::max<size_t>(1, auto_list.size()));
    hipError_t e;
    BatchCache &bc = ctx->batch;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise before batch planning");
    if (bc.exec) { (void)hipGraphExecDestroy(bc.exec); bc.exec = nullptr; }
    if (bc.graph) { (void)hipGraphDestroy(bc.graph); bc.graph = nullptr; }
    bc.valid = false;
    if (bc.dev_size < off) {
        if (bc.dev) (void)hipFree(bc.dev);
        bc.dev = nullptr;
        bc.dev_size = 0;
        if (hipMalloc(&bc.dev, off) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HTSVD_ENOMEM, "batch descriptor allocation");
        }
        bc.dev_size = off;
    }
    // device table of the chosen group sizes, referenced by the descriptors of auto images
    const int *d_ksel = (const int *)((char *)bc.dev + o_ksel);
    for (int i = 0; i < ni; ++i)
        if (P.im[i].auto_k) items[i].ksel = d_ksel + i;
    for (size_t k = 0; k < P.classes.size(); ++k)
        for (size_t j = 0; j < cls_items[k].size(); ++j)
            if (P.im[cls_src[k][j]].auto_k) cls_items[k][j].ksel = d_ksel + cls_src[k][j];
    for (size_t k = 0; k < sitems.size(); ++k)
        if (P.im[sitem_img[k]].auto_k) sitems[k].ksel = d_ksel + sitem_img[k];
    std::vector<unsigned char> host(off, 0);
    memcpy(host.data() + o_items, items.data(), sizeof(BatchItem) * ni);
    for (size_t k = 0; k < P.classes.size(); ++k) {
        memcpy(host.data() + o_citems[k], cls_items[k].data(), sizeof(BatchItem) * cls_items[k].size());
        memcpy(host.data() + o_cstart[k], cls_start[k].data(), sizeof(int) * cls_start[k].size());
    }
    memcpy(host.data() + o_bm, bm_start.data(), sizeof(int) * (ni + 1));
    memcpy(host.data() + o_ref, ref_start.data(), sizeof(int) * (ni + 1));
    memcpy(host.data() + o_pix, pix_start.data(), sizeof(int) * (ni + 1));
    memcpy(host.data() + o_sig, sigma_h.data(), sizeof(double) * ni);
    memcpy(host.data() + o_mult, mult_h.data(), sizeof(double) * ni);
    memcpy(host.data() + o_ksel, ksel_h.data(), sizeof(int) * ni);
    if (!auto_list.empty()) memcpy(host.data() + o_auto, auto_list.data(), sizeof(int) * auto_list.size());
    if (!sitems.empty()) memcpy(host.data() + o_sitems, sitems.data(), sizeof(SigmaItem) * sitems.size());
    for (size_t k = 0; k < P.cnn.size(); ++k)
        for (size_t n = 0; n < P.cnn[k].members.size(); ++n) {
            const ImageGeom &gk = P.im[P.cnn[k].members[n]].g;
            memcpy(host.data() + o_ctab[k] + n * sizeof(const uint8_t *), &gk.img, sizeof(const uint8_t *));
            memcpy(host.data() + o_cstr[k] + n * sizeof(int64_t), &gk.stride, sizeof(int64_t));
        }
    auto put_ints = [&](size_t o2, const std::vector<int> &v) {
        if (!v.empty()) memcpy(host.data() + o2, v.data(), sizeof(int) * v.size());
    };
    put_ints(o_cov_sel, cov_sel);
    put_ints(o_cov_st, cov_st);
    put_ints(o_tile_sel, tile_sel);
    put_ints(o_tile_st, tile_st);
    put_ints(o_ref_sel, ref_sel);
    put_ints(o_ref_st, ref_st);
    put_ints(o_aref_sel, aref_sel);
    put_ints(o_aref_st, aref_st);
    for (int v = 0; v < NVK; ++v) {
        put_ints(o_vote_sel[v], vote_sel[v]);
        put_ints(o_vote_st[v], vote_st[v]);
    }
    if ((e = hipMemcpy(bc.dev, host.data(), off, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "batch descriptor upload");
    bc.k_plan.assign(n, 0);
    bc.auto_k.assign(n, 0);
    bc.n_ref.assign(n, 0);
    bc.tau.assign(n, nullptr);
    bc.ksel.assign(n, nullptr);
    bc.mul_alt = p->tau_mult > 0.0 ? 1.0 : default_mult(C, 16) / default_mult(C, 32);
    for (int i = 0; i < ni; ++i) {
        const int src = P.im[i].src;
        bc.k_plan[src] = P.im[i].mp.K;
        bc.auto_k[src] = P.im[i].auto_k ? 1 : 0;
        bc.n_ref[src] = P.im[i].n_ref;
        bc.tau[src] = items[i].tau;
        bc.ksel[src] = P.im[i].auto_k ? d_ksel + i : nullptr;
    }
    char *D = (char *)bc.dev;
    const BatchItem *d_items = (const BatchItem *)(D + o_items);
    int *d_q = (int *)(D + o_q);
    int n_cu = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (n_cu < 1) n_cu = 1;
    const int grid = n_cu * o.blocks_per_cu;

    // the launch sequence (captured when use_graph)
    hipStream_t ls = st;
    const bool timing = ctx->timing;
    if (o.use_graph) {
        if (!ctx->cap_stream && (e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "capture stream");
        ls = ctx->cap_stream;
        ctx->timing = false;   // no event records inside the graph
        if ((e = hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            ctx->timing = timing;
            return hip_fail(e, "begin capture");
        }
    }
    auto enqueue = [&]() -> htsvd_status {
        hipError_t e2;
        if ((e2 = launch_zero(d_q, sizeof(int) * (1 + P.classes.size()), ls)) != hipSuccess) return hip_fail(e2, "queues");
        if ((e2 = launch_zero(ctx->d_guard, 2 * sizeof(unsigned long long), ls)) != hipSuccess) return hip_fail(e2, "counters");
        if ((e2 = launch_fill_tau_batched(d_items, ni, (const int *)(D + o_ref), ref_start[ni], (const double *)(D + o_sig),
                                          (const double *)(D + o_mult), ls)) != hipSuccess)
            return hip_fail(e2, "tau");
        if ((e2 = launch_block_match_batched(d_items, ni, (const int *)(D + o_bm), P.max_s, P.max_W, P.max_h, P.max_w,
                                             d_q, std::min(grid, bm_start[ni]), ls)) != hipSuccess)
            return hip_fail(e2, "batched block matching");
        // images whose noise level is estimated or adjusted: the network per learned image, then
        // every sub-image stage in one launch over all images
        if (!sitems.empty()) {
            StageScope sc(ctx, HTSVD_STAGE_SIGMA, ls);
            const int T = p->subimage;
            const SigmaItem *S = (const SigmaItem *)(D + o_sitems);
            // the network once per size class, writing the class's contiguous maps
            for (size_t k = 0; k < P.cnn.size(); ++k) {
                const CnnClass &cc = P.cnn[k];
                const int m = (int)cc.members.size();
                CnnBuffers cb = cnn_buffers(ctx->cnn, plan_cnn_ws(ctx->cnn.ws, m, cc.h, cc.w, C, false));
                cb.z = (float *)((char *)ctx->ws + P.im[cc.members[0]].off_z);
                if ((e2 = cnn_forward_tab(cb, (const uint8_t *const *)(D + o_ctab[k]), (const int64_t *)(D + o_cstr[k]),
                                          m, cc.h, cc.w, C, ls)) != hipSuccess)
                    return hip_fail(e2, "network forward");
            }
            auto I = [&](size_t o2) { return (const int *)(D + o2); };
            if ((e2 = launch_sigma_est_batched(S, I(o_cov_sel), I(o_cov_st), (int)cov_sel.size(), cov_st.back(), T,
                                               (int32_t *)((char *)ctx->ws + P.off_mom), ls)) != hipSuccess)
                return hip_fail(e2, "batched sigma estimation");
            if ((e2 = launch_sigma_tiles_batched(S, I(o_tile_sel), I(o_tile_st), (int)tile_sel.size(), tile_st.back(),
                                                 T, JUDGE_RATIO, ls)) != hipSuccess)
                return hip_fail(e2, "batched sigma tiles");
            // auto-K images: thresholds at the level before the vote, from which the group size is
            // chosen; the vote then runs on the groups of that size
            if ((e2 = launch_fill_tau_sigma_batched(S, I(o_aref_sel), I(o_aref_st), (int)aref_sel.size(),
                                                    aref_st.back(), T, ls)) != hipSuccess)
                return hip_fail(e2, "batched thresholds before the vote");
        }
        if ((e2 = launch_select_k(d_items, (const int *)(D + o_auto), (int)auto_list.size(), k_chunks,
                                  (double *)(D + o_kpart), (const double *)(D + o_mult), (double)o.k_sigma_cutoff,
                                  (int *)(D + o_ksel), ls)) != hipSuccess)
            return hip_fail(e2, "group size selection");
        if (!sitems.empty()) {
            StageScope sc(ctx, HTSVD_STAGE_SIGMA, ls);
            const int T = p->subimage;
            const SigmaItem *S = (const SigmaItem *)(D + o_sitems);
            auto I = [&](size_t o2) { return (const int *)(D + o2); };
            for (int v = 0; v < NVK; ++v)
                if ((e2 = launch_vote_batched(vK[v], S, I(o_vote_sel[v]), I(o_vote_st[v]), (int)vote_sel[v].size(),
                                              vote_st[v].back(), T, p->n_vote, p->vote_seed, p->gamma_rank, p->beta,
                                              ls)) != hipSuccess)
                    return hip_fail(e2, "batched vote");
            if ((e2 = launch_fill_tau_sigma_batched(S, I(o_ref_sel), I(o_ref_st), (int)ref_sel.size(), ref_st.back(), T,
                                                    ls)) != hipSuccess)
                return hip_fail(e2, "batched thresholds");
        }
        for (size_t k = 0; k < P.classes.size(); ++k) {
            const int units = cls_start[k].back();
            if ((e2 = launch_filter_batched(C, P.classes[k], (const BatchItem *)(D + o_citems[k]), (int)cls_items[k].size(),
                                            (const int *)(D + o_cstart[k]), cls_lds[k], ctx->basis[C == 3], ctx->d_guard,
                                            d_q + 1 + k, std::min(grid, units), ls)) != hipSuccess)
                return hip_fail(e2, "batched filtering");
        }
        if ((e2 = launch_gather_batched(C, d_items, ni, (const int *)(D + o_pix), pix_start[ni], ls)) != hipSuccess)
            return hip_fail(e2, "batched aggregation");
        return HTSVD_OK;
    };
    s = enqueue();
    if (o.use_graph) {
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(ls, &g);
        ctx->timing = timing;
        if (s != HTSVD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (ee != hipSuccess) return hip_fail(ee, "end capture");
        hipGraphExec_t ex = nullptr;
        if ((e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "graph instantiate");
        }
        bc.graph = g;
        bc.exec = ex;
        bc.sig = sig;
        bc.valid = true;
        if ((e = hipGraphLaunch(ex, st)) != hipSuccess) return hip_fail(e, "graph launch");
    }
    return s;
}

htsvd_status htsvd_batch_inspect(htsvd_ctx *ctx, int32_t image, int32_t *h_K, double *d_tau_ref, void *stream) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    const BatchCache &bc = ctx->batch;
    if (bc.k_plan.empty()) return fail(HTSVD_ESTATE, "no batch has been planned on this context");
    if (image < 0 || image >= (int32_t)bc.k_plan.size()) return fail(HTSVD_EINVAL, "image index out of range");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (d_tau_ref &&
        (e = launch_scale_tau(bc.tau[image], d_tau_ref, bc.n_ref[image], bc.ksel[image], 16, bc.mul_alt, st)) !=
            hipSuccess)
        return hip_fail(e, "thresholds");
    if (h_K) {
        int k = bc.k_plan[image];
        if (bc.ksel[image]) {
            if ((e = hipMemcpyAsync(&k, bc.ksel[image], sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
                return hip_fail(e, "group size");
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronise");
        }
        *h_K = k;
    }
    return HTSVD_OK;
}

int32_t htsvd_ra_param_count(int32_t c) { return (c == 1 || c == 3) ? ra_param_count(c) : 0; }

htsvd_status htsvd_ra_set_weights(htsvd_ctx *ctx, int32_t c, const float *h_params, int64_t n) {
    if (!ctx || !h_params) return fail(HTSVD_EINVAL, "null argument");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    const int N = ra_param_count(c), P = 64 * c, H = ra_hidden(c);
    if (n != N) return fail(HTSVD_EINVAL, "wrong parameter count");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(h_params[i])) return fail(HTSVD_EINVAL, "parameters must be finite");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    RaState &r = ctx->ra[c == 3];
    if (!r.w) {
        void *q[8] = {};
        const size_t bytes[8] = {sizeof(float) * N, sizeof(float) * N, sizeof(float) * N, sizeof(float) * N,
                                 sizeof(uint16_t) * ra_frag_halves(c), sizeof(uint16_t) * 2 * P * H,
                                 sizeof(float) * (2 * H + P), sizeof(float) * P};
        for (int i = 0; i < 8; ++i)
            if (hipMalloc(&q[i], bytes[i]) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipFree(q[j]);
                (void)hipGetLastError();
                return fail(HTSVD_ENOMEM, "network allocation");
            }
        r.w = (float *)q[0];
        r.m = (float *)q[1];
        r.v = (float *)q[2];
        r.grad = (float *)q[3];
        r.frag = (uint16_t *)q[4];
        r.frag3t = (uint16_t *)q[5];
        r.bias = (float *)q[6];
        r.bias3t = (float *)q[7];
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise before network upload");
    if ((e = hipMemcpy(r.w, h_params, sizeof(float) * N, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(r.m, 0, sizeof(float) * N)) != hipSuccess || (e = hipMemset(r.v, 0, sizeof(float) * N)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(e, "network upload");
    r.n = N;
    r.step = 0;
    ++r.wgen;
    return HTSVD_OK;
}

htsvd_status htsvd_ra_get_weights(htsvd_ctx *ctx, int32_t c, float *h_params, int64_t n) {
    if (!ctx || !h_params) return fail(HTSVD_EINVAL, "null argument");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    RaState &r = ctx->ra[c == 3];
    if (r.n == 0) return fail(HTSVD_ESTATE, "no RA network set for this channel count");
    if (n != r.n) return fail(HTSVD_EINVAL, "wrong parameter count");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h_params, r.w, sizeof(float) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "network download");
    return HTSVD_OK;
}

htsvd_status htsvd_ra_means(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t c,
                            int64_t in_stride, const int32_t *d_idx, int32_t K, int64_t n_ref, float *d_means,
                            void *stream) {
    if (!ctx || !d_in || !d_idx || !d_means) return fail(HTSVD_EINVAL, "null argument");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    if (h < PS || w < PS) return fail(HTSVD_ESHAPE, "image smaller than one patch");
    if (in_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "in_stride < w*c");
    if (K < 1 || K > 64) return fail(HTSVD_EINVAL, "K must be in [1, 64]");
    if (n_ref < 0) return fail(HTSVD_EINVAL, "n_ref must be >= 0");
    hipError_t e = launch_ra_means(d_in, in_stride, h, w, c, d_idx, K, K, n_ref, d_means, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mean patches");
    return HTSVD_OK;
}

htsvd_status htsvd_ra_forward(htsvd_ctx *ctx, int32_t c, const float *d_means, int64_t n, float *d_r, void *stream) {
    if (!ctx || !d_means || !d_r) return fail(HTSVD_EINVAL, "null argument");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    if (n < 0) return fail(HTSVD_EINVAL, "n must be >= 0");
    htsvd_status s = ra_prepare(ctx, c, false);
    if (s != HTSVD_OK) return s;
    hipError_t e = launch_ra_forward(c, ra_dev(ctx->ra[c == 3]), false, d_means, nullptr, 0, 0, 0, nullptr, 0, 1, n,
                                     nullptr, 0.0, 0.0, nullptr, d_r, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "refinement network");
    return HTSVD_OK;
}

htsvd_status htsvd_ra_gradients(htsvd_ctx *ctx, int32_t c, const float *d_noisy, const float *d_clean, int32_t n,
                                float *d_grad, double *h_loss, void *stream) {
    return ra_grad_impl(ctx, c, d_noisy, d_clean, n, d_grad, h_loss, (hipStream_t)stream);
}

htsvd_status htsvd_ra_train_step(htsvd_ctx *ctx, int32_t c, const float *d_noisy, const float *d_clean, int32_t n,
                                 float lr, double *h_loss, void *stream) {
    if (!ctx) return fail(HTSVD_EINVAL, "null argument");
    if (!(lr > 0.f)) return fail(HTSVD_EINVAL, "lr must be > 0");
    if (c != 1 && c != 3) return fail(HTSVD_EINVAL, "c must be 1 or 3");
    RaState &r = ctx->ra[c == 3];
    hipStream_t st = (hipStream_t)stream;
    htsvd_status s = ra_grad_impl(ctx, c, d_noisy, d_clean, n, r.grad, h_loss, st);
    if (s != HTSVD_OK) return s;
    hipError_t e = ra_adam(r.w, r.m, r.v, r.grad, r.n, lr, ++r.step, st);
    if (e != hipSuccess) return hip_fail(e, "adam");
    ++r.wgen;
    return HTSVD_OK;
}

// Band-wise noise levels (Sec. IV-D): every band through the plain sub-image estimator alone,
// sigma_b the mean of its sub-images' estimates.  Scratch at `scratch` (band_sigma_bytes);
// synchronises the stream to return the levels on the host.
constexpr int BAND_SIGMA_UNITS = 4096;   // (sub-image, band) units per launch: 68 MB of moments

static size_t band_sigma_bytes(int h, int w, int B, int tile) {
    const int64_t units = (int64_t)((h + tile - 1) / tile) * ((w + tile - 1) / tile) * B;
    return align256(sizeof(double) * units) +
           align256(sizeof(int32_t) * sigma_mom_ints() * std::min<int64_t>(units, BAND_SIGMA_UNITS));
}

// The cube is estimated as one B-channel image: unit t*B + b is band b of sub-image t, the same
// moments and eigenvalues as the band's plane alone, in launches of at most BAND_SIGMA_UNITS.
static htsvd_status band_sigmas(const uint8_t *d_in, int h, int w, int B, int64_t in_stride, int tile, void *scratch,
                         std::vector<double> &sig, hipStream_t st) {
    const int64_t n_tiles = (int64_t)((h + tile - 1) / tile) * ((w + tile - 1) / tile), units = n_tiles * B;
    double *s2 = (double *)scratch;
    int32_t *mom = (int32_t *)((char *)scratch + align256(sizeof(double) * units));
    ImageGeom g{};
    g.img = d_in;
    g.stride = in_stride;
    g.h = h;
    g.w = w;
    g.c = B;
    for (int64_t u0 = 0; u0 < units; u0 += BAND_SIGMA_UNITS) {
        const int n = (int)std::min<int64_t>(BAND_SIGMA_UNITS, units - u0);
        hipError_t e = launch_sigma2_units(g, tile, (int)u0, n, mom, s2 + u0, st);
        if (e != hipSuccess) return hip_fail(e, "band noise estimate");
    }
    std::vector<double> h_s2((size_t)units);
    hipError_t e;
    if ((e = hipMemcpyAsync(h_s2.data(), s2, sizeof(double) * h_s2.size(), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(e, "band noise download");
    sig.assign(B, 0.0);
    for (int k = 0; k < B; ++k) {
        double acc = 0.0;
        for (int64_t t = 0; t < n_tiles; ++t) {
            const double v = h_s2[(size_t)t * B + k];
            acc += v > 0.0 ? std::sqrt(v) : 0.0;
        }
        sig[k] = acc / (double)n_tiles;
    }
    return HTSVD_OK;
}

htsvd_status htsvd_band_sigma(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t bands,
                              int64_t in_stride, double *h_sigma, void *stream) {
    if (!ctx || !d_in || !h_sigma) return fail(HTSVD_EINVAL, "null argument");
    if (bands < 1 || bands > MAX_BANDS) return fail(HTSVD_EINVAL, "bands must be in [1, 64]");
    if (h < PS || w < PS) return fail(HTSVD_ESHAPE, "cube smaller than one patch");
    if (in_stride < (int64_t)w * bands) return fail(HTSVD_EINVAL, "in_stride < w*bands");
    if ((int64_t)h * w > (int64_t)1 << 30) return fail(HTSVD_ENOTSUP, "cube larger than 2^30 pixels");
    htsvd_status s = ensure_ws(ctx, band_sigma_bytes(h, w, bands, 128));
    if (s != HTSVD_OK) return s;
    std::vector<double> sig;
    if ((s = band_sigmas(d_in, h, w, bands, in_stride, 128, ctx->ws, sig, (hipStream_t)stream)) != HTSVD_OK) return s;
    memcpy(h_sigma, sig.data(), sizeof(double) * bands);
    return HTSVD_OK;
}

htsvd_status htsvd_band_guide(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t bands,
                              int64_t in_stride, uint8_t *d_guide, void *stream) {
    if (!ctx || !d_in || !d_guide) return fail(HTSVD_EINVAL, "null argument");
    if (bands < 1 || bands > MAX_BANDS) return fail(HTSVD_EINVAL, "bands must be in [1, 64]");
    if (h < 1 || w < 1) return fail(HTSVD_ESHAPE, "empty image");
    if (in_stride < (int64_t)w * bands) return fail(HTSVD_EINVAL, "in_stride < w*bands");
    hipError_t e = launch_band_guide(d_in, in_stride, h, w, bands, d_guide, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "band guide");
    return HTSVD_OK;
}

htsvd_status htsvd_set_band_memory(htsvd_ctx *ctx, int64_t bytes) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (bytes < ((int64_t)1 << 20)) return fail(HTSVD_EINVAL, "the band memory cap must be at least 1 MiB");
    ctx->band_cap = bytes;
    return HTSVD_OK;
}

htsvd_status htsvd_denoise_bands(htsvd_ctx *ctx, const uint8_t *d_in, int32_t h, int32_t w, int32_t bands,
                                 int64_t in_stride, float sigma, const htsvd_params *p, float *d_out,
                                 int64_t out_stride, void *stream) {
    if (!ctx || !d_in || !d_out || !p) return fail(HTSVD_EINVAL, "null argument");
    if (bands < 2 || bands > MAX_BANDS || bands == 3) return fail(HTSVD_EINVAL, "bands must be 2 or 4 .. 64");
    if (ctx->bands != bands) return fail(HTSVD_ESTATE, "no basis set for this band count");
    if (in_stride < (int64_t)w * bands) return fail(HTSVD_EINVAL, "in_stride < w*bands");
    if (out_stride < (int64_t)w * bands) return fail(HTSVD_EINVAL, "out_stride < w*bands");
    if ((!(sigma > 0.f) && sigma != HTSVD_SIGMA_AUTO) || !std::isfinite(sigma))
        return fail(HTSVD_EINVAL, "sigma must be > 0 or AUTO");
    if (p->adaptive || p->ra) return fail(HTSVD_ENOTSUP, "the band path takes no vote or refinement");
    const bool auto_sigma = sigma == HTSVD_SIGMA_AUTO;
    // the grouping checks run on the guide's geometry (one channel)
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate(ctx, d_in, h, w, 1, w, p, &g, &mp, false);
    if (s != HTSVD_OK) return s;
    const int64_t n_ref = (int64_t)g.ny * g.nx;
    const size_t off_idx = align256((size_t)h * w);
    const size_t off_ws = off_idx + align256(sizeof(int32_t) * n_ref * mp.K);
    const size_t off_auto = off_ws + align256(band_ws_bytes(h, w, bands, mp.K, n_ref, ctx->band_cap));
    const size_t off_sel = off_auto + align256(sizeof(float) * (size_t)h * w * bands);
    const size_t off_sig = off_sel + 256;
    if ((s = ensure_ws(ctx, auto_sigma ? off_sig + band_sigma_bytes(h, w, bands, p->subimage) : off_auto)) != HTSVD_OK)
        return s;
    uint8_t *guide = (uint8_t *)ctx->ws;
    int32_t *idx = (int32_t *)((char *)ctx->ws + off_idx);
    hipStream_t st = (hipStream_t)stream;
    // Band-wise noise levels (Sec. IV-D): the cube is filtered at the mean level sigma_mean; bands
    // estimated above 2 sigma_mean take the output filtered at the highest band level instead.
    double s_lo = sigma, s_hi = sigma;
    std::vector<uint8_t> severe(bands, 0);
    bool any_severe = false;
    if (auto_sigma) {
        std::vector<double> sig;
        if ((s = band_sigmas(d_in, h, w, bands, in_stride, p->subimage, (char *)ctx->ws + off_sig, sig, st)) !=
            HTSVD_OK)
            return s;
        double mean = 0.0;
        s_hi = 0.0;
        for (int k = 0; k < bands; ++k) {
            mean += sig[k] / bands;
            s_hi = std::max(s_hi, sig[k]);
        }
        s_lo = mean;
        for (int k = 0; k < bands; ++k) {
            severe[k] = sig[k] > 2.0 * mean;
            any_severe = any_severe || severe[k];
        }
    }
    hipError_t e = launch_band_guide(d_in, in_stride, h, w, bands, guide, st);
    if (e != hipSuccess) return hip_fail(e, "band guide");
    g.img = guide;
    {
        StageScope sc(ctx, HTSVD_STAGE_BM, st);
        if ((e = launch_block_match(g, mp, idx, nullptr, st)) != hipSuccess) return hip_fail(e, "block matching");
    }
    const double mult = p->tau_mult > 0.0 ? p->tau_mult : std::sqrt(2.0 * std::log((double)bands * mp.K * PS * PS));
    BandMaps bm;
    bm.nb = band_nb(bands);
    bm.D = ctx->d_band_maps;
    bm.Dinv = bm.D + bm.nb * bm.nb;
    bm.frag_fwd = bm.Dinv + bm.nb * bm.nb;
    bm.frag_inv = bm.frag_fwd + (size_t)(bands / 2 + 1) * 512;
    {
        StageScope sc(ctx, HTSVD_STAGE_FILTER, st);
        if ((e = launch_band_filter(bm, d_in, in_stride, h, w, bands, idx, n_ref, mp.K, s_lo * mult, ctx->band_cap,
                                    (char *)ctx->ws + off_ws, d_out, out_stride, st)) != hipSuccess)
            return hip_fail(e, "band filter");
        if (any_severe) {
            float *alt = (float *)((char *)ctx->ws + off_auto);
            uint8_t *sel = (uint8_t *)ctx->ws + off_sel;
            if ((e = launch_band_filter(bm, d_in, in_stride, h, w, bands, idx, n_ref, mp.K, s_hi * mult,
                                        ctx->band_cap, (char *)ctx->ws + off_ws, alt, (int64_t)w * bands, st)) !=
                    hipSuccess ||
                (e = hipMemcpyAsync(sel, severe.data(), bands, hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = launch_select_bands(alt, (int64_t)w * bands, sel, h, w, bands, d_out, out_stride, st)) !=
                    hipSuccess)
                return hip_fail(e, "band filter at the highest level");
            // the host vector must outlive the asynchronous copy
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "band selection");
        }
    }
    return HTSVD_OK;
}

// Checks of the video calls: frame geometry and method parameters as for one image, then the
// frame count, the temporal radius and the size of the stacked frames.
static htsvd_status validate_video(htsvd_ctx *ctx, const uint8_t *d_in, int32_t T, int32_t h, int32_t w, int32_t c,
                            int64_t in_stride, int32_t radius, const htsvd_params *p, ImageGeom *g, MethodParams *mp,
                            bool need_basis) {
    htsvd_status s = validate(ctx, d_in, h, w, c, in_stride, p, g, mp, need_basis);
    if (s != HTSVD_OK) return s;
    if (T < 1) return fail(HTSVD_ESHAPE, "a video needs at least one frame");
    if (radius < 0 || radius > 31) return fail(HTSVD_EINVAL, "radius must be in [0, 31]");
    if ((int64_t)T * h * w > (int64_t)1 << 30) return fail(HTSVD_ENOTSUP, "video larger than 2^30 pixels");
    return HTSVD_OK;
}

htsvd_status htsvd_block_match_video(htsvd_ctx *ctx, const uint8_t *d_in, int32_t T, int32_t h, int32_t w,
                                     int32_t c, int64_t in_stride, int32_t radius, const htsvd_params *p,
                                     int32_t *d_idx, int32_t *d_dist, void *stream) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate_video(ctx, d_in, T, h, w, c, in_stride, radius, p, &g, &mp, false);
    if (s != HTSVD_OK) return s;
    if (!d_idx) return fail(HTSVD_EINVAL, "null index output");
    hipError_t e = launch_block_match_video(g, mp, T, radius, d_idx, d_dist, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "spatio-temporal block matching");
    return HTSVD_OK;
}

htsvd_status htsvd_denoise_video(htsvd_ctx *ctx, const uint8_t *d_in, int32_t T, int32_t h, int32_t w, int32_t c,
                                 int64_t in_stride, int32_t radius, float sigma, const htsvd_params *p, float *d_out,
                                 int64_t out_stride, void *stream) {
    ImageGeom g;
    MethodParams mp;
    htsvd_status s = validate_video(ctx, d_in, T, h, w, c, in_stride, radius, p, &g, &mp, true);
    if (s != HTSVD_OK) return s;
    if (!d_out) return fail(HTSVD_EINVAL, "null output");
    if (out_stride < (int64_t)w * c) return fail(HTSVD_EINVAL, "out_stride < w*c");
    if (!(sigma > 0.f) && sigma != HTSVD_SIGMA_AUTO) return fail(HTSVD_EINVAL, "sigma must be > 0 or AUTO");
    if (!std::isfinite(sigma)) return fail(HTSVD_EINVAL, "sigma must be finite");
    if (p->estimator != 0 && p->estimator != 1) return fail(HTSVD_EINVAL, "estimator must be 0 or 1");
    const bool learned = sigma == HTSVD_SIGMA_AUTO && p->estimator == 1;
    // thresholds from each frame's own noise estimate (and vote), as for one image
    const bool per_frame = !(sigma > 0.f && !p->adaptive);
    const int tile = p->subimage;
    // The stacked frames as one image whose reference grid is T*ny x nx (frame-major).
    ImageGeom gv = g;
    gv.h = T * h;
    gv.ny = T * g.ny;
    const int64_t n_frame = (int64_t)g.ny * g.nx, n_ref = (int64_t)gv.ny * gv.nx, npx = (int64_t)gv.h * w;
    const size_t off_tau = align256(sizeof(int32_t) * n_ref * mp.K);
    const size_t off_acc = off_tau + align256(sizeof(double) * n_ref);
    const size_t off_hist = off_acc + align256(filter_mfma_global_bytes(gv, T, radius, mp.W, mp.K));
    const size_t off_ra = off_hist + align256(sizeof(int) * npx);
    const size_t off_frame = off_ra + (p->ra ? align256(ra_ws_bytes(gv)) : 0);
    const size_t frame_ws = per_frame ? plan_ws(nullptr, g, mp.W, mp.K, tile).total : 0;
    if ((s = ensure_ws(ctx, off_frame + frame_ws)) != HTSVD_OK) return s;
    char *ws = (char *)ctx->ws;
    int32_t *idx = (int32_t *)ws;
    double *tau = (double *)(ws + off_tau);
    void *accum = ws + off_acc;
    int *ghist = (int *)(ws + off_hist);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    {
        StageScope sc(ctx, HTSVD_STAGE_BM, st);
        if ((e = launch_block_match_video(g, mp, T, radius, idx, nullptr, st)) != hipSuccess)
            return hip_fail(e, "spatio-temporal block matching");
    }
    const double mult = p->tau_mult > 0.0 ? p->tau_mult : default_mult(c, mp.K);
    if (!per_frame) {
        if ((e = launch_fill_tau(tau, n_ref, nullptr, (double)sigma, mult, gv, tile, st)) != hipSuccess)
            return hip_fail(e, "tau");
    } else {
        // frame by frame: the noise estimate of the frame's sub-images, adjusted by the vote over
        // the frame's own (spatial) groups, gives the thresholds of its references
        for (int t = 0; t < T; ++t) {
            ImageGeom gt = g;
            gt.img = d_in + (int64_t)t * h * in_stride;
            Ws wt = plan_ws(ws + off_frame, gt, mp.W, mp.K, tile);
            const float *zmap = nullptr;
            if (learned && (s = run_cnn_map(ctx, gt, st, &zmap)) != HTSVD_OK) return s;
            if ((s = run_bm(ctx, gt, mp, wt, st)) != HTSVD_OK) return s;
            if ((s = run_sigma(ctx, gt, mp, p, sigma, wt, zmap, st)) != HTSVD_OK) return s;
            if (learned)
                e = launch_fill_tau_learned(tau + t * n_frame, gt, tile, zmap, wt.use_plain, wt.sig_est, wt.sig_hat,
                                            mult, st);
            else
                e = launch_fill_tau(tau + t * n_frame, n_frame, wt.sig_hat, 0.0, mult, gt, tile, st);
            if (e != hipSuccess) return hip_fail(e, "tau");
        }
    }
    const float *ra_d = nullptr;
    const uint8_t *ra_f = nullptr;
    if (p->ra) {
        Ws wv{};
        wv.idx = idx;
        if ((s = run_ra(ctx, gv, mp, wv, tau, ws + off_ra, mult, p->ra_sigma, st, &ra_d, &ra_f)) != HTSVD_OK) return s;
    }
    {
        StageScope sc(ctx, HTSVD_STAGE_CLEAR, st);
        if ((e = launch_zero(ctx->d_guard, 2 * sizeof(unsigned long long), st)) != hipSuccess ||
            (e = launch_zero(ghist, sizeof(int) * npx, st)) != hipSuccess)
            return hip_fail(e, "zero accumulators");
    }
    {
        StageScope sc(ctx, HTSVD_STAGE_FILTER, st);
        if ((e = launch_filter_mfma_global(gv, T, radius, mp.W, mp.K, ctx->basis[c == 3], idx, tau, accum, ghist,
                                           ctx->d_guard, d_out, out_stride, st, ra_d, ra_f)) != hipSuccess)
            return hip_fail(e, "video filter");
    }
    return HTSVD_OK;
}

htsvd_status htsvd_sync(htsvd_ctx *ctx, void *stream) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronise");
    return HTSVD_OK;
}

const char *htsvd_last_error(void) { return g_err.c_str(); }

htsvd_status htsvd_set_timing(htsvd_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(HTSVD_EINVAL, "null context");
    if (enable && !ctx->ev[0]) {
        for (int i = 0; i < 2 * HTSVD_N_STAGES; ++i) {
            hipError_t e = hipEventCreate(&ctx->ev[i]);
            if (e != hipSuccess) return hip_fail(e, "event creation");
        }
    }
    for (int s = 0; s < HTSVD_N_STAGES; ++s) {
        ctx->ev_pending[s] = false;
        ctx->stage_ms[s] = 0.0;
        ctx->stage_calls[s] = 0;
    }
    ctx->timing = enable != 0;
    return HTSVD_OK;
}

htsvd_status htsvd_stage_times(htsvd_ctx *ctx, double *h_ms, int64_t *h_calls) {
    if (!ctx || !h_ms) return fail(HTSVD_EINVAL, "null argument");
    for (int s = 0; s < HTSVD_N_STAGES; ++s) {
        harvest(ctx, s);
        h_ms[s] = ctx->stage_ms[s];
        if (h_calls) h_calls[s] = ctx->stage_calls[s];
    }
    return HTSVD_OK;
}

htsvd_status htsvd_last_guard_count(htsvd_ctx *ctx, int64_t *h_count) {
    if (!ctx || !h_count) return fail(HTSVD_EINVAL, "null argument");
    unsigned long long v[2];
    hipError_t e = hipMemcpy(v, ctx->d_guard, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "counter copy");
    h_count[0] = (int64_t)v[0];
    h_count[1] = (int64_t)v[1];
    return HTSVD_OK;
}

}  // extern "C"
