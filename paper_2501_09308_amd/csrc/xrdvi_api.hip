// C ABI of the single-analysis path: context, problem, tape, profile,
// window plan, ELBO forward (+ fused adjoint) and gradient.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "xrdvi.h"
#include "xrdvi_internal.h"

using namespace xrdvi;

struct xrdvi_ctx {
    int device = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // measurement: events around fused launches
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

struct xrdvi_problem {
    xrdvi_ctx *ctx = nullptr;
    int device = 0;           // destroy never dereferences ctx
    ProbDev P{};
    void *mem = nullptr;
    int *perm = nullptr;      // device: sorted peak -> caller's peak index
};

struct xrdvi_tape {
    const xrdvi_problem *prob = nullptr;
    int device = 0;           // destroy never dereferences prob
    StepDev st{};
    void *mem = nullptr;
    double *zeros = nullptr;  // D K zeros (mean and log-scale of a position)
    bool has_grad = false;
};

namespace xrdvi {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t step_bytes(const StepShape &sh) {
    const size_t S = sh.S, K = sh.K, D = (size_t)sh.D * K;
    const size_t NS = num_sums(sh.D), nt = sh.ntiles;
    const size_t kb = (K + kWave - 1) / kWave;
    const bool asym = sh.D == 5;
    size_t b = 0;
    b += align256(sizeof(double) * S * D);          // eps
    b += align256(sizeof(double) * S * D);          // phi
    b += align256(sizeof(float4) * S * K);          // pk
    b += align256(asym ? sizeof(float) * S * K : 4);  // pkr
    b += align256(sizeof(double) * S * K);          // lpj
    b += align256(sizeof(double) * S * kb);         // lpb
    b += 2 * align256(sizeof(int) * S * (size_t)std::max(sh.T, 1));  // lo, hi
    b += align256(sizeof(double) * S * nt);         // llp
    b += align256(sh.dense ? sizeof(float) * NS * nt * K * S : 4);  // part
    b += align256(sizeof(double) * D);              // sd
    // tile ranges: dense mode only (windowed tiles find their own)
    b += align256(sh.dense ? sizeof(int4) * S * nt * K : 4);            // rng
    b += align256(sh.dense && asym ? sizeof(int2) * S * nt * K : 4);    // rng2
    b += align256(sizeof(float) * S * (size_t)sh.N);  // rres
    b += align256(sizeof(double) * NS * K * S);     // pw
    b += align256(sh.sec ? sizeof(float4) * S * (size_t)std::max(sh.T, 1) : 4);  // psec
    const bool cand = !sh.dense && !sh.sec;
    b += align256(cand ? sizeof(int2) * nt * K : 4);                      // cab
    b += align256(cand ? sizeof(double) * kCandKeep * nt * K : 4);        // cp
    b += align256(cand ? sizeof(double4) * K : 4);                        // cext
    return b;
}

StepDev carve_step(void *base, const StepShape &sh) {
    char *p = static_cast<char *>(base);
    const size_t S = sh.S, K = sh.K, D = (size_t)sh.D * K;
    const size_t NS = num_sums(sh.D), nt = sh.ntiles;
    const size_t kb = (K + kWave - 1) / kWave;
    const bool asym = sh.D == 5;
    auto take = [&](size_t bytes) { char *r = p; p += align256(bytes); return r; };
    StepDev st{};
    st.S = sh.S;
    st.eps = (double *)take(sizeof(double) * S * D);
    st.phi = (double *)take(sizeof(double) * S * D);
    st.pk = (float4 *)take(sizeof(float4) * S * K);
    st.pkr = (float *)take(asym ? sizeof(float) * S * K : 4);
    st.lpj = (double *)take(sizeof(double) * S * K);
    st.lpb = (double *)take(sizeof(double) * S * kb);
    st.lo = (int *)take(sizeof(int) * S * (size_t)std::max(sh.T, 1));
    st.hi = (int *)take(sizeof(int) * S * (size_t)std::max(sh.T, 1));
    st.llp = (double *)take(sizeof(double) * S * nt);
    st.part = (float *)take(sh.dense ? sizeof(float) * NS * nt * K * S : 4);
    st.sd = (double *)take(sizeof(double) * D);
    st.rng = (int4 *)take(sh.dense ? sizeof(int4) * S * nt * K : 4);
    st.rng2 = (int2 *)take(sh.dense && asym ? sizeof(int2) * S * nt * K : 4);
    st.rres = (float *)take(sizeof(float) * S * (size_t)sh.N);
    st.pw = (double *)take(sizeof(double) * NS * K * S);
    st.psec = (float4 *)take(sh.sec ? sizeof(float4) * S * (size_t)std::max(sh.T, 1) : 4);
    const bool cand = !sh.dense && !sh.sec;
    st.cab = (int2 *)take(cand ? sizeof(int2) * nt * K : 4);
    st.cp = (double *)take(cand ? sizeof(double) * kCandKeep * nt * K : 4);
    st.cext = (double4 *)take(cand ? sizeof(double4) * K : 4);
    if (!cand) st.cab = nullptr;
    return st;
}

// Device layout of a prepared problem, in 256-byte aligned pieces.
struct ProblemLayout {
    size_t x, y, bg, lgy, u, ul, off, ph, pos, inten, pt, ptl, perm, ptab, total;
};

static ProblemLayout problem_layout(int N, int K, int T) {
    const int nt = num_tiles(N);
    const size_t T1 = (size_t)std::max(T, 1);
    ProblemLayout L{};
    size_t o = 0;
    auto slot = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    L.x = slot(8 * (size_t)N); L.y = slot(8 * (size_t)N);
    L.bg = slot(8 * (size_t)N); L.lgy = slot(8 * (size_t)N);
    L.u = slot(4 * (size_t)nt * kTile); L.ul = slot(4 * (size_t)nt * kTile);
    L.off = slot(4 * (size_t)(K + 1));
    L.ph = slot(4 * T1); L.pos = slot(8 * T1); L.inten = slot(4 * T1);
    L.pt = slot(4 * (size_t)nt * T1); L.ptl = slot(4 * (size_t)nt * T1);
    L.perm = slot(4 * T1);
    L.ptab = slot(4 * (size_t)K * (kTabBuckets + 1));
    L.total = o;
    return L;
}

size_t problem_bytes(int N, int K, int T) { return problem_layout(N, K, T).total; }

hipError_t upload_problem(const xrdvi_problem_desc &d, double lambda,
                          char *base, ProbDev &P, int **perm_out,
                          hipStream_t stream) {
    const int N = d.N, K = d.K, T = d.peak_off[K];
    const int T1 = std::max(T, 1);
    const ProblemLayout L = problem_layout(N, K, T);
    // peaks ordered by position within each phase (stable)
    std::vector<int> perm(T1, 0), phase(T1, 0);
    std::vector<double> pos(T1, 0.0);
    std::vector<float> inten(T1, 0.f);
    for (int k = 0; k < K; ++k) {
        const int a = d.peak_off[k], b = d.peak_off[k + 1];
        std::iota(perm.begin() + a, perm.begin() + b, a);
        std::stable_sort(perm.begin() + a, perm.begin() + b, [&](int i, int j) {
            return d.peak_pos[i] < d.peak_pos[j];
        });
        for (int j = a; j < b; ++j) {
            phase[j] = k;
            pos[j] = d.peak_pos[perm[j]];
            inten[j] = (float)d.peak_int[perm[j]];
        }
    }
    // position index per phase: first sorted peak at or after each of
    // kTabBuckets + 1 equally spaced positions spanning the grid
    const double tab_x0 = d.x[0];
    const double tab_inv = N > 1 ? kTabBuckets / (d.x[N - 1] - d.x[0]) : 0.0;
    std::vector<int> ptab((size_t)K * (kTabBuckets + 1));
    for (int k = 0; k < K; ++k) {
        const int a = d.peak_off[k], b = d.peak_off[k + 1];
        int j = a;
        for (int bb = 0; bb <= kTabBuckets; ++bb) {
            const double v = tab_inv > 0.0 ? tab_x0 + bb / tab_inv : tab_x0;
            while (j < b && pos[j] < v) ++j;
            ptab[(size_t)k * (kTabBuckets + 1) + bb] = j;
        }
    }
    auto up = [&](size_t o, const void *src, size_t bytes) {
        return hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, stream);
    };
    hipError_t e = up(L.x, d.x, 8 * (size_t)N);
    if (e == hipSuccess) e = up(L.y, d.y, 8 * (size_t)N);
    if (e == hipSuccess) e = up(L.bg, d.bg, 8 * (size_t)N);
    if (e == hipSuccess) e = up(L.off, d.peak_off, 4 * (size_t)(K + 1));
    if (e == hipSuccess) e = up(L.ph, phase.data(), 4 * (size_t)T1);
    if (e == hipSuccess) e = up(L.pos, pos.data(), 8 * (size_t)T1);
    if (e == hipSuccess) e = up(L.inten, inten.data(), 4 * (size_t)T1);
    if (e == hipSuccess) e = up(L.perm, perm.data(), 4 * (size_t)T1);
    if (e == hipSuccess) e = up(L.ptab, ptab.data(), 4 * ptab.size());
    // pageable sources: complete the copies before the vectors go away
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    P = ProbDev{};
    P.N = N; P.K = K; P.T = T; P.ntiles = num_tiles(N);
    P.D = latent_types(d);
    P.sec = d.width_law;
    P.cutoff = d.cutoff;
    P.x0 = d.x[0];
    P.inv_dx = N > 1 ? (double)(N - 1) / (d.x[N - 1] - d.x[0]) : 0.0;
    P.dx = N > 1 ? (d.x[N - 1] - d.x[0]) / (double)(N - 1) : 0.0;
    P.uniform = 1;
    for (int i = 1; i < N; ++i)
        if (!(std::fabs(d.x[i] - std::fma((double)i, P.dx, d.x[0])) <= 1e-9 * P.dx)) {
            P.uniform = 0;
            break;
        }
    P.formed_x = P.uniform && (P.sec || P.D == 5 || P.cutoff <= kF32Cutoff) ? 1 : 0;
    P.lambda = lambda;
    P.mu_sd = d.prior.mu_sd;
    P.w_shape = d.prior.w_shape;
    P.w_rate = d.prior.w_rate;
    P.c_h = std::log(lambda);
    P.c_mu = -std::log(d.prior.mu_sd) - 0.5 * std::log(2.0 * M_PI);
    P.c_w = d.prior.w_shape * std::log(d.prior.w_rate) - std::lgamma(d.prior.w_shape);
    if (P.D == 5) {
        P.a_mean = d.prior.alpha_mean;
        P.a_sd = d.prior.alpha_sd;
        P.c_a = -std::log(d.prior.alpha_sd) - 0.5 * std::log(2.0 * M_PI);
    }
    P.x = (const double *)(base + L.x);
    P.y = (const double *)(base + L.y);
    P.bg = (const double *)(base + L.bg);
    P.lgy = (const double *)(base + L.lgy);
    P.u = (const float *)(base + L.u);
    P.ul = (const float *)(base + L.ul);
    P.off = (const int *)(base + L.off);
    P.phase = (const int *)(base + L.ph);
    P.pos = (const double *)(base + L.pos);
    P.inten = (const float *)(base + L.inten);
    P.pt = (const float *)(base + L.pt);
    P.ptl = (const float *)(base + L.ptl);
    P.ptab = (const int *)(base + L.ptab);
    P.tab_x0 = tab_x0;
    P.tab_inv = tab_inv;
    if (perm_out) *perm_out = (int *)(base + L.perm);
    return launch_prepare(P, (double *)(base + L.lgy), (float *)(base + L.u),
                          (float *)(base + L.ul), (float *)(base + L.pt),
                          (float *)(base + L.ptl), stream);
}

}  // namespace xrdvi

// ---- scratch of the allocation-free profile entry ------------------------
//
// xrdvi_profile_static keeps its per-call state (phase constants, window
// plan, tile ranges, per-tile likelihoods) in this file-scope device array
// instead of the context workspace.  Each GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device memory: host code uses the per-device address
// that hipGetSymbolAddress returns (looked up once per device, with that
// device current, by xrdvi_ctx_create).
namespace xrdvi {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;   // 64 MiB
constexpr int kMaxDevices = 64;
}  // namespace xrdvi

static __device__ __align__(256) unsigned char scratch[xrdvi::kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[xrdvi::kMaxDevices] = {};

// Device address of this device's scratch (the current device must be
// `dev`); looked up on the first call per device.
hipError_t static_scratch_lookup(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

void *static_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

}  // namespace

namespace {

struct DeviceGuard {
    int old = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old)
            (void)hipSetDevice(old);
    }
};

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(XRDVI_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

// Host validation of a problem description; resolves lambda_h.
int validate_desc(const xrdvi_problem_desc *d, double *lambda_out,
                  double *ymax_out = nullptr) {
    if (!d) return fail(XRDVI_EINVAL, "problem description is NULL");
    if (d->N < 1) return fail(XRDVI_EINVAL, "N must be >= 1");
    if (d->K < 1) return fail(XRDVI_EINVAL, "K must be >= 1");
    if (!d->x || !d->y || !d->bg || !d->peak_off)
        return fail(XRDVI_EINVAL, "x, y, bg and peak_off must be non-NULL");
    for (int i = 0; i < d->N; ++i) {
        const double x = d->x[i];
        if (!std::isfinite(x) || !(x > 0.0) || !(x < 180.0))
            return fail(XRDVI_EINVAL, "x must be finite and inside (0, 180)");
        if (i > 0 && !(x > d->x[i - 1]))
            return fail(XRDVI_EINVAL, "x must be strictly ascending");
        if (!std::isfinite(d->y[i]) || d->y[i] < 0.0)
            return fail(XRDVI_EINVAL, "y must be finite and >= 0");
        if (!std::isfinite(d->bg[i]) || !(d->bg[i] > 0.0))
            return fail(XRDVI_EINVAL, "bg must be finite and > 0");
    }
    if (d->peak_off[0] != 0) return fail(XRDVI_EINVAL, "peak_off[0] must be 0");
    for (int k = 0; k < d->K; ++k)
        if (d->peak_off[k + 1] < d->peak_off[k])
            return fail(XRDVI_EINVAL, "peak_off must be non-decreasing");
    const int T = d->peak_off[d->K];
    if (T > 0 && (!d->peak_pos || !d->peak_int))
        return fail(XRDVI_EINVAL, "peak_pos and peak_int must be non-NULL");
    for (int j = 0; j < T; ++j) {
        if (!std::isfinite(d->peak_pos[j]))
            return fail(XRDVI_EINVAL, "peak_pos must be finite");
        const double I = d->peak_int[j];
        if (!std::isfinite(I) || I < 0.0 || I > 1.0)
            return fail(XRDVI_EINVAL, "peak_int must lie in [0, 1]");
    }
    if (!std::isfinite(d->cutoff) || d->cutoff < 0.0)
        return fail(XRDVI_EINVAL, "cutoff must be finite and >= 0");
    const xrdvi_prior &pr = d->prior;
    if (!std::isfinite(pr.lambda_h) || pr.lambda_h < 0.0)
        return fail(XRDVI_EINVAL, "prior.lambda_h must be >= 0");
    if (!(pr.mu_sd > 0.0) || !std::isfinite(pr.mu_sd))
        return fail(XRDVI_EINVAL, "prior.mu_sd must be > 0");
    if (!(pr.w_shape > 0.0) || !(pr.w_rate > 0.0) || !std::isfinite(pr.w_shape)
        || !std::isfinite(pr.w_rate))
        return fail(XRDVI_EINVAL, "prior.w_shape and prior.w_rate must be > 0");
    if (d->asymmetric != 0 && d->asymmetric != 1)
        return fail(XRDVI_EINVAL, "asymmetric must be 0 or 1");
    if (d->asymmetric && (!std::isfinite(pr.alpha_mean) || !(pr.alpha_sd > 0.0)
                          || !std::isfinite(pr.alpha_sd)))
        return fail(XRDVI_EINVAL,
                    "prior.alpha_mean must be finite and prior.alpha_sd > 0");
    if (d->width_law != 0 && d->width_law != 1)
        return fail(XRDVI_EINVAL, "width_law must be 0 or 1");
    if (d->width_law == 1)
        for (int j = 0; j < T; ++j)
            if (!(d->peak_pos[j] > 0.0) || !(d->peak_pos[j] < 180.0))
                return fail(XRDVI_EINVAL,
                            "peak_pos must lie inside (0, 180) with width_law 1");
    double lam = pr.lambda_h;
    double m = -INFINITY;
    for (int i = 0; i < d->N; ++i) m = std::max(m, d->y[i] - d->bg[i]);
    if (lam == 0.0) {
        if (!(m > 0.0))
            return fail(XRDVI_EINVAL,
                        "max(y - bg) must be > 0 when prior.lambda_h = 0");
        lam = 1.0 / m;
    }
    if (lambda_out) *lambda_out = lam;
    if (ymax_out) *ymax_out = m;
    return XRDVI_OK;
}

hipEvent_t take_event(xrdvi_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launches the fused kernel, bracketed by events when timing is enabled.
hipError_t timed_fused(xrdvi_ctx *ctx, const ProbDev &P, const StepDev &st,
                       bool grad, float *f_out, hipStream_t s) {
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
        a = take_event(ctx);
        b = take_event(ctx);
        if (a && b) (void)hipEventRecord(a, s);
    }
    hipError_t e = launch_fused(P, st, grad, f_out, s);
    if (ctx->timing && a && b) {
        (void)hipEventRecord(b, s);
        ctx->ev_pending.emplace_back(a, b);
    }
    return e;
}

bool ensure_ws(xrdvi_ctx *ctx, size_t bytes, int *rc) {
    if (ctx->ws_bytes >= bytes) return true;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && ctx->ws) e = hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (e == hipSuccess) e = hipMalloc(&ctx->ws, bytes);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        *rc = fail(XRDVI_ENOMEM, std::string("workspace allocation: ") +
                                     hipGetErrorString(e));
        return false;
    }
    ctx->ws_bytes = bytes;
    return true;
}

}  // namespace

int xrdvi::validate_problem(const xrdvi_problem_desc *d, double *lambda_out,
                            double *ymax) {
    return validate_desc(d, lambda_out, ymax);
}

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                                  \
    }                                                                  \
    catch (const std::bad_alloc &) {                                   \
        return fail(XRDVI_ENOMEM, "host allocation failed");           \
    }                                                                  \
    catch (...) {                                                      \
        return fail(XRDVI_EDEVICE, "unexpected internal exception");   \
    }

extern "C" {

const char *xrdvi_last_error(void) { return g_err.c_str(); }

int xrdvi_version(void) { return 1; }

int xrdvi_validate(const xrdvi_problem_desc *desc) {
    API_GUARD_BEGIN
    return validate_desc(desc, nullptr);
    API_GUARD_END
}

int xrdvi_ctx_create(int device, xrdvi_ctx **out) {
    API_GUARD_BEGIN
    if (!out) return fail(XRDVI_EINVAL, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(XRDVI_EINVAL, "device index out of range");
    if (device >= kMaxDevices)
        return fail(XRDVI_EINVAL, "device index beyond the library's 64-device table");
    {
        DeviceGuard g(device);
        void *ptr = nullptr;
        HIP_TRY(static_scratch_lookup(device, &ptr), "static scratch address");
    }
    auto *c = new xrdvi_ctx();
    c->device = device;
    *out = c;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_ctx_destroy(xrdvi_ctx *ctx) {
    API_GUARD_BEGIN
    if (!ctx) return XRDVI_OK;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    for (auto &pr : ctx->ev_pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_problem_create(xrdvi_ctx *ctx, const xrdvi_problem_desc *d,
                         xrdvi_problem **out) {
    API_GUARD_BEGIN
    if (!ctx || !out) return fail(XRDVI_EINVAL, "ctx and out must be non-NULL");
    double lam = 0.0;
    int rc = validate_desc(d, &lam);
    if (rc != XRDVI_OK) return rc;
    DeviceGuard g(ctx->device);
    const size_t bytes = problem_bytes(d->N, d->K, d->peak_off[d->K]);
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, bytes);
    if (e != hipSuccess)
        return fail(XRDVI_ENOMEM, std::string("problem allocation: ") + hipGetErrorString(e));
    auto *pb = new xrdvi_problem();
    pb->ctx = ctx;
    pb->device = ctx->device;
    pb->mem = mem;
    e = upload_problem(*d, lam, static_cast<char *>(mem), pb->P, &pb->perm, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        delete pb;
        return hip_fail(e, "problem upload");
    }
    *out = pb;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_problem_destroy(xrdvi_problem *prob) {
    API_GUARD_BEGIN
    if (!prob) return XRDVI_OK;
    DeviceGuard g(prob->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(prob->mem);
    delete prob;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_problem_info(const xrdvi_problem *prob, int32_t *N, int32_t *K,
                       int32_t *total_peaks, double *lambda_h) {
    if (!prob) return fail(XRDVI_EINVAL, "problem is NULL");
    if (N) *N = prob->P.N;
    if (K) *K = prob->P.K;
    if (total_peaks) *total_peaks = prob->P.T;
    if (lambda_h) *lambda_h = prob->P.lambda;
    return XRDVI_OK;
}

int xrdvi_problem_latents(const xrdvi_problem *prob) {
    if (!prob) return fail(XRDVI_EINVAL, "problem is NULL");
    return prob->P.D;
}

int xrdvi_tape_create(xrdvi_ctx *ctx, const xrdvi_problem *prob, int32_t S,
                      xrdvi_tape **out) {
    API_GUARD_BEGIN
    if (!ctx || !prob || !out) return fail(XRDVI_EINVAL, "NULL argument");
    if (S < 1 || S > kMaxSamples) return fail(XRDVI_EINVAL, "S must be in [1, 1024]");
    DeviceGuard g(ctx->device);
    const ProbDev &P = prob->P;
    const size_t bytes = step_bytes(step_shape(P, S));
    const size_t zbytes = sizeof(double) * P.D * (size_t)P.K;
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, bytes + zbytes);
    if (e == hipSuccess) e = hipMemset(static_cast<char *>(mem) + bytes, 0, zbytes);
    if (e != hipSuccess) {
        if (mem) (void)hipFree(mem);
        return fail(XRDVI_ENOMEM, std::string("tape allocation: ") + hipGetErrorString(e));
    }
    auto *t = new xrdvi_tape();
    t->prob = prob;
    t->device = ctx->device;
    t->mem = mem;
    t->st = carve_step(mem, step_shape(P, S));
    t->zeros = reinterpret_cast<double *>(static_cast<char *>(mem) + bytes);
    *out = t;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_tape_destroy(xrdvi_tape *tape) {
    API_GUARD_BEGIN
    if (!tape) return XRDVI_OK;
    DeviceGuard g(tape->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(tape->mem);
    delete tape;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_profile(xrdvi_ctx *ctx, const xrdvi_problem *prob, int32_t S,
                  const double *phi, float *f_out, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !prob || !phi || !f_out) return fail(XRDVI_EINVAL, "NULL argument");
    if (prob->ctx != ctx) return fail(XRDVI_EINVAL, "problem belongs to another context");
    if (S < 1 || S > kMaxSamples) return fail(XRDVI_EINVAL, "S must be in [1, 1024]");
    DeviceGuard g(ctx->device);
    const ProbDev &P = prob->P;
    int rc = XRDVI_OK;
    if (!ensure_ws(ctx, step_bytes(step_shape(P, S)), &rc)) return rc;
    StepDev st = carve_step(ctx->ws, step_shape(P, S));
    st.phi = const_cast<double *>(phi);   // read only: the kernels' samples
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_phi_consts(P, S, phi, st.pk, st.pkr, s), "phi constants");
    HIP_TRY(launch_peak_plan(P, st, phi, s), "window plan");
    HIP_TRY(launch_plan(P, st, phi, s), "tile plan");
    HIP_TRY(timed_fused(ctx, P, st, false, f_out, s), "profile");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_profile_static(xrdvi_ctx *ctx, const xrdvi_problem *prob, int32_t S,
                         const double *phi, float *f_out, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !prob || !phi || !f_out) return fail(XRDVI_EINVAL, "NULL argument");
    if (prob->ctx != ctx) return fail(XRDVI_EINVAL, "problem belongs to another context");
    if (S < 1 || S > kMaxSamples) return fail(XRDVI_EINVAL, "S must be in [1, 1024]");
    const ProbDev &P = prob->P;
    const StepShape sh = step_shape(P, S);
    const size_t bytes = step_bytes(sh);
    if (bytes > kStaticScratchBytes)
        return fail(XRDVI_EINVAL,
                    "xrdvi_profile_static: this problem and S need " +
                        std::to_string(bytes) + " bytes of scratch, more than the " +
                        std::to_string(kStaticScratchBytes) +
                        " of the static scratch (use xrdvi_profile or a smaller S)");
    void *base = static_scratch(ctx->device);
    if (!base) return fail(XRDVI_EDEVICE, "static scratch address not set up for this device");
    DeviceGuard g(ctx->device);
    StepDev st = carve_step(base, sh);
    st.phi = const_cast<double *>(phi);   // read only: the kernels' samples
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every scratch value these kernels read is written earlier in the same
    // sequence, so nothing needs clearing between calls
    HIP_TRY(launch_phi_consts(P, S, phi, st.pk, st.pkr, s), "phi constants");
    HIP_TRY(launch_peak_plan(P, st, phi, s), "window plan");
    HIP_TRY(launch_plan(P, st, phi, s), "tile plan");
    HIP_TRY(launch_fused(P, st, false, f_out, s), "profile");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_window_plan(xrdvi_ctx *ctx, const xrdvi_problem *prob, int32_t S,
                      const double *phi, int32_t *lo, int32_t *hi,
                      void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !prob || !phi || !lo || !hi) return fail(XRDVI_EINVAL, "NULL argument");
    if (prob->ctx != ctx) return fail(XRDVI_EINVAL, "problem belongs to another context");
    if (S < 1 || S > kMaxSamples) return fail(XRDVI_EINVAL, "S must be in [1, 1024]");
    DeviceGuard g(ctx->device);
    HIP_TRY(launch_windows(prob->P, S, phi, lo, hi, prob->perm,
                           static_cast<hipStream_t>(stream)),
            "window plan");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_elbo_fwd(xrdvi_ctx *ctx, const xrdvi_problem *prob, int32_t S,
                   const double *loc, const double *logscale,
                   const double *eps, uint64_t seed, uint64_t step,
                   int32_t need_grad, double *elbo_out, double *loglik_out,
                   xrdvi_tape *tape, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !prob || !loc || !logscale || !elbo_out || !tape)
        return fail(XRDVI_EINVAL, "NULL argument");
    if (prob->ctx != ctx) return fail(XRDVI_EINVAL, "problem belongs to another context");
    if (tape->prob != prob) return fail(XRDVI_EINVAL, "tape belongs to another problem");
    if (S != tape->st.S) return fail(XRDVI_EINVAL, "S differs from the tape's S");
    DeviceGuard g(ctx->device);
    const ProbDev &P = prob->P;
    const StepDev &st = tape->st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    tape->has_grad = false;
    HIP_TRY(launch_sample(P, st, loc, logscale, eps, seed, step, s), "sample");
    HIP_TRY(launch_peak_plan(P, st, st.phi, s), "window plan");
    HIP_TRY(launch_plan(P, st, st.phi, s), "tile plan");
    HIP_TRY(timed_fused(ctx, P, st, need_grad != 0, nullptr, s),
            "fused profile/adjoint");
    HIP_TRY(launch_elbo(P, st, logscale, elbo_out, loglik_out, s), "elbo");
    tape->has_grad = need_grad != 0;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_elbo_bwd(xrdvi_ctx *ctx, const xrdvi_tape *tape, double grad_scale,
                   const double *grad_scale_dev, double *grad_loc,
                   double *grad_logscale, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !tape || !grad_loc || !grad_logscale)
        return fail(XRDVI_EINVAL, "NULL argument");
    if (tape->prob->ctx != ctx) return fail(XRDVI_EINVAL, "tape belongs to another context");
    if (!tape->has_grad)
        return fail(XRDVI_EINVAL, "the last xrdvi_elbo_fwd on this tape had need_grad = 0");
    if (!std::isfinite(grad_scale)) return fail(XRDVI_EINVAL, "grad_scale must be finite");
    DeviceGuard g(ctx->device);
    HIP_TRY(launch_grad(tape->prob->P, tape->st, grad_scale, grad_scale_dev,
                        grad_loc, grad_logscale,
                        static_cast<hipStream_t>(stream)),
            "gradient");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_logpost(xrdvi_ctx *ctx, const xrdvi_problem *prob, int32_t S,
                  const double *z, double *logp_out, double *grad_out,
                  xrdvi_tape *tape, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !prob || !z || !logp_out || !tape)
        return fail(XRDVI_EINVAL, "NULL argument");
    if (prob->ctx != ctx) return fail(XRDVI_EINVAL, "problem belongs to another context");
    if (tape->prob != prob) return fail(XRDVI_EINVAL, "tape belongs to another problem");
    if (S != tape->st.S) return fail(XRDVI_EINVAL, "S differs from the tape's S");
    DeviceGuard g(ctx->device);
    tape->has_grad = false;
    HIP_TRY(launch_logpost(prob->P, tape->st, tape->zeros, z, logp_out, grad_out,
                           static_cast<hipStream_t>(stream)),
            "log posterior");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_tape_samples(xrdvi_ctx *ctx, const xrdvi_tape *tape,
                       double *phi_out, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !tape || !phi_out) return fail(XRDVI_EINVAL, "NULL argument");
    DeviceGuard g(ctx->device);
    const ProbDev &P = tape->prob->P;
    const size_t bytes = sizeof(double) * P.D * (size_t)P.K * tape->st.S;
    HIP_TRY(hipMemcpyAsync(phi_out, tape->st.phi, bytes, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)),
            "copy samples");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_timing_enable(xrdvi_ctx *ctx, int32_t enable) {
    API_GUARD_BEGIN
    if (!ctx) return fail(XRDVI_EINVAL, "ctx is NULL");
    ctx->timing = enable != 0;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_timing_read(xrdvi_ctx *ctx, double *ms_total, int64_t *launches,
                      int32_t reset) {
    API_GUARD_BEGIN
    if (!ctx) return fail(XRDVI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    for (auto &pr : ctx->ev_pending) {
        HIP_TRY(hipEventSynchronize(pr.second), "timing event");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second), "timing elapsed");
        ctx->timed_ms += ms;
        ctx->timed_launches += 1;
        ctx->ev_pool.push_back(pr.first);
        ctx->ev_pool.push_back(pr.second);
    }
    ctx->ev_pending.clear();
    if (ms_total) *ms_total = ctx->timed_ms;
    if (launches) *launches = ctx->timed_launches;
    if (reset) {
        ctx->timed_ms = 0.0;
        ctx->timed_launches = 0;
    }
    return XRDVI_OK;
    API_GUARD_END
}

}  // extern "C"
