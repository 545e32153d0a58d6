// Hamiltonian Monte Carlo over the same posterior, reusing the fused
// forward + adjoint step for every gradient (the sampling alternative the
// paper compares its stochastic VI with, Sec. 4 and Table 1).
//
// Every chain is one "sample" of the step kernels: its position z is passed
// as the noise of a zero-mean, unit-scale draw, so the per-sample log
// posterior and its gradient in z come out of the ELBO kernels unchanged.
// One iteration: momentum p ~ N(0, I) from Philox4x32-10 keyed by (seed,
// iteration), n_leapfrog leapfrog steps, and a Metropolis correction with a
// uniform from a second Philox stream.  Step sizes adapt per chain during
// warm-up by dual averaging (Hoffman and Gelman, JMLR 2014) and are frozen
// at their averaged value for the kept draws.
#include <cmath>
#include <string>
#include <vector>

#include "xrdvi.h"
#include "xrdvi_internal.h"

namespace xrdvi {

namespace {

constexpr int kHmcBlock = 256;
// Key offset of the Metropolis uniforms (a different stream than momenta).
constexpr uint64_t kUniformKey = 0x9E3779B97F4A7C15ull;

struct HmcDev {
    int C, n;                       // chains, coordinates per chain
    int n_warmup;
    int *iter;                      // current iteration (device counter)
    double *z, *z0, *g, *g0, *p;    // [C][n]
    double *logp, *logp0, *h0;      // [C]
    double *eps, *leps_bar, *hbar;  // [C] step, log averaged step, statistic
    int *accepted;                  // [C] accepted kept iterations
    double mu, gamma, t0, kappa, delta;
};

// Sum over the block of v (kHmcBlock threads); valid in every thread.
__device__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kHmcBlock / kWave; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Momentum draw, Hamiltonian at the start, first half step and position step.
__global__ __launch_bounds__(kHmcBlock) void k_hmc_begin(HmcDev H,
                                                         uint64_t seed) {
#pragma clang fp contract(off)
    __shared__ double red[kHmcBlock / kWave];
    const uint64_t iter = (uint64_t)*H.iter;
    const int c = blockIdx.x;
    const size_t o = (size_t)c * H.n;
    const double eps = H.eps[c];
    double kin = 0.0;
    for (int j = threadIdx.x; j < H.n; j += kHmcBlock) {
        const double pj = philox_normal(seed, iter, c, j);
        kin += pj * pj;
        H.z0[o + j] = H.z[o + j];
        H.g0[o + j] = H.g[o + j];
        const double ph = pj + 0.5 * eps * H.g[o + j];
        H.p[o + j] = ph;
        H.z[o + j] += eps * ph;
    }
    kin = block_sum(kin, red);
    if (threadIdx.x == 0) {
        H.logp0[c] = H.logp[c];
        H.h0[c] = -H.logp[c] + 0.5 * kin;
    }
}

// Full momentum step and position step between two gradients.
__global__ __launch_bounds__(kHmcBlock) void k_hmc_mid(HmcDev H) {
#pragma clang fp contract(off)
    const int c = blockIdx.x;
    const size_t o = (size_t)c * H.n;
    const double eps = H.eps[c];
    for (int j = threadIdx.x; j < H.n; j += kHmcBlock) {
        const double ph = H.p[o + j] + eps * H.g[o + j];
        H.p[o + j] = ph;
        H.z[o + j] += eps * ph;
    }
}

// Last half step, Metropolis correction, step-size adaptation during
// warm-up (frozen at the averaged step after the last warm-up iteration)
// and the kept draw.
__global__ __launch_bounds__(kHmcBlock) void k_hmc_end(
    HmcDev H, uint64_t seed, double *draws, double *logp_draws) {
#pragma clang fp contract(off)
    __shared__ double red[kHmcBlock / kWave];
    __shared__ int acc_s;
    const int it = *H.iter;
    const uint64_t iter = (uint64_t)it;
    const int warm = it < H.n_warmup ? it + 1 : 0;     // 1-based warm-up step
    const int d = it >= H.n_warmup ? it - H.n_warmup : -1;   // kept draw
    const int c = blockIdx.x;
    const size_t o = (size_t)c * H.n;
    const double eps = H.eps[c];
    double kin = 0.0;
    for (int j = threadIdx.x; j < H.n; j += kHmcBlock) {
        const double ph = H.p[o + j] + 0.5 * eps * H.g[o + j];
        kin += ph * ph;
    }
    kin = block_sum(kin, red);
    if (threadIdx.x == 0) {
        const double h1 = -H.logp[c] + 0.5 * kin;
        const double dh = H.h0[c] - h1;
        const bool finite = std::isfinite(h1) && std::isfinite(dh);
        const double alpha = finite ? (dh >= 0.0 ? 1.0 : exp(dh)) : 0.0;
        uint32_t v[4] = {0u, (uint32_t)c, (uint32_t)iter, (uint32_t)(iter >> 32)};
        const uint64_t key = seed ^ kUniformKey;
        philox10(v, (uint32_t)key, (uint32_t)(key >> 32));
        const double u = ((double)v[0] + 0.5) * 2.3283064365386962890625e-10;
        const int acc = finite && log(u) < dh;
        acc_s = acc;
        if (!acc) H.logp[c] = H.logp0[c];
        if (warm > 0) {
            const double m = (double)warm;
            const double w = 1.0 / (m + H.t0);
            H.hbar[c] = (1.0 - w) * H.hbar[c] + w * (H.delta - alpha);
            const double leps = H.mu - sqrt(m) / H.gamma * H.hbar[c];
            const double eta = pow(m, -H.kappa);
            H.leps_bar[c] = eta * leps + (1.0 - eta) * H.leps_bar[c];
            H.eps[c] = exp(leps);
            if (warm == H.n_warmup) H.eps[c] = exp(H.leps_bar[c]);
        }
        if (d >= 0) {
            H.accepted[c] += acc;
            if (logp_draws) logp_draws[(size_t)d * H.C + c] = H.logp[c];
        }
    }
    __syncthreads();
    const int acc = acc_s;
    for (int j = threadIdx.x; j < H.n; j += kHmcBlock) {
        if (!acc) {
            H.z[o + j] = H.z0[o + j];
            H.g[o + j] = H.g0[o + j];
        }
        if (d >= 0 && draws) draws[((size_t)d * H.C + c) * H.n + j] = H.z[o + j];
    }
}

// Next iteration.
__global__ void k_hmc_tick(HmcDev H) {
    if (threadIdx.x == 0) *H.iter += 1;
}

// Initial per-chain state.
__global__ void k_hmc_init(HmcDev H, double eps0) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) *H.iter = 0;
    if (c < H.C) {
        H.eps[c] = eps0;
        H.leps_bar[c] = 0.0;
        H.hbar[c] = 0.0;
        H.accepted[c] = 0;
    }
}

int hfail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

}  // namespace

}  // namespace xrdvi

using namespace xrdvi;

extern "C" int xrdvi_hmc(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                         const xrdvi_hmc_config *cfg, double *z,
                         double *draws, double *logp_draws,
                         double *accept_out, double *step_out, void *stream) {
    try {
        if (!ctx || !prob || !cfg || !z) return hfail(XRDVI_EINVAL, "NULL argument");
        const int C = cfg->chains;
        if (C < 1 || C > kMaxSamples) return hfail(XRDVI_EINVAL, "chains must be in [1, 1024]");
        if (cfg->n_warmup < 0 || cfg->n_draws < 0 || cfg->n_leapfrog < 1)
            return hfail(XRDVI_EINVAL, "n_warmup, n_draws >= 0 and n_leapfrog >= 1 required");
        if (!(cfg->step_size > 0.0) || !std::isfinite(cfg->step_size))
            return hfail(XRDVI_EINVAL, "step_size must be > 0");
        const double delta = cfg->target_accept == 0.0 ? 0.8 : cfg->target_accept;
        if (!(delta > 0.0 && delta < 1.0))
            return hfail(XRDVI_EINVAL, "target_accept must lie in (0, 1)");
        int32_t K = 0;
        int rc = xrdvi_problem_info(prob, nullptr, &K, nullptr, nullptr);
        if (rc != XRDVI_OK) return rc;
        const int D = xrdvi_problem_latents(prob);
        const int n = D * K;
        hipStream_t s = static_cast<hipStream_t>(stream);
        xrdvi_tape *tape = nullptr;
        rc = xrdvi_tape_create(ctx, prob, C, &tape);
        if (rc != XRDVI_OK) return rc;
        const size_t cn = (size_t)C * n;
        double *mem = nullptr;
        if (hipMalloc(&mem, sizeof(double) * (4 * cn + 6 * (size_t)C) + sizeof(int) * (C + 1)) !=
            hipSuccess) {
            xrdvi_tape_destroy(tape);
            return hfail(XRDVI_ENOMEM, "hmc: state allocation failed");
        }
        HmcDev H{};
        H.C = C;
        H.n = n;
        H.z = z;
        H.z0 = mem;
        H.g = mem + cn;
        H.g0 = mem + 2 * cn;
        H.p = mem + 3 * cn;
        double *sc = mem + 4 * cn;
        H.logp = sc;
        H.logp0 = sc + C;
        H.h0 = sc + 2 * C;
        H.eps = sc + 3 * C;
        H.leps_bar = sc + 4 * C;
        H.hbar = sc + 5 * C;
        H.accepted = reinterpret_cast<int *>(sc + 6 * C);
        H.mu = std::log(10.0 * cfg->step_size);
        H.gamma = 0.05;
        H.t0 = 10.0;
        H.kappa = 0.75;
        H.delta = delta;
        H.n_warmup = cfg->n_warmup;
        H.iter = H.accepted + C;
        // The iterations run on a private stream (ordered after the caller's
        // work) as replays of one captured iteration: begin, n_leapfrog
        // gradients with the steps between them, end, and the counter tick.
        hipStream_t hs = nullptr;
        hipEvent_t ev = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&hs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(hs, ev, 0);
        if (e == hipSuccess) {
            k_hmc_init<<<(C + 255) / 256, 256, 0, hs>>>(H, cfg->step_size);
            e = hipGetLastError();
        }
        if (e == hipSuccess) rc = xrdvi_logpost(ctx, prob, C, H.z, H.logp, H.g, tape, hs);
        const int total = cfg->n_warmup + cfg->n_draws;
        if (rc == XRDVI_OK && e == hipSuccess && total > 0) {
            e = hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                k_hmc_begin<<<C, kHmcBlock, 0, hs>>>(H, cfg->seed);
                for (int l = 1; rc == XRDVI_OK && l <= cfg->n_leapfrog; ++l) {
                    rc = xrdvi_logpost(ctx, prob, C, H.z, H.logp, H.g, tape, hs);
                    if (rc == XRDVI_OK && l < cfg->n_leapfrog)
                        k_hmc_mid<<<C, kHmcBlock, 0, hs>>>(H);
                }
                k_hmc_end<<<C, kHmcBlock, 0, hs>>>(H, cfg->seed, draws, logp_draws);
                k_hmc_tick<<<1, 1, 0, hs>>>(H);
                const hipError_t el = hipGetLastError();
                e = hipStreamEndCapture(hs, &graph);
                if (e == hipSuccess) e = el;
            }
            if (e == hipSuccess && rc == XRDVI_OK)
                e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
            for (int it = 0; rc == XRDVI_OK && e == hipSuccess && it < total; ++it)
                e = hipGraphLaunch(gexec, hs);
        }
        std::vector<int> acc(C);
        std::vector<double> eps(C);
        if (rc == XRDVI_OK && e == hipSuccess)
            e = hipMemcpyAsync(acc.data(), H.accepted, sizeof(int) * C,
                               hipMemcpyDeviceToHost, hs);
        if (rc == XRDVI_OK && e == hipSuccess)
            e = hipMemcpyAsync(eps.data(), H.eps, sizeof(double) * C,
                               hipMemcpyDeviceToHost, hs);
        if (hs) {
            const hipError_t es = hipStreamSynchronize(hs);
            if (e == hipSuccess) e = es;
        }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev) (void)hipEventDestroy(ev);
        if (hs) (void)hipStreamDestroy(hs);
        (void)hipFree(mem);
        xrdvi_tape_destroy(tape);
        if (rc != XRDVI_OK) return rc;
        if (e != hipSuccess)
            return hfail(XRDVI_EDEVICE, std::string("hmc: ") + hipGetErrorString(e));
        for (int c = 0; c < C; ++c) {
            if (accept_out)
                accept_out[c] = cfg->n_draws > 0 ? (double)acc[c] / cfg->n_draws : 0.0;
            if (step_out) step_out[c] = eps[c];
        }
        return XRDVI_OK;
    } catch (const std::bad_alloc &) {
        return hfail(XRDVI_ENOMEM, "host allocation failed");
    } catch (...) {
        return hfail(XRDVI_EDEVICE, "unexpected internal exception");
    }
}
