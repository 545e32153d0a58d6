// Global kernels of one analysis step (gfx950).  See xrdvi_device.h for the
// per-tile work and the data layout.
#include "xrdvi_device.h"
#include "xrdvi_internal.h"
#include "xrdvi_steps.h"

namespace xrdvi {

// Problem preparation: ln y!, tile-relative FP32 grid and peak positions.
__global__ void k_prepare_points(ProbDev P, double *lgy, float *u, float *ul) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.ntiles * kTile) return;
    const int t = i / kTile;
    const double xref = P.x[min(t * kTile + kTile / 2, P.N - 1)];
    if (i < P.N) {
        lgy[i] = lgamma(P.y[i] + 1.0);
        const double v = P.x[i] - xref;
        const float vh = (float)v;
        u[i] = vh;
        ul[i] = (float)(v - (double)vh);
    } else {
        u[i] = 0.f;
        ul[i] = 0.f;
    }
}

__global__ void k_prepare_peaks(ProbDev P, float *pt, float *ptl) {
    const int t = blockIdx.y;
    const double xref = P.x[min(t * kTile + kTile / 2, P.N - 1)];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < P.T;
         j += gridDim.x * blockDim.x) {
        const double v = P.pos[j] - xref;
        const float vh = (float)v;
        pt[(size_t)t * P.T + j] = vh;
        ptl[(size_t)t * P.T + j] = (float)(v - (double)vh);
    }
}

// a1: grid (ceil(K/64), S), 256 threads.
__global__ __launch_bounds__(256) void k_sample(
    ProbDev P, StepDev st, const double *__restrict__ loc,
    const double *__restrict__ logscale, const double *__restrict__ eps_in,
    uint64_t seed, uint64_t step) {
    __shared__ SampleSmem sm;
    sample_block(P, st, loc, logscale, eps_in, seed, step, blockIdx.y,
                 blockIdx.x, gridDim.x, sm);
}

// Constants of given constrained samples (profile entry).
__global__ void k_phi_consts(ProbDev P, int S, const double *__restrict__ phi,
                             float4 *pk, float *pkr) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= P.K || s >= S) return;
    const double *ph = phi + (size_t)s * P.D * P.K;
    const size_t o = (size_t)s * P.K + k;
    if (P.D == 5) {
        const double al = ph[4 * P.K + k];
        pk[o] = phase_consts(ph[k], ph[P.K + k], ph[2 * P.K + k],
                             ph[3 * P.K + k], asym_norm(al));
        pkr[o] = asym_iw2(ph[2 * P.K + k], al);
    } else {
        pk[o] = phase_consts(ph[k], ph[P.K + k], ph[2 * P.K + k],
                             ph[3 * P.K + k]);
    }
}

// a2: one thread per (sample, peak).  perm != NULL writes the caller's
// peak order; psec != NULL also writes the sec-law peak records.
template <bool SEC>
__global__ void k_windows(ProbDev P, int S, const double *__restrict__ phi,
                          int *lo, int *hi, const int *__restrict__ perm,
                          float4 *psec) {
    const size_t n = (size_t)S * P.T;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        windows_elem<SEC>(P, phi, lo, hi, perm, g, psec);
}

// a2 (cont.): peak ranges of every (sample, tile, phase).
template <bool SEC>
__global__ void k_plan(ProbDev P, StepDev st, const double *__restrict__ phi) {
    const size_t n = (size_t)st.S * P.ntiles * P.K;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        plan_elem<SEC>(P, st, phi, g);
}

// a2 (windowed, constant width): the window step and the phases' extremes
// over the samples in one launch.  Blocks [0, next) take 64 phases each,
// the others one thread per (sample, peak) as k_windows.
__global__ __launch_bounds__(kCandThreads) void k_windows_ext(ProbDev P, StepDev st,
                                                              const double *__restrict__ phi,
                                                              int next) {
    __shared__ CandExtSmem sm;
    if ((int)blockIdx.x < next) {
        cand_ext_block(P, st, phi, blockIdx.x * kWave, sm);
        return;
    }
    const size_t n = (size_t)st.S * P.T;
    const size_t nb = gridDim.x - next;
    for (size_t g = (size_t)(blockIdx.x - next) * blockDim.x + threadIdx.x; g < n;
         g += nb * blockDim.x)
        windows_elem<false>(P, phi, st.lo, st.hi, nullptr, g, nullptr);
}

// The candidate ranges, grid (ceil(K / 256), ntiles), one thread per
// (tile, phase).
__global__ __launch_bounds__(kCandThreads) void k_cand(ProbDev P, StepDev st) {
    const int k = blockIdx.x * kCandThreads + threadIdx.x;
    if (k < P.K) cand_elem(P, st, blockIdx.y, k);
}

// a3 + a4 (+ a6): grid (ntiles, S), kBlock threads, blocks ordered by XCD
// (the samples of a tile share its positions and counts in one L2, and
// their adjoint partials, adjacent in memory, merge there before write-back).
template <bool WIN, bool GRAD, bool ASYM, bool SEC>
__global__ __launch_bounds__(kBlock) void k_fused(ProbDev P, StepDev st,
                                                  float *f_out) {
    __shared__ FusedSmem sm;
    const int2 ts = xcd_tile_sample(P.ntiles, st.S);
    fused_tile<WIN, GRAD, ASYM, SEC>(P, st, ts.x, ts.y, f_out, sm);
}

// Dense a3 + a4 + a6 with kWideWaves waves per tile, for grids of too few
// (tile, sample) blocks to fill the GPU (the log-posterior path of
// Hamiltonian Monte Carlo with a few chains); kWideWaves * 64 threads.
constexpr int kWideWaves = 16;
template <bool GRAD, bool ASYM, bool SEC>
__global__ __launch_bounds__(kWideWaves * kWave) void k_fused_wide(ProbDev P, StepDev st,
                                                                  float *f_out) {
    __shared__ FusedSmemT<kWideWaves> sm;
    fused_tile<false, GRAD, ASYM, SEC, kWideWaves>(P, st, blockIdx.x, blockIdx.y, f_out, sm);
}

// a3 + a4 (windowed): forward tile over its staged peak records; grid
// (ntiles, S), kBlock threads, blocks ordered by XCD (constant width).  The
// register budget is held to the occupancy the staging space allows (seven
// blocks per CU, six with asymmetric records; the sec-law variants are
// left unbounded).
template <bool ASYM, bool SEC, bool UNIF>
__global__ __launch_bounds__(kBlock, SEC ? 1 : (ASYM ? 6 : 7)) void k_win(ProbDev P, StepDev st,
                                                float *f_out) {
    __shared__ WinSmem<ASYM> sm;
    // the sec-law variant reads per-sample window and peak records, which
    // the default order (tile fastest) keeps to a few samples per L2
    const int2 ts = SEC ? make_int2(blockIdx.x, blockIdx.y)
                  : st.S % kXcds == 0 ? xcd_sample_group(st.S)
                                      : xcd_tile_sample(P.ntiles, st.S);
    win_tile<ASYM, SEC, UNIF>(P, st, ts.x, ts.y, f_out, sm);
}

// a6 (windowed): peak-major adjoint, one block per (sample, phase);
// grid (K, S), kBlock threads.
template <bool ASYM, bool SEC>
__global__ __launch_bounds__(kBlock) void k_adjoint_win(ProbDev P, StepDev st) {
    __shared__ double red[kWaves][12];
    adjoint_phase<ASYM, SEC>(P, st, blockIdx.y, blockIdx.x, red);
}

// a5: one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_elbo(ProbDev P, StepDev st,
                                               const double *__restrict__ logscale,
                                               double *elbo_out,
                                               double *loglik_out,
                                               double *logp_out) {
    __shared__ ElboSmem sm;
    const double e = elbo_block(P, st, logscale, loglik_out, sm, logp_out);
    if (threadIdx.x == 0 && elbo_out) *elbo_out = e;
}

// a7: one block of 256 threads per phase.
__global__ __launch_bounds__(256) void k_grad(ProbDev P, StepDev st,
                                              double scale,
                                              const double *scale_dev,
                                              double *gloc,
                                              double *glogscale,
                                              double *gz_out) {
    __shared__ GradSmem sm;
    grad_block(P, st, blockIdx.x, scale, scale_dev, gloc, glogscale, nullptr,
               nullptr, nullptr, sm, gz_out);
}

// a7, windowed: one wave per phase, grid ceil(K / 4).
__global__ __launch_bounds__(256) void k_grad_win(ProbDev P, StepDev st,
                                                  double scale,
                                                  const double *scale_dev,
                                                  double *gloc,
                                                  double *glogscale,
                                                  double *gz_out) {
    const int k = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
    if (k < P.K)
        grad_wave(P, st, k, scale, scale_dev, gloc, glogscale, nullptr, nullptr,
                  nullptr, gz_out);
}

// a8: Adam ascent step on n coordinates.
__global__ void k_adam(int n, double *theta, double *m1, double *m2,
                       const double *__restrict__ g, int t, double lr,
                       double b1, double b2, double eps) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) adam_update(theta[j], m1[j], m2[j], g[j], t, lr, b1, b2, eps);
}

// ---- launchers ------------------------------------------------------------

hipError_t launch_prepare(const ProbDev &P, double *lgy, float *u, float *ul,
                          float *pt, float *ptl, hipStream_t stream) {
    const int np = P.ntiles * kTile;
    k_prepare_points<<<(np + 255) / 256, 256, 0, stream>>>(P, lgy, u, ul);
    if (P.T > 0) {
        dim3 g((P.T + 255) / 256 < 64 ? (P.T + 255) / 256 : 64, P.ntiles);
        k_prepare_peaks<<<g, 256, 0, stream>>>(P, pt, ptl);
    }
    return hipGetLastError();
}

hipError_t launch_sample(const ProbDev &P, const StepDev &st,
                         const double *loc, const double *logscale,
                         const double *eps, uint64_t seed, uint64_t step,
                         hipStream_t stream) {
    dim3 g((P.K + kWave - 1) / kWave, st.S);
    k_sample<<<g, 256, 0, stream>>>(P, st, loc, logscale, eps, seed, step);
    return hipGetLastError();
}

hipError_t launch_phi_consts(const ProbDev &P, int S, const double *phi,
                             float4 *pk, float *pkr, hipStream_t stream) {
    dim3 g((P.K + kWave - 1) / kWave, S);
    k_phi_consts<<<g, kWave, 0, stream>>>(P, S, phi, pk, pkr);
    return hipGetLastError();
}

hipError_t launch_windows(const ProbDev &P, int S, const double *phi, int *lo,
                          int *hi, const int *perm, hipStream_t stream,
                          float4 *psec) {
    const size_t n = (size_t)S * P.T;
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (P.sec)
        k_windows<true><<<(unsigned)blocks, 256, 0, stream>>>(P, S, phi, lo, hi,
                                                              perm, psec);
    else
        k_windows<false><<<(unsigned)blocks, 256, 0, stream>>>(P, S, phi, lo, hi,
                                                               perm, nullptr);
    return hipGetLastError();
}

// The window step.  Windowed with a constant width it also finds the
// phases' extremes over the samples (for launch_plan, which follows it).
hipError_t launch_peak_plan(const ProbDev &P, const StepDev &st,
                            const double *phi, hipStream_t stream) {
    if (P.cutoff == 0.0 && !P.sec) return hipSuccess;
    if (P.cutoff > 0.0 && !P.sec && st.cab) {
        const int next = (P.K + kWave - 1) / kWave;
        size_t blocks = ((size_t)st.S * P.T + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        if (blocks == 0) blocks = 1;
        k_windows_ext<<<(unsigned)(next + blocks), kCandThreads, 0, stream>>>(P, st, phi,
                                                                              next);
        return hipGetLastError();
    }
    return launch_windows(P, st.S, phi, P.cutoff > 0.0 ? st.lo : nullptr,
                          st.hi, nullptr, stream, P.sec ? st.psec : nullptr);
}

// Dense mode: the tile plan.  Windowed mode with a constant width: the
// candidate ranges of each (tile, phase) over the step's samples, from the
// phases' extremes that launch_peak_plan found (the windowed forward tile
// then finds its exact ranges among them).
hipError_t launch_plan(const ProbDev &P, const StepDev &st, const double *phi,
                       hipStream_t stream) {
    if (P.cutoff > 0.0) {
        if (!P.sec && st.cab) {
            dim3 g((P.K + kCandThreads - 1) / kCandThreads, P.ntiles);
            k_cand<<<g, kCandThreads, 0, stream>>>(P, st);
        }
        return hipGetLastError();
    }
    const size_t n = (size_t)st.S * P.ntiles * P.K;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (P.sec) k_plan<true><<<(unsigned)blocks, 256, 0, stream>>>(P, st, phi);
    else k_plan<false><<<(unsigned)blocks, 256, 0, stream>>>(P, st, phi);
    return hipGetLastError();
}

// Dense: one fused forward + adjoint launch.  Windowed: the forward writes
// the residual, the peak-major adjoint follows when `grad` is set.
template <bool ASYM, bool SEC>
static void launch_fused_t(const ProbDev &P, const StepDev &st, bool grad,
                           float *f_out, hipStream_t stream, bool wide) {
    dim3 g(P.ntiles, st.S);
    if (P.cutoff > 0.0) {
        StepDev sf = st;
        if (!grad) sf.rres = nullptr;
        // records in grid steps on a uniform grid (constant width only)
        if (!SEC && uses_grid_steps(P))
            k_win<ASYM, SEC, !SEC><<<g, kBlock, 0, stream>>>(P, sf, f_out);
        else
            k_win<ASYM, SEC, false><<<g, kBlock, 0, stream>>>(P, sf, f_out);
        if (grad) {
            dim3 ga(P.K, st.S);
            k_adjoint_win<ASYM, SEC><<<ga, kBlock, 0, stream>>>(P, st);
        }
    } else {
        StepDev sd = st;
        sd.rres = nullptr;      // dense: the residual stays in LDS
        if (wide) {
            const int nt = kWideWaves * kWave;
            if (grad) k_fused_wide<true, ASYM, SEC><<<g, nt, 0, stream>>>(P, sd, f_out);
            else k_fused_wide<false, ASYM, SEC><<<g, nt, 0, stream>>>(P, sd, f_out);
        } else if (grad) {
            k_fused<false, true, ASYM, SEC><<<g, kBlock, 0, stream>>>(P, sd, f_out);
        } else {
            k_fused<false, false, ASYM, SEC><<<g, kBlock, 0, stream>>>(P, sd, f_out);
        }
    }
}

hipError_t launch_fused(const ProbDev &P, const StepDev &st, bool grad,
                        float *f_out, hipStream_t stream, bool wide) {
    if (P.D == 5) {
        if (P.sec) launch_fused_t<true, true>(P, st, grad, f_out, stream, wide);
        else launch_fused_t<true, false>(P, st, grad, f_out, stream, wide);
    } else {
        if (P.sec) launch_fused_t<false, true>(P, st, grad, f_out, stream, wide);
        else launch_fused_t<false, false>(P, st, grad, f_out, stream, wide);
    }
    return hipGetLastError();
}

hipError_t launch_elbo(const ProbDev &P, const StepDev &st,
                       const double *logscale, double *elbo_out,
                       double *loglik_out, hipStream_t stream,
                       double *logp_out) {
    k_elbo<<<1, 1024, 0, stream>>>(P, st, logscale, elbo_out, loglik_out,
                                   logp_out);
    return hipGetLastError();
}

hipError_t launch_grad(const ProbDev &P, const StepDev &st, double scale,
                       const double *scale_dev, double *gloc,
                       double *glogscale, hipStream_t stream,
                       double *gz_out) {
    if (P.cutoff > 0.0)
        k_grad_win<<<(P.K + kWaves - 1) / kWaves, 256, 0, stream>>>(
            P, st, scale, scale_dev, gloc, glogscale, gz_out);
    else
        k_grad<<<P.K, 256, 0, stream>>>(P, st, scale, scale_dev, gloc, glogscale,
                                        gz_out);
    return hipGetLastError();
}

hipError_t launch_adam(int n, double *theta, double *m1, double *m2,
                       const double *g, int t, double lr, double b1, double b2,
                       double eps, hipStream_t stream) {
    k_adam<<<(n + 255) / 256, 256, 0, stream>>>(n, theta, m1, m2, g, t, lr, b1,
                                                 b2, eps);
    return hipGetLastError();
}

}  // namespace xrdvi

namespace xrdvi {

// Log posterior density ln p(Y|phi) + ln p(phi) + ln|J| and its gradient in
// z at the positions z [S][D K] (one per sample): the sampling step with a
// zero mean and unit scale reproduces z exactly, the rest is the ELBO
// step's fused forward, adjoint and chain rule, with per-sample outputs.
hipError_t launch_logpost(const ProbDev &P, const StepDev &st,
                          const double *zeros, const double *z, double *logp,
                          double *gz, hipStream_t stream) {
    hipError_t e = launch_sample(P, st, zeros, zeros, z, 0, 0, stream);
    if (e == hipSuccess) e = launch_peak_plan(P, st, st.phi, stream);
    if (e == hipSuccess) e = launch_plan(P, st, st.phi, stream);
    // a few chains give too few (tile, sample) blocks to fill the GPU: the
    // dense tile then splits its phases over more waves
    const bool wide = P.cutoff == 0.0 && (long long)P.ntiles * st.S < 4LL * 256;
    if (e == hipSuccess) e = launch_fused(P, st, gz != nullptr, nullptr, stream, wide);
    if (e == hipSuccess)
        e = launch_elbo(P, st, zeros, nullptr, nullptr, stream, logp);
    if (e == hipSuccess && gz)
        e = launch_grad(P, st, 1.0, nullptr, nullptr, nullptr, stream, gz);
    return e;
}

}  // namespace xrdvi
