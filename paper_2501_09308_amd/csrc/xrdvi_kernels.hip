// Global kernels of one analysis step (gfx950).  See xrdvi_device.h for the
// per-tile work and the data layout.
#include "xrdvi_device.h"
#include "xrdvi_internal.h"

namespace xrdvi {

// Problem preparation: ln y!, tile-relative FP32 grid and peak positions.
__global__ void k_prepare_points(ProbDev P, double *lgy, float *u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.ntiles * kTile) return;
    const int t = i / kTile;
    const double xref = P.x[min(t * kTile + kTile / 2, P.N - 1)];
    if (i < P.N) {
        lgy[i] = lgamma(P.y[i] + 1.0);
        u[i] = (float)(P.x[i] - xref);
    } else {
        u[i] = 0.f;
    }
}

__global__ void k_prepare_peaks(ProbDev P, float *pt) {
    const int t = blockIdx.y;
    const double xref = P.x[min(t * kTile + kTile / 2, P.N - 1)];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < P.T;
         j += gridDim.x * blockDim.x)
        pt[(size_t)t * P.T + j] = (float)(P.pos[j] - xref);
}

// a1: sample and transform.  Block of 256 threads = 64 phases x 4 latent
// types of one sample; grid (ceil(K/64), S).  Each thread draws one
// coordinate z = loc + exp(logscale) eps, maps it to its constrained value
// and adds its log prior + log|dphi/dz| term; lane 0 of each phase then
// writes the FP32 kernel constants.
__global__ __launch_bounds__(256) void k_sample(
    ProbDev P, StepDev st, const double *__restrict__ loc,
    const double *__restrict__ logscale, const double *__restrict__ eps_in,
    uint64_t seed, uint64_t step) {
#pragma clang fp contract(off)
    __shared__ double val[4][kWave];
    __shared__ double lpt[4][kWave];
    const int t = threadIdx.x / kWave, kk = threadIdx.x % kWave;
    const int k = blockIdx.x * kWave + kk;
    const int s = blockIdx.y;
    const int K = P.K, D = 4 * K;
    double v = 0.0, lp = 0.0;
    if (k < K) {
        const int j = t * K + k;
        const double e = eps_in ? eps_in[(size_t)s * D + j]
                                : philox_normal(seed, step, s, j);
        const double sd = exp(logscale[j]);
        const double dz = sd * e;
        const double z = loc[j] + dz;
        st.eps[(size_t)s * D + j] = e;
        if (s == 0) st.sd[j] = sd;
        if (t == 0) {            // h = e^z, h ~ Exp(lambda); |dh/dz| = h
            v = exp(z);
            lp = P.c_h - P.lambda * v + z;
        } else if (t == 1) {     // mu = z, mu ~ N(0, mu_sd)
            const double um = z / P.mu_sd;
            v = z;
            lp = P.c_mu - 0.5 * um * um;
        } else if (t == 2) {     // w = e^z, w ~ Gamma(shape, rate); |dw/dz| = w
            v = exp(z);
            lp = P.c_w + (P.w_shape - 1.0) * z - P.w_rate * v + z;
        } else {                 // r = logistic(z), r ~ U(0,1); |dr/dz| = r(1-r)
            v = 1.0 / (1.0 + exp(-z));
            lp = -softplus(-z) - softplus(z);
        }
        st.phi[(size_t)s * D + j] = v;
    }
    val[t][kk] = v;
    lpt[t][kk] = lp;
    __syncthreads();
    if (t == 0) {
        double lpk = 0.0;
        if (k < K) {
            st.pk[(size_t)s * K + k] =
                phase_consts(val[0][kk], val[1][kk], val[2][kk], val[3][kk]);
            lpk = lpt[0][kk] + lpt[1][kk] + lpt[2][kk] + lpt[3][kk];
            st.lpj[(size_t)s * K + k] = lpk;
        }
        lpk = wave_sum(lpk);
        if (kk == 0) st.lpb[(size_t)s * gridDim.x + blockIdx.x] = lpk;
    }
}

// Constants of given constrained samples (profile entry).
__global__ void k_phi_consts(ProbDev P, int S, const double *__restrict__ phi,
                             float4 *pk) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= P.K || s >= S) return;
    const double *ph = phi + (size_t)s * 4 * P.K;
    pk[(size_t)s * P.K + k] =
        phase_consts(ph[k], ph[P.K + k], ph[2 * P.K + k], ph[3 * P.K + k]);
}

// a2: one thread per (sample, peak).  perm != NULL writes the caller's
// peak order.
__global__ void k_windows(ProbDev P, int S, const double *__restrict__ phi,
                          int *lo, int *hi, const int *__restrict__ perm) {
    const size_t n = (size_t)S * P.T;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(g / P.T), j = (int)(g % P.T);
        const int k = P.phase[j];
        const double *ph = phi + (size_t)s * 4 * P.K;
        const int2 wnd = window_of(P, P.pos[j], ph[P.K + k], ph[2 * P.K + k]);
        const size_t o = (size_t)s * P.T + (perm ? perm[j] : j);
        lo[o] = wnd.x;
        hi[o] = wnd.y;
    }
}

// a2 (cont.): peak ranges of every (sample, tile, phase).
__global__ void k_plan(ProbDev P, StepDev st, const double *__restrict__ phi) {
    const size_t n = (size_t)st.S * P.ntiles * P.K;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(g % P.K);
        const size_t st_idx = g / P.K;
        const int t = (int)(st_idx % P.ntiles), s = (int)(st_idx / P.ntiles);
        st.rng[g] = tile_range(P, st, phi, s, t, k);
    }
}

// a3 + a4 (+ a6): grid (ntiles, S), kBlock threads.
template <bool WIN, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_fused(ProbDev P, StepDev st,
                                                  float *f_out) {
    __shared__ FusedSmem sm;
    fused_tile<WIN, GRAD>(P, st, blockIdx.x, blockIdx.y, f_out, sm);
}

// a5: ELBO assembly, one block of 1024 threads.  Each sample is summed by
// a group of G consecutive lanes (G a power of two, G * S <= 1024) and the
// groups combine with a butterfly; totals over samples use a fixed tree.
__global__ __launch_bounds__(1024) void k_elbo(ProbDev P, StepDev st,
                                               const double *__restrict__ logscale,
                                               double *elbo_out,
                                               double *loglik_out) {
    __shared__ double tot[1024];
    __shared__ double red[1024 / kWave];
    const int S = st.S;
    int G = 1;
    while (G < kWave && 2 * G * S <= 1024) G *= 2;
    const int tid = threadIdx.x, s = tid / G, g = tid % G;
    const int kb = (P.K + kWave - 1) / kWave;
    double l = 0.0, p = 0.0;
    if (s < S) {
        for (int t = g; t < P.ntiles; t += G) l += st.llp[(size_t)s * P.ntiles + t];
        for (int b = g; b < kb; b += G) p += st.lpb[(size_t)s * kb + b];
    }
    for (int o = G / 2; o >= 1; o >>= 1) {
        l += __shfl_xor(l, o, kWave);
        p += __shfl_xor(p, o, kWave);
    }
    tot[tid] = 0.0;
    __syncthreads();
    if (g == 0 && s < S) {
        if (loglik_out) loglik_out[s] = l;
        tot[s] = l + p;
    }
    double ent = 0.0;
    for (int j = tid; j < 4 * P.K; j += blockDim.x) ent += logscale[j];
    ent = wave_sum(ent);
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = ent;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (tid < w) tot[tid] += tot[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        double e = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w) e += red[w];
        const double D = 4.0 * P.K;
        *elbo_out = tot[0] / S + e + 0.5 * D * (1.0 + kLn2Pi);
    }
}

// a7: gradient.  One block of 256 threads per phase: SG = min(S, 64)
// samples per pass, 256 / SG threads per sample each summing a stripe of
// tiles; stripes, samples and tiles are combined in FP64 in fixed order,
// then the chain rule runs through the prior, Jacobian and
// reparameterisation.
__global__ __launch_bounds__(256) void k_grad(ProbDev P, StepDev st,
                                              double scale,
                                              const double *scale_dev,
                                              double *gloc,
                                              double *glogscale) {
    __shared__ double red[256][6];
    const int k = blockIdx.x;
    const int K = P.K, D = 4 * K, S = st.S;
    const int SG = S < kWave ? S : kWave;
    const int G = 256 / SG;
    const int tid = threadIdx.x, sl = tid % SG, g = tid / SG;
    double am[4] = {0, 0, 0, 0}, as[4] = {0, 0, 0, 0};
    for (int s0 = 0; s0 < S; s0 += SG) {
        const int s = s0 + sl;
        double E[6] = {0, 0, 0, 0, 0, 0};
        if (g < G && s < S) {
            for (int t = g; t < P.ntiles; t += G) {
                const float *src = st.part + (((size_t)t * K + k) * S + s) * 6;
#pragma unroll
                for (int c = 0; c < 6; ++c) E[c] += (double)src[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) red[tid][c] = E[c];
        __syncthreads();
        if (g == 0 && s < S) {
#pragma unroll
            for (int c = 0; c < 6; ++c) E[c] = 0.0;
            for (int gg = 0; gg < G; ++gg)
#pragma unroll
                for (int c = 0; c < 6; ++c) E[c] += red[gg * SG + sl][c];
            const double *ph = st.phi + (size_t)s * D;
            const double h = ph[k], mu = ph[K + k], w = ph[2 * K + k],
                         r = ph[3 * K + k];
            const double iw = 1.0 / w, iw2 = iw * iw;
            // d lnL / d(h, mu, w, r) from the six sums
            // E0 = sum R e, E1 = sum R e q2, E2 = sum R e q2^2,
            // L0 = sum R l, L1 = sum R l^2 q2, L2 = sum R l^2, R = (y/f - 1) I
            const double gh = (1.0 - r) * kCG * iw * E[0] + r * kCL * iw * E[3];
            const double gmu = h * iw2 * ((1.0 - r) * kCG * 4.0 * kLn2 * E[1]
                                          + r * kCL * 4.0 * E[4]);
            const double gw = h * iw2 * ((1.0 - r) * kCG * (2.0 * kLn2 * E[2] - E[0])
                                         + r * kCL * (E[3] - 2.0 * E[5]));
            const double gr = h * iw * (kCL * E[3] - kCG * E[0]);
            double gz[4];
            gz[0] = h * gh - P.lambda * h + 1.0;
            gz[1] = gmu - mu / (P.mu_sd * P.mu_sd);
            gz[2] = w * gw + (P.w_shape - 1.0) - P.w_rate * w + 1.0;
            gz[3] = r * (1.0 - r) * gr + 1.0 - 2.0 * r;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = t * K + k;
                am[t] += gz[t];
                as[t] += gz[t] * st.eps[(size_t)s * D + j] * st.sd[j];
            }
        }
        __syncthreads();
    }
    if (tid < kWave) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            am[t] = wave_sum(am[t]);
            as[t] = wave_sum(as[t]);
        }
        if (tid == 0) {
            if (scale_dev) scale *= *scale_dev;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                gloc[t * K + k] = scale * (am[t] / S);
                glogscale[t * K + k] = scale * (as[t] / S + 1.0);
            }
        }
    }
}

// ---- launchers ------------------------------------------------------------

hipError_t launch_prepare(const ProbDev &P, double *lgy, float *u, float *pt,
                          hipStream_t stream) {
    const int np = P.ntiles * kTile;
    k_prepare_points<<<(np + 255) / 256, 256, 0, stream>>>(P, lgy, u);
    if (P.T > 0) {
        dim3 g((P.T + 255) / 256 < 64 ? (P.T + 255) / 256 : 64, P.ntiles);
        k_prepare_peaks<<<g, 256, 0, stream>>>(P, pt);
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
                             float4 *pk, hipStream_t stream) {
    dim3 g((P.K + kWave - 1) / kWave, S);
    k_phi_consts<<<g, kWave, 0, stream>>>(P, S, phi, pk);
    return hipGetLastError();
}

hipError_t launch_windows(const ProbDev &P, int S, const double *phi, int *lo,
                          int *hi, const int *perm, hipStream_t stream) {
    const size_t n = (size_t)S * P.T;
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_windows<<<(unsigned)blocks, 256, 0, stream>>>(P, S, phi, lo, hi, perm);
    return hipGetLastError();
}

hipError_t launch_plan(const ProbDev &P, const StepDev &st, const double *phi,
                       hipStream_t stream) {
    const size_t n = (size_t)st.S * P.ntiles * P.K;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_plan<<<(unsigned)blocks, 256, 0, stream>>>(P, st, phi);
    return hipGetLastError();
}

hipError_t launch_fused(const ProbDev &P, const StepDev &st, bool grad,
                        float *f_out, hipStream_t stream) {
    dim3 g(P.ntiles, st.S);
    const bool win = P.cutoff > 0.0;
    if (win && grad) k_fused<true, true><<<g, kBlock, 0, stream>>>(P, st, f_out);
    else if (win) k_fused<true, false><<<g, kBlock, 0, stream>>>(P, st, f_out);
    else if (grad) k_fused<false, true><<<g, kBlock, 0, stream>>>(P, st, f_out);
    else k_fused<false, false><<<g, kBlock, 0, stream>>>(P, st, f_out);
    return hipGetLastError();
}

hipError_t launch_elbo(const ProbDev &P, const StepDev &st,
                       const double *logscale, double *elbo_out,
                       double *loglik_out, hipStream_t stream) {
    k_elbo<<<1, 1024, 0, stream>>>(P, st, logscale, elbo_out, loglik_out);
    return hipGetLastError();
}

hipError_t launch_grad(const ProbDev &P, const StepDev &st, double scale,
                       const double *scale_dev, double *gloc,
                       double *glogscale, hipStream_t stream) {
    k_grad<<<P.K, 256, 0, stream>>>(P, st, scale, scale_dev, gloc, glogscale);
    return hipGetLastError();
}

}  // namespace xrdvi
