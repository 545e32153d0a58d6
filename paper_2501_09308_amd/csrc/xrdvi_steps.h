// Per-step work units shared by the single-analysis kernels and the
// batched serving kernels (each unit is what one block or one thread does).
#pragma once

#include "xrdvi_device.h"

namespace xrdvi {

// ---- a1: sample and transform ---------------------------------------------
//
// Block of 256 threads = 64 phases x 4 of sample s, phases kb*64 .. kb*64+63;
// the thread of type t draws latent types t and t + 4 (< D).  Each draw is
// z = loc + exp(logscale) eps, mapped to its constrained value, with its
// log prior + log|dphi/dz| term; the first wave then writes the FP32 kernel
// constants and the block's sum of those terms.
struct SampleSmem {
    double val[5][kWave];
    double lpt[5][kWave];
};

__device__ inline void sample_block(const ProbDev &P, const StepDev &st,
                                    const double *__restrict__ loc,
                                    const double *__restrict__ logscale,
                                    const double *__restrict__ eps_in,
                                    uint64_t seed, uint64_t step, int s, int kb,
                                    int nkb, SampleSmem &sm) {
#pragma clang fp contract(off)
    const int t0 = threadIdx.x / kWave, kk = threadIdx.x % kWave;
    const int k = kb * kWave + kk;
    const int K = P.K, D = P.D * K;
    for (int t = t0; t < P.D; t += 4) {
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
            } else if (t == 3) {     // r = logistic(z), r ~ U(0,1); |dr/dz| = r(1-r)
                v = 1.0 / (1.0 + exp(-z));
                lp = -softplus(-z) - softplus(z);
            } else {                 // alpha = e^z, alpha ~ N(a_mean, a_sd); |J| = alpha
                v = exp(z);
                const double ua = (v - P.a_mean) / P.a_sd;
                lp = P.c_a - 0.5 * ua * ua + z;
            }
            st.phi[(size_t)s * D + j] = v;
        }
        sm.val[t][kk] = v;
        sm.lpt[t][kk] = lp;
    }
    __syncthreads();
    if (t0 == 0) {
        double lpk = 0.0;
        if (k < K) {
            const size_t o = (size_t)s * K + k;
            lpk = sm.lpt[0][kk] + sm.lpt[1][kk] + sm.lpt[2][kk] + sm.lpt[3][kk];
            if (P.D == 5) {
                const double al = sm.val[4][kk];
                lpk += sm.lpt[4][kk];
                st.pk[o] = phase_consts(sm.val[0][kk], sm.val[1][kk],
                                        sm.val[2][kk], sm.val[3][kk],
                                        asym_norm(al));
                st.pkr[o] = asym_iw2(sm.val[2][kk], al);
            } else {
                st.pk[o] = phase_consts(sm.val[0][kk], sm.val[1][kk],
                                        sm.val[2][kk], sm.val[3][kk]);
            }
            st.lpj[o] = lpk;
        }
        lpk = wave_sum(lpk);
        if (kk == 0) st.lpb[(size_t)s * nkb + kb] = lpk;
    }
}

// ---- a2: window plan element g = s * T + j ---------------------------------
// lo/hi: the peak's grid window (windowed mode; NULL skips it).  SEC (sec
// width law): psec (NULL skips it) receives the peak's record
// (c, I c, tan(theta) (pi/360) w, 0) with c = |cos theta|, theta = rho / 2,
// in sorted peak order.  The
// constant-width kernels are a separate instantiation, so they keep the
// register budget of the window search alone.
template <bool SEC>
__device__ inline void windows_elem(const ProbDev &P, const double *phi,
                                    int *lo, int *hi, const int *perm,
                                    size_t g, float4 *psec) {
#pragma clang fp contract(off)
    const int s = (int)(g / P.T), j = (int)(g % P.T);
    const int k = P.phase[j];
    const double *ph = phi + (size_t)s * P.D * P.K;
    const double mu = ph[P.K + k], w = ph[2 * P.K + k];
    if (lo) {
        const int2 wnd = window_of<SEC>(P, P.pos[j], mu, w,
                                   P.D == 5 ? ph[4 * P.K + k] : 1.0);
        const size_t o = (size_t)s * P.T + (perm ? perm[j] : j);
        lo[o] = wnd.x;
        hi[o] = wnd.y;
    }
    if (SEC && psec) {
        const double th = (P.pos[j] + mu) * kHalfDegRad;
        const double c = fabs(cos(th));
        psec[(size_t)s * P.T + j] =
            make_float4((float)c, (float)((double)P.inten[j] * c),
                        (float)(tan(th) * kHalfDegRad * w), 0.f);
    }
}

// ---- a2 (cont.): range element g = (s * ntiles + t) * K + k ---------------
template <bool SEC>
__device__ inline void plan_elem(const ProbDev &P, const StepDev &st,
                                 const double *phi, size_t g) {
    const int k = (int)(g % P.K);
    const size_t st_idx = g / P.K;
    const int t = (int)(st_idx % P.ntiles), s = (int)(st_idx / P.ntiles);
    if (P.D == 5) {
        int2 side;
        st.rng[g] = tile_range<SEC>(P, st, phi, s, t, k, &side);
        st.rng2[g] = side;
    } else {
        st.rng[g] = tile_range<SEC>(P, st, phi, s, t, k, nullptr);
    }
}

// ---- a5: ELBO assembly, block of 1024 threads --------------------------------
//
// Each sample is summed by a group of G consecutive lanes (G a power of
// two, G * S <= 1024) and the groups combine with a butterfly; totals over
// samples use a fixed tree.
struct ElboSmem {
    double tot[1024];
    double red[1024 / kWave];
};

// logp_out (may be NULL) receives each sample's ln p(Y|phi_s) + ln p(phi_s)
// + ln|J(z_s)|: the unnormalised log posterior density at z_s.
__device__ inline double elbo_block(const ProbDev &P, const StepDev &st,
                                    const double *__restrict__ logscale,
                                    double *loglik_out, ElboSmem &sm,
                                    double *logp_out = nullptr) {
#pragma clang fp contract(off)
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
    sm.tot[tid] = 0.0;
    __syncthreads();
    if (g == 0 && s < S) {
        if (loglik_out) loglik_out[s] = l;
        if (logp_out) logp_out[s] = l + p;
        sm.tot[s] = l + p;
    }
    double ent = 0.0;
    for (int j = tid; j < P.D * P.K; j += 1024) ent += logscale[j];
    ent = wave_sum(ent);
    if ((tid & (kWave - 1)) == 0) sm.red[tid / kWave] = ent;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (tid < w) sm.tot[tid] += sm.tot[tid + w];
        __syncthreads();
    }
    double e = 0.0;
    for (int w = 0; w < 1024 / kWave; ++w) e += sm.red[w];
    const double D = (double)P.D * P.K;
    return sm.tot[0] / S + e + 0.5 * D * (1.0 + kLn2Pi);   // valid in all threads
}

// ---- a8: Adam (Kingma & Ba) ascent step on one coordinate --------------------
struct AdamArgs {
    double *m1_loc, *m2_loc, *m1_ls, *m2_ls;   // [D K] moment estimates
    int t;                                      // 1-based step
    double lr, b1, b2, eps;
};

__device__ inline void adam_update(double &theta, double &m1, double &m2,
                                   double g, int t, double lr, double b1,
                                   double b2, double eps) {
#pragma clang fp contract(off)
    m1 = b1 * m1 + (1.0 - b1) * g;
    m2 = b2 * m2 + (1.0 - b2) * g * g;
    const double mh = m1 / (1.0 - pow(b1, (double)t));
    const double vh = m2 / (1.0 - pow(b2, (double)t));
    theta += lr * mh / (sqrt(vh) + eps);
}

// ---- a7: gradient of phase k, block of 256 threads ----------------------------
//
// SG = min(S, 64) samples per pass, 256 / SG threads per sample each summing
// a stripe of tiles (dense) or reading the phase's sums (windowed); stripes,
// samples and tiles are combined in FP64 in fixed order, then the chain
// rule runs through the prior, Jacobian and reparameterisation.  With
// `adam`, the gradient of the phase's 2 D parameters updates loc/logscale
// in place instead of being stored.  gz_out (may be NULL) receives every
// sample's gradient of the log posterior density in z, [S][D K].
struct GradSmem {
    double red[256][12];
};

// d lnL / d(h, mu, w, r[, alpha]) of one (sample, phase) from the adjoint
// sums E (sums over points and peaks with R = (y/f - 1) I):
//   E0 = sum R e, E1 = sum R e q2 / A, E2 = sum R e q2^2,
//   L0 = sum R l, L1 = sum R l^2 q2 / A, L2 = sum R l^2,
// and for asymmetric peaks the high-side parts E2u = sum_{x >= rho} R e q2^2
// and Q2u = sum_{x >= rho} R l^2 q2^2 = sum_{x >= rho} R (l - l^2).
__device__ inline void phase_grad(const ProbDev &P, const double *E, double h,
                                  double w, double r, double alpha,
                                  double g[5]) {
#pragma clang fp contract(off)
    // the Gaussian sums E[0..2] (E[6..8]) were accumulated with
    // 2^(-1 - q2^2), half the Gaussian's 2^(-q2^2): doubled here (exactly)
    double E0, E1, E2, L0, L1, L2, nrm = 1.0;
    if (P.D == 5) {
        const double ia = 1.0 / alpha;
        E0 = 2.0 * (E[0] + E[6]);  E1 = 2.0 * (E[1] + ia * E[7]);
        E2 = 2.0 * (E[2] + E[8]);
        L0 = E[3] + E[9];  L1 = E[4] + ia * E[10]; L2 = E[5] + E[11];
        nrm = asym_norm(alpha);
    } else {
        E0 = 2.0 * E[0]; E1 = 2.0 * E[1]; E2 = 2.0 * E[2];
        L0 = E[3]; L1 = E[4]; L2 = E[5];
    }
    const double iw = 1.0 / w, iw2 = iw * iw;
    const double cg = (1.0 - r) * kCG * nrm, cl = r * kCL * nrm;
    g[0] = cg * iw * E0 + cl * iw * L0;
    g[1] = h * iw2 * (cg * 4.0 * kLn2 * E1 + cl * 4.0 * L1);
    g[2] = h * iw2 * (cg * (2.0 * kLn2 * E2 - E0) + cl * (L0 - 2.0 * L2));
    g[3] = h * iw * nrm * (kCL * L0 - kCG * E0);
    if (P.D == 5) {
        const double E2u = 2.0 * E[8], Q2u = E[9] - E[11];
        g[4] = h * iw * (-(cg * E0 + cl * L0) / (1.0 + alpha)
                         + (cg * 2.0 * kLn2 * E2u + cl * 2.0 * Q2u) / alpha);
    }
}

// The part of phase k's gradient from sample s with adjoint sums E: the
// chain rule through the transforms, the prior and the Jacobian, added to
// this lane's sums am (for loc) and as (for logscale).
__device__ inline void grad_sample(const ProbDev &P, const StepDev &st, int k, int s,
                                   const double (&E)[12], double (&am)[5],
                                   double (&as)[5], double *gz_out) {
#pragma clang fp contract(off)
    const int K = P.K, D = P.D * K, NT = P.D;
    const double *ph = st.phi + (size_t)s * D;
    const double h = ph[k], mu = ph[K + k], w = ph[2 * K + k], r = ph[3 * K + k];
    const double al = P.D == 5 ? ph[4 * K + k] : 1.0;
    double gp[5];
    phase_grad(P, E, h, w, r, al, gp);
    double gz[5];
    gz[0] = h * gp[0] - P.lambda * h + 1.0;
    gz[1] = gp[1] - mu / (P.mu_sd * P.mu_sd);
    gz[2] = w * gp[2] + (P.w_shape - 1.0) - P.w_rate * w + 1.0;
    gz[3] = r * (1.0 - r) * gp[3] + 1.0 - 2.0 * r;
    gz[4] = P.D == 5
        ? al * gp[4] - al * (al - P.a_mean) / (P.a_sd * P.a_sd) + 1.0
        : 0.0;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        if (t >= NT) break;
        const int j = t * K + k;
        if (gz_out) gz_out[(size_t)s * D + j] = gz[t];
        am[t] += gz[t];
        as[t] += gz[t] * st.eps[(size_t)s * D + j] * st.sd[j];
    }
}

// One wave: sums am and as over its lanes (every lane receives the sums);
// then lane t < D stores the gradient of phase k's loc of latent type t and
// lane 32 + t that of its logscale, or with `adam` updates them in place.
__device__ inline void grad_finish(const ProbDev &P, const StepDev &st, int k,
                                   double scale, const double *scale_dev,
                                   double *gloc, double *glogscale, double *loc,
                                   double *logscale, const AdamArgs *adam,
                                   double (&am)[5], double (&as)[5]) {
#pragma clang fp contract(off)
    const int K = P.K, S = st.S, NT = P.D;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        am[t] = wave_sum(am[t]);
        as[t] = wave_sum(as[t]);
    }
    const int lane = threadIdx.x & (kWave - 1), t = lane & 31;
    const bool ls = lane >= 32;   // the logscale half of the wave
    if (t >= NT) return;
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < 5; ++u)
        if (u == t) a = ls ? as[u] : am[u];
    if (scale_dev) scale *= *scale_dev;
    const int j = t * K + k;
    const double g = ls ? scale * (a / S + 1.0) : scale * (a / S);
    if (adam) {
        if (ls)
            adam_update(logscale[j], adam->m1_ls[j], adam->m2_ls[j], g,
                        adam->t, adam->lr, adam->b1, adam->b2, adam->eps);
        else
            adam_update(loc[j], adam->m1_loc[j], adam->m2_loc[j], g,
                        adam->t, adam->lr, adam->b1, adam->b2, adam->eps);
    } else if (gloc) {
        (ls ? glogscale : gloc)[j] = g;
    }
}

__device__ inline void grad_block(const ProbDev &P, const StepDev &st, int k,
                                  double scale, const double *scale_dev,
                                  double *gloc, double *glogscale,
                                  double *loc, double *logscale,
                                  const AdamArgs *adam, GradSmem &sm,
                                  double *gz_out = nullptr) {
#pragma clang fp contract(off)
    const int K = P.K, S = st.S;
    const int NS = num_sums(P.D);
    const int SG = S < kWave ? S : kWave;
    const int G = 256 / SG;
    const int tid = threadIdx.x, sl = tid % SG, g = tid / SG;
    double am[5] = {0, 0, 0, 0, 0}, as[5] = {0, 0, 0, 0, 0};
    for (int s0 = 0; s0 < S; s0 += SG) {
        const int s = s0 + sl;
        // E stays in registers: every loop over it has a constant trip count
        double E[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (g < G && s < S) {
            if (P.cutoff > 0.0) {
                if (g == 0) {
                    const double *src = st.pw + ((size_t)k * S + s) * NS;
#pragma unroll
                    for (int c = 0; c < 12; ++c)
                        if (c < NS) E[c] = src[c];
                }
            } else {
                for (int t = g; t < P.ntiles; t += G) {
                    const float *src = st.part + (((size_t)t * K + k) * S + s) * NS;
#pragma unroll
                    for (int c = 0; c < 12; ++c)
                        if (c < NS) E[c] += (double)src[c];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) sm.red[tid][c] = E[c];
        __syncthreads();
        if (g == 0 && s < S) {
#pragma unroll
            for (int c = 0; c < 12; ++c) E[c] = 0.0;
            for (int gg = 0; gg < G; ++gg)
#pragma unroll
                for (int c = 0; c < 12; ++c) E[c] += sm.red[gg * SG + sl][c];
            grad_sample(P, st, k, s, E, am, as, gz_out);
        }
        __syncthreads();
    }
    if (tid < kWave)
        grad_finish(P, st, k, scale, scale_dev, gloc, glogscale, loc, logscale, adam,
                    am, as);
}

// The gradient of phase k of a windowed analysis by one wave: its adjoint
// sums are already per (phase, sample), so the lanes take the samples (64
// per pass) and no block-wide reduction is needed.  The same arithmetic, in
// the same order, as grad_block.
__device__ inline void grad_wave(const ProbDev &P, const StepDev &st, int k,
                                 double scale, const double *scale_dev,
                                 double *gloc, double *glogscale, double *loc,
                                 double *logscale, const AdamArgs *adam,
                                 double *gz_out = nullptr) {
#pragma clang fp contract(off)
    const int S = st.S, NS = num_sums(P.D);
    const int lane = threadIdx.x & (kWave - 1);
    double am[5] = {0, 0, 0, 0, 0}, as[5] = {0, 0, 0, 0, 0};
    for (int s0 = 0; s0 < S; s0 += kWave) {
        const int s = s0 + lane;
        if (s < S) {
            // (0 + sum, as grad_block's combination of its groups forms it)
            double E[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            const double *src = st.pw + ((size_t)k * S + s) * NS;
#pragma unroll
            for (int c = 0; c < 12; ++c)
                if (c < NS) E[c] = 0.0 + src[c];
            grad_sample(P, st, k, s, E, am, as, gz_out);
        }
    }
    grad_finish(P, st, k, scale, scale_dev, gloc, glogscale, loc, logscale, adam, am, as);
}

}  // namespace xrdvi
