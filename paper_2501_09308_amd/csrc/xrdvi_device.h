// Device-side layout and per-tile work of the xrdvi hot path (gfx950).
//
// One step of the method over S Monte-Carlo samples (Sec. 3.2, App. A):
//   sample   z = loc + exp(logscale) eps, phi = T(z), log prior + log|J|
//   windows  per (sample, peak): grid range inside rho +- c w (FP64 bounds)
//   fused    per (2-theta tile, sample): profile f = B + sum_k h_k C_k in
//            FP32, Poisson log-likelihood and residual y/f - 1 in FP64, then
//            the adjoint recomputes every peak value and accumulates six
//            FP32 sums per (sample, phase) -- the S x K x N basis is never
//            stored
//   grad     FP64 reduction of the tile sums in fixed order and the chain
//            rule to (loc, logscale)
//   elbo     FP64 assembly of the estimate
//
// Peak shape (Appendix A.2, pseudo-Voigt): with q2 = 2 (x - rho) / w,
//   G = (cG / w) 2^(-q2^2),  L = (cL / w) / (1 + q2^2),
//   cG = 2 sqrt(ln2 / pi), cL = 2 / pi
// (unit-area Gaussian and Lorentzian of full width at half maximum w).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xrdvi {

constexpr int kWave = 64;
constexpr int kPPL = 2;                   // 2-theta points per lane
constexpr int kTile = kWave * kPPL;       // points per tile (one block)
constexpr int kWaves = 4;                 // waves per block, splitting phases
constexpr int kBlock = kWave * kWaves;
constexpr int kChunk = 1024;              // phases per LDS range chunk
// The Gaussian term is evaluated only while some lane has 1 + q2^2 < this
// bound; beyond it 2^(-q2^2) < 2^-80 of the peak height, far below the FP32
// resolution of any profile value f >= B > 0.
constexpr float kGaussTMax = 81.0f;

constexpr double kCG = 0.93943727869965133377;   // 2 sqrt(ln 2 / pi)
constexpr double kCL = 0.63661977236758134308;   // 2 / pi
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLn2Pi = 1.83787706640934548356;  // ln(2 pi)
constexpr double kTwoPi = 6.28318530717958647693;

// A prepared problem in device memory (peaks ordered by position within
// each phase).
struct ProbDev {
    int N, K, T, ntiles;
    double cutoff;
    double lambda, mu_sd, w_shape, w_rate, lgamma_w_shape;
    const double *x, *y, *bg, *lgy;   // [N]; lgy = ln y!
    const float *u;                   // [ntiles * kTile] x_i - xref_tile
    const int *off;                   // [K + 1]
    const int *phase;                 // [T] phase of each peak
    const double *pos;                // [T]
    const float *inten;               // [T]
    const float *pt;                  // [ntiles][T] p_j - xref_tile
};

// Per-step state of one analysis with S samples.
struct StepDev {
    int S;
    double *eps;      // [S][4K] noise used
    double *phi;      // [S][4K] constrained samples (h, mu, w, r rows)
    float4 *pk;       // [S][K] (2/w, h(1-r)cG/w, h r cL/w, mu) in FP32
    double *lpj;      // [S][K] log prior + log|J|
    double *lpb;      // [S][ceil(K/64)] per-wave sums of lpj
    int *lo, *hi;     // [S][T] window plan (sorted peak order)
    double *llp;      // [S][ntiles] per-tile log-likelihood
    float *part;      // [ntiles][K][S][6] adjoint tile sums
    double *sd;       // [4K] exp(logscale)
};

// Read-only view of data that no kernel of the current launch writes:
// uniform loads through it become scalar loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
    return (cptr<T>)p;
}

__device__ __forceinline__ float rcp_f32(float v) {
    return __builtin_amdgcn_rcpf(v);
}
__device__ __forceinline__ float exp2_f32(float v) {
    return __builtin_amdgcn_exp2f(v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// ---- Philox4x32-10 (Salmon et al., SC'11) + Box-Muller ------------------

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = c[0], b = c[2];
        const uint32_t hiA = __umulhi(0xD2511F53u, a), loA = 0xD2511F53u * a;
        const uint32_t hiB = __umulhi(0xCD9E8D57u, b), loB = 0xCD9E8D57u * b;
        c[0] = hiB ^ c[1] ^ k0;
        c[1] = loB;
        c[2] = hiA ^ c[3] ^ k1;
        c[3] = loA;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Standard normal number j of sample s at (seed, step): Philox block j/4,
// uniform pair (j & 3) >> 1, cosine branch for even j, sine for odd j.
__device__ inline double philox_normal(uint64_t seed, uint64_t step, int s,
                                       int j) {
#pragma clang fp contract(off)
    uint32_t c[4] = {(uint32_t)(j >> 2), (uint32_t)s, (uint32_t)step,
                     (uint32_t)(step >> 32)};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const int pr = (j & 3) >> 1;
    const double ua = ((double)c[2 * pr] + 0.5) * 2.3283064365386962890625e-10;
    const double ub = ((double)c[2 * pr + 1] + 0.5) * 2.3283064365386962890625e-10;
    const double rad = sqrt(-2.0 * log(ua));
    const double ang = kTwoPi * ub;
    return (j & 1) ? rad * sin(ang) : rad * cos(ang);
}

// ---- transforms and priors (Sec. 2.2, Sec. 3.2, Appendix B.2) ----------

__device__ __forceinline__ double softplus(double a) {
    return a > 0.0 ? a + log1p(exp(-a)) : log1p(exp(a));
}

// FP32 kernel constants of one (sample, phase).
__device__ __forceinline__ float4 phase_consts(double h, double mu, double w,
                                               double r) {
    const double iw = 1.0 / w;
    return make_float4((float)(2.0 * iw), (float)(h * (1.0 - r) * kCG * iw),
                       (float)(h * r * kCL * iw), (float)mu);
}

__device__ __forceinline__ double log_prior_phase(const ProbDev &P, double h,
                                                  double mu, double w) {
    const double um = mu / P.mu_sd;
    return (log(P.lambda) - P.lambda * h)
         + (-log(P.mu_sd) - 0.5 * kLn2Pi - 0.5 * um * um)
         + (P.w_shape * log(P.w_rate) - P.lgamma_w_shape
            + (P.w_shape - 1.0) * log(w) - P.w_rate * w);
}

// ---- window plan ---------------------------------------------------------

// First i with x[i] >= v.
__device__ inline int lower_bound_x(const double *x, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// First i with x[i] > v.
__device__ inline int upper_bound_x(const double *x, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Grid range [lo, hi) with rho - c w <= x_i <= rho + c w; each bound is one
// rounded FP64 operation (no contraction), as in the model's definition.
__device__ inline int2 window_of(const ProbDev &P, double p, double mu,
                                 double w) {
#pragma clang fp contract(off)
    if (P.cutoff == 0.0) return make_int2(0, P.N);
    const double rho = p + mu;
    const double hw = P.cutoff * w;
    const double a = rho - hw;
    const double b = rho + hw;
    const int lo = lower_bound_x(P.x, P.N, a);
    int hi = upper_bound_x(P.x, P.N, b);
    if (hi < lo) hi = lo;
    return make_int2(lo, hi);
}

// Peaks [ja, jb) of phase k whose windows (for sample s) can reach the
// tile's points [i0, i1): windows are monotone in the sorted peak order.
__device__ inline int2 tile_peak_range(const int *lo, const int *hi, int a,
                                       int b, int i0, int i1) {
    int l = a, r = b;                   // first j with hi[j] > i0
    while (l < r) {
        const int mid = (l + r) >> 1;
        if (hi[mid] > i0) r = mid; else l = mid + 1;
    }
    const int ja = l;
    r = b;                              // first j with lo[j] >= i1
    while (l < r) {
        const int mid = (l + r) >> 1;
        if (lo[mid] >= i1) r = mid; else l = mid + 1;
    }
    return make_int2(ja, l);
}

struct FusedSmem {
    float sig[kWaves][kTile];
    float rres[kTile];
    double red[kWaves];
    int2 rng[kChunk];
};

// Fills smem.rng[0..kn) with the tile's peak range of phases kc..kc+kn-1.
template <bool WIN>
__device__ __forceinline__ void load_ranges(const ProbDev &P,
                                            const StepDev &st, int s, int i0,
                                            int kc, int kn, FusedSmem &sm) {
    if (!WIN) return;
    __syncthreads();
    const int *lo = st.lo + (size_t)s * P.T;
    const int *hi = st.hi + (size_t)s * P.T;
    const int i1 = min(i0 + kTile, P.N);
    for (int kk = threadIdx.x; kk < kn; kk += kBlock) {
        const int k = kc + kk;
        sm.rng[kk] = tile_peak_range(lo, hi, P.off[k], P.off[k + 1], i0, i1);
    }
    __syncthreads();
}

// ---- fused profile + likelihood + adjoint of one (tile, sample) ---------
//
// Four waves split the phases (k = wave, wave + 4, ...).  Every wave holds
// the same kTile points, kPPL per lane (point i0 + p*64 + lane).  Peak data
// are wave-uniform (scalar loads).  WIN: only peaks whose window reaches
// the tile are visited and each lane is masked by the exact window.
template <bool WIN, bool GRAD>
__device__ void fused_tile(const ProbDev &P, const StepDev &st, int t, int s,
                           float *f_out, FusedSmem &sm) {
    const int lane = threadIdx.x & (kWave - 1);
    // wave index as a wave-uniform (scalar) value: loops over phases and
    // peaks then run on the scalar unit and peak data use scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i0 = t * kTile;
    cptr<float> pk = as_const(reinterpret_cast<const float *>(st.pk + (size_t)s * P.K));
    cptr<float> ptt = as_const(P.pt + (size_t)t * P.T);
    cptr<float> inten = as_const(P.inten);
    cptr<int> off = as_const(P.off);
    cptr<int> wlo = as_const(st.lo + (size_t)s * P.T);
    cptr<int> whi = as_const(st.hi + (size_t)s * P.T);

    float u[kPPL];
    int idx[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        idx[p] = i0 + p * kWave + lane;
        u[p] = P.u[idx[p]];
    }

    // forward: per-lane partial signal over this wave's phases
    float sig[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) sig[p] = 0.f;

    for (int kc = 0; kc < P.K; kc += kChunk) {
        const int kn = min(kChunk, P.K - kc);
        load_ranges<WIN>(P, st, s, i0, kc, kn, sm);
        for (int kk = wv; kk < kn; kk += kWaves) {
            const int k = kc + kk;
            int ja, jb;
            if (WIN) { ja = sm.rng[kk].x; jb = sm.rng[kk].y; }
            else { ja = off[k]; jb = off[k + 1]; }
            if (ja >= jb) continue;
            const float4 c = make_float4(pk[4 * k], pk[4 * k + 1], pk[4 * k + 2],
                                         pk[4 * k + 3]);
            float uq[kPPL], accL[kPPL], accG[kPPL];
#pragma unroll
            for (int p = 0; p < kPPL; ++p) {
                uq[p] = (u[p] - c.w) * c.x;
                accL[p] = 0.f;
                accG[p] = 0.f;
            }
            for (int j = ja; j < jb; ++j) {
                const float ptj = ptt[j];
                const float I = inten[j];
                float q2[kPPL], tt[kPPL];
                bool near = false;
#pragma unroll
                for (int p = 0; p < kPPL; ++p) {
                    q2[p] = fmaf(-ptj, c.x, uq[p]);
                    tt[p] = fmaf(q2[p], q2[p], 1.0f);
                    if (WIN) {
                        const int l0 = wlo[j], l1 = whi[j];
                        const bool in = (unsigned)(idx[p] - l0) <
                                        (unsigned)(l1 - l0);
                        tt[p] = in ? tt[p] : __builtin_huge_valf();
                    }
                    near |= tt[p] < kGaussTMax;
                }
#pragma unroll
                for (int p = 0; p < kPPL; ++p)
                    accL[p] = fmaf(I, rcp_f32(tt[p]), accL[p]);
                if (__builtin_expect(__any(near), 0)) {
#pragma unroll
                    for (int p = 0; p < kPPL; ++p)
                        accG[p] = fmaf(I, exp2_f32(1.0f - tt[p]), accG[p]);
                }
            }
#pragma unroll
            for (int p = 0; p < kPPL; ++p)
                sig[p] = fmaf(c.z, accL[p], fmaf(c.y, accG[p], sig[p]));
        }
    }

#pragma unroll
    for (int p = 0; p < kPPL; ++p) sm.sig[wv][p * kWave + lane] = sig[p];
    __syncthreads();

    // point stage: f = B + signal (FP64), log-likelihood, residual
    double ll = 0.0;
    for (int q = threadIdx.x; q < kTile; q += kBlock) {
        const int i = i0 + q;
        float rr = 0.f;
        if (i < P.N) {
            double sg = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) sg += (double)sm.sig[w][q];
            const double f = P.bg[i] + sg;
            if (f_out) f_out[(size_t)s * P.N + i] = (float)f;
            const double y = P.y[i];
            ll += (y != 0.0 ? y * log(f) : 0.0) - f - P.lgy[i];
            rr = (float)(y / f - 1.0);
        }
        sm.rres[q] = rr;
    }
    ll = wave_sum(ll);
    if (lane == 0) sm.red[wv] = ll;
    __syncthreads();
    if (threadIdx.x == 0 && st.llp) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) tot += sm.red[w];
        st.llp[(size_t)s * P.ntiles + t] = tot;
    }
    if (!GRAD) return;

    // adjoint: recompute every peak value, six sums per (sample, phase)
    float rres[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) rres[p] = sm.rres[p * kWave + lane];

    for (int kc = 0; kc < P.K; kc += kChunk) {
        const int kn = min(kChunk, P.K - kc);
        if (P.K > kChunk) load_ranges<WIN>(P, st, s, i0, kc, kn, sm);
        for (int kk = wv; kk < kn; kk += kWaves) {
            const int k = kc + kk;
            float *dst = st.part + (((size_t)t * P.K + k) * st.S + s) * 6;
            int ja, jb;
            if (WIN) { ja = sm.rng[kk].x; jb = sm.rng[kk].y; }
            else { ja = off[k]; jb = off[k + 1]; }
            if (ja >= jb) {
                if (lane < 6) dst[lane] = 0.f;
                continue;
            }
            const float4 c = make_float4(pk[4 * k], pk[4 * k + 1], pk[4 * k + 2],
                                         pk[4 * k + 3]);
            float uq[kPPL];
#pragma unroll
            for (int p = 0; p < kPPL; ++p) uq[p] = (u[p] - c.w) * c.x;
            float e0 = 0.f, e1 = 0.f, e2 = 0.f, l0s = 0.f, l1s = 0.f, l2s = 0.f;
            for (int j = ja; j < jb; ++j) {
                const float ptj = ptt[j];
                const float I = inten[j];
                float q2[kPPL], tt[kPPL];
                bool near = false;
#pragma unroll
                for (int p = 0; p < kPPL; ++p) {
                    q2[p] = fmaf(-ptj, c.x, uq[p]);
                    tt[p] = fmaf(q2[p], q2[p], 1.0f);
                    if (WIN) {
                        const int a = wlo[j], b = whi[j];
                        const bool in = (unsigned)(idx[p] - a) <
                                        (unsigned)(b - a);
                        tt[p] = in ? tt[p] : __builtin_huge_valf();
                    }
                    near |= tt[p] < kGaussTMax;
                }
#pragma unroll
                for (int p = 0; p < kPPL; ++p) {
                    const float R = rres[p] * I;
                    const float l = rcp_f32(tt[p]);
                    const float Rl = R * l;
                    const float Rll = Rl * l;
                    l0s += Rl;
                    l2s += Rll;
                    l1s = fmaf(Rll, q2[p], l1s);
                }
                if (__builtin_expect(__any(near), 0)) {
#pragma unroll
                    for (int p = 0; p < kPPL; ++p) {
                        const float R = rres[p] * I;
                        const float Re = R * exp2_f32(1.0f - tt[p]);
                        const float Req = Re * q2[p];
                        e0 += Re;
                        e1 += Req;
                        e2 = fmaf(Req, q2[p], e2);
                    }
                }
            }
            e0 = wave_sum(e0); e1 = wave_sum(e1); e2 = wave_sum(e2);
            l0s = wave_sum(l0s); l1s = wave_sum(l1s); l2s = wave_sum(l2s);
            if (lane == 0) {
                dst[0] = e0; dst[1] = e1; dst[2] = e2;
                dst[3] = l0s; dst[4] = l1s; dst[5] = l2s;
            }
        }
    }
}

}  // namespace xrdvi
