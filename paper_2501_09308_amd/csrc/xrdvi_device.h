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
// The Gaussian term of a peak is evaluated for a tile only when the peak
// lies within kGaussReach FWHM of one of the tile's points: beyond 4.47 w,
// 2^(-q2^2) < 2^-80 of the peak height, far below the FP32 resolution of
// any profile value f >= B > 0 (the extra 0.13 w absorbs rounding).
constexpr double kGaussReach = 4.6;

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
    double lambda, mu_sd, w_shape, w_rate;
    // log-density constants: ln lambda, -ln(mu_sd sqrt(2 pi)),
    // shape ln(rate) - lgamma(shape)
    double c_h, c_mu, c_w;
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
    int4 *rng;        // [S][ntiles][K] peak ranges (ja, ga, gb, jb) of a
                      // tile: [ja, jb) reach the tile, [ga, gb) need G
    float *rres;      // [S][N] residual y/f - 1 (windowed mode)
    double *pw;       // [K][S][6] adjoint sums per (phase, sample)
                      // (windowed mode)
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

// ---- per-(sample, tile, phase) peak ranges ---------------------------------
//
// Peaks are ordered by position inside each phase, so for a fixed sample
// the window bounds are monotone in the peak index and both the peaks whose
// window reaches a tile and the peaks whose Gaussian matters there form
// contiguous index ranges.

// First j in [a, b) with v[j] > key (v non-decreasing).
__device__ inline int first_greater(const int *v, int a, int b, int key) {
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (v[mid] > key) b = mid; else a = mid + 1;
    }
    return a;
}
// First j in [a, b) with v[j] >= key.
__device__ inline int first_not_less(const int *v, int a, int b, int key) {
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (v[mid] >= key) b = mid; else a = mid + 1;
    }
    return a;
}
__device__ inline int first_not_less_d(const double *v, int a, int b,
                                       double key) {
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (v[mid] >= key) b = mid; else a = mid + 1;
    }
    return a;
}
__device__ inline int first_greater_d(const double *v, int a, int b,
                                      double key) {
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (v[mid] > key) b = mid; else a = mid + 1;
    }
    return a;
}

// Range entry of (sample s, tile t, phase k); phi: [S][4][K].
__device__ inline int4 tile_range(const ProbDev &P, const StepDev &st,
                                  const double *phi, int s, int t, int k) {
    const int a = P.off[k], b = P.off[k + 1];
    const int i0 = t * kTile, i1 = min(i0 + kTile, P.N);
    int ja = a, jb = b;
    if (P.cutoff > 0.0) {
        const int *lo = st.lo + (size_t)s * P.T;
        const int *hi = st.hi + (size_t)s * P.T;
        ja = first_greater(hi, a, b, i0);
        jb = first_not_less(lo, ja, b, i1);
    }
    const double *ph = phi + (size_t)s * 4 * P.K;
    const double mu = ph[P.K + k], w = ph[2 * P.K + k];
    const double reach = kGaussReach * w;
    // Gaussian relevant: p + mu + reach >= x[i0] and p + mu - reach <= x[i1-1]
    const int ga = first_not_less_d(P.pos, ja, jb, P.x[i0] - mu - reach);
    const int gb = first_greater_d(P.pos, ga, jb, P.x[i1 - 1] - mu + reach);
    return make_int4(ja, ga, gb, jb);
}

// ---- wave reductions ------------------------------------------------------

template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v),
                                                      CTRL, ROWS, 0xf, BOUND));
}

// Sum over the 64 lanes with DPP row shifts and row broadcasts (inclusive
// scan inside each row of 16, then across rows); the total ends in lane 63
// and is returned as a wave-uniform value.
__device__ __forceinline__ float wave_total_f32(float v) {
    v += dpp_f32<0x111, 0xf, true>(v);   // row_shr:1
    v += dpp_f32<0x112, 0xf, true>(v);   // row_shr:2
    v += dpp_f32<0x114, 0xf, true>(v);   // row_shr:4
    v += dpp_f32<0x118, 0xf, true>(v);   // row_shr:8
    v += dpp_f32<0x142, 0xa, false>(v);  // row_bcast:15
    v += dpp_f32<0x143, 0xc, false>(v);  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Keeps a wave-uniform value in a vector register, so that an instruction
// combining it with a scalar operand needs no extra move.
__device__ __forceinline__ float in_vgpr(float v) {
    asm volatile("" : "+v"(v));
    return v;
}

struct FusedSmem {
    float sig[kWaves][kTile];
    float rres[kTile];
    double red[kWaves];
};

// ---- fused profile + likelihood + adjoint of one (tile, sample) ---------
//
// Four waves split the phases (k = wave, wave + 4, ...).  Every wave holds
// the same kTile points, kPPL per lane (point i0 + p*64 + lane).  Peak data
// are wave-uniform (scalar loads).  Per phase the peaks run in three
// segments: [ja, ga) and [gb, jb) need only the Lorentzian, [ga, gb) both
// components.  WIN: each lane is masked by the peak's exact window.
template <bool WIN>
struct PeakMask {
    int lo, hi;
    __device__ __forceinline__ float apply(int i, float t) const {
        if (!WIN) return t;
        return (unsigned)(i - lo) < (unsigned)(hi - lo) ? t
                                                        : __builtin_huge_valf();
    }
};

template <bool WIN, bool GRAD>
__device__ void fused_tile(const ProbDev &P, const StepDev &st, int t, int s,
                           float *f_out, FusedSmem &sm) {
    const int lane = threadIdx.x & (kWave - 1);
    // wave index as a wave-uniform (scalar) value: loops over phases and
    // peaks then run on the scalar unit and peak data use scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i0 = t * kTile;
    cptr<float> pk = as_const(reinterpret_cast<const float *>(st.pk + (size_t)s * P.K));
    cptr<int> rg = as_const(reinterpret_cast<const int *>(
        st.rng + ((size_t)s * P.ntiles + t) * P.K));
    cptr<float> ptt = as_const(P.pt + (size_t)t * P.T);
    cptr<float> inten = as_const(P.inten);
    cptr<int> wlo = as_const(st.lo + (size_t)s * P.T);
    cptr<int> whi = as_const(st.hi + (size_t)s * P.T);

    float u[kPPL];
    int idx[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        idx[p] = i0 + p * kWave + lane;
        u[p] = P.u[idx[p]];
    }

    // ---------------- forward: partial signal over this wave's phases
    float sig[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) sig[p] = 0.f;

    for (int k = wv; k < P.K; k += kWaves) {
        const int ja = rg[4 * k], ga = rg[4 * k + 1], gb = rg[4 * k + 2],
                  jb = rg[4 * k + 3];
        if (ja >= jb) continue;
        const float iw2 = in_vgpr(pk[4 * k]);
        const float aG = pk[4 * k + 1], aL = pk[4 * k + 2], mu = pk[4 * k + 3];
        float uq[kPPL], accL[kPPL], accG[kPPL];
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            uq[p] = (u[p] - mu) * iw2;
            accL[p] = 0.f;
            accG[p] = 0.f;
        }
        // Lorentzian-only and full segments
        for (int seg = 0; seg < 3; ++seg) {
            const int j0 = seg == 0 ? ja : (seg == 1 ? ga : gb);
            const int j1 = seg == 0 ? ga : (seg == 1 ? gb : jb);
            const bool gauss = seg == 1;
#pragma unroll 2
            for (int j = j0; j < j1; ++j) {
                const float ptj = ptt[j];
                const float I = inten[j];
                PeakMask<WIN> mk;
                if (WIN) { mk.lo = wlo[j]; mk.hi = whi[j]; }
#pragma unroll
                for (int p = 0; p < kPPL; ++p) {
                    const float q2 = fmaf(-ptj, iw2, uq[p]);
                    const float tt = mk.apply(idx[p], fmaf(q2, q2, 1.0f));
                    accL[p] = fmaf(I, rcp_f32(tt), accL[p]);
                    if (gauss) accG[p] = fmaf(I, exp2_f32(1.0f - tt), accG[p]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < kPPL; ++p)
            sig[p] = fmaf(aL, accL[p], fmaf(aG, accG[p], sig[p]));
    }

#pragma unroll
    for (int p = 0; p < kPPL; ++p) sm.sig[wv][p * kWave + lane] = sig[p];
    __syncthreads();

    // ---------------- point stage: f = B + signal (FP64), likelihood, residual
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
            if (st.rres) st.rres[(size_t)s * P.N + i] = rr;
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

    // ---------------- adjoint: recompute every peak value
    // per point and phase: yl = sum I l, yl1 = sum I l^2 q2, yl2 = sum I l^2,
    // ye = sum I e, ye1 = sum I e q2, ye2 = sum I e q2^2; the phase's six
    // sums are then sum_points (y/f - 1) * (...), reduced over the wave.
    float rres[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) rres[p] = sm.rres[p * kWave + lane];

    for (int k = wv; k < P.K; k += kWaves) {
        float *dst = st.part + (((size_t)t * P.K + k) * st.S + s) * 6;
        const int ja = rg[4 * k], ga = rg[4 * k + 1], gb = rg[4 * k + 2],
                  jb = rg[4 * k + 3];
        if (ja >= jb) {
            if (lane < 6) dst[lane] = 0.f;
            continue;
        }
        const float iw2 = in_vgpr(pk[4 * k]);
        const float mu = pk[4 * k + 3];
        float uq[kPPL], yl0[kPPL], yl1[kPPL], yl2[kPPL], ye0[kPPL], ye1[kPPL],
            ye2[kPPL];
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            uq[p] = (u[p] - mu) * iw2;
            yl0[p] = yl1[p] = yl2[p] = 0.f;
            ye0[p] = ye1[p] = ye2[p] = 0.f;
        }
        for (int seg = 0; seg < 3; ++seg) {
            const int j0 = seg == 0 ? ja : (seg == 1 ? ga : gb);
            const int j1 = seg == 0 ? ga : (seg == 1 ? gb : jb);
            const bool gauss = seg == 1;
#pragma unroll 2
            for (int j = j0; j < j1; ++j) {
                const float ptj = ptt[j];
                const float I = inten[j];
                PeakMask<WIN> mk;
                if (WIN) { mk.lo = wlo[j]; mk.hi = whi[j]; }
#pragma unroll
                for (int p = 0; p < kPPL; ++p) {
                    const float q2 = fmaf(-ptj, iw2, uq[p]);
                    const float tt = mk.apply(idx[p], fmaf(q2, q2, 1.0f));
                    const float l = rcp_f32(tt);
                    const float Il = I * l;
                    const float Ill = Il * l;
                    yl0[p] += Il;
                    yl2[p] += Ill;
                    yl1[p] = fmaf(Ill, q2, yl1[p]);
                    if (gauss) {
                        const float Ie = I * exp2_f32(1.0f - tt);
                        const float Ieq = Ie * q2;
                        ye0[p] += Ie;
                        ye1[p] += Ieq;
                        ye2[p] = fmaf(Ieq, q2, ye2[p]);
                    }
                }
            }
        }
        float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f;
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            v0 = fmaf(rres[p], ye0[p], v0);
            v1 = fmaf(rres[p], ye1[p], v1);
            v2 = fmaf(rres[p], ye2[p], v2);
            v3 = fmaf(rres[p], yl0[p], v3);
            v4 = fmaf(rres[p], yl1[p], v4);
            v5 = fmaf(rres[p], yl2[p], v5);
        }
        v0 = wave_total_f32(v0); v1 = wave_total_f32(v1);
        v2 = wave_total_f32(v2); v3 = wave_total_f32(v3);
        v4 = wave_total_f32(v4); v5 = wave_total_f32(v5);
        if (lane == 0) {
            dst[0] = v0; dst[1] = v1; dst[2] = v2;
            dst[3] = v3; dst[4] = v4; dst[5] = v5;
        }
    }
}

// ---- peak-major adjoint (windowed mode) -----------------------------------
//
// One block of kWaves waves per (sample s, phase k); wave w takes peaks
// a + w, a + w + kWaves, ...  For every peak the lanes cover consecutive
// points of its window (64 at a time); x - rho is formed in FP64 and
// rounded to FP32.  Six sums accumulate per lane over the wave's peaks, are
// reduced over the wave, then over the waves in fixed order.
__device__ inline void adjoint_phase(const ProbDev &P, const StepDev &st,
                                     int s, int k, double (*red)[6]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int K = P.K;
    const double *ph = st.phi + (size_t)s * 4 * K;
    const double mu = ph[K + k];
    const float iw2 = (float)(2.0 / ph[2 * K + k]);
    const float *__restrict__ rres = st.rres + (size_t)s * P.N;
    cptr<int> wlo = as_const(st.lo + (size_t)s * P.T);
    cptr<int> whi = as_const(st.hi + (size_t)s * P.T);
    cptr<double> pos = as_const(P.pos);
    cptr<float> inten = as_const(P.inten);
    const int a = P.off[k], b = P.off[k + 1];
    float e0 = 0.f, e1 = 0.f, e2 = 0.f, l0 = 0.f, l1 = 0.f, l2 = 0.f;
    for (int j = a + wv; j < b; j += kWaves) {
        const int lo = wlo[j], hi = whi[j];
        const float I = inten[j];
        const double rho = pos[j] + mu;
        for (int c = lo; c < hi; c += kWave) {
            const int i = c + lane;
            const bool valid = i < hi;
            const int ii = valid ? i : lo;
            const float R = valid ? rres[ii] * I : 0.f;
            const float q2 = (float)(P.x[ii] - rho) * iw2;
            const float tt = fmaf(q2, q2, 1.0f);
            const float l = rcp_f32(tt);
            const float Rl = R * l;
            const float Rll = Rl * l;
            l0 += Rl;
            l2 += Rll;
            l1 = fmaf(Rll, q2, l1);
            if (__builtin_expect(__any(valid && tt < 81.0f), 0)) {
                const float Re = R * exp2_f32(1.0f - tt);
                const float Req = Re * q2;
                e0 += Re;
                e1 += Req;
                e2 = fmaf(Req, q2, e2);
            }
        }
    }
    e0 = wave_total_f32(e0); e1 = wave_total_f32(e1); e2 = wave_total_f32(e2);
    l0 = wave_total_f32(l0); l1 = wave_total_f32(l1); l2 = wave_total_f32(l2);
    if (lane == 0) {
        red[wv][0] = e0; red[wv][1] = e1; red[wv][2] = e2;
        red[wv][3] = l0; red[wv][4] = l1; red[wv][5] = l2;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0.0;
        for (int w = 0; w < kWaves; ++w) v += red[w][threadIdx.x];
        st.pw[((size_t)k * st.S + s) * 6 + threadIdx.x] = v;
    }
}

}  // namespace xrdvi
