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
//
// Asymmetric peaks (Appendix A.2, asymmetry factor A(x; alpha): alpha on the
// high-angle side of the peak, 1 below it): the full width is w below rho
// and alpha w from rho up, and the peak is scaled by 2 / (1 + alpha) so that
// it keeps unit area; the same formulas hold with q2 = 2 (x - rho) / (A w)
// and the prefactors multiplied by 2 / (1 + alpha).  Each phase then has a
// fifth latent, alpha = exp(z_alpha) with a normal prior.
//
// Angle-dependent width (Appendix A.2 uses sec(x) = 1/cos(x) in the lost
// width formula): with the sec law the full width of peak m of phase k is
// W = w sec(theta), theta = rho / 2, taken as w / |cos(rho pi / 360)|.
// Writing c = |cos theta|, the peak is the same function of
// q2 = 2 c (x - rho) / (A w) with its intensity scaled by c, so the phase
// constants stay per phase and each peak carries (c, I c); the shift's
// gradient gains the term of dW/drho = W tan(theta) pi / 360.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
constexpr double kHalfDegRad = 3.14159265358979323846 / 360.0;  // rad per deg / 2

// A prepared problem in device memory (peaks ordered by position within
// each phase).
struct ProbDev {
    int N, K, T, ntiles;
    int D;                            // latent types per phase: 4, or 5 with
                                      // the asymmetry alpha
    int sec;                          // 1: width w sec(rho / 2); 0: width w
    double cutoff;
    double lambda, mu_sd, w_shape, w_rate;
    double a_mean, a_sd;              // normal prior on alpha (D = 5)
    // log-density constants: ln lambda, -ln(mu_sd sqrt(2 pi)),
    // shape ln(rate) - lgamma(shape), -ln(a_sd sqrt(2 pi))
    double c_h, c_mu, c_w, c_a;
    const double *x, *y, *bg, *lgy;   // [N]; lgy = ln y!
    double x0, inv_dx;                // x[0] and (N - 1) / (x[N-1] - x[0])
                                      // (0 for N = 1): grid-search guesses
    double dx;                        // (x[N-1] - x[0]) / (N - 1) (0 for N = 1)
    int uniform;                      // 1: every x_i lies within 1e-9 dx of
                                      // x0 + i dx
    int formed_x;                     // 1: the windowed adjoint forms x_i
                                      // instead of loading it (a uniform
                                      // grid; symmetric peaks of constant
                                      // width, whose q2 it then forms in
                                      // FP32, only with windows of at most
                                      // kF32Cutoff FWHM)
    const float *u;                   // [ntiles * kTile] x_i - xref_tile
                                      // (FP32, rounded)
    const float *ul;                  // [ntiles * kTile] its rounding
                                      // error: (x_i - xref) - u_i in FP32
    const int *off;                   // [K + 1]
    const int *phase;                 // [T] phase of each peak
    const double *pos;                // [T]
    const float *inten;               // [T]
    const float *pt;                  // [ntiles][T] p_j - xref_tile
    const float *ptl;                 // [ntiles][T] its rounding error
    // position index of each phase's sorted peaks: ptab[k][b] is the first
    // peak j of phase k with pos[j] >= tab_x0 + b / tab_inv (b = 0 ..
    // kTabBuckets), a starting guess for searches over positions
    const int *ptab;
    double tab_x0, tab_inv;
};

constexpr int kTabBuckets = 128;

// Per-step state of one analysis with S samples.
// Number of adjoint sums per (sample, phase): six, or six per side of the
// peak (below / above rho) for asymmetric peaks.
__host__ __device__ inline int num_sums(int D) { return D == 5 ? 12 : 6; }

struct StepDev {
    int S;
    double *eps;      // [S][D K] noise used
    double *phi;      // [S][D K] constrained samples (h, mu, w, r[, alpha])
    float4 *pk;       // [S][K] (2/w, h(1-r)cG n/w, h r cL n/w, mu) in FP32,
                      // n = 2/(1+alpha) (1 for symmetric peaks)
    float *pkr;       // [S][K] 2/(alpha w): the high-angle side (D = 5)
    double *lpj;      // [S][K] log prior + log|J|
    double *lpb;      // [S][ceil(K/64)] per-wave sums of lpj
    int *lo, *hi;     // [S][T] window plan (sorted peak order)
    int4 *rng;        // dense mode: [S][ntiles][K] peak ranges (ja, ga, gb, jb) of a
                      // tile: [ja, jb) reach the tile, [ga, gb) need G
    int2 *rng2;       // [S][ntiles][K] (jr, jl) for D = 5: peaks before jr
                      // lie at or below every point of the tile, peaks from
                      // jl above every point
    float4 *psec;     // [S][T] sec width law, per (sample, peak):
                      // (c, I c, tan(theta) (pi/360) w, 0), c = |cos theta|
    float *rres;      // [S][N] residual y/f - 1 (windowed mode)
    double *pw;       // [K][S][num_sums] adjoint sums per (phase, sample)
                      // (windowed mode)
    double *llp;      // [S][ntiles] per-tile log-likelihood
    float *part;      // [ntiles][K][S][num_sums] adjoint tile sums
    double *sd;       // [D K] exp(logscale)
    // windowed mode, constant width: the candidate peaks of each (tile,
    // phase) over the step's samples, laid out [..][ntiles][K] so that the
    // forward's threads (one per phase of a tile) read them coalesced:
    int2 *cab;        // [ntiles][K] candidates [ca, cb)
    double *cp;       // [kCandKeep][ntiles][K] positions of the first ones
    double4 *cext;    // [K] (min mu, max mu, max w, max w alpha) over samples
};

// Candidate peaks [ca, cb) of one phase for one tile are those whose window
// can reach the tile at some sample of the step; the positions of the first
// four of them are kept beside the range, so that the windowed forward finds
// its exact ranges without a search when a tile has at most four candidates
// (the usual case).
constexpr int kCandKeep = 4;
struct CandRec {
    int ca, cb;
    double p[kCandKeep];
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

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
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
// nrm = 2 / (1 + alpha) for asymmetric peaks, 1 otherwise.  The kernels
// evaluate the Gaussian as 2^(-tt) = 2^(-1 - q2^2) with tt = 1 + q2^2 (the
// Lorentzian's denominator, and the exponent's negation is free), so its
// amplitude here is twice h (1 - r) cG n / w, and the adjoint's Gaussian
// sums are half those of 2^(-q2^2) (phase_grad doubles them).
__device__ __forceinline__ float4 phase_consts(double h, double mu, double w,
                                               double r, double nrm = 1.0) {
    const double iw = 1.0 / w;
    return make_float4((float)(2.0 * iw),
                       (float)(2.0 * h * (1.0 - r) * kCG * iw * nrm),
                       (float)(h * r * kCL * iw * nrm), (float)mu);
}
__device__ __forceinline__ double asym_norm(double alpha) {
    return 2.0 / (1.0 + alpha);
}
__device__ __forceinline__ float asym_iw2(double w, double alpha) {
    return (float)(2.0 / (alpha * w));
}

// ---- window plan ---------------------------------------------------------

// Grid searches.  The grid is ascending and usually close to uniform, so a
// search starts at the index a uniform grid would give and checks the true
// values there (grid_range below); the result is the exact bound for any
// ascending grid.

// Index guess for value v on a grid starting at x0 with inv_dx points per
// unit (clamped to [0, n]; NaN gives 0).
__host__ __device__ inline int grid_guess(double x0, double inv_dx, int n,
                                          double v) {
    const double g = (v - x0) * inv_dx;
    if (!(g > 0.0)) return 0;
    if (!(g < (double)n)) return n;
    return (int)g;
}

// Batched searches.  A search from a good guess costs one round trip to
// memory when the entries around the guess are loaded together: a probe
// loads NP consecutive entries from j0 (several searches issue their probes
// before any result is needed), and the answer is read off the probe when
// it lies inside.  Otherwise the search moves a whole probe towards it (two
// more probes at most) and bisects what remains.  Entries are read clamped
// to [a, b - 1] (entry 0 when the range is empty), so every load stays in
// bounds for any j0.
template <int NP, typename T>
struct Probe {
    int j0;
    T v[NP];
};

template <int NP, typename T>
__host__ __device__ __forceinline__ Probe<NP, T> probe_at(const T *v, int a,
                                                         int b, int j0) {
    Probe<NP, T> p;
    p.j0 = j0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int j = j0 + i < a ? a : (j0 + i > b - 1 ? b - 1 : j0 + i);
        p.v[i] = v[a < b ? j : 0];
    }
    return p;
}

// The number of leading entries of a probe (loaded by probe_at with the
// same a and b) whose predicate is false, pred false and then true over
// [a, b): entries below a count as false and entries at or past b as true.
// Evaluating every probe this way first leaves one integer per search live
// instead of the probed values.
template <int NP, typename T, typename F>
__host__ __device__ __forceinline__ int probe_count(const Probe<NP, T> &p,
                                                   int a, int b, F pred) {
    int nf = 0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int j = p.j0 + i;
        nf += (j >= b || (j >= a && pred(p.v[i]))) ? 0 : 1;
    }
    return nf;
}

// First j in [a, b) with pred(v[j]) true, b if none, given the count nf of
// a probe at j0: the answer j0 + nf when it lies inside the probe, otherwise
// the search goes on by whole probes (two more at most), then bisects.
template <int NP, typename T, typename F>
__host__ __device__ inline int probe_settle(const T *v, int a, int b, int j0,
                                            int nf, F pred) {
    if (a >= b) return a;
    int lo = a, hi = b;                     // the answer lies in [lo, hi]
    for (int round = 0;; ++round) {
        if (nf > 0 && nf < NP) return j0 + nf;
        if (nf == 0) hi = j0 < hi ? j0 : hi;               // at or left of j0
        else lo = j0 + NP > lo ? j0 + NP : lo;             // right of the probe
        if (lo >= hi || round == 2) break;
        j0 = nf == 0 ? (hi - NP > lo ? hi - NP : lo) : lo;
        nf = probe_count(probe_at<NP>(v, a, b, j0), a, b, pred);
    }
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pred(v[mid])) hi = mid; else lo = mid + 1;
    }
    return lo;
}

template <int NP, typename T, typename F>
__host__ __device__ inline int probe_result(const T *v, int a, int b,
                                            const Probe<NP, T> &p, F pred) {
    return probe_settle<NP>(v, a, b, p.j0, probe_count(p, a, b, pred), pred);
}

// Grid range [lo, hi) of the points with va <= x_i <= vb (lo = first i with
// x[i] >= va, hi = first i with x[i] > vb; both written as negated "before"
// tests, so a NaN bound gives 0), each bound from a two-point probe at the
// uniform-grid guess.  grid_probe issues both probes, grid_finish reads the bounds off
// them, so that the probes of several ranges can be in flight together.
struct GridProbe {
    Probe<2, double> a, b;
    double va, vb;
};
__host__ __device__ __forceinline__ GridProbe grid_probe(const double *x, int n,
                                                        double x0, double inv_dx,
                                                        double va, double vb) {
    return GridProbe{probe_at<2>(x, 0, n, grid_guess(x0, inv_dx, n, va)),
                     probe_at<2>(x, 0, n, grid_guess(x0, inv_dx, n, vb)), va, vb};
}
__host__ __device__ inline int2 grid_finish(const double *x, int n,
                                            const GridProbe &g) {
    const double va = g.va, vb = g.vb;
    auto ge = [&](double xi) { return !(xi < va); };
    auto gt = [&](double xi) { return !(xi <= vb); };
    const int na = probe_count(g.a, 0, n, ge), nb = probe_count(g.b, 0, n, gt);
    return make_int2(probe_settle<2>(x, 0, n, g.a.j0, na, ge),
                     probe_settle<2>(x, 0, n, g.b.j0, nb, gt));
}
__host__ __device__ inline int2 grid_range(const double *x, int n, double x0,
                                           double inv_dx, double va,
                                           double vb) {
    return grid_finish(x, n, grid_probe(x, n, x0, inv_dx, va, vb));
}

// Full width of a peak centred at rho: w, or w / |cos(rho pi / 360)| with
// the sec law (SEC).
template <bool SEC>
__device__ __forceinline__ double peak_width(double rho, double w) {
#pragma clang fp contract(off)
    return SEC ? w / fabs(cos(rho * kHalfDegRad)) : w;
}

// Grid range [lo, hi) with rho - c W <= x_i <= rho + c W (rho + (c W) alpha
// for asymmetric peaks, alpha > 0; pass 1 otherwise), W the peak's full
// width; each bound is one rounded FP64 operation (no contraction), as in
// the model's definition.
// The window's bounds a = rho - c W and b = rho + c W (rho + (c W) alpha for
// asymmetric peaks).
template <bool SEC>
__device__ __forceinline__ double2 window_bounds(const ProbDev &P, double p,
                                                 double mu, double w,
                                                 double alpha) {
#pragma clang fp contract(off)
    const double rho = p + mu;
    const double hw = P.cutoff * peak_width<SEC>(rho, w);
    return make_double2(rho - hw, rho + (P.D == 5 ? hw * alpha : hw));
}

template <bool SEC>
__device__ inline int2 window_of(const ProbDev &P, double p, double mu,
                                 double w, double alpha) {
    if (P.cutoff == 0.0) return make_int2(0, P.N);
    const double2 ab = window_bounds<SEC>(P, p, mu, w, alpha);
    int2 r = grid_range(P.x, P.N, P.x0, P.inv_dx, ab.x, ab.y);
    if (r.y < r.x) r.y = r.x;
    return r;
}

// ---- per-(sample, tile, phase) peak ranges ---------------------------------
//
// Peaks are ordered by position inside each phase, so for a fixed sample
// the window bounds are monotone in the peak index and both the peaks whose
// window reaches a tile and the peaks whose Gaussian matters there form
// contiguous index ranges.

// First j in [a, b) with p[j] + mu > key (FP64 sum, as the peak centre
// rho is formed everywhere else); monotone because p is sorted.
__device__ inline int first_centre_above(const double *p, int a, int b,
                                         double mu, double key) {
#pragma clang fp contract(off)
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (p[mid] + mu > key) b = mid; else a = mid + 1;
    }
    return a;
}

// With the sec law a peak's reach [rho - R W, rho + R alpha W] has bounds
// that move with rho at slopes 1 - R W tau and 1 + R alpha W tau
// (tau = tan(theta) pi / 360).  For centres inside (-180, 180) deg, W tau
// increases with rho, so both bounds are monotone over a phase (and the
// searches over its sorted peaks valid) when the slopes are positive at the
// last and the first centre respectively.
__device__ inline bool sec_monotone(double rf, double rl, double w, double R,
                                    double alpha) {
#pragma clang fp contract(off)
    if (!(rf > -180.0) || !(rl < 180.0)) return false;
    const double tf = rf * kHalfDegRad, tl = rl * kHalfDegRad;
    const double up = 1.0 + R * alpha * (w / fabs(cos(tf))) * tan(tf) * kHalfDegRad;
    const double dn = 1.0 - R * (w / fabs(cos(tl))) * tan(tl) * kHalfDegRad;
    return up > 0.0 && dn > 0.0;
}

// Probe start for the first peak of phase k (peaks [a, b)) whose position
// is >= v: one before the bucket's first peak, so that the probe also
// covers an answer one to the left of it.
__device__ __forceinline__ int tab_guess(const ProbDev &P, int k, double v,
                                         int a, int b) {
    const double g = (v - P.tab_x0) * P.tab_inv;
    const int u = !(g > 0.0) ? 0 : (g < (double)kTabBuckets ? (int)g : kTabBuckets);
    const int j = P.ptab[k * (kTabBuckets + 1) + u];
    return (j < a ? a : (j > b ? b : j)) - 1;
}

// The peaks of phase k whose windows reach the points [xa, xb] = x[i0 ..
// i1-1] of a tile (sample row ph of phi, window arrays wlo / whi of that
// sample): [ja, jb), from two searches whose probes go out together, each
// predicate monotone over the whole phase:
//   ja: first peak whose window reaches the tile, hi_j > i0 <=> xa <= b_j,
//   jb: first peak whose window starts past it, lo_j >= i1 <=> a_j > xb,
// with the window bounds (a_j, b_j) formed as the window step forms them.
// The searches start from position-index guesses.  With a constant width
// they test the positions; under the sec law (whose bounds need a cosine
// per peak) they test the window step's index arrays.  The whole phase
// when there is no window or its sec-law bounds are not monotone.  Also
// returns the phase's FP64 shift, width and alpha, and whether the reach
// of the Gaussian is monotone (sec law).
struct PhaseWin {
    int a, b, ja, jb;
    double mu, w, alpha;
    bool g_mono;
};

template <bool SEC>
__device__ inline PhaseWin phase_window(const ProbDev &P, const double *ph,
                                        int k, int i0, int i1, const int *wlo,
                                        const int *whi) {
#pragma clang fp contract(off)
    PhaseWin r;
    r.a = P.off[k];
    r.b = P.off[k + 1];
    const int a = r.a, b = r.b;
    r.mu = ph[P.K + k];
    r.w = ph[2 * P.K + k];
    r.alpha = P.D == 5 ? ph[4 * P.K + k] : 1.0;
    const double mu = r.mu, w = r.w, alpha = r.alpha;
    const double xa = P.x[i0], xb = P.x[i1 - 1];
    bool win_mono = true;
    r.g_mono = true;
    if (SEC && a < b) {
        const double rf = P.pos[a] + mu, rl = P.pos[b - 1] + mu;
        win_mono = sec_monotone(rf, rl, w, P.cutoff, alpha);
        r.g_mono = sec_monotone(rf, rl, w, kGaussReach, alpha);
    }
    r.ja = a;
    r.jb = b;
    if (!(P.cutoff > 0.0) || !win_mono) return r;
    const double Wt = SEC ? peak_width<SEC>(xa, w) : w;   // a guess only
    const double hw = P.cutoff * Wt, hwu = P.D == 5 ? hw * alpha : hw;
    const int g_a = tab_guess(P, k, xa - mu - hwu, a, b);
    const int g_b = tab_guess(P, k, xb - mu + hw, a, b);
    if (SEC) {
        const Probe<4, int> pja = probe_at<4>(whi, a, b, g_a);
        const Probe<4, int> pjb = probe_at<4>(wlo, a, b, g_b);
        auto reach_a = [&](int hi) { return hi > i0; };
        auto past_b = [&](int lo) { return lo >= i1; };
        const int nja = probe_count(pja, a, b, reach_a);
        const int njb = probe_count(pjb, a, b, past_b);
        r.ja = probe_settle<4>(whi, a, b, pja.j0, nja, reach_a);
        r.jb = probe_settle<4>(wlo, a, b, pjb.j0, njb, past_b);
    } else {
        const Probe<4, double> pja = probe_at<4>(P.pos, a, b, g_a);
        const Probe<4, double> pjb = probe_at<4>(P.pos, a, b, g_b);
        auto reach_a = [&](double p) {
            return xa <= window_bounds<SEC>(P, p, mu, w, alpha).y;
        };
        auto past_b = [&](double p) {
            return window_bounds<SEC>(P, p, mu, w, alpha).x > xb;
        };
        const int nja = probe_count(pja, a, b, reach_a);
        const int njb = probe_count(pjb, a, b, past_b);
        r.ja = probe_settle<4>(P.pos, a, b, pja.j0, nja, reach_a);
        r.jb = probe_settle<4>(P.pos, a, b, pjb.j0, njb, past_b);
    }
    if (r.jb < r.ja) r.jb = r.ja;
    return r;
}

// The peaks of [ja, jb) whose Gaussian reaches the tile [xa, xb]: [ga, gb),
// clamped into [ja, jb).  Reach of a peak: [rho - R W, rho + R alpha W] with
// R = kGaussReach; ga is the first peak whose reach ends at or past xa, gb
// the first whose reach starts past xb.  With a constant width, searched
// like [ja, jb) over the positions; under the sec law by bisection of the
// few peaks of [ja, jb) (a cosine per test), and all of them when the reach
// is not monotone.
template <bool SEC>
__device__ inline int2 gauss_range(const ProbDev &P, const PhaseWin &pw, int k,
                                   double xa, double xb) {
#pragma clang fp contract(off)
    const int a = pw.a, b = pw.b, ja = pw.ja, jb = pw.jb;
    const double mu = pw.mu, w = pw.w, alpha = pw.alpha;
    if (SEC) {
        if (!pw.g_mono) return make_int2(ja, jb);
        auto bisect = [&](int lo, int hi, auto pred) {
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (pred(P.pos[mid])) hi = mid; else lo = mid + 1;
            }
            return lo;
        };
        const int ga = bisect(ja, jb, [&](double p) {
            const double rho = p + mu;
            return rho + kGaussReach * peak_width<SEC>(rho, w) * alpha >= xa;
        });
        const int gb = bisect(ga, jb, [&](double p) {
            const double rho = p + mu;
            return rho - kGaussReach * peak_width<SEC>(rho, w) > xb;
        });
        return make_int2(ga, gb);
    }
    const double rg = kGaussReach * w, rgu = rg * alpha;
    const Probe<4, double> pga = probe_at<4>(P.pos, a, b, tab_guess(P, k, xa - mu - rgu, a, b));
    const Probe<4, double> pgb = probe_at<4>(P.pos, a, b, tab_guess(P, k, xb - mu + rg, a, b));
    auto g_a = [&](double p) { return p >= xa - mu - kGaussReach * w * alpha; };
    auto g_b = [&](double p) { return p > xb - mu + kGaussReach * w; };
    const int nga = probe_count(pga, a, b, g_a);
    const int ngb = probe_count(pgb, a, b, g_b);
    int ga = probe_settle<4>(P.pos, a, b, pga.j0, nga, g_a);
    int gb = probe_settle<4>(P.pos, a, b, pgb.j0, ngb, g_b);
    ga = ga < ja ? ja : (ga > jb ? jb : ga);
    gb = gb < ga ? ga : (gb > jb ? jb : gb);
    return make_int2(ga, gb);
}

// ---- candidate ranges (windowed mode, constant width) --------------------
//
// The peaks of a phase whose window reaches a tile at sample s lie among
// those whose window could reach it at any sample of the step: positions p
// with xa - max_s(mu) - c max_s(w alpha) <= p <= xb - min_s(mu) + c max_s(w)
// (widened by a margin far above FP64 rounding).  Found once per step for
// every (tile, phase), so that each (tile, sample) of the windowed forward
// reads them with coalesced loads instead of searching the phase with
// scattered ones.
constexpr int kCandThreads = 256;

// The extremes of each phase over the step's samples: (min mu, max mu,
// max w, max w alpha) to st.cext[k].  Block of kCandThreads threads: 64
// phases (starting at k0) times 4 slices of the samples, combined in LDS.
struct CandExtSmem {
    double v[4][4][kWave];
};
__device__ inline void cand_ext_block(const ProbDev &P, const StepDev &st,
                                      const double *phi, int k0,
                                      CandExtSmem &sm) {
    const int kk = threadIdx.x % kWave, sl = threadIdx.x / kWave;
    const int k = k0 + kk;
    const size_t row = (size_t)P.D * P.K;
    double mn = __builtin_huge_val(), mx = -__builtin_huge_val(), wm = 0.0, wam = 0.0;
    if (k < P.K) {
        for (int s = sl; s < st.S; s += 4) {
            const double mu = phi[s * row + P.K + k], w = phi[s * row + 2 * P.K + k];
            const double al = P.D == 5 ? phi[s * row + 4 * P.K + k] : 1.0;
            mn = fmin(mn, mu);
            mx = fmax(mx, mu);
            wm = fmax(wm, w);
            wam = fmax(wam, w * al);
        }
    }
    sm.v[0][sl][kk] = mn; sm.v[1][sl][kk] = mx; sm.v[2][sl][kk] = wm; sm.v[3][sl][kk] = wam;
    __syncthreads();
    if (sl == 0 && k < P.K) {
#pragma unroll
        for (int o = 1; o < 4; ++o) {
            mn = fmin(mn, sm.v[0][o][kk]);
            mx = fmax(mx, sm.v[1][o][kk]);
            wm = fmax(wm, sm.v[2][o][kk]);
            wam = fmax(wam, sm.v[3][o][kk]);
        }
        st.cext[k] = make_double4(mn, mx, wm, wam);
    }
}

// Candidate range of (tile t, phase k) from the phase's extremes.
__device__ inline void cand_elem(const ProbDev &P, const StepDev &st, int t,
                                 int k) {
#pragma clang fp contract(off)
    const double4 e = st.cext[k];
    const double lo_off = e.y + P.cutoff * e.w;
    const double hi_off = P.cutoff * e.z - e.x;
    const int a = P.off[k], b = P.off[k + 1];
    const int i0 = t * kTile, i1 = min(i0 + kTile, P.N);
    const double xa = P.x[i0], xb = P.x[i1 - 1];
    const double pl = xa - lo_off - (1e-9 + 1e-12 * fabs(xa));
    const double pu = xb + hi_off + (1e-9 + 1e-12 * fabs(xb));
    auto ge = [&](double p) { return !(p < pl); };
    auto gt = [&](double p) { return p > pu; };
    const Probe<4, double> pa = probe_at<4>(P.pos, a, b, tab_guess(P, k, pl, a, b));
    const Probe<4, double> pb = probe_at<4>(P.pos, a, b, tab_guess(P, k, pu, a, b));
    const int na = probe_count(pa, a, b, ge), nb = probe_count(pb, a, b, gt);
    const int ca = probe_settle<4>(P.pos, a, b, pa.j0, na, ge);
    int cb = probe_settle<4>(P.pos, a, b, pb.j0, nb, gt);
    cb = cb < ca ? ca : cb;
    const size_t ci = (size_t)t * P.K + k, ntk = (size_t)P.ntiles * P.K;
    st.cab[ci] = make_int2(ca, cb);
#pragma unroll
    for (int q = 0; q < kCandKeep; ++q)
        st.cp[q * ntk + ci] = ca + q < cb ? P.pos[ca + q] : 0.0;
}

// The candidates of (tile t, phase k) as the forward's staging thread reads
// them.
__device__ __forceinline__ CandRec cand_read(const ProbDev &P, const StepDev &st,
                                             int t, int k) {
    const size_t ci = (size_t)t * P.K + k, ntk = (size_t)P.ntiles * P.K;
    CandRec r;
    const int2 ab = st.cab[ci];
    r.ca = ab.x;
    r.cb = ab.y;
#pragma unroll
    for (int q = 0; q < kCandKeep; ++q) r.p[q] = st.cp[q * ntk + ci];
    return r;
}

// The ranges [ja, jb) and [ga, gb) of phase_window and gauss_range
// (constant width), searched within the candidates [ca, cb) of the tile:
// from the candidates' own positions when there are at most four, else by
// the batched searches restricted to the candidates.  The predicates are
// those of phase_window and gauss_range, monotone over the phase, so the
// ranges are the same as from searches over the whole phase.
__device__ inline PhaseWin phase_window_cand(const ProbDev &P, const double *ph,
                                             int k, double xa, double xb,
                                             const CandRec &cand, int2 *gr) {
#pragma clang fp contract(off)
    PhaseWin r;
    r.a = P.off[k];
    r.b = P.off[k + 1];
    r.mu = ph[P.K + k];
    r.w = ph[2 * P.K + k];
    r.alpha = P.D == 5 ? ph[4 * P.K + k] : 1.0;
    r.g_mono = true;
    const double mu = r.mu, w = r.w, alpha = r.alpha;
    const int ca = cand.ca, cb = cand.cb;
    auto reach_a = [&](double p) { return xa <= window_bounds<false>(P, p, mu, w, alpha).y; };
    auto past_b = [&](double p) { return window_bounds<false>(P, p, mu, w, alpha).x > xb; };
    auto g_a = [&](double p) { return p >= xa - mu - kGaussReach * w * alpha; };
    auto g_b = [&](double p) { return p > xb - mu + kGaussReach * w; };
    int ja, jb, ga, gb;
    if (cb - ca <= kCandKeep) {
        Probe<kCandKeep, double> pr;
        pr.j0 = ca;
#pragma unroll
        for (int q = 0; q < kCandKeep; ++q) pr.v[q] = cand.p[q];
        ja = ca + probe_count(pr, ca, cb, reach_a);
        jb = ca + probe_count(pr, ca, cb, past_b);
        ga = ca + probe_count(pr, ca, cb, g_a);
        gb = ca + probe_count(pr, ca, cb, g_b);
    } else {
        const double hw = P.cutoff * w, hwu = P.D == 5 ? hw * alpha : hw;
        const double rg = kGaussReach * w, rgu = rg * alpha;
        ja = probe_result<4>(P.pos, ca, cb, probe_at<4>(P.pos, ca, cb,
                             tab_guess(P, k, xa - mu - hwu, ca, cb)), reach_a);
        jb = probe_result<4>(P.pos, ca, cb, probe_at<4>(P.pos, ca, cb,
                             tab_guess(P, k, xb - mu + hw, ca, cb)), past_b);
        ga = probe_result<4>(P.pos, ca, cb, probe_at<4>(P.pos, ca, cb,
                             tab_guess(P, k, xa - mu - rgu, ca, cb)), g_a);
        gb = probe_result<4>(P.pos, ca, cb, probe_at<4>(P.pos, ca, cb,
                             tab_guess(P, k, xb - mu + rg, ca, cb)), g_b);
    }
    if (jb < ja) jb = ja;
    ga = ga < ja ? ja : (ga > jb ? jb : ga);
    gb = gb < ga ? ga : (gb > jb ? jb : gb);
    r.ja = ja;
    r.jb = jb;
    *gr = make_int2(ga, gb);
    return r;
}

// Range entry of (sample s, tile t, phase k); phi: [S][D][K].  For
// asymmetric peaks *side receives (jr, jl) with ga <= jr <= jl <= gb.
// Ranges may be wider than needed (the windowed kernels mask each peak by
// its exact window); with the sec law they cover the whole phase when its
// bounds are not monotone.  [ja, jb) as phase_window, [ga, gb) as
// gauss_range.
template <bool SEC>
__device__ inline int4 tile_range(const ProbDev &P, const StepDev &st,
                                  const double *phi, int s, int t, int k,
                                  int2 *side) {
#pragma clang fp contract(off)
    const int i0 = t * kTile, i1 = min(i0 + kTile, P.N);
    const double xa = P.x[i0], xb = P.x[i1 - 1];
    const PhaseWin pw = phase_window<SEC>(P, phi + (size_t)s * P.D * P.K, k, i0, i1,
                                          st.lo + (size_t)s * P.T,
                                          st.hi + (size_t)s * P.T);
    const int2 g = gauss_range<SEC>(P, pw, k, xa, xb);
    if (side) {
        const int jr = first_centre_above(P.pos, g.x, g.y, pw.mu, xa);
        const int jl = first_centre_above(P.pos, jr, g.y, pw.mu, xb);
        *side = make_int2(jr, jl);
    }
    return make_int4(pw.ja, g.x, g.y, pw.jb);
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

// NW waves per block (kWaves, or more for grids too small to fill the GPU).
template <int NW>
struct FusedSmemT {
    float sig[NW][kTile];
    float rres[kTile];
    double red[NW];
};
using FusedSmem = FusedSmemT<kWaves>;

// ---- fused profile + likelihood + adjoint of one (tile, sample) ---------
//
// NW waves (kWaves = 4 unless the grid is too small to fill the GPU) split
// the phases (k = wave, wave + NW, ...).  Every wave holds
// the same kTile points, kPPL per lane (point i0 + p*64 + lane).  Peak data
// are wave-uniform (scalar loads).  Per phase the peaks run in segments:
// [ja, ga) and [gb, jb) need only the Lorentzian, [ga, gb) both components.
// For asymmetric peaks [ga, gb) splits further at jr and jl: the tile lies
// above the centres of [ja, jr), straddles those of [jr, jl) and lies below
// those of [jl, jb), so only [jr, jl) picks the width per point.
// WIN: each lane is masked by the peak's exact window.  The step kernels use
// this tile for the dense mode (WIN = false, every peak reaches every
// point); the windowed forward is win_tile below, whose global-memory path
// reuses the segment loops with WIN = true.
template <bool WIN>
struct PeakMask {
    int lo, hi;
    __device__ __forceinline__ float apply(int i, float t) const {
        if (!WIN) return t;
        return (unsigned)(i - lo) < (unsigned)(hi - lo) ? t
                                                        : __builtin_huge_valf();
    }
};

// One peak as a segment loop sees it: tile-relative position (and, for the
// peaks near the tile, the rounding error of that position), intensity,
// (windowed mode) its grid window [lo, hi) and, with the sec width law,
// c = |cos theta| and tw = tan(theta) (pi/360) w (the intensity is then
// I c).
struct PeakRec {
    float pt, ptl, I;
    int lo, hi;
    float c, tw;
};

struct SegPeaks {
    cptr<float> pt;       // tile-relative positions
    cptr<float> ptl;      // their rounding errors
    cptr<float> inten;
    cptr<int> wlo, whi;   // windows (WIN)
    cptr<float> sec;      // per-sample sec-law records, 4 floats each (SEC)
    // scalar loads (unused fields are never loaded)
    template <bool SEC, bool NEAR>
    __device__ __forceinline__ PeakRec rec(int j) const {
        const float l = NEAR ? ptl[j] : 0.f;
        if (SEC)
            return PeakRec{pt[j], l, sec[4 * j + 1], wlo[j], whi[j], sec[4 * j],
                           sec[4 * j + 2]};
        return PeakRec{pt[j], l, inten[j], wlo[j], whi[j], 1.f, 0.f};
    }
};

// Side of a segment: the points lie below the peak centres (or the peaks are
// symmetric), above them, or on both sides (chosen per point).
enum { kBelow = 0, kAbove = 1, kBoth = 2 };

// The lane's points as one phase's segment loops see them (mu: the phase's
// FP32 shift; iw2, iw2r: 2 / (A w) below and above the centre).  Two forms
// of q2 = 2 (x - rho) / (A w) for a peak at tile-relative position pt:
//   far:  q2 = fma(-pt, iw2, uq),                   uq  = (u - mu) iw2,
//   near: q2 = fma(u - pt, iw2, fma(-ptl, iw2, uql)), uql = (ul - mu) iw2.
// The far form carries the rounding of u, pt and uq, an absolute error in
// x - rho of a few 1e-8 times the tile's extent in degrees: harmless where
// q2 is large, but near the centre of a narrow peak, where the Gaussian is
// steep, it would set the profile's error.  The near form subtracts the
// rounded parts first (u - pt is exact or carries only its own relative
// rounding) and adds the small rounding errors ul and ptl separately, so
// that x - rho keeps a relative error of a few units of FP32 rounding.
// Peaks whose Gaussian reaches the tile take the near form (two more VALU
// operations per point), the others the far form.
struct PhasePts {
    float uq[kPPL], uqr[kPPL], uql[kPPL], uqlr[kPPL];
    __device__ __forceinline__ void set(const float (&u)[kPPL],
                                        const float (&ul)[kPPL], float mu,
                                        float iw2, float iw2r, bool asym) {
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            const float um = u[p] - mu, ulm = ul[p] - mu;
            uq[p] = um * iw2;
            uql[p] = ulm * iw2;
            uqr[p] = asym ? um * iw2r : uq[p];
            uqlr[p] = asym ? ulm * iw2r : uql[p];
        }
    }
};

// q2 of point p for peak r, and whether the point lies at or above the
// centre (the side of an asymmetric peak).  Sec law: the constant-width q2
// scaled by the peak's c.
struct SegQ {
    float q2;
    bool up;
};
template <int SIDE, bool NEAR, bool SEC>
__device__ __forceinline__ SegQ seg_q(const PeakRec &r, float u,
                                      const PhasePts &pp, int p, float iw2,
                                      float iw2r) {
    float ql = 0.f, qr = 0.f;
    if (NEAR) {
        const float d = u - r.pt;
        if (SIDE != kAbove) ql = fmaf(d, iw2, fmaf(-r.ptl, iw2, pp.uql[p]));
        if (SIDE != kBelow) qr = fmaf(d, iw2r, fmaf(-r.ptl, iw2r, pp.uqlr[p]));
    } else {
        if (SIDE != kAbove) ql = fmaf(-r.pt, iw2, pp.uq[p]);
        if (SIDE != kBelow) qr = fmaf(-r.pt, iw2r, pp.uqr[p]);
    }
    const bool up = SIDE == kAbove || (SIDE == kBoth && ql >= 0.f);
    const float q = SIDE == kBelow ? ql : (SIDE == kAbove ? qr : (up ? qr : ql));
    return SegQ{SEC ? r.c * q : q, up};
}

// Forward terms of the peaks [j0, j1) of one phase: accL += I l, accG += I e
// (GAUSS) with l = 1 / (1 + q2^2), e = 2^(-1 - q2^2) (see phase_consts);
// GAUSS segments take the near form of q2.
template <bool WIN, bool GAUSS, int SIDE, bool SEC, typename PK>
__device__ __forceinline__ void fwd_segment(const PK &pk, int j0, int j1,
                                            const int (&idx)[kPPL],
                                            const float (&u)[kPPL],
                                            const PhasePts &pp,
                                            float iw2, float iw2r,
                                            float (&accL)[kPPL],
                                            float (&accG)[kPPL]) {
#pragma unroll 2
    for (int j = j0; j < j1; ++j) {
        const PeakRec r = pk.template rec<SEC, GAUSS>(j);
        const float I = r.I;
        PeakMask<WIN> mk;
        if (WIN) { mk.lo = r.lo; mk.hi = r.hi; }
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            const float q2 = seg_q<SIDE, GAUSS, SEC>(r, u[p], pp, p, iw2, iw2r).q2;
            const float tt = mk.apply(idx[p], fmaf(q2, q2, 1.0f));
            accL[p] = fmaf(I, rcp_f32(tt), accL[p]);
            if (GAUSS) accG[p] = fmaf(I, exp2_f32(-tt), accG[p]);
        }
    }
}

// Per point and phase: l0 = sum I l, l1 = sum I l^2 q2, l2 = sum I l^2,
// e0 = sum I e, e1 = sum I e q2, e2 = sum I e q2^2 (e = 2^(-1 - q2^2),
// l = 1/(1 + q2^2)).
struct Acc6 {
    float l0[kPPL], l1[kPPL], l2[kPPL], e0[kPPL], e1[kPPL], e2[kPPL];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int p = 0; p < kPPL; ++p)
            l0[p] = l1[p] = l2[p] = e0[p] = e1[p] = e2[p] = 0.f;
    }
};

// Sec law: the shift moves the centre and, through W(rho), the width, so
// the mu sums take per-peak weights (side A: A = 1 below, alpha above):
//   e1 += I e (c q2 + kG (2 ln2 q2^2 - 1)),  kG = A tw / (4 ln2),
//   l1 += I l (c q2 l + kL (1 - 2 l)),       kL = A tw / 4,
// which phase_grad turns into d/dmu exactly as the plain sums (c = 1,
// tw = 0).  With q2^2 = tt - 1 the Gaussian weight is
// c q2 + bG tt + gG, bG = A tw / 2, gG = -A tw (1/2 + 1/(4 ln2)).
struct SecW {
    float bG, gG, kL;
    __device__ __forceinline__ static SecW of(float tws) {
        constexpr float kInv4Ln2 = 0.36067376022224085f;   // 1 / (4 ln 2)
        return SecW{0.5f * tws, -tws * (0.5f + kInv4Ln2), 0.25f * tws};
    }
};

// Adds the peak terms of [j0, j1) to `lo` (points below the centres, or
// symmetric peaks) or `hi` (points above).  ka: alpha of the phase (sec law
// with asymmetric peaks; 1 otherwise).
template <bool WIN, bool GAUSS, int SIDE, bool SEC>
__device__ __forceinline__ void adj_segment(const SegPeaks &pk, int j0, int j1,
                                            const int (&idx)[kPPL],
                                            const float (&u)[kPPL],
                                            const PhasePts &pp,
                                            float iw2, float iw2r, float ka,
                                            Acc6 &lo, Acc6 &hi) {
#pragma unroll 2
    for (int j = j0; j < j1; ++j) {
        const PeakRec r = pk.template rec<SEC, GAUSS>(j);
        const float I = r.I;
        SecW wl{0.f, 0.f, 0.f}, wh{0.f, 0.f, 0.f};
        if (SEC) {
            if (SIDE != kAbove) wl = SecW::of(r.tw);
            if (SIDE != kBelow) wh = SecW::of(r.tw * ka);
        }
        PeakMask<WIN> mk;
        if (WIN) { mk.lo = r.lo; mk.hi = r.hi; }
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            const SegQ sq = seg_q<SIDE, GAUSS, SEC>(r, u[p], pp, p, iw2, iw2r);
            const float q2 = sq.q2;
            const float tt = mk.apply(idx[p], fmaf(q2, q2, 1.0f));
            const float l = rcp_f32(tt);
            const float Il = I * l;
            const float Ill = Il * l;
            float Ie = 0.f, Ieq = 0.f;
            if (GAUSS) {
                Ie = I * exp2_f32(-tt);
                Ieq = Ie * q2;
            }
            if (SIDE != kBoth) {
                Acc6 &a = SIDE == kAbove ? hi : lo;
                a.l0[p] += Il;
                a.l2[p] += Ill;
                if (SEC) {
                    const SecW &sw = SIDE == kAbove ? wh : wl;
                    a.l1[p] = fmaf(Ill, fmaf(r.c, q2, -2.f * sw.kL), a.l1[p]);
                    a.l1[p] = fmaf(Il, sw.kL, a.l1[p]);
                } else {
                    a.l1[p] = fmaf(Ill, q2, a.l1[p]);
                }
                if (GAUSS) {
                    a.e0[p] += Ie;
                    if (SEC) {
                        const SecW &sw = SIDE == kAbove ? wh : wl;
                        a.e1[p] = fmaf(Ie, fmaf(r.c, q2, fmaf(sw.bG, tt, sw.gG)),
                                       a.e1[p]);
                    } else {
                        a.e1[p] += Ieq;
                    }
                    a.e2[p] = fmaf(Ieq, q2, a.e2[p]);
                }
            } else {
                const float Ieqq = Ieq * q2;
                const bool up = sq.up;
                const float fu = up ? 1.f : 0.f;
                const float fd = 1.f - fu;
                float m1L, m1G = 0.f;
                if (SEC) {
                    const float kL = up ? wh.kL : wl.kL;
                    m1L = fmaf(Ill, fmaf(r.c, q2, -2.f * kL), Il * kL);
                    if (GAUSS) {
                        const float bG = up ? wh.bG : wl.bG;
                        const float gG = up ? wh.gG : wl.gG;
                        m1G = Ie * fmaf(r.c, q2, fmaf(bG, tt, gG));
                    }
                } else {
                    m1L = Ill * q2;
                    m1G = Ieq;
                }
                hi.l0[p] = fmaf(fu, Il, hi.l0[p]);
                lo.l0[p] = fmaf(fd, Il, lo.l0[p]);
                hi.l2[p] = fmaf(fu, Ill, hi.l2[p]);
                lo.l2[p] = fmaf(fd, Ill, lo.l2[p]);
                hi.l1[p] = fmaf(fu, m1L, hi.l1[p]);
                lo.l1[p] = fmaf(fd, m1L, lo.l1[p]);
                if (GAUSS) {
                    hi.e0[p] = fmaf(fu, Ie, hi.e0[p]);
                    lo.e0[p] = fmaf(fd, Ie, lo.e0[p]);
                    hi.e1[p] = fmaf(fu, m1G, hi.e1[p]);
                    lo.e1[p] = fmaf(fd, m1G, lo.e1[p]);
                    hi.e2[p] = fmaf(fu, Ieqq, hi.e2[p]);
                    lo.e2[p] = fmaf(fd, Ieqq, lo.e2[p]);
                }
            }
        }
    }
}

// The six residual-weighted sums of `a` over the tile, wave totals written by
// lane 0 to dst[0..5] in the order (e0, e1, e2, l0, l1, l2).
__device__ __forceinline__ void store_sums(const Acc6 &a,
                                           const float (&rres)[kPPL],
                                           int lane, float *dst) {
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f;
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        v0 = fmaf(rres[p], a.e0[p], v0);
        v1 = fmaf(rres[p], a.e1[p], v1);
        v2 = fmaf(rres[p], a.e2[p], v2);
        v3 = fmaf(rres[p], a.l0[p], v3);
        v4 = fmaf(rres[p], a.l1[p], v4);
        v5 = fmaf(rres[p], a.l2[p], v5);
    }
    v0 = wave_total_f32(v0); v1 = wave_total_f32(v1);
    v2 = wave_total_f32(v2); v3 = wave_total_f32(v3);
    v4 = wave_total_f32(v4); v5 = wave_total_f32(v5);
    if (lane == 0) {
        dst[0] = v0; dst[1] = v1; dst[2] = v2;
        dst[3] = v3; dst[4] = v4; dst[5] = v5;
    }
}

// Point stage of a tile, after the waves' partial signals are in sig:
// f = B + signal in FP64, the tile's Poisson log-likelihood (to st.llp) and
// the residual y/f - 1 (to rres_lds, and to st.rres when it is set).
template <int NW = kWaves>
__device__ __forceinline__ void tile_points(const ProbDev &P, const StepDev &st,
                                            int t, int s, float *f_out,
                                            const float (*sig)[kTile],
                                            float *rres_lds, double *red) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i0 = t * kTile;
    double ll = 0.0;
    for (int q = threadIdx.x; q < kTile; q += NW * kWave) {
        const int i = i0 + q;
        float rr = 0.f;
        if (i < P.N) {
            double sg = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) sg += (double)sig[w][q];
            const double f = P.bg[i] + sg;
            if (f_out) f_out[(size_t)s * P.N + i] = (float)f;
            const double y = P.y[i];
            ll += (y != 0.0 ? y * log(f) : 0.0) - f - P.lgy[i];
            rr = (float)(y / f - 1.0);
            if (st.rres) st.rres[(size_t)s * P.N + i] = rr;
        }
        rres_lds[q] = rr;
    }
    ll = wave_sum(ll);
    if (lane == 0) red[wv] = ll;
    __syncthreads();
    if (threadIdx.x == 0 && st.llp) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) tot += red[w];
        st.llp[(size_t)s * P.ntiles + t] = tot;
    }
}

template <bool WIN, bool GRAD, bool ASYM, bool SEC, int NW = kWaves>
__device__ void fused_tile(const ProbDev &P, const StepDev &st, int t, int s,
                           float *f_out, FusedSmemT<NW> &sm) {
    const int lane = threadIdx.x & (kWave - 1);
    // wave index as a wave-uniform (scalar) value: loops over phases and
    // peaks then run on the scalar unit and peak data use scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i0 = t * kTile;
    cptr<float> pk = as_const(reinterpret_cast<const float *>(st.pk + (size_t)s * P.K));
    cptr<int> rg = as_const(reinterpret_cast<const int *>(
        st.rng + ((size_t)s * P.ntiles + t) * P.K));
    cptr<float> pkr = nullptr;
    cptr<int> rg2 = nullptr;
    if (ASYM) {
        pkr = as_const(st.pkr + (size_t)s * P.K);
        rg2 = as_const(reinterpret_cast<const int *>(
            st.rng2 + ((size_t)s * P.ntiles + t) * P.K));
    }
    SegPeaks sp;
    sp.pt = as_const(P.pt + (size_t)t * P.T);
    sp.ptl = as_const(P.ptl + (size_t)t * P.T);
    sp.inten = as_const(P.inten);
    sp.wlo = as_const(st.lo + (size_t)s * P.T);
    sp.whi = as_const(st.hi + (size_t)s * P.T);
    sp.sec = SEC ? as_const(reinterpret_cast<const float *>(st.psec + (size_t)s * P.T))
                 : nullptr;

    float u[kPPL], ul[kPPL];
    int idx[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        idx[p] = i0 + p * kWave + lane;
        u[p] = P.u[idx[p]];
        ul[p] = P.ul[idx[p]];
    }

    // ---------------- forward: partial signal over this wave's phases
    float sig[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) sig[p] = 0.f;

    for (int k = wv; k < P.K; k += NW) {
        const int ja = rg[4 * k], ga = rg[4 * k + 1], gb = rg[4 * k + 2],
                  jb = rg[4 * k + 3];
        if (ja >= jb) continue;
        const float iw2 = in_vgpr(pk[4 * k]);
        const float aG = pk[4 * k + 1], aL = pk[4 * k + 2], mu = pk[4 * k + 3];
        const float iw2r = ASYM ? in_vgpr(pkr[k]) : iw2;
        PhasePts pp;
        pp.set(u, ul, mu, iw2, iw2r, ASYM);
        float accL[kPPL], accG[kPPL];
#pragma unroll
        for (int p = 0; p < kPPL; ++p) {
            accL[p] = 0.f;
            accG[p] = 0.f;
        }
        if (ASYM) {
            const int jr = rg2[2 * k], jl = rg2[2 * k + 1];
            fwd_segment<WIN, false, kAbove, SEC>(sp, ja, ga, idx, u, pp, iw2, iw2r, accL, accG);
            fwd_segment<WIN, true, kAbove, SEC>(sp, ga, jr, idx, u, pp, iw2, iw2r, accL, accG);
            fwd_segment<WIN, true, kBoth, SEC>(sp, jr, jl, idx, u, pp, iw2, iw2r, accL, accG);
            fwd_segment<WIN, true, kBelow, SEC>(sp, jl, gb, idx, u, pp, iw2, iw2r, accL, accG);
            fwd_segment<WIN, false, kBelow, SEC>(sp, gb, jb, idx, u, pp, iw2, iw2r, accL, accG);
        } else {
            fwd_segment<WIN, false, kBelow, SEC>(sp, ja, ga, idx, u, pp, iw2, iw2r, accL, accG);
            fwd_segment<WIN, true, kBelow, SEC>(sp, ga, gb, idx, u, pp, iw2, iw2r, accL, accG);
            fwd_segment<WIN, false, kBelow, SEC>(sp, gb, jb, idx, u, pp, iw2, iw2r, accL, accG);
        }
#pragma unroll
        for (int p = 0; p < kPPL; ++p)
            sig[p] = fmaf(aL, accL[p], fmaf(aG, accG[p], sig[p]));
    }

#pragma unroll
    for (int p = 0; p < kPPL; ++p) sm.sig[wv][p * kWave + lane] = sig[p];
    __syncthreads();

    tile_points<NW>(P, st, t, s, f_out, sm.sig, sm.rres, sm.red);
    if (!GRAD) return;

    // ---------------- adjoint: recompute every peak value; the phase's sums
    // are sum_points (y/f - 1) * (per-point sums), reduced over the wave
    constexpr int NS = ASYM ? 12 : 6;
    float rres[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) rres[p] = sm.rres[p * kWave + lane];

    for (int k = wv; k < P.K; k += NW) {
        float *dst = st.part + (((size_t)t * P.K + k) * st.S + s) * NS;
        const int ja = rg[4 * k], ga = rg[4 * k + 1], gb = rg[4 * k + 2],
                  jb = rg[4 * k + 3];
        if (ja >= jb) {
            if (lane < NS) dst[lane] = 0.f;
            continue;
        }
        const float iw2 = in_vgpr(pk[4 * k]);
        const float mu = pk[4 * k + 3];
        const float iw2r = ASYM ? in_vgpr(pkr[k]) : iw2;
        PhasePts pp;
        pp.set(u, ul, mu, iw2, iw2r, ASYM);
        const float ka = ASYM && SEC ? iw2 / iw2r : 1.f;   // alpha
        Acc6 lo, hi;
        lo.zero();
        if (ASYM) {
            hi.zero();
            const int jr = rg2[2 * k], jl = rg2[2 * k + 1];
            adj_segment<WIN, false, kAbove, SEC>(sp, ja, ga, idx, u, pp, iw2, iw2r, ka, lo, hi);
            adj_segment<WIN, true, kAbove, SEC>(sp, ga, jr, idx, u, pp, iw2, iw2r, ka, lo, hi);
            adj_segment<WIN, true, kBoth, SEC>(sp, jr, jl, idx, u, pp, iw2, iw2r, ka, lo, hi);
            adj_segment<WIN, true, kBelow, SEC>(sp, jl, gb, idx, u, pp, iw2, iw2r, ka, lo, hi);
            adj_segment<WIN, false, kBelow, SEC>(sp, gb, jb, idx, u, pp, iw2, iw2r, ka, lo, hi);
        } else {
            adj_segment<WIN, false, kBelow, SEC>(sp, ja, ga, idx, u, pp, iw2, iw2r, ka, lo, hi);
            adj_segment<WIN, true, kBelow, SEC>(sp, ga, gb, idx, u, pp, iw2, iw2r, ka, lo, hi);
            adj_segment<WIN, false, kBelow, SEC>(sp, gb, jb, idx, u, pp, iw2, iw2r, ka, lo, hi);
        }
        store_sums(lo, rres, lane, dst);
        if (ASYM) store_sums(hi, rres, lane, dst + 6);
    }
}

// ---- windowed forward tile: flat peak records in LDS ------------------------
//
// In windowed mode only one or two peaks of a phase reach a tile, so a loop
// over phases would spend most of its time on per-phase set-up.  The block
// instead stages, 256 phases at a time, one record per peak that reaches the
// tile, holding all that its evaluation needs from its phase: the centre
// relative to the tile, 2 c / (A w) below and above the centre (c = 1 without
// the sec law; A = 1 below, alpha above), the Lorentzian and Gaussian
// amplitudes I h r cL n / w and I h (1 - r) cG n / w (times c with the sec
// law) and the window.  One thread per phase finds its phase's peak ranges
// over the tile and writes its records: those whose Gaussian reaches the
// tile from the front of the list, the others (Lorentzian only) from the
// back, so that each part is evaluated by a loop without a per-record
// branch.  The waves then share both parts.  Phases whose records do not
// fit the staging space (they come last in the chunk) are evaluated from
// global memory, phase by phase.
constexpr int kWinChunk = kBlock;   // phases staged at a time (one per thread)
// LDS for the staged peak records of a chunk, the same for the
// single-analysis and the batched forward: which phases take the
// global-memory path, and so the order in which a point's terms are summed,
// depends on it, and a served analysis gives the same bits as its
// one-at-a-time run only if both kernels stage alike.  21 KB hold 896
// symmetric or 672 asymmetric records (seven blocks per CU; the asymmetric
// forward's registers hold it to six).
constexpr int kWinRecBytes = 21 * 1024;

// A staged record.  Its FP32 centre relative to the tile is rounded;
// records whose Gaussian reaches the tile also carry that rounding error cl
// (x - rho is then formed as (u - centre) + (ul - cl), or on a uniform grid
// in grid steps as (u - centre) - cl with u exact, see win_record).
// Symmetric records keep the centre times the scale below (without the
// Gaussian) or cl times that scale (with it), so that q2 takes fused
// multiply-adds (see win_record).  The window is kept relative to the
// tile: its first point and length, both in [0, kTile], packed as
// first | length << 16.  One record is read with one address: 24 bytes
// (symmetric) or 32 (asymmetric: the scale above the centre as well).
template <bool ASYM>
struct alignas(8) WinRecord {
    float c, s, aL, aG;   // centre (or centre times s), 2c/(A w) below, amplitudes
    int wnd;              // window: first | length << 16
    float cl;             // the centre's rounding error (times s if symmetric)
    __device__ __forceinline__ float ahi() const { return s; }
    __device__ __forceinline__ static WinRecord make(float c, float s, float aL, float aG,
                                                     int wnd, float, float cl) {
        return WinRecord{c, s, aL, aG, wnd, cl};
    }
};
template <>
struct alignas(16) WinRecord<true> {
    float c, s, aL, aG;
    int wnd;
    float cl;
    float ah;             // 2c/(alpha w): the scale above the centre
    float pad;
    __device__ __forceinline__ float ahi() const { return ah; }
    __device__ __forceinline__ static WinRecord make(float c, float s, float aL, float aG,
                                                     int wnd, float ah, float cl) {
        return WinRecord{c, s, aL, aG, wnd, cl, ah, 0.f};
    }
};

// The window [lo, hi) of grid indices relative to the tile starting at i0,
// clamped to it, as a record holds it.
__device__ __forceinline__ int win_rel(int lo, int hi, int i0) {
    const int rl = min(max(lo - i0, 0), kTile), rh = min(max(hi - i0, 0), kTile);
    return rl | ((rh - rl) << 16);
}

template <bool ASYM>
struct WinSmem {
    static constexpr int kCap = kWinRecBytes / sizeof(WinRecord<ASYM>);
    struct Sums {
        float sig[kWaves][kTile];   // the waves' partial sums at the points
        float rres[kTile];
    };
    // the last chunk's records are consumed before the sums are written
    union {
        WinRecord<ASYM> rec[kCap];
        Sums e;
    };
    int wmax[kWaves], wmaxn[kWaves], wcnt[kWaves], wcntg[kWaves];
    double red[kWaves];
};

// The forward of one phase over the tile's points from global memory
// (phases whose records did not fit the staging space).
template <bool ASYM, bool SEC>
__device__ void win_phase_global(const SegPeaks &sp, int4 r, int2 r2,
                                 float4 cst, float iw2r,
                                 const float (&u)[kPPL], const float (&ul)[kPPL],
                                 const int (&idx)[kPPL], float (&sig)[kPPL]) {
    const int ja = __builtin_amdgcn_readfirstlane(r.x);
    const int ga = __builtin_amdgcn_readfirstlane(r.y);
    const int gb = __builtin_amdgcn_readfirstlane(r.z);
    const int jb = __builtin_amdgcn_readfirstlane(r.w);
    const float iw2 = cst.x, aG = cst.y, aL = cst.z, mu = cst.w;
    PhasePts pp;
    pp.set(u, ul, mu, iw2, iw2r, ASYM);
    float accL[kPPL], accG[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        accL[p] = 0.f;
        accG[p] = 0.f;
    }
    if (ASYM) {
        const int jr = __builtin_amdgcn_readfirstlane(r2.x);
        const int jl = __builtin_amdgcn_readfirstlane(r2.y);
        fwd_segment<true, false, kAbove, SEC>(sp, ja, ga, idx, u, pp, iw2, iw2r, accL, accG);
        fwd_segment<true, true, kAbove, SEC>(sp, ga, jr, idx, u, pp, iw2, iw2r, accL, accG);
        fwd_segment<true, true, kBoth, SEC>(sp, jr, jl, idx, u, pp, iw2, iw2r, accL, accG);
        fwd_segment<true, true, kBelow, SEC>(sp, jl, gb, idx, u, pp, iw2, iw2r, accL, accG);
        fwd_segment<true, false, kBelow, SEC>(sp, gb, jb, idx, u, pp, iw2, iw2r, accL, accG);
    } else {
        fwd_segment<true, false, kBelow, SEC>(sp, ja, ga, idx, u, pp, iw2, iw2r, accL, accG);
        fwd_segment<true, true, kBelow, SEC>(sp, ga, gb, idx, u, pp, iw2, iw2r, accL, accG);
        fwd_segment<true, false, kBelow, SEC>(sp, gb, jb, idx, u, pp, iw2, iw2r, accL, accG);
    }
#pragma unroll
    for (int p = 0; p < kPPL; ++p)
        sig[p] = fmaf(aL, accL[p], fmaf(aG, accG[p], sig[p]));
}

// One staged record's terms at the lane's points (lane and lane + 64 of
// the tile).  Only the lanes whose point lies in the window take part: a
// half tile the window misses is skipped by the whole wave.
// UNIF (a uniform grid): u holds the points' exact offsets from the
// tile's reference point in grid steps, and the records hold the centre,
// its rounding error and the scales in grid steps as well, so the points
// carry no rounding error of their own.
template <bool ASYM, bool GAUSS, bool UNIF>
__device__ __forceinline__ void win_record(const WinRecord<ASYM> r,
                                           const float (&u)[kPPL],
                                           const float (&ul)[kPPL], int lane,
                                           float (&sig)[kPPL]) {
    const float ah = r.ahi();
    const int d0 = lane - (r.wnd & 0xffff), len = r.wnd >> 16;
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        const bool in = (unsigned)(d0 + p * kWave) < (unsigned)len;
        if (GAUSS) {
            if (in) {
                asm volatile("");   // a branch, as below
                float q2;
                if (ASYM) {
                    const float d = UNIF ? (u[p] - r.c) - r.cl
                                         : (u[p] - r.c) + (ul[p] - r.cl);
                    q2 = d * (d >= 0.f ? ah : r.s);
                } else if (UNIF) {
                    // (u - centre) s - cl s, cl s kept in the record
                    q2 = fmaf(u[p] - r.c, r.s, -r.cl);
                } else {
                    // (u - centre) s + (ul s - cl s), cl s kept in the record
                    q2 = fmaf(u[p] - r.c, r.s, fmaf(ul[p], r.s, -r.cl));
                }
                const float tt = fmaf(q2, q2, 1.0f);
                sig[p] = fmaf(r.aL, rcp_f32(tt), sig[p]);
                sig[p] = fmaf(r.aG, exp2_f32(-tt), sig[p]);
            }
        } else if (in) {
            // (an empty volatile statement keeps a short body a branch, which
            // the wave skips when the half misses the window; the compiler
            // would otherwise evaluate it at both halves and select)
            asm volatile("");
            float q2;
            if (ASYM) {
                const float d = u[p] - r.c;
                q2 = d * (d >= 0.f ? ah : r.s);
            } else {
                // u s - centre s, centre s kept in the record (far peaks)
                q2 = fmaf(u[p], r.s, -r.c);
            }
            sig[p] = fmaf(r.aL, rcp_f32(fmaf(q2, q2, 1.0f)), sig[p]);
        }
    }
}

// Block order of the kernels over (tile, sample) grids.  The hardware deals
// consecutive blocks to the 8 XCDs in turn; block b takes (tile, sample)
// pairs from the (b mod 8)-th contiguous run of the tile-major,
// sample-fastest order, so each XCD's L2 holds the peak data near its own
// run of tiles.
constexpr int kXcds = 8;
__device__ __forceinline__ int2 xcd_tile_sample(int ntiles, int S) {
    const int nb = ntiles * S;
    const int b = blockIdx.x + blockIdx.y * gridDim.x;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    const int q = x * per + min(x, rem) + i;
    return make_int2(q / S, q % S);
}

// Block order of the windowed forward when S is a multiple of 8: XCD x
// takes samples [x S/8, (x+1) S/8) of every tile, tile by tile.  Its L2 then
// holds the window arrays of its own samples (each staged record reads its
// window's ends from them, one cache line per phase), which tile-major runs
// over all samples overflow when the phases are many.
__device__ __forceinline__ int2 xcd_sample_group(int S) {
    const int b = blockIdx.x + blockIdx.y * gridDim.x;
    const int G = S / kXcds, i = b / kXcds;
    return make_int2(i / G, (b % kXcds) * G + i % G);
}

// Whether the windowed forward stages its records in grid steps: a uniform
// grid of more than one point.
__host__ __device__ inline bool uses_grid_steps(const ProbDev &P) {
    return P.uniform != 0 && P.N > 1;
}

// UNIF (constant width, uniform grid): the staged records and the points
// are in grid steps relative to the tile's reference point (see win_record).
template <bool ASYM, bool SEC, bool UNIF, typename SM>
__device__ void win_tile(const ProbDev &P, const StepDev &st, int t, int s,
                         float *f_out, SM &sm) {
    static_assert(!(UNIF && SEC), "grid-step records need a constant width");
    constexpr int kCap = SM::kCap;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int i0 = t * kTile;
    const int K = P.K;
    const float4 *pkv = st.pk + (size_t)s * K;
    const float *pkrv = ASYM ? st.pkr + (size_t)s * K : nullptr;
    const float *ptt = P.pt + (size_t)t * P.T;
    const int *wlo = st.lo + (size_t)s * P.T;
    const int *whi = st.hi + (size_t)s * P.T;
    const float *psec = SEC ? reinterpret_cast<const float *>(st.psec + (size_t)s * P.T)
                            : nullptr;
    const double *ph = st.phi + (size_t)s * P.D * K;
    const int iref = min(i0 + kTile / 2, P.N - 1);
    const double xref = P.x[iref];   // the tile's reference
    const int i1 = min(i0 + kTile, P.N);
    const double xa = P.x[i0], xb = P.x[i1 - 1];
    SegPeaks sp;
    sp.pt = as_const(ptt);
    sp.ptl = as_const(P.ptl + (size_t)t * P.T);
    sp.inten = as_const(P.inten);
    sp.wlo = as_const(wlo);
    sp.whi = as_const(whi);
    sp.sec = as_const(psec);

    float u[kPPL], ul[kPPL], ug[kPPL];
    int idx[kPPL];
    float sig[kPPL];
#pragma unroll
    for (int p = 0; p < kPPL; ++p) {
        idx[p] = i0 + p * kWave + lane;
        u[p] = P.u[idx[p]];
        ul[p] = P.ul[idx[p]];
        ug[p] = (float)(idx[p] - iref);   // exact
        sig[p] = 0.f;
    }
    // grid steps per degree (uniform grid)
    const double gpd = P.inv_dx;

    for (int c0 = 0; c0 < K; c0 += kWinChunk) {
        const int nk = min(kWinChunk, K - c0);
        // this thread's phase: the peaks whose windows reach the tile and,
        // among them, those whose Gaussian does (found here: the windowed
        // forward is their only user), constants and counts
        PhaseWin pw{0, 0, 0, 0, 0.0, 0.0, 1.0, true};
        int2 gr = make_int2(0, 0);
        float4 cst = make_float4(0.f, 0.f, 0.f, 0.f);
        float iw2r = 0.f;
        if (tid < nk) {
            cst = pkv[c0 + tid];
            if (ASYM) iw2r = pkrv[c0 + tid];
            if constexpr (!SEC) {
                // constant width: among the step's candidates (written by
                // the candidate kernel before this one)
                pw = phase_window_cand(P, ph, c0 + tid, xa, xb,
                                       cand_read(P, st, t, c0 + tid), &gr);
            } else {
                pw = phase_window<SEC>(P, ph, c0 + tid, i0, i1, wlo, whi);
                gr = gauss_range<SEC>(P, pw, c0 + tid, xa, xb);
            }
        }
        const int cnt = pw.jb - pw.ja, cg = gr.y - gr.x;
        // inclusive prefixes over the block of the record counts and of the
        // Gaussian record counts
        int incl = cnt, inclg = cg;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int v = __shfl_up(incl, o, kWave);
            const int vg = __shfl_up(inclg, o, kWave);
            if (lane >= o) { incl += v; inclg += vg; }
        }
        if (lane == kWave - 1) { sm.wcnt[wv] = incl; sm.wcntg[wv] = inclg; }
        __syncthreads();
        for (int w = 0; w < wv; ++w) { incl += sm.wcnt[w]; inclg += sm.wcntg[w]; }
        const int excl = incl - cnt, exclg = inclg - cg, excln = excl - exclg;
        // records of the phases that fit (a prefix of the chunk: incl grows
        // with the phase index).  Records with a Gaussian fill the list from
        // the front, the others from the back, each in phase and peak order.
        const bool fits = tid < nk && incl <= kCap;
        if (fits) {
            const float iw2 = cst.x, aG = cst.y, aL = cst.z;
            // The tile-relative centre comes from the FP64 position and
            // shift (rounded once, its rounding error kept for the records
            // with the Gaussian), the window from the window step's arrays
            // (a load instead of a search: the forward is bound by VALU
            // issue), and the side of an asymmetric peak from the predicates
            // of the tile plan's side searches.
            for (int q = 0; q < cnt; ++q) {
                const int j = pw.ja + q;
                const double pj = P.pos[j];
                const float I = SEC ? psec[4 * j + 1] : P.inten[j];
                const float c = SEC ? psec[4 * j] : 1.f;
                // (in grid steps the scales are 2 dx / w: the degree scales
                // times dx)
                const float iw2u = UNIF ? (float)((double)iw2 * P.dx) : iw2;
                const float iw2ru = UNIF ? (float)((double)iw2r * P.dx) : iw2r;
                float alo = iw2u * c, ahi = alo;
                if (ASYM) {
                    // centre at or below the tile's first point: the tile
                    // lies above it; at or below its last: it straddles it
                    const float ar = iw2ru * c;
                    const double rho = pj + pw.mu;
                    if (!(rho > xa)) alo = ahi = ar;
                    else if (!(rho > xb)) ahi = ar;
                }
                const bool gauss = j >= gr.x && j < gr.y;
                const int slot = gauss ? exclg + (j - gr.x)
                                       : kCap - 1 - excln -
                                             (j < gr.x ? j - pw.ja : q - cg);
                const double cxd = (pj - xref) + pw.mu;
                const double cx = UNIF ? cxd * gpd : cxd;   // grid steps if UNIF
                const float cxf = (float)cx;
                // symmetric peaks keep the centre times the scale (records
                // without the Gaussian) or the rounding error of the centre
                // times the scale (with it), so that q2 takes fused
                // multiply-adds (see win_record)
                const int2 wnd = make_int2(wlo[j], whi[j]);
                const int whi_j = wnd.y < wnd.x ? wnd.x : wnd.y;
                const double cld = cx - (double)cxf;
                const float cl = (float)(ASYM ? cld : cld * (double)alo);
                sm.rec[slot] = WinRecord<ASYM>::make(
                    ASYM || gauss ? cxf : (float)(cx * (double)alo), alo, I * aL,
                    gauss ? I * aG : 0.f, win_rel(wnd.x, whi_j, i0), ahi, gauss ? cl : 0.f);
            }
        }
        // staged record counts and number of fitting phases
        const int ng = wave_max_i32(fits ? inclg : 0);
        const int nn = wave_max_i32(fits ? incl - inclg : 0);
        const int nfit = __builtin_popcountll(__ballot(fits));
        __syncthreads();                       // prefix words read, records written
        if (lane == 0) { sm.wmax[wv] = ng; }
        if (lane == 1) { sm.wmaxn[wv] = nn; }
        if (lane == 2) { sm.wcnt[wv] = nfit; }
        __syncthreads();
        int n_g = 0, n_n = 0, n_fit = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            n_g = max(n_g, sm.wmax[w]);
            n_n = max(n_n, sm.wmaxn[w]);
            n_fit += sm.wcnt[w];
        }
        n_g = __builtin_amdgcn_readfirstlane(n_g);
        n_n = __builtin_amdgcn_readfirstlane(n_n);
        n_fit = __builtin_amdgcn_readfirstlane(n_fit);

        // the waves share the two lists
        // (two records per pass, unrolled by hand: the volatile statements
        // in the record bodies keep the compiler from unrolling)
        const float (&uu)[kPPL] = UNIF ? ug : u;
        int f = wv;
        for (; f + kWaves < n_g; f += 2 * kWaves) {
            const WinRecord<ASYM> r0 = sm.rec[f], r1 = sm.rec[f + kWaves];
            win_record<ASYM, true, UNIF>(r0, uu, ul, lane, sig);
            win_record<ASYM, true, UNIF>(r1, uu, ul, lane, sig);
        }
        if (f < n_g) win_record<ASYM, true, UNIF>(sm.rec[f], uu, ul, lane, sig);
        for (f = wv; f + kWaves < n_n; f += 2 * kWaves) {
            const WinRecord<ASYM> r0 = sm.rec[kCap - 1 - f], r1 = sm.rec[kCap - 1 - f - kWaves];
            win_record<ASYM, false, UNIF>(r0, uu, ul, lane, sig);
            win_record<ASYM, false, UNIF>(r1, uu, ul, lane, sig);
        }
        if (f < n_n) win_record<ASYM, false, UNIF>(sm.rec[kCap - 1 - f], uu, ul, lane, sig);
        // phases that did not fit (every lane finds the same ranges)
        for (int kl = n_fit + wv; kl < nk; kl += kWaves) {
            const int k = c0 + kl;
            int2 rk2 = make_int2(0, 0);
            const int4 rk = tile_range<SEC>(P, st, st.phi, s, t, k, ASYM ? &rk2 : nullptr);
            win_phase_global<ASYM, SEC>(sp, rk, rk2, pkv[k], ASYM ? pkrv[k] : 0.f,
                                        u, ul, idx, sig);
        }
        __syncthreads();                       // records consumed
    }

#pragma unroll
    for (int p = 0; p < kPPL; ++p) sm.e.sig[wv][p * kWave + lane] = sig[p];
    __syncthreads();
    tile_points(P, st, t, s, f_out, sm.e.sig, sm.e.rres, sm.red);
}

// ---- peak-major adjoint (windowed mode) -----------------------------------
//
// One block of kWaves waves per (sample s, phase k); the phase's peaks go
// in groups of kAdjPeaks consecutive ones, group g to wave g mod kWaves.
// For every peak the lanes cover consecutive points of its window (64 at a
// time); x - rho is formed in FP64 and rounded to FP32 (its sign picks the
// side of an asymmetric peak), or for symmetric peaks of constant width on
// a uniform grid from FP32 offsets each rounded once (adjoint_phase).  Six
// sums (twelve: six per side) accumulate per lane over the wave's peaks,
// are reduced over the wave, then over the waves in fixed order.
// R = 0 for lanes outside the window (their terms vanish).  SEC: iw2 and
// iw2r carry the peak's c, and wl / wh are the mu-sum weights of the two
// sides (see SecW).  The Lorentzian terms and the Gaussian terms are two
// steps, so that a chunk of points where no Gaussian matters can skip the
// second.
struct AdjPt {
    float R, q2, tt;
    bool up;
};

template <bool ASYM, bool SEC>
__device__ __forceinline__ AdjPt adj_point_L(float R, float d, float iw2,
                                             float iw2r, float c,
                                             const SecW &wl, const SecW &wh,
                                             float (&acc)[ASYM ? 12 : 6]) {
    const bool up = ASYM && d >= 0.f;
    const float q2 = d * (up ? iw2r : iw2);
    const float tt = fmaf(q2, q2, 1.0f);
    const float l = rcp_f32(tt);
    const float Rl = R * l;
    const float Rll = Rl * l;
    float m1L;
    if (SEC) {
        const float kL = up ? wh.kL : wl.kL;
        m1L = fmaf(Rll, fmaf(c, q2, -2.f * kL), Rl * kL);
    } else {
        m1L = Rll * q2;
    }
    if (!ASYM) {
        acc[3] += Rl;
        acc[5] += Rll;
        if (SEC) acc[4] += m1L;
        else acc[4] = fmaf(Rll, q2, acc[4]);
    } else {
        const float fu = up ? 1.f : 0.f, fd = 1.f - fu;
        acc[3] = fmaf(fd, Rl, acc[3]);
        acc[9] = fmaf(fu, Rl, acc[9]);
        acc[5] = fmaf(fd, Rll, acc[5]);
        acc[11] = fmaf(fu, Rll, acc[11]);
        acc[4] = fmaf(fd, m1L, acc[4]);
        acc[10] = fmaf(fu, m1L, acc[10]);
    }
    return AdjPt{R, q2, tt, up};
}

template <bool ASYM, bool SEC>
__device__ __forceinline__ void adj_point_G(const AdjPt &pt, float c,
                                            const SecW &wl, const SecW &wh,
                                            float (&acc)[ASYM ? 12 : 6]) {
    const float q2 = pt.q2, tt = pt.tt;
    const float Re = pt.R * exp2_f32(-tt);
    const float Req = Re * q2;
    float m1G;
    if (SEC) {
        const float bG = pt.up ? wh.bG : wl.bG;
        const float gG = pt.up ? wh.gG : wl.gG;
        m1G = Re * fmaf(c, q2, fmaf(bG, tt, gG));
    } else {
        m1G = Req;
    }
    if (!ASYM) {
        acc[0] += Re;
        acc[1] += m1G;
        acc[2] = fmaf(Req, q2, acc[2]);
    } else {
        const float Reqq = Req * q2;
        const float fu = pt.up ? 1.f : 0.f, fd = 1.f - fu;
        acc[0] = fmaf(fd, Re, acc[0]);
        acc[6] = fmaf(fu, Re, acc[6]);
        acc[1] = fmaf(fd, m1G, acc[1]);
        acc[7] = fmaf(fu, m1G, acc[7]);
        acc[2] = fmaf(fd, Reqq, acc[2]);
        acc[8] = fmaf(fu, Reqq, acc[8]);
    }
}

// The Gaussian matters where |x - rho| <= kGaussReach w (the forward's
// rule): 1 + q2^2 <= 1 + (2 kGaussReach)^2.
constexpr float kGaussTT = (float)(1.0 + 4.0 * kGaussReach * kGaussReach);

// Word 3 of a gfx9-family buffer resource (32-bit data format, raw access).
constexpr int kBufferFlags = 0x00020000;

// Peaks a wave handles together: their scalar data and grid loads are issued
// back to back, so one memory latency covers all of them.
constexpr int kAdjPeaks = 4;

// Windows of at most this many FWHM each side (symmetric peaks of constant
// width on a uniform grid): the adjoint forms q2 = 2 (x - rho) / w in FP32.
// |q2| is at most 2c inside a window and its chunk offsets at most 4c, so
// each of its three roundings errs by at most 4c 2^-24: q2 is exact to
// 12c 2^-24, about 6e-6 at c = 8 and 1.1e-5 at this bound (a relative
// gradient error of that order, against a bar of 1e-4).
constexpr double kF32Cutoff = 16.0;

template <bool ASYM, bool SEC>
__device__ inline void adjoint_phase(const ProbDev &P, const StepDev &st,
                                     int s, int k, double (*red)[12]) {
    constexpr int NS = ASYM ? 12 : 6;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int K = P.K;
    const double *ph = st.phi + (size_t)s * P.D * K;
    const double mu = ph[K + k];
    const float iw2 = (float)(2.0 / ph[2 * K + k]);
    const float iw2r = ASYM ? asym_iw2(ph[2 * K + k], ph[4 * K + k]) : iw2;
    // constant width: x - rho is formed already scaled by 2/w in FP64, so
    // that q2 below the centre is one rounding of it (above the centre of an
    // asymmetric peak it is that times 1/alpha); symmetric peaks on a uniform
    // grid take FP32 from there (the chunk loop)
    const double iw2d = 2.0 / ph[2 * K + k];
    const float up_ratio = ASYM ? (float)(1.0 / ph[4 * K + k]) : 1.f;
    // bounded buffer views of the residual (one per peak, below) and the
    // grid: 32-bit offsets, and reads past the end return 0
    const float *rres_s = st.rres + (size_t)s * P.N;
    const __amdgpu_buffer_rsrc_t x_rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)P.x, (short)0, P.N * 8, kBufferFlags);
    cptr<int> wlo = as_const(st.lo + (size_t)s * P.T);
    cptr<int> whi = as_const(st.hi + (size_t)s * P.T);
    cptr<double> pos = as_const(P.pos);
    cptr<float> inten = as_const(P.inten);
    cptr<float> psec = SEC ? as_const(reinterpret_cast<const float *>(st.psec + (size_t)s * P.T))
                           : nullptr;
    const float ka = ASYM ? (float)ph[4 * K + k] : 1.f;
    const bool unif = P.formed_x != 0;
    const double xl = fma((double)lane, P.dx, P.x0);   // uniform grid: x0 + lane dx
    const double dxw = kWave * P.dx;                     // one chunk of points
    const int a = P.off[k], b = P.off[k + 1];
    float acc[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) acc[c] = 0.f;
    // the phase's peaks in groups of kAdjPeaks consecutive ones (neighbours
    // in position, with windows of one length), group g to wave g mod 4: only
    // the phase's last group can be short
    for (int j0 = a + kAdjPeaks * wv; j0 < b; j0 += kWaves * kAdjPeaks) {
        int lo[kAdjPeaks], len[kAdjPeaks];
        float I[kAdjPeaks], cq[kAdjPeaks], tw[kAdjPeaks];
        double rho[kAdjPeaks];
        int span = 0;
#pragma unroll
        for (int q = 0; q < kAdjPeaks; ++q) {
            const int j = j0 + q;
            const bool ok = j < b;
            const int jj = ok ? j : j0;
            lo[q] = wlo[jj];
            len[q] = ok ? whi[jj] - lo[q] : 0;
            if (SEC) {
                cq[q] = psec[4 * jj];
                I[q] = psec[4 * jj + 1];
                tw[q] = psec[4 * jj + 2];
            } else {
                cq[q] = 1.f;
                I[q] = inten[jj];
                tw[q] = 0.f;
            }
            rho[q] = pos[jj] + mu;
            span = max(span, len[q]);
        }
        // each peak's residuals through a buffer view that ends with its
        // window: lanes past the window read 0 and so weigh their point by 0
        __amdgpu_buffer_rsrc_t rq[kAdjPeaks];
        // x_i - rho = e + t in FP64.  On a uniform grid x_i is formed, not
        // loaded, so only the residuals are read: e is the lane's offset in
        // the first chunk, x0 + (lo + lane) dx - rho, and t the chunk's c dx;
        // otherwise e = -rho and t = x_i, loaded.  With a constant width e
        // and t carry the factor 2/w (e by a multiply here, c dx by the
        // chunk step, a loaded x_i by a fused multiply-add)
        double e[kAdjPeaks];
#pragma unroll
        for (int q = 0; q < kAdjPeaks; ++q) {
            rq[q] = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(rres_s + lo[q]), (short)0, len[q] * 4, kBufferFlags);
            e[q] = unif ? fma((double)lo[q], P.dx, xl) - rho[q] : -rho[q];
            if (!SEC) e[q] *= iw2d;
        }
        // the chunks of the peaks' windows, one loop per kind of grid
        auto chunks = [&](auto unif_tag) {
            constexpr bool UNIF = decltype(unif_tag)::value;
            // symmetric peaks of constant width on a uniform grid: q2 is
            // formed in FP32 as the chunk's index times the chunk step plus
            // the lane's offset, each rounded once (one fused multiply-add
            // per point instead of an FP64 sum and a conversion; no side of
            // a peak depends on its sign)
            constexpr bool F32 = UNIF && !SEC && !ASYM;
            // the chunk's c dx (scaled by 2/w with a constant width)
            const double step = SEC ? dxw : dxw * iw2d;
            const float stepf = (float)step;
            float ef[kAdjPeaks];
#pragma unroll
            for (int q = 0; q < kAdjPeaks; ++q) ef[q] = (float)e[q];
            double cdx = 0.0;
            float cf = 0.f;
            for (int c = 0; c < span; c += kWave, cdx += step, cf += 1.f) {
                float R[kAdjPeaks], rv[kAdjPeaks], d[kAdjPeaks];
                double xv[kAdjPeaks];
#pragma unroll
                for (int q = 0; q < kAdjPeaks; ++q) {
                    // every lane loads; points past the grid's end (a window
                    // ending at N, or lo = N for an empty one) read 0 from
                    // the bounded grid view, and their residual is 0
                    rv[q] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(rq[q], (c + lane) * 4, 0, 0));
                    if (!UNIF)
                        xv[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                               x_rs, (lo[q] + c + lane) * 8, 0, 0));
                }
                // all loads are issued before the first use, so one memory
                // latency covers them
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < kAdjPeaks; ++q) {
                    R[q] = rv[q] * I[q];
                    // sec law: x - rho; constant width: (x - rho) 2/w
                    d[q] = F32 ? fmaf(cf, stepf, ef[q])
                               : (float)(SEC || UNIF ? e[q] + (UNIF ? cdx : xv[q])
                                                     : fma(xv[q], iw2d, e[q]));
                }
                AdjPt pt[kAdjPeaks];
                SecW wl[kAdjPeaks], wh[kAdjPeaks];
                bool gauss = false;
#pragma unroll
                for (int q = 0; q < kAdjPeaks; ++q) {
                    wl[q] = SecW::of(SEC ? tw[q] : 0.f);
                    wh[q] = SecW::of(SEC ? tw[q] * ka : 0.f);
                    pt[q] = SEC ? adj_point_L<ASYM, SEC>(R[q], d[q], iw2 * cq[q], iw2r * cq[q],
                                                         cq[q], wl[q], wh[q], acc)
                                : adj_point_L<ASYM, SEC>(R[q], d[q], 1.f, up_ratio, 1.f,
                                                         wl[q], wh[q], acc);
                    // (points outside the window lie beyond 8 FWHM: no effect)
                    gauss = gauss | (pt[q].tt <= kGaussTT);
                }
                // one wave-uniform branch over the four peaks' Gaussian terms
                // (a ballot is a scalar value: no lane-to-scalar move)
                if (__builtin_amdgcn_ballot_w64(gauss) != 0) {
#pragma unroll
                    for (int q = 0; q < kAdjPeaks; ++q)
                        adj_point_G<ASYM, SEC>(pt[q], cq[q], wl[q], wh[q], acc);
                }
            }
        };
        if (unif)
            chunks(std::true_type{});
        else
            chunks(std::false_type{});
    }
#pragma unroll
    for (int c = 0; c < NS; ++c) acc[c] = wave_total_f32(acc[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NS; ++c) red[wv][c] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double v = 0.0;
        for (int w = 0; w < kWaves; ++w) v += red[w][threadIdx.x];
        st.pw[((size_t)k * st.S + s) * NS + threadIdx.x] = v;
    }
}

}  // namespace xrdvi
