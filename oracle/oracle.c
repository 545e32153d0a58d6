/*
 * FP64 CPU oracle for the variational phase-identification hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, constant or helper
 * with the HIP library.
 *
 * Plain, slow, obviously correct: every quantity is computed in double
 * precision directly from its definition, with loops in the order the
 * paper writes its sums (phases k, peaks m, points i).  Build with
 * -O2 -fno-fast-math -ffp-contract=off so that no multiply-add is fused.
 *
 * Notation follows the paper (Appendix A): grid x_i, counts y_i,
 * background B_i, candidate phase k with peaks (p_m^(k), I_m^(k)),
 * per-phase latents h_k (weight), mu_k (shift), w_k (width), r_k
 * (Lorentz fraction), rho_mk = p_m^(k) + mu_k.
 *
 * Readings of the paper that this file relies on (each is listed, with
 * its reason, in the design notes):
 *  - G and L are unit-area Gaussian and Lorentzian sharing FWHM = w_k
 *    (the standard pseudo-Voigt the paper cites; its formulas are lost).
 *  - V = (1-r) G + r L: r is the Lorentz fraction (Appendix A.2).
 *  - Gamma priors use a rate: p(h) = lambda exp(-lambda h) (Sec. 2.2),
 *    w ~ Gam(shape 3, rate 100) (Appendix B.2).
 *  - mean-field Gaussian q in an unconstrained space z with
 *    h = exp(z_h), mu = z_mu, w = exp(z_w), r = logistic(z_r); the ELBO
 *    is the reparameterised Monte-Carlo estimate with analytic Gaussian
 *    entropy (Sec. 3.2).
 *  - an optional window: peak m of phase k contributes at x_i only when
 *    rho - c w <= x_i <= rho + c w (c = 0 means every point, the paper's
 *    dense sum).
 *  - optional width law: FWHM w_k sec(rho_mk / 2), with rho in degrees
 *    2-theta (Appendix A.2 defines sec; the formula using it is lost).
 *
 * Parity status: the peak shape, window rule, likelihood, priors, ELBO
 * assembly and gradient are pinned by the CPU tests (closed-form areas and
 * limits, library densities, identities, central finite differences,
 * brute-force subset enumeration).  Philox4x32-10 is pinned to the
 * published known-answer vectors.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- peak shape (Appendix A.2, pseudo-Voigt) -------------------------- */

/* Unit-area Gaussian with full width at half maximum w, centred at 0. */
static double gauss_fwhm(double d, double w)
{
    const double sigma = w / (2.0 * sqrt(2.0 * log(2.0)));
    return exp(-0.5 * (d / sigma) * (d / sigma)) / (sigma * sqrt(2.0 * M_PI));
}

/* Unit-area Lorentzian (Cauchy) with FWHM w, i.e. half width gamma = w/2. */
static double lorentz_fwhm(double d, double w)
{
    const double gamma = 0.5 * w;
    return gamma / (M_PI * (d * d + gamma * gamma));
}

/* Window rule: true when x lies in [rho - c w, rho + c w]; c = 0 keeps
 * every point.  Each bound is one rounded double operation. */
static int in_window(double x, double rho, double w, double c)
{
    if (c == 0.0) return 1;
    const double hw = c * w;
    const double lo = rho - hw;
    const double hi = rho + hw;
    return (lo <= x) && (x <= hi);
}

/* ---- profile f = S + B (Appendix A.2, signal eq.) --------------------- */

/* f[s][i] = B_i + sum_k h_k sum_m I_m V(x_i; rho_mk, w_k, r_k),
 * phi[s][4][K] holds the constrained (h, mu, w, r) of sample s. */
int oracle_profile(int N, int K, const double *x, const double *B,
                   const int *peak_off, const double *p, const double *I,
                   double c, int S, const double *phi, double *f)
{
    if (N < 1 || K < 1 || S < 1) return -1;
    #pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < S; ++s) {
        const double *h = phi + (size_t)s * 4 * K;
        const double *mu = h + K, *w = h + 2 * K, *r = h + 3 * K;
        double *fs = f + (size_t)s * N;
        for (int i = 0; i < N; ++i) fs[i] = B[i];
        for (int k = 0; k < K; ++k) {
            for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                const double rho = p[m] + mu[k];
                for (int i = 0; i < N; ++i) {
                    if (!in_window(x[i], rho, w[k], c)) continue;
                    const double d = x[i] - rho;
                    const double V = (1.0 - r[k]) * gauss_fwhm(d, w[k])
                                   + r[k] * lorentz_fwhm(d, w[k]);
                    fs[i] += h[k] * I[m] * V;
                }
            }
        }
    }
    return 0;
}

/* Window plan: lo[s][m] = first i inside, hi[s][m] = one past the last
 * (lo = hi when no point is inside), by a plain scan of the grid. */
int oracle_windows(int N, int K, const double *x, const int *peak_off,
                   const double *p, double c, int S, const double *phi,
                   int *lo, int *hi)
{
    const int T = peak_off[K];
    for (int s = 0; s < S; ++s) {
        const double *mu = phi + (size_t)s * 4 * K + K;
        const double *w = mu + K;
        for (int k = 0; k < K; ++k) {
            for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                const double rho = p[m] + mu[k];
                int first = -1, last = -1;
                for (int i = 0; i < N; ++i) {
                    if (in_window(x[i], rho, w[k], c)) {
                        if (first < 0) first = i;
                        last = i;
                    }
                }
                int *l = lo + (size_t)s * T + m, *u = hi + (size_t)s * T + m;
                if (first < 0) {
                    /* empty: both at the insertion point of rho */
                    int ins = 0;
                    while (ins < N && x[ins] < rho) ++ins;
                    *l = ins; *u = ins;
                } else {
                    *l = first; *u = last + 1;
                }
            }
        }
    }
    return 0;
}

/* ---- Poisson log-likelihood (Appendix A.2, likelihood eqs.) ---------- */

static double poisson_loglik(int N, const double *y, const double *f)
{
    double l = 0.0;
    for (int i = 0; i < N; ++i) {
        const double ylnf = (y[i] == 0.0) ? 0.0 : y[i] * log(f[i]);
        l += ylnf - f[i] - lgamma(y[i] + 1.0);
    }
    return l;
}

int oracle_loglik(int N, int S, const double *y, const double *f,
                  double *loglik)
{
    for (int s = 0; s < S; ++s)
        loglik[s] = poisson_loglik(N, y, f + (size_t)s * N);
    return 0;
}

/* ---- priors (Sec. 2.2 and Appendix B.2) -------------------------------- */

static double log_gamma_pdf(double v, double shape, double rate)
{
    return shape * log(rate) - lgamma(shape) + (shape - 1.0) * log(v)
         - rate * v;
}

static double log_normal_pdf(double v, double mean, double sd)
{
    const double u = (v - mean) / sd;
    return -log(sd * sqrt(2.0 * M_PI)) - 0.5 * u * u;
}

/* log prior of one phase: h ~ Gam(1, lambda) (exponential), mu ~ N(0, sd),
 * r ~ U(0,1), w ~ Gam(shape, rate). */
double oracle_log_prior(double h, double mu, double w, double r,
                        double lambda, double mu_sd, double w_shape,
                        double w_rate)
{
    (void)r;  /* uniform on [0,1]: log density 0 inside the support */
    return log_gamma_pdf(h, 1.0, lambda) + log_normal_pdf(mu, 0.0, mu_sd)
         + log_gamma_pdf(w, w_shape, w_rate);
}

/* ---- transforms of the mean-field Gaussian (Sec. 3.2) ----------------- */

static double softplus(double a)
{
    return a > 0.0 ? a + log1p(exp(-a)) : log1p(exp(a));
}

/* z -> (h, mu, w, r) and log|det J| of that map. */
static void transform(double zh, double zmu, double zw, double zr,
                      double *h, double *mu, double *w, double *r,
                      double *logjac)
{
    *h = exp(zh);
    *mu = zmu;
    *w = exp(zw);
    *r = 1.0 / (1.0 + exp(-zr));
    /* d h/dz = h, d w/dz = w, d r/dz = r (1-r) */
    *logjac = zh + zw - softplus(-zr) - softplus(zr);
}

/* ---- ELBO and its gradient --------------------------------------------- */

typedef struct {
    int N, K;
    const double *x, *y, *B;
    const int *peak_off;
    const double *p, *I;
    double c;
    double lambda, mu_sd, w_shape, w_rate;
} prob_t;

static double max_signal(const prob_t *P)
{
    double v = -INFINITY;
    for (int i = 0; i < P->N; ++i)
        if (P->y[i] - P->B[i] > v) v = P->y[i] - P->B[i];
    return v;
}

/*
 * ELBO estimate with S reparameterised samples z_s = m + exp(omega) eps_s:
 *   L = (1/S) sum_s [ ln p(Y|phi_s) + sum_k ln p(phi_sk) + ln|J(z_s)| ]
 *       + sum_j omega_j + (P/2)(1 + ln 2 pi),        P = 4K.
 * The last two terms are the entropy of the Gaussian q (Sec. 3.2: the
 * ELBO is E_q[ln p(Y,Phi) - ln q(Phi)]).
 *
 * When grad_loc/grad_logscale are non-NULL the exact gradient of this
 * estimate (window edges held fixed) is written as well.
 * loc, logscale: [4][K] (rows h, mu, w, r); eps: [S][4][K].
 */
int oracle_elbo(int N, int K, const double *x, const double *y,
                const double *B, const int *peak_off, const double *p,
                const double *I, double c, double lambda, double mu_sd,
                double w_shape, double w_rate, int S, const double *loc,
                const double *logscale, const double *eps, double *elbo,
                double *loglik, double *grad_loc, double *grad_logscale)
{
    if (N < 1 || K < 1 || S < 1) return -1;
    prob_t P = {N, K, x, y, B, peak_off, p, I, c, lambda, mu_sd, w_shape,
                w_rate};
    if (P.lambda == 0.0) {
        const double ymax = max_signal(&P);
        if (!(ymax > 0.0)) return -2;
        P.lambda = 1.0 / ymax;
    }
    const int D = 4 * K;
    double *phi = malloc(sizeof(double) * (size_t)S * D);
    double *z = malloc(sizeof(double) * (size_t)S * D);
    double *lpj = malloc(sizeof(double) * (size_t)S);
    double *ll = malloc(sizeof(double) * (size_t)S);
    double *gz = malloc(sizeof(double) * (size_t)S * D);
    double *f = malloc(sizeof(double) * (size_t)S * N);
    if (!phi || !z || !lpj || !ll || !gz || !f) {
        free(phi); free(z); free(lpj); free(ll); free(gz); free(f);
        return -3;
    }

    /* sample and transform */
    for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            double zz[4];
            for (int t = 0; t < 4; ++t) {
                const int j = t * K + k;
                const double sd = exp(logscale[j]);
                const double step = sd * eps[(size_t)s * D + j];
                zz[t] = loc[j] + step;
                z[(size_t)s * D + j] = zz[t];
            }
            double h, mu, w, r, lj;
            transform(zz[0], zz[1], zz[2], zz[3], &h, &mu, &w, &r, &lj);
            double *ph = phi + (size_t)s * D;
            ph[k] = h; ph[K + k] = mu; ph[2 * K + k] = w; ph[3 * K + k] = r;
            acc += oracle_log_prior(h, mu, w, r, P.lambda, mu_sd, w_shape,
                                    w_rate) + lj;
        }
        lpj[s] = acc;
    }

    /* profile and likelihood */
    oracle_profile(N, K, x, B, peak_off, p, I, c, S, phi, f);
    oracle_loglik(N, S, y, f, ll);

    double mean = 0.0;
    for (int s = 0; s < S; ++s) mean += ll[s] + lpj[s];
    mean /= (double)S;
    double ent = 0.0;
    for (int j = 0; j < D; ++j) ent += logscale[j];
    ent += 0.5 * (double)D * (1.0 + log(2.0 * M_PI));
    *elbo = mean + ent;
    if (loglik) for (int s = 0; s < S; ++s) loglik[s] = ll[s];

    if (grad_loc && grad_logscale) {
        const double ln2 = log(2.0);
        /* d lnL / d phi for every (s, k), then the chain rule to z */
        #pragma omp parallel for collapse(2) schedule(dynamic)
        for (int s = 0; s < S; ++s) {
            for (int k = 0; k < K; ++k) {
                const double *ph = phi + (size_t)s * D;
                const double h = ph[k], mu = ph[K + k], w = ph[2 * K + k],
                             r = ph[3 * K + k];
                const double *fs = f + (size_t)s * N;
                double gh = 0.0, gmu = 0.0, gw = 0.0, gr = 0.0;
                for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                    const double rho = p[m] + mu;
                    for (int i = 0; i < N; ++i) {
                        if (!in_window(x[i], rho, w, c)) continue;
                        const double rres = y[i] / fs[i] - 1.0;
                        const double d = x[i] - rho;
                        const double q = d / w;
                        const double G = gauss_fwhm(d, w);
                        const double L = lorentz_fwhm(d, w);
                        const double l = 1.0 / (1.0 + 4.0 * q * q);
                        const double a = rres * I[m];
                        /* f depends on phi through h V */
                        gh += a * ((1.0 - r) * G + r * L);
                        /* dG/dmu = G 8 ln2 q / w, dL/dmu = L 8 q l / w */
                        gmu += a * h * ((1.0 - r) * G * 8.0 * ln2 * q / w
                                        + r * L * 8.0 * q * l / w);
                        /* dG/dw = (G/w)(8 ln2 q^2 - 1),
                           dL/dw = (L/w)(8 q^2 l - 1) */
                        gw += a * h * ((1.0 - r) * (G / w)
                                           * (8.0 * ln2 * q * q - 1.0)
                                       + r * (L / w) * (8.0 * q * q * l - 1.0));
                        gr += a * h * (L - G);
                    }
                }
                /* chain to z, adding d/dz of log prior + log Jacobian */
                double *g = gz + (size_t)s * D;
                g[k] = h * gh - P.lambda * h + 1.0;
                g[K + k] = gmu - mu / (mu_sd * mu_sd);
                g[2 * K + k] = w * gw + (w_shape - 1.0) - w_rate * w + 1.0;
                g[3 * K + k] = r * (1.0 - r) * gr + 1.0 - 2.0 * r;
            }
        }
        for (int j = 0; j < D; ++j) {
            double gm = 0.0, go = 0.0;
            const double sd = exp(logscale[j]);
            for (int s = 0; s < S; ++s) {
                gm += gz[(size_t)s * D + j];
                go += gz[(size_t)s * D + j] * eps[(size_t)s * D + j] * sd;
            }
            grad_loc[j] = gm / (double)S;
            grad_logscale[j] = go / (double)S + 1.0;
        }
    }
    free(phi); free(z); free(lpj); free(ll); free(gz); free(f);
    return 0;
}

/* ---- asymmetric peaks (Appendix A.2, asymmetry factor A(x; alpha)) ----- */
/*
 * Reading of the lost equation that uses A: the peak keeps width w below
 * rho and takes width alpha w above it (A = alpha for x >= rho, 1 below),
 * with one common height at rho and the normalisation 2 / (1 + alpha), so
 * every peak keeps unit area:
 *   V(d) = 2/(1+alpha) * (w_A / w) * [(1-r) G(d; w_A) + r L(d; w_A)],
 *   w_A = w A(d).
 * alpha = 1 gives the symmetric pseudo-Voigt.  The window of a peak spans
 * rho - c w .. rho + (c w) alpha.  Latents per phase: (h, mu, w, r, alpha),
 * alpha = exp(z_alpha) with prior N(alpha_mean, alpha_sd) (Appendix B.2).
 */
static double voigt_asym(double d, double w, double r, double alpha)
{
    const double wA = (d >= 0.0) ? alpha * w : w;
    return 2.0 / (1.0 + alpha) * (wA / w)
         * ((1.0 - r) * gauss_fwhm(d, wA) + r * lorentz_fwhm(d, wA));
}

static int in_window_asym(double x, double rho, double w, double alpha,
                          double c)
{
    if (c == 0.0) return 1;
    const double hw = c * w;
    const double lo = rho - hw;
    const double hwr = hw * alpha;
    const double hi = rho + hwr;
    return (lo <= x) && (x <= hi);
}

/* f[s][i] with phi[s][5][K] rows (h, mu, w, r, alpha). */
int oracle_profile_asym(int N, int K, const double *x, const double *B,
                        const int *peak_off, const double *p,
                        const double *I, double c, int S, const double *phi,
                        double *f)
{
    if (N < 1 || K < 1 || S < 1) return -1;
    #pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < S; ++s) {
        const double *h = phi + (size_t)s * 5 * K;
        const double *mu = h + K, *w = h + 2 * K, *r = h + 3 * K,
                     *al = h + 4 * K;
        double *fs = f + (size_t)s * N;
        for (int i = 0; i < N; ++i) fs[i] = B[i];
        for (int k = 0; k < K; ++k) {
            for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                const double rho = p[m] + mu[k];
                for (int i = 0; i < N; ++i) {
                    if (!in_window_asym(x[i], rho, w[k], al[k], c)) continue;
                    fs[i] += h[k] * I[m] * voigt_asym(x[i] - rho, w[k], r[k],
                                                      al[k]);
                }
            }
        }
    }
    return 0;
}

int oracle_windows_asym(int N, int K, const double *x, const int *peak_off,
                        const double *p, double c, int S, const double *phi,
                        int *lo, int *hi)
{
    const int T = peak_off[K];
    for (int s = 0; s < S; ++s) {
        const double *mu = phi + (size_t)s * 5 * K + K;
        const double *w = mu + K, *al = mu + 3 * K;
        for (int k = 0; k < K; ++k) {
            for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                const double rho = p[m] + mu[k];
                int first = -1, last = -1;
                for (int i = 0; i < N; ++i) {
                    if (in_window_asym(x[i], rho, w[k], al[k], c)) {
                        if (first < 0) first = i;
                        last = i;
                    }
                }
                int *l = lo + (size_t)s * T + m, *u = hi + (size_t)s * T + m;
                if (first < 0) {
                    int ins = 0;
                    while (ins < N && x[ins] < rho) ++ins;
                    *l = ins; *u = ins;
                } else {
                    *l = first; *u = last + 1;
                }
            }
        }
    }
    return 0;
}

/*
 * ELBO of the asymmetric model (P = 5K coordinates) and its gradient; the
 * same estimator as oracle_elbo with alpha ~ N(alpha_mean, alpha_sd),
 * alpha = exp(z_alpha).  loc, logscale: [5][K]; eps: [S][5][K].
 */
int oracle_elbo_asym(int N, int K, const double *x, const double *y,
                     const double *B, const int *peak_off, const double *p,
                     const double *I, double c, double lambda, double mu_sd,
                     double w_shape, double w_rate, double alpha_mean,
                     double alpha_sd, int S, const double *loc,
                     const double *logscale, const double *eps, double *elbo,
                     double *loglik, double *grad_loc, double *grad_logscale)
{
    if (N < 1 || K < 1 || S < 1) return -1;
    prob_t P = {N, K, x, y, B, peak_off, p, I, c, lambda, mu_sd, w_shape,
                w_rate};
    if (P.lambda == 0.0) {
        const double ymax = max_signal(&P);
        if (!(ymax > 0.0)) return -2;
        P.lambda = 1.0 / ymax;
    }
    const int D = 5 * K;
    double *phi = malloc(sizeof(double) * (size_t)S * D);
    double *lpj = malloc(sizeof(double) * (size_t)S);
    double *ll = malloc(sizeof(double) * (size_t)S);
    double *gz = malloc(sizeof(double) * (size_t)S * D);
    double *f = malloc(sizeof(double) * (size_t)S * N);
    if (!phi || !lpj || !ll || !gz || !f) {
        free(phi); free(lpj); free(ll); free(gz); free(f);
        return -3;
    }
    for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            double zz[5];
            for (int t = 0; t < 5; ++t) {
                const int j = t * K + k;
                const double sd = exp(logscale[j]);
                const double step = sd * eps[(size_t)s * D + j];
                zz[t] = loc[j] + step;
            }
            double h, mu, w, r, lj;
            transform(zz[0], zz[1], zz[2], zz[3], &h, &mu, &w, &r, &lj);
            const double al = exp(zz[4]);
            double *ph = phi + (size_t)s * D;
            ph[k] = h; ph[K + k] = mu; ph[2 * K + k] = w; ph[3 * K + k] = r;
            ph[4 * K + k] = al;
            acc += oracle_log_prior(h, mu, w, r, P.lambda, mu_sd, w_shape,
                                    w_rate)
                 + log_normal_pdf(al, alpha_mean, alpha_sd) + lj + zz[4];
        }
        lpj[s] = acc;
    }
    oracle_profile_asym(N, K, x, B, peak_off, p, I, c, S, phi, f);
    oracle_loglik(N, S, y, f, ll);
    double mean = 0.0;
    for (int s = 0; s < S; ++s) mean += ll[s] + lpj[s];
    mean /= (double)S;
    double ent = 0.0;
    for (int j = 0; j < D; ++j) ent += logscale[j];
    ent += 0.5 * (double)D * (1.0 + log(2.0 * M_PI));
    *elbo = mean + ent;
    if (loglik) for (int s = 0; s < S; ++s) loglik[s] = ll[s];

    if (grad_loc && grad_logscale) {
        const double ln2 = log(2.0);
        const double cG = 2.0 * sqrt(ln2 / M_PI), cL = 2.0 / M_PI;
        #pragma omp parallel for collapse(2) schedule(dynamic)
        for (int s = 0; s < S; ++s) {
            for (int k = 0; k < K; ++k) {
                const double *ph = phi + (size_t)s * D;
                const double h = ph[k], mu = ph[K + k], w = ph[2 * K + k],
                             r = ph[3 * K + k], al = ph[4 * K + k];
                const double Na = 2.0 / (1.0 + al);
                const double *fs = f + (size_t)s * N;
                double gh = 0.0, gmu = 0.0, gw = 0.0, gr = 0.0, ga = 0.0;
                for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                    const double rho = p[m] + mu;
                    for (int i = 0; i < N; ++i) {
                        if (!in_window_asym(x[i], rho, w, al, c)) continue;
                        const double rres = y[i] / fs[i] - 1.0;
                        const double d = x[i] - rho;
                        const int right = d >= 0.0;
                        const double wA = right ? al * w : w;
                        const double q = d / wA;
                        /* V = Na v(q) / w with v = (1-r) cG g + r cL lam */
                        const double g = exp(-4.0 * ln2 * q * q);
                        const double lam = 1.0 / (1.0 + 4.0 * q * q);
                        const double v = (1.0 - r) * cG * g + r * cL * lam;
                        const double dv = (1.0 - r) * cG * (-8.0 * ln2 * q) * g
                                        + r * cL * (-8.0 * q) * lam * lam;
                        const double a = rres * I[m];
                        gh += a * Na * v / w;
                        gmu += a * h * Na * dv * (-1.0 / wA) / w;
                        gw += a * h * (-Na / (w * w)) * (v + q * dv);
                        gr += a * h * Na / w * (cL * lam - cG * g);
                        ga += a * h * (-Na / (1.0 + al) * v / w
                                       + (right ? Na / w * dv * (-q / al) : 0.0));
                    }
                }
                double *gzz = gz + (size_t)s * D;
                gzz[k] = h * gh - P.lambda * h + 1.0;
                gzz[K + k] = gmu - mu / (mu_sd * mu_sd);
                gzz[2 * K + k] = w * gw + (w_shape - 1.0) - w_rate * w + 1.0;
                gzz[3 * K + k] = r * (1.0 - r) * gr + 1.0 - 2.0 * r;
                gzz[4 * K + k] = al * ga
                               - al * (al - alpha_mean) / (alpha_sd * alpha_sd)
                               + 1.0;
            }
        }
        for (int j = 0; j < D; ++j) {
            double gm = 0.0, go = 0.0;
            const double sd = exp(logscale[j]);
            for (int s = 0; s < S; ++s) {
                gm += gz[(size_t)s * D + j];
                go += gz[(size_t)s * D + j] * eps[(size_t)s * D + j] * sd;
            }
            grad_loc[j] = gm / (double)S;
            grad_logscale[j] = go / (double)S + 1.0;
        }
    }
    free(phi); free(lpj); free(ll); free(gz); free(f);
    return 0;
}

/* ---- width growing with the Bragg angle (Appendix A.2, sec(x)) --------- */
/*
 * Reading of the lost width law that uses sec(x) = 1/cos(x): the full width
 * at half maximum of peak m of phase k follows the Scherrer-type law
 *   W_mk = w_k sec(theta_mk),   theta_mk = rho_mk / 2  (rho in deg 2-theta),
 * taken as w_k / |cos(rho_mk pi / 360)|, which stays positive for a shifted
 * centre past 180 deg.  The shape is the pseudo-Voigt (or its asymmetric
 * form) with W_mk in place of w_k, so every peak keeps unit area, and the
 * window of a peak spans rho - c W .. rho + (c W) alpha.  w_k is the width
 * at 2-theta -> 0.  D = 4 (h, mu, w, r) or 5 (with alpha).
 */
static double sec_width(double rho, double w)
{
    return w / fabs(cos(rho * (M_PI / 360.0)));
}

/* dW/drho = W tau with tau = tan(theta) pi / 360 (either sign of cos). */
static double sec_tau(double rho)
{
    return tan(rho * (M_PI / 360.0)) * (M_PI / 360.0);
}

static int in_window_sec(double x, double rho, double W, double alpha,
                         int D, double c)
{
    if (c == 0.0) return 1;
    const double hw = c * W;
    const double lo = rho - hw;
    const double hi = rho + (D == 5 ? hw * alpha : hw);
    return (lo <= x) && (x <= hi);
}

/* One peak of unit area at offset d = x - rho with FWHM W. */
static double shape_sec(double d, double W, double r, double alpha, int D)
{
    if (D == 5) return voigt_asym(d, W, r, alpha);
    return (1.0 - r) * gauss_fwhm(d, W) + r * lorentz_fwhm(d, W);
}

/* f[s][i] with phi[s][D][K]. */
int oracle_profile_sec(int N, int K, const double *x, const double *B,
                       const int *peak_off, const double *p, const double *I,
                       double c, int D, int S, const double *phi, double *f)
{
    if (N < 1 || K < 1 || S < 1 || (D != 4 && D != 5)) return -1;
    #pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < S; ++s) {
        const double *h = phi + (size_t)s * D * K;
        const double *mu = h + K, *w = h + 2 * K, *r = h + 3 * K;
        const double *al = D == 5 ? h + 4 * K : NULL;
        double *fs = f + (size_t)s * N;
        for (int i = 0; i < N; ++i) fs[i] = B[i];
        for (int k = 0; k < K; ++k) {
            const double a = al ? al[k] : 1.0;
            for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                const double rho = p[m] + mu[k];
                const double W = sec_width(rho, w[k]);
                for (int i = 0; i < N; ++i) {
                    if (!in_window_sec(x[i], rho, W, a, D, c)) continue;
                    fs[i] += h[k] * I[m] * shape_sec(x[i] - rho, W, r[k], a, D);
                }
            }
        }
    }
    return 0;
}

int oracle_windows_sec(int N, int K, const double *x, const int *peak_off,
                       const double *p, double c, int D, int S,
                       const double *phi, int *lo, int *hi)
{
    if (D != 4 && D != 5) return -1;
    const int T = peak_off[K];
    for (int s = 0; s < S; ++s) {
        const double *mu = phi + (size_t)s * D * K + K;
        const double *w = mu + K;
        const double *al = D == 5 ? mu + 3 * K : NULL;
        for (int k = 0; k < K; ++k) {
            for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                const double rho = p[m] + mu[k];
                const double W = sec_width(rho, w[k]);
                int first = -1, last = -1;
                for (int i = 0; i < N; ++i) {
                    if (in_window_sec(x[i], rho, W, al ? al[k] : 1.0, D, c)) {
                        if (first < 0) first = i;
                        last = i;
                    }
                }
                int *l = lo + (size_t)s * T + m, *u = hi + (size_t)s * T + m;
                if (first < 0) {
                    int ins = 0;
                    while (ins < N && x[ins] < rho) ++ins;
                    *l = ins; *u = ins;
                } else {
                    *l = first; *u = last + 1;
                }
            }
        }
    }
    return 0;
}

/*
 * ELBO and gradient of the model with the sec width law (D = 4 or 5; the
 * same estimator and priors as oracle_elbo / oracle_elbo_asym).  The shift
 * mu moves each peak and, through W(rho), widens or narrows it; both parts
 * enter d/dmu.
 */
int oracle_elbo_sec(int N, int K, const double *x, const double *y,
                    const double *B, const int *peak_off, const double *p,
                    const double *I, double c, double lambda, double mu_sd,
                    double w_shape, double w_rate, double alpha_mean,
                    double alpha_sd, int D, int S, const double *loc,
                    const double *logscale, const double *eps, double *elbo,
                    double *loglik, double *grad_loc, double *grad_logscale)
{
    if (N < 1 || K < 1 || S < 1 || (D != 4 && D != 5)) return -1;
    prob_t P = {N, K, x, y, B, peak_off, p, I, c, lambda, mu_sd, w_shape,
                w_rate};
    if (P.lambda == 0.0) {
        const double ymax = max_signal(&P);
        if (!(ymax > 0.0)) return -2;
        P.lambda = 1.0 / ymax;
    }
    const int DK = D * K;
    double *phi = malloc(sizeof(double) * (size_t)S * DK);
    double *lpj = malloc(sizeof(double) * (size_t)S);
    double *ll = malloc(sizeof(double) * (size_t)S);
    double *gz = malloc(sizeof(double) * (size_t)S * DK);
    double *f = malloc(sizeof(double) * (size_t)S * N);
    if (!phi || !lpj || !ll || !gz || !f) {
        free(phi); free(lpj); free(ll); free(gz); free(f);
        return -3;
    }
    for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            double zz[5];
            for (int t = 0; t < D; ++t) {
                const int j = t * K + k;
                const double sd = exp(logscale[j]);
                const double step = sd * eps[(size_t)s * DK + j];
                zz[t] = loc[j] + step;
            }
            double h, mu, w, r, lj;
            transform(zz[0], zz[1], zz[2], zz[3], &h, &mu, &w, &r, &lj);
            double *ph = phi + (size_t)s * DK;
            ph[k] = h; ph[K + k] = mu; ph[2 * K + k] = w; ph[3 * K + k] = r;
            acc += oracle_log_prior(h, mu, w, r, P.lambda, mu_sd, w_shape,
                                    w_rate) + lj;
            if (D == 5) {
                const double al = exp(zz[4]);
                ph[4 * K + k] = al;
                acc += log_normal_pdf(al, alpha_mean, alpha_sd) + zz[4];
            }
        }
        lpj[s] = acc;
    }
    oracle_profile_sec(N, K, x, B, peak_off, p, I, c, D, S, phi, f);
    oracle_loglik(N, S, y, f, ll);
    double mean = 0.0;
    for (int s = 0; s < S; ++s) mean += ll[s] + lpj[s];
    mean /= (double)S;
    double ent = 0.0;
    for (int j = 0; j < DK; ++j) ent += logscale[j];
    ent += 0.5 * (double)DK * (1.0 + log(2.0 * M_PI));
    *elbo = mean + ent;
    if (loglik) for (int s = 0; s < S; ++s) loglik[s] = ll[s];

    if (grad_loc && grad_logscale) {
        const double ln2 = log(2.0);
        const double cG = 2.0 * sqrt(ln2 / M_PI), cL = 2.0 / M_PI;
        #pragma omp parallel for collapse(2) schedule(dynamic)
        for (int s = 0; s < S; ++s) {
            for (int k = 0; k < K; ++k) {
                const double *ph = phi + (size_t)s * DK;
                const double h = ph[k], mu = ph[K + k], w = ph[2 * K + k],
                             r = ph[3 * K + k];
                const double al = D == 5 ? ph[4 * K + k] : 1.0;
                const double Na = D == 5 ? 2.0 / (1.0 + al) : 1.0;
                const double *fs = f + (size_t)s * N;
                double gh = 0.0, gmu = 0.0, gw = 0.0, gr = 0.0, ga = 0.0;
                for (int m = peak_off[k]; m < peak_off[k + 1]; ++m) {
                    const double rho = p[m] + mu;
                    const double W = sec_width(rho, w);
                    const double tau = sec_tau(rho);
                    for (int i = 0; i < N; ++i) {
                        if (!in_window_sec(x[i], rho, W, al, D, c)) continue;
                        const double rres = y[i] / fs[i] - 1.0;
                        const double d = x[i] - rho;
                        const int right = D == 5 && d >= 0.0;
                        const double A = right ? al : 1.0;
                        const double q = d / (A * W);
                        /* V = Na v(q) / W, v = (1-r) cG g + r cL lam */
                        const double g = exp(-4.0 * ln2 * q * q);
                        const double lam = 1.0 / (1.0 + 4.0 * q * q);
                        const double v = (1.0 - r) * cG * g + r * cL * lam;
                        const double dv = (1.0 - r) * cG * (-8.0 * ln2 * q) * g
                                        + r * cL * (-8.0 * q) * lam * lam;
                        const double a = rres * I[m];
                        /* dV/dd at fixed W, dV/dW at fixed d */
                        const double dVdd = Na * dv / (A * W * W);
                        const double dVdW = -Na / (W * W) * (v + q * dv);
                        gh += a * Na * v / W;
                        /* drho/dmu = 1, dW/dmu = W tau */
                        gmu += a * h * (-dVdd + dVdW * W * tau);
                        /* dW/dw = W / w */
                        gw += a * h * dVdW * W / w;
                        gr += a * h * Na / W * (cL * lam - cG * g);
                        if (D == 5)
                            ga += a * h * (-Na / (1.0 + al) * v / W
                                           + (right ? Na / W * dv * (-q / al)
                                                    : 0.0));
                    }
                }
                double *gzz = gz + (size_t)s * DK;
                gzz[k] = h * gh - P.lambda * h + 1.0;
                gzz[K + k] = gmu - mu / (mu_sd * mu_sd);
                gzz[2 * K + k] = w * gw + (w_shape - 1.0) - w_rate * w + 1.0;
                gzz[3 * K + k] = r * (1.0 - r) * gr + 1.0 - 2.0 * r;
                if (D == 5)
                    gzz[4 * K + k] = al * ga
                                   - al * (al - alpha_mean)
                                     / (alpha_sd * alpha_sd) + 1.0;
            }
        }
        for (int j = 0; j < DK; ++j) {
            double gm = 0.0, go = 0.0;
            const double sd = exp(logscale[j]);
            for (int s = 0; s < S; ++s) {
                gm += gz[(size_t)s * DK + j];
                go += gz[(size_t)s * DK + j] * eps[(size_t)s * DK + j] * sd;
            }
            grad_loc[j] = gm / (double)S;
            grad_logscale[j] = go / (double)S + 1.0;
        }
    }
    free(phi); free(lpj); free(ll); free(gz); free(f);
    return 0;
}

/* ---- posterior readout (Sec. 4: selection by area ratio) -------------- */

/*
 * With h = exp(z), z ~ N(m, s^2) under q: E[h] = exp(m + s^2/2) and
 * sd[h] = E[h] sqrt(exp(s^2) - 1) (log-normal moments).  Unit-area peaks
 * make phase k's area E[h_k] sum_m I_m; ratio = area / total area;
 * selected = ratio > threshold.  Returns -1 when the total is not positive.
 */
int oracle_readout(int K, const int *peak_off, const double *I,
                   const double *m, const double *logscale, double threshold,
                   double *mean_h, double *sd_h, double *ratio, int *selected)
{
    double total = 0.0;
    for (int k = 0; k < K; ++k) {
        const double s = exp(logscale[k]);
        mean_h[k] = exp(m[k] + 0.5 * s * s);
        sd_h[k] = mean_h[k] * sqrt(exp(s * s) - 1.0);
        double isum = 0.0;
        for (int j = peak_off[k]; j < peak_off[k + 1]; ++j) isum += I[j];
        ratio[k] = mean_h[k] * isum;
        total += ratio[k];
    }
    if (!(total > 0.0)) return -1;
    for (int k = 0; k < K; ++k) {
        ratio[k] /= total;
        selected[k] = ratio[k] > threshold;
    }
    return 0;
}

/* ---- Adam (Kingma & Ba 2015) on the maximisation of the ELBO ----------- */

/* One ascent step on theta with gradient g; m1, m2 are the moment
 * estimates, t the 1-based step count. */
void oracle_adam(int n, double *theta, double *m1, double *m2,
                 const double *g, int t, double lr, double b1, double b2,
                 double e)
{
    for (int j = 0; j < n; ++j) {
        m1[j] = b1 * m1[j] + (1.0 - b1) * g[j];
        m2[j] = b2 * m2[j] + (1.0 - b2) * g[j] * g[j];
        const double mh = m1[j] / (1.0 - pow(b1, (double)t));
        const double vh = m2[j] / (1.0 - pow(b2, (double)t));
        theta[j] += lr * mh / (sqrt(vh) + e);
    }
}

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------- */

/* Ten rounds of the Philox-4x32 bijection on counter ctr with key key. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n1 = lo1;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        const uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Standard-normal noise eps[s][j], j < D (j = t*K + k), for one step of one
 * analysis: counter (j / 4, s, step low, step high), key (seed low, seed
 * high); the four 32-bit words map to uniforms u = (v + 0.5) / 2^32 and
 * the pairs (u0,u1), (u2,u3) to normals by the Box-Muller transform
 * (cos then sin).
 */
void oracle_eps_philox_n(int S, int D, uint64_t seed, uint64_t step,
                         double *eps)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int s = 0; s < S; ++s) {
        for (int blk = 0; blk * 4 < D; ++blk) {
            const uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)s,
                                     (uint32_t)step, (uint32_t)(step >> 32)};
            uint32_t v[4];
            oracle_philox4x32_10(ctr, key, v);
            double u[4];
            for (int t = 0; t < 4; ++t)
                u[t] = ((double)v[t] + 0.5) / 4294967296.0;
            double n[4];
            for (int t = 0; t < 4; t += 2) {
                const double rad = sqrt(-2.0 * log(u[t]));
                n[t] = rad * cos(2.0 * M_PI * u[t + 1]);
                n[t + 1] = rad * sin(2.0 * M_PI * u[t + 1]);
            }
            for (int t = 0; t < 4; ++t) {
                const int j = blk * 4 + t;
                if (j < D) eps[(size_t)s * D + j] = n[t];
            }
        }
    }
}

/* Noise of the symmetric model: D = 4 K numbers per sample. */
void oracle_eps_philox(int S, int K, uint64_t seed, uint64_t step,
                       double *eps)
{
    oracle_eps_philox_n(S, 4 * K, seed, step, eps);
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
