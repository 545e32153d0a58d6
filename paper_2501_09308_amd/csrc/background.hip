// Background estimation before the analysis (App. A.2: the background is
// estimated beforehand by an iterative least-squares method): asymmetric
// least squares (Eilers and Boelens, 2005).  Repeatedly solve
//     (W + lambda D^T D) z = W y,   D the second-difference operator,
// and set w_i = p where y_i > z_i and 1 - p elsewhere (w = 1 at the start),
// so that the smooth curve z hugs the data from below.
//
// The system is symmetric positive definite and pentadiagonal; one thread
// per spectrum factors it as L D L^T (unit lower L of bandwidth 2) and
// solves in FP64.  Loads of the inputs are independent of the recurrence,
// so the unrolled loops issue them ahead of the dependent arithmetic.
#include <cmath>
#include <string>

#include "xrdvi.h"
#include "xrdvi_internal.h"

namespace xrdvi {

namespace {

// (D^T D)_{ij} for |i - j| <= 2, D the (N-2) x N second-difference matrix
// with rows (1, -2, 1) at columns k, k+1, k+2.
__device__ inline double dtd(int i, int j, int N) {
    const double c[3] = {1.0, -2.0, 1.0};
    const int k0 = max(max(i, j) - 2, 0), k1 = min(min(i, j), N - 3);
    double s = 0.0;
    for (int k = k0; k <= k1; ++k) s += c[i - k] * c[j - k];
    return s;
}

// One thread per spectrum b: n_iter reweighting iterations.  Scratch
// arrays [B][N]: w (weights), dg (pivots), l1 = L_{i,i-1}, l2 = L_{i,i-2}.
__global__ void k_asls(int B, int N, const double *__restrict__ y,
                       double *w, double *dg, double *l1, double *l2,
                       double *z, double lambda, double p, int n_iter) {
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const size_t o = (size_t)b * N;
    const double *yb = y + o;
    double *wb = w + o, *db = dg + o, *l1b = l1 + o, *l2b = l2 + o, *zb = z + o;
    if (N < 3) {                       // no second differences: z = y
        for (int i = 0; i < N; ++i) zb[i] = yb[i];
        return;
    }
    for (int i = 0; i < N; ++i) wb[i] = 1.0;
    for (int it = 0; it < n_iter; ++it) {
        // factor A = L D L^T and solve L u = W y in one forward sweep
        double dm1 = 0.0, dm2 = 0.0, lm1 = 0.0, um1 = 0.0, um2 = 0.0;
#pragma unroll 4
        for (int i = 0; i < N; ++i) {
            const double a = wb[i] + lambda * dtd(i, i, N);
            double L2 = 0.0, L1 = 0.0;
            if (i >= 2) L2 = lambda * dtd(i, i - 2, N) / dm2;
            if (i >= 1) L1 = (lambda * dtd(i, i - 1, N) - L2 * lm1 * dm2) / dm1;
            const double d = a - L1 * L1 * dm1 - L2 * L2 * dm2;
            const double u = wb[i] * yb[i] - L1 * um1 - L2 * um2;
            db[i] = d;
            l1b[i] = L1;
            l2b[i] = L2;
            zb[i] = u;
            dm2 = dm1; dm1 = d;
            lm1 = L1;
            um2 = um1; um1 = u;
        }
        // back substitution: z_i = u_i / d_i - L_{i+1,i} z_{i+1} - L_{i+2,i} z_{i+2}
        double zp1 = 0.0, zp2 = 0.0;
#pragma unroll 4
        for (int i = N - 1; i >= 0; --i) {
            const double c1 = i + 1 < N ? l1b[i + 1] : 0.0;
            const double c2 = i + 2 < N ? l2b[i + 2] : 0.0;
            const double zi = zb[i] / db[i] - c1 * zp1 - c2 * zp2;
            zb[i] = zi;
            zp2 = zp1; zp1 = zi;
        }
        if (it + 1 < n_iter)
            for (int i = 0; i < N; ++i) wb[i] = yb[i] > zb[i] ? p : 1.0 - p;
    }
}

}  // namespace

}  // namespace xrdvi

using namespace xrdvi;

extern "C" int xrdvi_background(xrdvi_ctx *ctx, int32_t B, int32_t N,
                                const double *y, double lambda, double p,
                                int32_t n_iter, double *bg_out,
                                void *scratch, void *stream) {
    try {
        if (!ctx || !y || !bg_out || !scratch) {
            set_error("background: NULL argument");
            return XRDVI_EINVAL;
        }
        if (B < 1 || N < 1 || n_iter < 1) {
            set_error("background: B, N and n_iter must be >= 1");
            return XRDVI_EINVAL;
        }
        if (!(lambda >= 0.0) || !std::isfinite(lambda) || !(p > 0.0 && p < 0.5)) {
            set_error("background: lambda must be >= 0 and p in (0, 0.5)");
            return XRDVI_EINVAL;
        }
        const size_t bn = (size_t)B * N;
        double *w = static_cast<double *>(scratch);
        k_asls<<<(B + 63) / 64, 64, 0, static_cast<hipStream_t>(stream)>>>(
            B, N, y, w, w + bn, w + 2 * bn, w + 3 * bn, bg_out, lambda, p, n_iter);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error(std::string("background: ") + hipGetErrorString(e));
            return XRDVI_EDEVICE;
        }
        return XRDVI_OK;
    } catch (...) {
        set_error("background: unexpected internal exception");
        return XRDVI_EDEVICE;
    }
}
