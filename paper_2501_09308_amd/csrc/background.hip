// Background estimation before the analysis (App. A.2: the background is
// estimated beforehand by an iterative least-squares method): asymmetric
// least squares (Eilers and Boelens, 2005).  Repeatedly solve
//     (W + lambda D^T D) z = W y,   D the second-difference operator,
// and set w_i = p where y_i > z_i and 1 - p elsewhere (w = 1 at the start),
// so that the smooth curve z hugs the data from below.
//
// The system A z = r is symmetric positive definite and pentadiagonal.  One
// wave per spectrum solves it in parallel by a symmetric reordering: the
// rows split into P interior blocks separated by 2-row separators (with
// bandwidth 2, removing two consecutive rows decouples the blocks).
//  1. Each lane factors its block A_p = L D L^T and, in the same forward
//     sweep, forms the corner 2 x 2 blocks of A_p^{-1} that couple it to
//     its separators, (A_p^{-1})_{ab} = sum_i (L^{-1})_{ia} (L^{-1})_{ib} /
//     d_i, and the corresponding entries of A_p^{-1} r_p.
//  2. The Schur complement on the separators, a block tridiagonal SPD
//     system of 2 x 2 blocks: its blocks one lane per separator, then block
//     elimination by one lane.
//  3. Each lane solves its block with the separator values moved to the
//     right-hand side.
// Every step is elimination without pivoting on a symmetric reordering of
// an SPD matrix, the stable case.  FP64 throughout.
#include <cmath>
#include <string>

#include "xrdvi.h"
#include "xrdvi_internal.h"

namespace xrdvi {

namespace {

constexpr int kBgLanes = 64;      // one wave per spectrum, one lane per block

// (D^T D)_{ij} for |i - j| <= 2, D the (N-2) x N second-difference matrix
// with rows (1, -2, 1) at columns k, k+1, k+2.
__device__ inline double dtd(int i, int j, int N) {
    const double c[3] = {1.0, -2.0, 1.0};
    const int k0 = max(max(i, j) - 2, 0), k1 = min(min(i, j), N - 3);
    double s = 0.0;
    for (int k = k0; k <= k1; ++k) s += c[i - k] * c[j - k];
    return s;
}

struct M2 {
    double a, b, c, d;     // [[a, b], [c, d]]
};
__device__ inline M2 mul(const M2 &x, const M2 &y) {
    return M2{x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d,
              x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
__device__ inline M2 tr(const M2 &x) { return M2{x.a, x.c, x.b, x.d}; }
__device__ inline M2 sub(const M2 &x, const M2 &y) {
    return M2{x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d};
}
__device__ inline M2 inv(const M2 &x) {
    const double det = x.a * x.d - x.b * x.c;
    return M2{x.d / det, -x.b / det, -x.c / det, x.a / det};
}
__device__ inline double2 mulv(const M2 &x, double2 v) {
    return make_double2(x.a * v.x + x.b * v.y, x.c * v.x + x.d * v.y);
}

// Block p of the partition: first row and row count.  P blocks share the
// N - 2 (P - 1) interior rows as evenly as possible.
__device__ inline int2 block_of(int p, int P, int N) {
    const int nint = N - 2 * (P - 1);
    const int base = nint / P, extra = nint % P;
    return make_int2(p * (base + 2) + min(p, extra), base + (p < extra ? 1 : 0));
}

// Per-block results of the forward sweep: corner blocks of A_p^{-1}
// (top-left, top-right, bottom-right) and the first / last two entries of
// A_p^{-1} r_p.
struct BlockInv {
    M2 tl, trr, br;
    double2 xf, xl;
};

// Blocks per spectrum: at most one per lane, at least 8 rows each.
__device__ inline int num_blocks(int N) { return max(1, min(kBgLanes, (N + 2) / 10)); }

// One wave per spectrum b: n_iter reweighting iterations.  Scratch arrays
// [B][N]: w (weights), dg (pivots), l1 = L_{i,i-1}, l2 = L_{i,i-2}.
__global__ __launch_bounds__(kBgLanes) void k_asls(
    int B, int N, const double *__restrict__ y, double *w, double *dg,
    double *l1, double *l2, double *z, double lambda, double p, int n_iter) {
#pragma clang fp contract(off)
    __shared__ BlockInv inv_s[kBgLanes];
    __shared__ M2 dp_s[kBgLanes], off_s[kBgLanes];
    __shared__ double2 yv_s[kBgLanes], zs_s[kBgLanes];
    const int b = blockIdx.x, t = threadIdx.x;
    if (b >= B) return;
    const size_t o = (size_t)b * N;
    const double *yb = y + o;
    double *wb = w + o, *db = dg + o, *l1b = l1 + o, *l2b = l2 + o, *zb = z + o;
    if (N < 3) {                       // no second differences: z = y
        for (int i = t; i < N; i += kBgLanes) zb[i] = yb[i];
        return;
    }
    const int P = num_blocks(N);
    auto A = [&](int i, int j) {       // entry of W + lambda D^T D
        const double v = lambda * dtd(i, j, N);
        return i == j ? v + wb[i] : v;
    };
    // couplings of block q's first two rows to the separator before it, and
    // of its last two rows to the separator after it
    auto CL = [&](int q) {
        const int r0 = block_of(q, P, N).x;
        return M2{A(r0, r0 - 2), A(r0, r0 - 1), 0.0, A(r0 + 1, r0 - 1)};
    };
    auto CR = [&](int q) {
        const int2 bq = block_of(q, P, N);
        const int e = bq.x + bq.y;
        return M2{A(e - 2, e), 0.0, A(e - 1, e), A(e - 1, e + 1)};
    };
    for (int i = t; i < N; i += kBgLanes) wb[i] = 1.0;
    __syncthreads();
    for (int it = 0; it < n_iter; ++it) {
        // 1. factor each block; corner blocks of its inverse
        if (t < P) {
            const int2 bk = block_of(t, P, N);
            const int r0 = bk.x, n = bk.y;
            double dm1 = 0.0, dm2 = 0.0, lm1 = 0.0;
            double um1 = 0.0, um2 = 0.0, a1 = 0.0, a2 = 0.0, c1 = 0.0, c2 = 0.0;
            M2 tl{0.0, 0.0, 0.0, 0.0};
            double2 xf = make_double2(0.0, 0.0);
#pragma unroll 4
            for (int i = 0; i < n; ++i) {
                const int g = r0 + i;
                double L2 = 0.0, L1 = 0.0;
                if (i >= 2) L2 = A(g, g - 2) / dm2;
                if (i >= 1) L1 = (A(g, g - 1) - L2 * lm1 * dm2) / dm1;
                const double d = A(g, g) - L1 * L1 * dm1 - L2 * L2 * dm2;
                const double u = wb[g] * yb[g] - L1 * um1 - L2 * um2;
                // columns 0 and 1 of L^{-1}
                const double ca = (i == 0 ? 1.0 : 0.0) - L1 * a1 - L2 * a2;
                const double cb = (i == 1 ? 1.0 : 0.0) - L1 * c1 - L2 * c2;
                db[g] = d;
                l1b[g] = L1;
                l2b[g] = L2;
                tl.a += ca * ca / d;
                tl.b += ca * cb / d;
                tl.d += cb * cb / d;
                xf.x += ca * u / d;
                xf.y += cb * u / d;
                dm2 = dm1; dm1 = d; lm1 = L1;
                um2 = um1; um1 = u;
                a2 = a1; a1 = ca;
                c2 = c1; c1 = cb;
            }
            tl.c = tl.b;
            // columns n-2 and n-1 of L^{-1} are (1, -L_{n-1,n-2}) and (0, 1)
            // on the last two rows and 0 above them
            const double lnm1 = lm1;                  // L_{n-1, n-2}
            const double dn2 = dm2, dn1 = dm1;
            const double m2a = 1.0, m2b = -lnm1;      // column n-2, rows n-2, n-1
            BlockInv bi;
            bi.tl = tl;
            // rows 0, 1 of columns n-2, n-1 of A^{-1}: sum over rows n-2, n-1
            bi.trr = M2{a2 * m2a / dn2 + a1 * m2b / dn1, a1 / dn1,
                        c2 * m2a / dn2 + c1 * m2b / dn1, c1 / dn1};
            bi.br = M2{m2a * m2a / dn2 + m2b * m2b / dn1, m2b / dn1,
                       m2b / dn1, 1.0 / dn1};
            bi.xf = xf;
            bi.xl = make_double2(m2a * um2 / dn2 + m2b * um1 / dn1, um1 / dn1);
            inv_s[t] = bi;
        }
        __syncthreads();
        // 2. Schur complement on the separators (separator q lies between
        //    blocks q and q + 1): its blocks in parallel, one lane per
        //    separator, then block elimination by one lane
        if (t < P - 1) {
            const int q = t;
            const int2 bq = block_of(q, P, N);
            const int e = bq.x + bq.y;
            const M2 cr = CR(q), cl = CL(q + 1);
            const M2 ass{A(e, e), A(e, e + 1), A(e + 1, e), A(e + 1, e + 1)};
            dp_s[q] = sub(sub(ass, mul(tr(cr), mul(inv_s[q].br, cr))),
                          mul(tr(cl), mul(inv_s[q + 1].tl, cl)));
            const double2 ccr = mulv(tr(cr), inv_s[q].xl);
            const double2 ccl = mulv(tr(cl), inv_s[q + 1].xf);
            yv_s[q] = make_double2(wb[e] * yb[e] - ccr.x - ccl.x,
                                   wb[e + 1] * yb[e + 1] - ccr.y - ccl.y);
            if (q + 1 < P - 1) {               // coupling to separator q + 1
                const M2 zero{0.0, 0.0, 0.0, 0.0};
                off_s[q] = sub(zero, mul(tr(cl), mul(inv_s[q + 1].trr, CR(q + 1))));
            }
        }
        __syncthreads();
        if (t == 0) {
            for (int q = 1; q < P - 1; ++q) {
                const M2 Lq = mul(tr(off_s[q - 1]), inv(dp_s[q - 1]));
                dp_s[q] = sub(dp_s[q], mul(Lq, off_s[q - 1]));
                const double2 lv = mulv(Lq, yv_s[q - 1]);
                yv_s[q] = make_double2(yv_s[q].x - lv.x, yv_s[q].y - lv.y);
            }
            for (int q = P - 2; q >= 0; --q) {
                double2 rhs = yv_s[q];
                if (q + 1 < P - 1) {
                    const double2 c = mulv(off_s[q], zs_s[q + 1]);
                    rhs = make_double2(rhs.x - c.x, rhs.y - c.y);
                }
                zs_s[q] = mulv(inv(dp_s[q]), rhs);
            }
        }
        __syncthreads();
        if (t < P - 1) {
            const int2 bq = block_of(t, P, N);
            const int e = bq.x + bq.y;
            zb[e] = zs_s[t].x;
            zb[e + 1] = zs_s[t].y;
        }
        // 3. each block with its separators' values on the right-hand side
        if (t < P) {
            const int2 bk = block_of(t, P, N);
            const int r0 = bk.x, n = bk.y;
            double2 fl = make_double2(0.0, 0.0), fr = make_double2(0.0, 0.0);
            if (t > 0) fl = mulv(CL(t), zs_s[t - 1]);
            if (t < P - 1) fr = mulv(CR(t), zs_s[t]);
            double um1 = 0.0, um2 = 0.0;
#pragma unroll 4
            for (int i = 0; i < n; ++i) {
                const int g = r0 + i;
                double r = wb[g] * yb[g];
                if (i == 0) r -= fl.x;
                if (i == 1) r -= fl.y;
                if (i == n - 2) r -= fr.x;
                if (i == n - 1) r -= fr.y;
                const double u = r - l1b[g] * um1 - l2b[g] * um2;
                zb[g] = u;
                um2 = um1; um1 = u;
            }
            double zp1 = 0.0, zp2 = 0.0;
#pragma unroll 4
            for (int i = n - 1; i >= 0; --i) {
                const int g = r0 + i;
                const double c1 = i + 1 < n ? l1b[g + 1] : 0.0;
                const double c2 = i + 2 < n ? l2b[g + 2] : 0.0;
                const double zi = zb[g] / db[g] - c1 * zp1 - c2 * zp2;
                zb[g] = zi;
                zp2 = zp1; zp1 = zi;
            }
        }
        __syncthreads();
        if (it + 1 < n_iter)
            for (int i = t; i < N; i += kBgLanes) wb[i] = yb[i] > zb[i] ? p : 1.0 - p;
        __syncthreads();
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
        k_asls<<<B, kBgLanes, 0, static_cast<hipStream_t>(stream)>>>(
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
