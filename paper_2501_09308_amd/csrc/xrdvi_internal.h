// Host-side internals shared by the C ABI, the launchers and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "xrdvi.h"
#include "xrdvi_device.h"

namespace xrdvi {

// Per-problem tables: ln y!, the tile-relative FP32 grid and peak positions
// and the rounding errors of both.
hipError_t launch_prepare(const ProbDev &P, double *lgy, float *u, float *ul,
                          float *pt, float *ptl, hipStream_t stream);
hipError_t launch_sample(const ProbDev &P, const StepDev &st,
                         const double *loc, const double *logscale,
                         const double *eps, uint64_t seed, uint64_t step,
                         hipStream_t stream);
hipError_t launch_phi_consts(const ProbDev &P, int S, const double *phi,
                             float4 *pk, float *pkr, hipStream_t stream);
// Window plan of S samples (lo/hi NULL: none) under the problem's width
// law and, with psec (sec law only), the sec-law peak records.
hipError_t launch_windows(const ProbDev &P, int S, const double *phi, int *lo,
                          int *hi, const int *perm, hipStream_t stream,
                          float4 *psec = nullptr);
// Per-(sample, peak) step of a2 for st: windows (windowed mode) and sec-law
// records (sec law); nothing for a dense constant-width problem.
hipError_t launch_peak_plan(const ProbDev &P, const StepDev &st,
                            const double *phi, hipStream_t stream);
hipError_t launch_plan(const ProbDev &P, const StepDev &st, const double *phi,
                       hipStream_t stream);
// wide: dense tiles with more waves each (small grids; other summation
// order of the partial signals, so not for results that must match across
// paths bit for bit).
hipError_t launch_fused(const ProbDev &P, const StepDev &st, bool grad,
                        float *f_out, hipStream_t stream, bool wide = false);
// logp_out: per-sample log posterior density; gz_out: per-sample gradient
// of it in z, [S][D K] (both optional).
hipError_t launch_elbo(const ProbDev &P, const StepDev &st,
                       const double *logscale, double *elbo_out,
                       double *loglik_out, hipStream_t stream,
                       double *logp_out = nullptr);
hipError_t launch_grad(const ProbDev &P, const StepDev &st, double scale,
                       const double *scale_dev, double *gloc,
                       double *glogscale, hipStream_t stream,
                       double *gz_out = nullptr);

// Per-sample log posterior density and (gz != NULL) its gradient in z at
// positions z [S][D K]; zeros: D K zeros.
hipError_t launch_logpost(const ProbDev &P, const StepDev &st,
                          const double *zeros, const double *z, double *logp,
                          double *gz, hipStream_t stream);

hipError_t launch_adam(int n, double *theta, double *m1, double *m2,
                       const double *g, int t, double lr, double b1, double b2,
                       double eps, hipStream_t stream);

void set_error(const std::string &msg);

constexpr int kMaxSamples = 1024;

// Sizes that fix the per-step device state of one analysis.
struct StepShape {
    int ntiles, K, T, S, N;
    int D;          // latent types per phase (4, or 5 with asymmetry)
    bool dense;     // cutoff 0: the adjoint keeps per-tile partial sums
    bool sec;       // sec width law: per-(sample, peak) records
};
inline StepShape step_shape(const ProbDev &P, int S) {
    return StepShape{P.ntiles, P.K, P.T, S, P.N, P.D, P.cutoff == 0.0,
                     P.sec != 0};
}
// Bytes of per-step device state, laid out by carve_step.
size_t step_bytes(const StepShape &sh);
// Carves StepDev buffers out of `base` (256-byte aligned pieces).
StepDev carve_step(void *base, const StepShape &sh);

inline int num_tiles(int N) { return (N + kTile - 1) / kTile; }

// Latent types per phase of a description.
inline int latent_types(const xrdvi_problem_desc &d) {
    return d.asymmetric ? 5 : 4;
}

// Device bytes of a prepared problem and its upload (validated desc,
// resolved lambda) into `base`; fills P and the sorted-to-caller peak
// permutation.  Synchronises `stream` before returning (pageable sources).
size_t problem_bytes(int N, int K, int T);
hipError_t upload_problem(const xrdvi_problem_desc &d, double lambda,
                          char *base, ProbDev &P, int **perm_out,
                          hipStream_t stream);
// Host validation of a problem description; resolves lambda_h (0 -> 1 /
// max(y - bg)) and returns max(y - bg) in *ymax when non-NULL.
int validate_problem(const xrdvi_problem_desc *d, double *lambda_out,
                     double *ymax);

}  // namespace xrdvi
