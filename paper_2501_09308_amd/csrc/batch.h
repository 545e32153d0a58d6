// Device-side tables of the batched serving step.
#pragma once

#include <hip/hip_runtime.h>

#include "xrdvi_device.h"

namespace xrdvi {

constexpr int kMaxSlots = 512;

// Kernel kinds of one batched step, each with its own work prefix.  The
// fused tile and the peak-major adjoint have one kernel per variant
// (windowed or dense, symmetric or asymmetric peaks), so that each kernel
// keeps the register budget of its single-analysis counterpart.
enum BatchKind { kSample = 0, kWindows, kPlan, kFusedWin, kFusedDense,
                 kFusedWinAsym, kFusedDenseAsym, kAdjoint, kAdjointAsym,
                 kElbo, kGrad, kKinds };

constexpr int fused_kind(bool win, bool asym) {
    return asym ? (win ? kFusedWinAsym : kFusedDenseAsym)
                : (win ? kFusedWin : kFusedDense);
}

// Fixed persistent grids (blocks) of the batched kernels.
constexpr int kGridSmall = 1024;
constexpr int kGridLarge = 2048;
constexpr int kGridElbo = 256;

// One resident analysis: its problem, per-step state and optimiser state.
struct SlotDev {
    ProbDev P;
    StepDev st;
    double *loc, *logscale;                      // [D K] variational params
    double *m1_loc, *m2_loc, *m1_ls, *m2_ls;     // [D K] Adam moments
    double *trace;                               // [steps] ELBO per step
    int *step;                                   // steps done so far
    int steps;
    uint64_t seed;
    double lr;
};

// Membership of the next batched step: resident slot ids and, per kernel
// kind, the prefix of work units over them.
struct SchedDev {
    int n;
    int slot[kMaxSlots];
    int pre[kKinds][kMaxSlots + 1];
};

// Work units of each kind for one analysis.
inline void batch_units(const ProbDev &P, int S, int units[kKinds]) {
    const bool win = P.cutoff > 0.0, asym = P.D == 5;
    const long long nkb = (P.K + kWave - 1) / kWave;
    for (int k = 0; k < kKinds; ++k) units[k] = 0;
    units[kSample] = (int)(S * nkb);
    units[kWindows] = win ? (int)(((long long)S * P.T + 255) / 256) : 0;
    units[kPlan] = (int)(((long long)S * P.ntiles * P.K + 255) / 256);
    units[fused_kind(win, asym)] = P.ntiles * S;
    if (win) units[asym ? kAdjointAsym : kAdjoint] = P.K * S;
    units[kElbo] = 1;
    units[kGrad] = P.K;
}

hipError_t launch_batch_step(const SlotDev *tab, const SchedDev *sch,
                             hipStream_t stream);

}  // namespace xrdvi
