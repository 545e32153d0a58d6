// Device-side tables of the batched serving step.
#pragma once

#include <hip/hip_runtime.h>

#include "xrdvi_device.h"

namespace xrdvi {

constexpr int kMaxSlots = 512;

// Kernel kinds of one batched step, each with its own work prefix.  The
// fused tile and the peak-major adjoint have one kernel per variant
// (windowed or dense, symmetric or asymmetric peaks, constant or sec-law
// width), so that each kernel keeps the register budget of its
// single-analysis counterpart.
enum BatchKind { kSample = 0, kWindows, kWindowsSec, kPlan, kPlanSec, kCand,
                 kFusedWin, kFusedDense, kFusedWinAsym, kFusedDenseAsym,
                 kFusedWinSec, kFusedDenseSec, kFusedWinAsymSec,
                 kFusedDenseAsymSec,
                 kAdjoint, kAdjointAsym, kAdjointSec, kAdjointAsymSec,
                 kElbo, kGrad, kKinds };

constexpr int fused_kind(bool win, bool asym, bool sec) {
    return kFusedWin + (win ? 0 : 1) + (asym ? 2 : 0) + (sec ? 4 : 0);
}
constexpr int adjoint_kind(bool asym, bool sec) {
    return kAdjoint + (asym ? 1 : 0) + (sec ? 2 : 0);
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
    const bool win = P.cutoff > 0.0, asym = P.D == 5, sec = P.sec != 0;
    const long long nkb = (P.K + kWave - 1) / kWave;
    for (int k = 0; k < kKinds; ++k) units[k] = 0;
    units[kSample] = (int)(S * nkb);
    if (win || sec)
        units[sec ? kWindowsSec : kWindows] = (int)(((long long)S * P.T + 255) / 256);
    if (!win)   // the windowed forward tile finds its own ranges
        units[sec ? kPlanSec : kPlan] = (int)(((long long)S * P.ntiles * P.K + 255) / 256);
    if (win && !sec) {   // ... among candidates found once per step
        // the phases' extremes over the samples, 64 phases per unit, run as
        // the window step's first units
        units[kWindows] += (int)nkb;
        units[kCand] = (int)(((long long)P.K + kCandThreads - 1) / kCandThreads) * P.ntiles;
    }
    units[fused_kind(win, asym, sec)] = P.ntiles * S;
    if (win) units[adjoint_kind(asym, sec)] = P.K * S;
    units[kElbo] = 1;
    units[kGrad] = win ? (P.K + kWaves - 1) / kWaves : P.K;   // windowed: a phase per wave
}

// Variant class of an analysis (0..7): windowed (bit 0), asymmetric peaks
// (bit 1), sec-law width (bit 2).  Each class has its own fused and adjoint
// kernels; a batched step launches only those of the resident classes.
inline int batch_class(const ProbDev &P) {
    return (P.cutoff > 0.0 ? 1 : 0) | (P.D == 5 ? 2 : 0) | (P.sec != 0 ? 4 : 0);
}

// One batched step over the resident analyses, whose classes are the set
// bits of `classes` (bit c: some resident analysis has class c).
hipError_t launch_batch_step(const SlotDev *tab, const SchedDev *sch,
                             hipStream_t stream, unsigned classes);

}  // namespace xrdvi
