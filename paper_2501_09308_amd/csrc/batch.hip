// Batched optimisation step over every resident analysis of the server.
//
// Persistent kernels with fixed grids: each reads the slot table and the
// per-kernel work prefix from device memory, so one captured graph serves
// any membership.  Unit u of a kernel belongs to resident slot i when
// pre[i] <= u < pre[i + 1]; units of analyses that have run all their steps
// do nothing.  The per-unit work is the same device code as the
// single-analysis kernels, and the noise of step n of an analysis is keyed
// by (its seed, n), so an analysis computes the same result alone or in
// any mix.
#include <type_traits>

#include "batch.h"
#include "xrdvi_steps.h"

namespace xrdvi {

namespace {

// Stages the prefix of kernel `kind` and the slot ids in LDS.
struct PrefixSmem {
    int pre[kMaxSlots + 1];
    int slot[kMaxSlots];
    int n;
};

__device__ void load_prefix(const SchedDev *sch, int kind, PrefixSmem &ps) {
    const int n = sch->n;
    for (int i = threadIdx.x; i <= n; i += blockDim.x) ps.pre[i] = sch->pre[kind][i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) ps.slot[i] = sch->slot[i];
    if (threadIdx.x == 0) ps.n = n;
    __syncthreads();
}

__device__ __forceinline__ int uniform(int v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// Resident index i with pre[i] <= u < pre[i + 1] (u is block-uniform, so
// the result is wave-uniform).
__device__ int find_slot(const PrefixSmem &ps, int u) {
    int lo = 0, hi = ps.n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ps.pre[mid] <= u) lo = mid; else hi = mid;
    }
    return uniform(lo);
}

// Slot table entry of resident index i.  The table does not change while a
// kernel runs, and the index is uniform, so the copy is made of scalar loads
// and the problem and step descriptors stay in scalar registers, as the
// arguments of the single-analysis kernels do.
__device__ __forceinline__ const SlotDev &slot_entry(const SlotDev *tab,
                                                     const PrefixSmem &ps,
                                                     int i) {
    return *(const SlotDev *)(as_const(tab) + uniform(ps.slot[i]));
}

// Unit index of u inside resident index i.
__device__ __forceinline__ int local_unit(const PrefixSmem &ps, int i, int u) {
    return uniform(u - ps.pre[i]);
}

__device__ inline bool running(const SlotDev &d) {
    return uniform(*d.step) < d.steps;
}

}  // namespace

__global__ __launch_bounds__(256) void kb_sample(const SlotDev *tab,
                                                 const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    __shared__ SampleSmem sm;
    load_prefix(sch, kSample, ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        const int local = local_unit(ps, i, u);
        const int nkb = (d.P.K + kWave - 1) / kWave;
        if (local / nkb >= d.st.S) continue;
        sample_block(d.P, d.st, d.loc, d.logscale, nullptr, d.seed,
                     (uint64_t)*d.step, local / nkb, local % nkb, nkb, sm);
        __syncthreads();
    }
}

// The window step.  With a constant width (windowed analyses) an
// analysis's first ceil(K / 64) units find its phases' extremes over the
// samples instead, 64 phases each (see batch_units).
template <bool SEC>
__global__ __launch_bounds__(256) void kb_windows(const SlotDev *tab,
                                                  const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    __shared__ typename std::conditional<SEC, char, CandExtSmem>::type sm;
    load_prefix(sch, SEC ? kWindowsSec : kWindows, ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        int local = local_unit(ps, i, u);
        if constexpr (!SEC) {
            const int next = (d.P.K + kWave - 1) / kWave;
            if (local < next) {
                if (d.st.cab) cand_ext_block(d.P, d.st, d.st.phi, local * kWave, sm);
                __syncthreads();   // the extremes' LDS is reused by the next unit
                continue;
            }
            local -= next;
        }
        const size_t g = (size_t)local * 256 + threadIdx.x;
        if (g < (size_t)d.st.S * d.P.T)
            windows_elem<SEC>(d.P, d.st.phi, d.P.cutoff > 0.0 ? d.st.lo : nullptr,
                              d.st.hi, nullptr, g, d.st.psec);
    }
}

template <bool SEC>
__global__ __launch_bounds__(256) void kb_plan(const SlotDev *tab,
                                               const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    load_prefix(sch, SEC ? kPlanSec : kPlan, ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        const size_t g = (size_t)local_unit(ps, i, u) * 256 + threadIdx.x;
        if (g < (size_t)d.st.S * d.P.ntiles * d.P.K) plan_elem<SEC>(d.P, d.st, d.st.phi, g);
    }
}

__global__ __launch_bounds__(kCandThreads) void kb_cand(const SlotDev *tab,
                                                        const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    load_prefix(sch, kCand, ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d) || !d.st.cab) continue;
        const int local = local_unit(ps, i, u);
        const int nkb = (d.P.K + kCandThreads - 1) / kCandThreads;
        const int t = local / nkb, k = (local % nkb) * kCandThreads + threadIdx.x;
        if (t < d.P.ntiles && k < d.P.K) cand_elem(d.P, d.st, t, k);
    }
}

// The windowed constant-width variants are held to the six blocks per CU
// their LDS allows (80 VGPRs; six 8-byte values are spilled once per block
// and reloaded once per unit, outside the record loops): their waves wait
// on memory more than their single-analysis counterpart's.
template <bool WIN, bool ASYM, bool SEC>
__global__ __launch_bounds__(kBlock, WIN && !SEC ? 6 : 1) void kb_fused(const SlotDev *tab,
                                                                        const SchedDev *sch) {
    using Smem = typename std::conditional<WIN, WinSmem<ASYM>,
                                           FusedSmem>::type;
    __shared__ PrefixSmem ps;
    __shared__ Smem sm;
    load_prefix(sch, fused_kind(WIN, ASYM, SEC), ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        const int local = local_unit(ps, i, u);
        int t = local % d.P.ntiles, s = local / d.P.ntiles;
        if (WIN && !SEC && d.st.S % kXcds == 0) {
            // a block runs on XCD u mod 8, and u - local is the same for all
            // of an analysis's units: the units with one value of local mod 8
            // share an XCD, which takes one eighth of the samples of every
            // tile (its L2 keeps those samples' window arrays)
            const int G = d.st.S / kXcds, q = local / kXcds;
            t = q / G;
            s = (local % kXcds) * G + q % G;
        }
        if (s >= d.st.S) continue;
        // windowed: forward only (the adjoint is peak-major); dense: fused
        if constexpr (WIN) {
            // records in grid steps on a uniform grid (constant width only)
            if (!SEC && uses_grid_steps(d.P))
                win_tile<ASYM, SEC, !SEC>(d.P, d.st, t, s, nullptr, sm);
            else
                win_tile<ASYM, SEC, false>(d.P, d.st, t, s, nullptr, sm);
        } else {
            fused_tile<false, true, ASYM, SEC>(d.P, d.st, t, s, nullptr, sm);
        }
        __syncthreads();
    }
}

template <bool ASYM, bool SEC>
__global__ __launch_bounds__(kBlock) void kb_adjoint(const SlotDev *tab,
                                                     const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    __shared__ double red[kWaves][12];
    load_prefix(sch, adjoint_kind(ASYM, SEC), ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        const int local = local_unit(ps, i, u);
        if (local / d.P.K >= d.st.S || d.P.cutoff == 0.0) continue;
        adjoint_phase<ASYM, SEC>(d.P, d.st, local / d.P.K, local % d.P.K, red);
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void kb_elbo(const SlotDev *tab,
                                                const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    __shared__ ElboSmem sm;
    load_prefix(sch, kElbo, ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        const double e = elbo_block(d.P, d.st, d.logscale, nullptr, sm);
        if (threadIdx.x == 0) d.trace[*d.step] = e;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void kb_grad_adam(const SlotDev *tab,
                                                    const SchedDev *sch) {
    __shared__ PrefixSmem ps;
    __shared__ GradSmem sm;
    load_prefix(sch, kGrad, ps);
    const int total = uniform(ps.pre[ps.n]);
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = find_slot(ps, u);
        const SlotDev &d = slot_entry(tab, ps, i);
        if (!running(d)) continue;
        AdamArgs a;
        a.m1_loc = d.m1_loc; a.m2_loc = d.m2_loc;
        a.m1_ls = d.m1_ls; a.m2_ls = d.m2_ls;
        a.t = *d.step + 1;
        a.lr = d.lr; a.b1 = 0.9; a.b2 = 0.999; a.eps = 1e-8;
        if (d.P.cutoff > 0.0) {
            // windowed: one phase per wave
            const int k = local_unit(ps, i, u) * kWaves + (int)(threadIdx.x / kWave);
            if (k < d.P.K)
                grad_wave(d.P, d.st, k, 1.0, nullptr, nullptr, nullptr, d.loc,
                          d.logscale, &a);
        } else {
            const int k = local_unit(ps, i, u);
            if (k >= d.P.K) continue;
            grad_block(d.P, d.st, k, 1.0, nullptr, nullptr, nullptr,
                       d.loc, d.logscale, &a, sm);
        }
        __syncthreads();
    }
}

// Last kernel of a step: every running analysis moves to its next step.
__global__ void kb_advance(const SlotDev *tab, const SchedDev *sch) {
    const int n = sch->n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x) {
        const SlotDev &d = tab[sch->slot[i]];
        if (*d.step < d.steps) *d.step += 1;
    }
}

hipError_t launch_batch_step(const SlotDev *tab, const SchedDev *sch,
                             hipStream_t s, unsigned classes) {
    // whether a resident class satisfies the windowed / sec-law test
    const auto any = [classes](int want_win, int want_sec) {
        for (int c = 0; c < 8; ++c)
            if ((classes >> c & 1u) && (want_win < 0 || (c & 1) == want_win) &&
                (want_sec < 0 || (c >> 2 & 1) == want_sec))
                return true;
        return false;
    };
    const auto has = [classes](bool win, bool asym, bool sec) {
        return (classes >> ((win ? 1 : 0) | (asym ? 2 : 0) | (sec ? 4 : 0)) & 1u) != 0;
    };
    kb_sample<<<kGridSmall, 256, 0, s>>>(tab, sch);
    if (any(1, 0)) kb_windows<false><<<kGridLarge, 256, 0, s>>>(tab, sch);
    if (any(-1, 1)) kb_windows<true><<<kGridLarge, 256, 0, s>>>(tab, sch);
    if (any(0, 0)) kb_plan<false><<<kGridLarge, 256, 0, s>>>(tab, sch);
    if (any(0, 1)) kb_plan<true><<<kGridLarge, 256, 0, s>>>(tab, sch);
    if (any(1, 0)) kb_cand<<<kGridLarge, kCandThreads, 0, s>>>(tab, sch);
    if (has(true, false, false)) kb_fused<true, false, false><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(false, false, false)) kb_fused<false, false, false><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, true, false)) kb_fused<true, true, false><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(false, true, false)) kb_fused<false, true, false><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, false, true)) kb_fused<true, false, true><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(false, false, true)) kb_fused<false, false, true><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, true, true)) kb_fused<true, true, true><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(false, true, true)) kb_fused<false, true, true><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, false, false)) kb_adjoint<false, false><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, true, false)) kb_adjoint<true, false><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, false, true)) kb_adjoint<false, true><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    if (has(true, true, true)) kb_adjoint<true, true><<<kGridLarge, kBlock, 0, s>>>(tab, sch);
    kb_elbo<<<kGridElbo, 1024, 0, s>>>(tab, sch);
    kb_grad_adam<<<kGridLarge, 256, 0, s>>>(tab, sch);
    kb_advance<<<1, 1024, 0, s>>>(tab, sch);
    return hipGetLastError();
}

}  // namespace xrdvi
