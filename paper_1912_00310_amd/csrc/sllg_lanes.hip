// Single-cell levels, one realization per lane.
//
// A level of one cell (the single-macrospin limit of the coarse-graining
// rule: the whole rod as one cell that feels anisotropy, the applied field
// and the thermal field only) has no neighbour to wait for, so each lane
// integrates one realization on its own: the state and the level constants
// stay in registers for a launch of many steps, and nothing is shared
// between realizations.  The per-step chain is the per-cell arithmetic of
// every other kernel (the same functions, so the states are bit-identical to
// the resident plan's): the thermal field of step n + 1 is drawn while step n
// is corrected (it does not depend on m).
//
// A workgroup is two waves for 64 realizations.  The first (the stepping
// wave) integrates; per chunk of kLanesChunk steps it leaves the ordinate m_z
// of every step in LDS.  The second (the loop wave) folds the previous
// chunk's ordinates into the FP64 loop accumulators of the same
// realizations, lane for lane, and tabulates the applied field of the next
// chunk, so the FP64 loop update is off the stepping chain; a barrier per
// chunk hands the buffers over (the ordinates and the field tables are
// double-buffered by chunk parity).  When the realizations of a workgroup
// have different levels, each lane evaluates its own schedule instead of the
// table.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

constexpr int kLanesThreads = 64;   // realizations per workgroup (two waves)
constexpr int kLanesChunk = 64;     // steps per hand-over

__global__ __launch_bounds__(2 * kLanesThreads) void k_lanes(const InstDev* __restrict__ insts, int inst0,
                                                            int ninst, const LevelDev* __restrict__ levels,
                                                            float* __restrict__ buf0, float* __restrict__ buf1,
                                                            const float* __restrict__ axes,
                                                            double* __restrict__ records, AccDev* __restrict__ accs,
                                                            float* __restrict__ ckpt, int ckpt_every, int64_t n0,
                                                            int64_t nsteps, int* __restrict__ status)
{
    __shared__ float s_hz[2][kLanesChunk + 1];    // applied field (A/m, FP32) of a chunk's steps
    __shared__ double s_H[2][kLanesChunk + 1];    // the same in Oe, FP64, for the loop
    __shared__ float s_mz[2][kLanesChunk][kLanesThreads];   // ordinate of every step of a chunk
    const int lane = static_cast<int>(threadIdx.x) & (kLanesThreads - 1);
    const bool stepper = threadIdx.x < kLanesThreads;
    const int k = static_cast<int>(blockIdx.x) * kLanesThreads + lane;
    const bool act = k < ninst;
    const int inst = inst0 + (act ? k : 0);
    const InstDev I = insts[inst];
    const LevelDev L = levels[I.level];
    // one level for the whole workgroup? (lane 0 is always a realization;
    // lanes past the last one step a copy of it and write nothing)
    const int lev0 = __shfl(I.level, 0);
    const bool shared_field = __ballot(act && I.level != lev0) == 0;
    const LevelDev& L0 = levels[lev0];
    const int64_t nchunks = (nsteps + kLanesChunk - 1) / kLanesChunk;
    // the applied field of chunk c (steps n0 + c K .. + K, the last one
    // included) into buffer c & 1, by the loop wave
    auto table = [&](int64_t c) {
        const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - c * kLanesChunk));
        for (int t = lane; t <= cn; t += kLanesThreads) {
            const double wt = wave_at(L0, n0 + c * kLanesChunk + t);
            s_hz[c & 1][t] = static_cast<float>(L0.hz_amp * wt);
            s_H[c & 1][t] = L0.hz_oe * wt;
        }
    };
    if (stepper) {
        const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
        V3 m = V3{mi[0], mi[1], mi[2]};
        const V3 u = L.has_axes ? V3{axes[L.axes_off], axes[L.axes_off + 1], axes[L.axes_off + 2]}
                                : V3{L.ux, L.uy, L.uz};
        float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n0));
        V3 hth = thermal_field(L, I.seed, 0u, n0);
        __syncthreads();   // the first table
        for (int64_t c = 0; c < nchunks; ++c) {
            const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - c * kLanesChunk));
            for (int t = 0; t < cn; ++t) {
                const int64_t n = n0 + c * kLanesChunk + t;
                if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                    float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3;
                    if (act) {
                        cp[0] = m.x;
                        cp[1] = m.y;
                        cp[2] = m.z;
                    }
                }
                const float hz1 = shared_field ? s_hz[c & 1][t + 1]
                                               : static_cast<float>(L.hz_amp * wave_at(L, n + 1));
                // a single cell is its own neighbour on every face: the
                // exchange sum is formed as in every other kernel (zero up to
                // FP32 rounding)
                V3 mp, q;
                heun_predict(L, m, nb_sum(m, m, m, m, m, m, m), u, hz0, hth, mp, q);
                const V3 hth_next = thermal_field(L, I.seed, 0u, n + 1);
                m = heun_correct(L, mp, nb_sum(mp, mp, mp, mp, mp, mp, mp), u, hz1, hth, q);
                s_mz[c & 1][t][lane] = m.z;
                hth = hth_next;
                hz0 = hz1;
            }
            __syncthreads();   // chunk c's ordinates and chunk c + 1's table are in place
        }
        if (act) {
            float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
            mo[0] = m.x;
            mo[1] = m.y;
            mo[2] = m.z;
        }
    } else {
        AccDev a = accs[inst];
        double* rec = records + I.rec_off;
        // fold chunk c (its ordinates and, with one level, its field table)
        auto fold = [&](int64_t c) {
            const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - c * kLanesChunk));
            double H0 = shared_field ? s_H[c & 1][0] : L.hz_oe * wave_at(L, n0 + c * kLanesChunk);
            for (int t = 0; t < cn; ++t) {
                const double H1 = shared_field ? s_H[c & 1][t + 1]
                                               : L.hz_oe * wave_at(L, n0 + c * kLanesChunk + t + 1);
                if (act) loop_accumulate_h(a, L, H0, H1, static_cast<double>(s_mz[c & 1][t][lane]), rec);
                H0 = H1;
            }
        };
        if (shared_field && nchunks > 0) table(0);
        __syncthreads();
        for (int64_t c = 0; c < nchunks; ++c) {
            // while the stepping wave runs chunk c: fold chunk c - 1, then
            // tabulate chunk c + 1 into the buffers chunk c - 1 used
            if (c > 0) fold(c - 1);
            if (shared_field && c + 1 < nchunks) table(c + 1);
            __syncthreads();
        }
        if (nchunks > 0) fold(nchunks - 1);
        if (act) {
            accs[inst] = a;
            if (!isfinite(a.m_prev)) atomicOr(status, 1);
        }
    }
}

}  // namespace sllg
