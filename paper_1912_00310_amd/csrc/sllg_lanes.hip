// Single-cell levels, one realization per lane.
//
// A level of one cell (the single-macrospin limit of the coarse-graining
// rule: the whole rod as one cell that feels anisotropy, the applied field
// and the thermal field only) has no neighbour to wait for, so each lane
// integrates one realization on its own: the state, the loop accumulators
// and the level constants stay in registers for a launch of many steps, and
// nothing is shared between lanes.  The per-step chain is the per-cell
// arithmetic of every other kernel (the same functions, so the states are
// bit-identical to the resident plan's): the thermal field of step n + 1 is
// drawn while step n is corrected (it does not depend on m), and the loop is
// accumulated in FP64 every step with the ordinate m_z of the single cell.
// The applied field is the same for every lane of one level: when all lanes
// of a wave belong to one level, the wave tabulates the FP64 schedule for
// the next kLanesChunk steps in LDS (each lane a few entries) and the step
// chain reads it back, instead of every lane evaluating it every step.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

constexpr int kLanesThreads = 64;
constexpr int kLanesChunk = 256;   // steps per applied-field table

__global__ __launch_bounds__(kLanesThreads) void k_lanes(const InstDev* __restrict__ insts, int inst0, int ninst,
                                                        const LevelDev* __restrict__ levels,
                                                        float* __restrict__ buf0, float* __restrict__ buf1,
                                                        const float* __restrict__ axes,
                                                        double* __restrict__ records, AccDev* __restrict__ accs,
                                                        float* __restrict__ ckpt, int ckpt_every, int64_t n0,
                                                        int64_t nsteps, int* __restrict__ status)
{
    __shared__ float s_hz[kLanesChunk + 1];    // applied field (A/m, FP32) of the chunk's steps
    __shared__ double s_H[kLanesChunk + 1];    // the same in Oe, FP64, for the loop
    const int lane = static_cast<int>(threadIdx.x);
    const int k = static_cast<int>(blockIdx.x) * kLanesThreads + lane;
    const bool act = k < ninst;
    const int inst = inst0 + (act ? k : 0);
    const InstDev I = insts[inst];
    const LevelDev L = levels[I.level];
    // one level for the whole wave? (lane 0 is always a realization; lanes
    // past the last one step a copy of it and write nothing)
    const int lev0 = __shfl(I.level, 0);
    const bool shared_field = __ballot(act && I.level != lev0) == 0;
    const LevelDev& L0 = levels[lev0];
    const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
    V3 m = V3{mi[0], mi[1], mi[2]};
    const V3 u = L.has_axes ? V3{axes[L.axes_off], axes[L.axes_off + 1], axes[L.axes_off + 2]}
                            : V3{L.ux, L.uy, L.uz};
    AccDev a = accs[inst];
    double* rec = records + I.rec_off;
    double w = wave_at(L, n0);
    float hz0 = static_cast<float>(L.hz_amp * w);
    double H0 = L.hz_oe * w;
    V3 hth = thermal_field(L, I.seed, 0u, n0);
    for (int64_t c0 = 0; c0 < nsteps; c0 += kLanesChunk) {
        const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - c0));
        if (shared_field) {
            __syncthreads();   // the previous chunk's reads are done
            for (int t = lane; t <= cn; t += kLanesThreads) {
                const double wt = wave_at(L0, n0 + c0 + t);
                s_hz[t] = static_cast<float>(L0.hz_amp * wt);
                s_H[t] = L0.hz_oe * wt;
            }
            __syncthreads();
        }
        for (int t = 0; t < cn; ++t) {
            const int64_t n = n0 + c0 + t;
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3;
                if (act) {
                    cp[0] = m.x;
                    cp[1] = m.y;
                    cp[2] = m.z;
                }
            }
            float hz1;
            double H1;
            if (shared_field) {
                hz1 = s_hz[t + 1];
                H1 = s_H[t + 1];
            } else {
                w = wave_at(L, n + 1);
                hz1 = static_cast<float>(L.hz_amp * w);
                H1 = L.hz_oe * w;
            }
            // a single cell is its own neighbour on every face: the exchange
            // sum is formed as in every other kernel (zero up to FP32 rounding)
            V3 mp, q;
            heun_predict(L, m, nb_sum(m, m, m, m, m, m, m), u, hz0, hth, mp, q);
            const V3 hth_next = thermal_field(L, I.seed, 0u, n + 1);
            m = heun_correct(L, mp, nb_sum(mp, mp, mp, mp, mp, mp, mp), u, hz1, hth, q);
            if (act) loop_accumulate_h(a, L, H0, H1, static_cast<double>(m.z), rec);
            hth = hth_next;
            hz0 = hz1;
            H0 = H1;
        }
    }
    if (!act) return;
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    mo[0] = m.x;
    mo[1] = m.y;
    mo[2] = m.z;
    accs[inst] = a;
    if (!isfinite(a.m_prev)) atomicOr(status, 1);
}

}  // namespace sllg
