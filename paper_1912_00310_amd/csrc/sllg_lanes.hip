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
// drawn while step n is corrected (it does not depend on m), the applied
// field comes from the FP64 schedule, and the loop is accumulated in FP64
// every step with the ordinate m_z of the single cell.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

constexpr int kLanesThreads = 64;

__global__ __launch_bounds__(kLanesThreads) void k_lanes(const InstDev* __restrict__ insts, int inst0, int ninst,
                                                        const LevelDev* __restrict__ levels,
                                                        float* __restrict__ buf0, float* __restrict__ buf1,
                                                        const float* __restrict__ axes,
                                                        double* __restrict__ records, AccDev* __restrict__ accs,
                                                        float* __restrict__ ckpt, int ckpt_every, int64_t n0,
                                                        int64_t nsteps, int* __restrict__ status)
{
    const int k = static_cast<int>(blockIdx.x) * kLanesThreads + static_cast<int>(threadIdx.x);
    if (k >= ninst) return;
    const int inst = inst0 + k;
    const InstDev I = insts[inst];
    const LevelDev L = levels[I.level];
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
    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
            float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3;
            cp[0] = m.x;
            cp[1] = m.y;
            cp[2] = m.z;
        }
        w = wave_at(L, n + 1);
        const float hz1 = static_cast<float>(L.hz_amp * w);
        const double H1 = L.hz_oe * w;
        // a single cell is its own neighbour on every face: the exchange sum
        // is formed as in every other kernel (zero up to FP32 rounding)
        V3 mp, q;
        heun_predict(L, m, nb_sum(m, m, m, m, m, m, m), u, hz0, hth, mp, q);
        const V3 hth_next = thermal_field(L, I.seed, 0u, n + 1);
        m = heun_correct(L, mp, nb_sum(mp, mp, mp, mp, mp, mp, mp), u, hz1, hth, q);
        loop_accumulate_h(a, L, H0, H1, static_cast<double>(m.z), rec);
        hth = hth_next;
        hz0 = hz1;
        H0 = H1;
    }
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    mo[0] = m.x;
    mo[1] = m.y;
    mo[2] = m.z;
    accs[inst] = a;
    if (!isfinite(a.m_prev)) atomicOr(status, 1);
}

}  // namespace sllg
