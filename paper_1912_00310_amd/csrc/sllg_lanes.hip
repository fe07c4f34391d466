// Single-cell levels, one realization per quad of lanes.
//
// A level of one cell (the single-macrospin limit of the coarse-graining
// rule: the whole rod as one cell that feels anisotropy, the applied field
// and the thermal field only) has no neighbour to wait for, so each
// realization is integrated on its own for a launch of many steps: the state
// and the level constants stay in registers and nothing is shared between
// realizations.  Four lanes carry one realization: lanes 0, 1, 2 of the quad
// hold the x, y, z components of m, m', q and of the fields, and each
// evaluates its own component of the per-cell functions of every other
// kernel, with the same operations in the same order, so the states are
// bit-identical to the resident plan's; lane 3 computes a copy that is never
// used.  The components a lane needs from the others (the cross products'
// neighbours, the three terms of a dot product) come from DPP quad
// permutes.  Every lane draws the (shared) thermal field of its realization,
// for step n + 1 while step n is corrected.  The step is bound by the
// latency of its dependent chain (one stepping wave per SIMD): the quads
// shorten it by 7 % against one realization per lane.
//
// A workgroup is four stepping waves (16 realizations each) and one loop
// wave for 64 realizations.  Per chunk of kLanesChunk steps the stepping
// waves leave the ordinate m_z of every step in LDS; the loop wave folds the
// previous chunk's ordinates into the FP64 loop accumulators, lane for
// realization, and tabulates the applied field of the next chunk, so the
// FP64 loop update is off the stepping chain; a barrier per chunk hands the
// buffers over (the ordinates and the field tables are double-buffered by
// chunk parity).  When the realizations of a workgroup have different
// levels, each lane evaluates its own schedule instead of the table.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

constexpr int kLanesThreads = 64;   // realizations per workgroup (four stepping waves and a loop wave)
constexpr int kLanesChunk = 64;     // steps per hand-over

// Component c of a quad-distributed vector, in every lane of the quad
// (quad_perm selecting lane c); and components c + 1 and c + 2 (mod 3) of
// the lane's own component c (lane 3 reads itself).
template <int C>
__device__ __forceinline__ float q_comp(float v)
{
    return dpp_mov<C * 0x55>(v);
}
__device__ __forceinline__ float q_next(float v) { return dpp_mov<0xC9>(v); }   // quad_perm [1,2,0,3]
__device__ __forceinline__ float q_prev(float v) { return dpp_mov<0xD2>(v); }   // quad_perm [2,0,1,3]

// dot3 of two quad-distributed vectors, the same terms in the same order
// (z product first), in every lane
__device__ __forceinline__ float q_dot(float a, float b)
{
    return fmaf(q_comp<0>(a), q_comp<0>(b), fmaf(q_comp<1>(a), q_comp<1>(b), q_comp<2>(a) * q_comp<2>(b)));
}

// component c of cross3(a, b): fmaf(a_{c+1}, b_{c+2}, -a_{c+2} b_{c+1})
__device__ __forceinline__ float q_cross(float a, float b)
{
    return fmaf(q_next(a), q_prev(b), -q_prev(a) * q_next(b));
}

// component c of x + dt f(m, H), f = -g1 m x H - ag1 m x (m x H), as llg_rhs
// and the Heun updates of the per-cell functions form it
__device__ __forceinline__ float q_rhs(const LevelDev& L, float m, float H)
{
    const float t = q_cross(m, H);
    const float d = q_cross(m, t);
    return -fmaf(L.g1, t, L.ag1 * d);
}

// component c of the effective field (eff_field): hb is the thermal field's
// component, plus the applied field on z
__device__ __forceinline__ float q_field(const LevelDev& L, float m, float u, float hb)
{
    const float ex = fmaf(-6.0f, m, ((m + m) + (m + m)) + (m + m));   // nb_sum of a cell with itself
    const float a = L.hk * q_dot(m, u);
    return fmaf(L.c_ex, ex, fmaf(a, u, hb));
}

__global__ __launch_bounds__(5 * 64) void k_lanes(const InstDev* __restrict__ insts, int inst0, int ninst,
                                                 const LevelDev* __restrict__ levels, float* __restrict__ buf0,
                                                 float* __restrict__ buf1, const float* __restrict__ axes,
                                                 double* __restrict__ records, AccDev* __restrict__ accs,
                                                 float* __restrict__ ckpt, int ckpt_every, int64_t n0,
                                                 int64_t nsteps, int* __restrict__ status)
{
    __shared__ float s_hz[2][kLanesChunk + 1];    // applied field (A/m, FP32) of a chunk's steps
    __shared__ double s_H[2][kLanesChunk + 1];    // the same in Oe, FP64, for the loop
    __shared__ float s_mz[2][kLanesChunk][kLanesThreads];   // ordinate of every step of a chunk
    __shared__ int s_lev[kLanesThreads];
    const int tid = static_cast<int>(threadIdx.x);
    const int wave = tid >> 6, lane = tid & 63;
    const bool stepper = wave < 4;
    // the realization of the thread within the workgroup: a quad of a
    // stepping wave, or a lane of the loop wave
    const int kr = stepper ? wave * 16 + (lane >> 2) : lane;
    const int c = lane & 3;   // the component of a stepping lane (3: unused copy)
    const int k = static_cast<int>(blockIdx.x) * kLanesThreads + kr;
    const bool act = k < ninst;
    const int inst = inst0 + (act ? k : 0);
    const InstDev I = insts[inst];
    const LevelDev L = levels[I.level];
    // one level for the whole workgroup? (realization 0 always exists;
    // realizations past the last one step a copy of it and write nothing)
    if (!stepper) s_lev[lane] = act ? I.level : -1;
    __syncthreads();
    const int lev0 = s_lev[0];
    bool shared_field = true;
    for (int r = 1; r < kLanesThreads; ++r) shared_field = shared_field && (s_lev[r] < 0 || s_lev[r] == lev0);
    const LevelDev& L0 = levels[lev0];
    const int64_t nchunks = (nsteps + kLanesChunk - 1) / kLanesChunk;
    // the applied field of chunk q (steps n0 + q K .. + K, the last one
    // included) into buffer q & 1, by the loop wave
    auto table = [&](int64_t q) {
        const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - q * kLanesChunk));
        for (int t = lane; t <= cn; t += 64) {
            const double wt = wave_at(L0, n0 + q * kLanesChunk + t);
            s_hz[q & 1][t] = static_cast<float>(L0.hz_amp * wt);
            s_H[q & 1][t] = L0.hz_oe * wt;
        }
    };
    if (stepper) {
        const int cc = c < 3 ? c : 0;
        const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
        float m = mi[cc];
        const float u = L.has_axes ? axes[L.axes_off + cc] : (cc == 0 ? L.ux : (cc == 1 ? L.uy : L.uz));
        float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n0));
        // the lane's component of a thermal field V3
        auto comp = [&](V3 h) { return c == 0 ? h.x : (c == 1 ? h.y : h.z); };
        float hth = comp(thermal_field(L, I.seed, 0u, n0));
        __syncthreads();   // the first table
        for (int64_t q = 0; q < nchunks; ++q) {
            const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - q * kLanesChunk));
            for (int t = 0; t < cn; ++t) {
                const int64_t n = n0 + q * kLanesChunk + t;
                if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                    float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3;
                    if (act && c < 3) cp[c] = m;
                }
                const float hz1 = shared_field ? s_hz[q & 1][t + 1]
                                               : static_cast<float>(L.hz_amp * wave_at(L, n + 1));
                // predictor (heun_predict)
                const float H = q_field(L, m, u, c == 2 ? hth + hz0 : hth);
                const float f = q_rhs(L, m, H);
                const float p = fmaf(L.dt, f, m);
                const float mp = p * __builtin_amdgcn_rsqf(q_dot(p, p));
                const float qv = fmaf(L.half_dt, f, m);
                const float hth_next = comp(thermal_field(L, I.seed, 0u, n + 1));
                // corrector (heun_correct)
                const float H1 = q_field(L, mp, u, c == 2 ? hth + hz1 : hth);
                const float f1 = q_rhs(L, mp, H1);
                const float pc = fmaf(L.half_dt, f1, qv);
                m = pc * __builtin_amdgcn_rsqf(q_dot(pc, pc));
                if (c == 2) s_mz[q & 1][t][kr] = m;
                hth = hth_next;
                hz0 = hz1;
            }
            __syncthreads();   // chunk q's ordinates and chunk q + 1's table are in place
        }
        if (act && c < 3) {
            float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
            mo[c] = m;
        }
    } else {
        AccDev a = accs[inst];
        double* rec = records + I.rec_off;
        // fold chunk q (its ordinates and, with one level, its field table)
        auto fold = [&](int64_t q) {
            const int cn = static_cast<int>(min<int64_t>(kLanesChunk, nsteps - q * kLanesChunk));
            double H0 = shared_field ? s_H[q & 1][0] : L.hz_oe * wave_at(L, n0 + q * kLanesChunk);
            for (int t = 0; t < cn; ++t) {
                const double H1 = shared_field ? s_H[q & 1][t + 1]
                                               : L.hz_oe * wave_at(L, n0 + q * kLanesChunk + t + 1);
                if (act) loop_accumulate_h(a, L, H0, H1, static_cast<double>(s_mz[q & 1][t][lane]), rec);
                H0 = H1;
            }
        };
        if (shared_field && nchunks > 0) table(0);
        __syncthreads();
        for (int64_t q = 0; q < nchunks; ++q) {
            // while the stepping waves run chunk q: fold chunk q - 1, then
            // tabulate chunk q + 1 into the buffers chunk q - 1 used
            if (q > 0) fold(q - 1);
            if (shared_field && q + 1 < nchunks) table(q + 1);
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
