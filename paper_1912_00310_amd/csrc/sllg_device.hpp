// Per-cell device arithmetic of the stochastic LLG step for gfx950.
//
// Every kernel of the library calls these functions, so the FP32 arithmetic
// of a cell is the same whichever execution plan runs it (the library is
// built with -ffp-contract=off; fused multiply-adds are written out).
#pragma once
#include <hip/hip_runtime.h>

#include "sllg_types.hpp"

namespace sllg {

struct V3 {
    float x, y, z;
};

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }

__device__ __forceinline__ V3 cross3(V3 a, V3 b)
{
    return V3{fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x)};
}

__device__ __forceinline__ float dot3(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter words 0 and 2
// are multiplied by the round multipliers; the new word 0 is hi(word2 product)
// ^ word1 ^ key0, word 1 the low half of that product, word 2 hi(word0
// product) ^ word3 ^ key1, word 3 its low half; the key then advances by the
// Weyl constants.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t a, b, c, d;
};

// A copy of a wave-uniform value in a vector register: the compiler cannot
// re-read it from memory inside a loop (a scalar reload waits on the same
// counter as the LDS reads of the step).
__device__ __forceinline__ float vreg(float x)
{
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Three-input exclusive or in one gfx950 VALU instruction (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox10(U4 w, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p = static_cast<uint64_t>(0xD2511F53u) * w.a;
        const uint64_t s = static_cast<uint64_t>(0xCD9E8D57u) * w.c;
        U4 n;
        if (r < 2) {
            // the first rounds mix wave-uniform counter words (step, tags),
            // which plain operators keep on the scalar unit
            n.a = static_cast<uint32_t>(s >> 32) ^ w.b ^ k0;
            n.c = static_cast<uint32_t>(p >> 32) ^ w.d ^ k1;
        } else {
            n.a = xor3(static_cast<uint32_t>(s >> 32), w.b, k0);
            n.c = xor3(static_cast<uint32_t>(p >> 32), w.d, k1);
        }
        n.b = static_cast<uint32_t>(s);
        n.d = static_cast<uint32_t>(p);
        w = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return w;
}

// Raw words for (seed, level tag, purpose tag, cell, step).
__device__ __forceinline__ U4 philox_cell(uint64_t seed, uint32_t level, uint32_t tag,
                                          uint32_t cell, uint64_t step)
{
    U4 ctr;
    ctr.a = cell;
    ctr.b = static_cast<uint32_t>(step);
    ctr.c = (static_cast<uint32_t>(step >> 32) & 0xFFFFu) | ((level & 0xFFu) << 16) | (tag << 24);
    ctr.d = 0u;
    return philox10(ctr, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
}

// 23 random bits with a half-step offset: (2k+1)/2^24, exact in FP32.  One
// funnel shift puts the top 23 bits k of w under the exponent of 1.0, giving
// 1 + k 2^-23; subtracting 1 - 2^-24 is exact (Sterbenz) and leaves
// (2k + 1) 2^-24.
__device__ __forceinline__ float unit_open(uint32_t w)
{
    const float one_k = __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u));
    return one_k - 0.999999940395355224609375f;
}

// Box-Muller with the hardware transcendentals: v_log_f32 is log2, v_sin_f32
// and v_cos_f32 take the angle in revolutions (so 2*pi*u needs no reduction).
__device__ __forceinline__ V3 gauss3(U4 w)
{
    const float u0 = unit_open(w.a), u1 = unit_open(w.b);
    const float u2 = unit_open(w.c), u3 = unit_open(w.d);
    const float kMinus2Ln2 = -1.3862943611198906f;  // -2 ln 2
    const float r0 = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u0));
    const float r2 = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u2));
    return V3{r0 * __builtin_amdgcn_cosf(u1), r0 * __builtin_amdgcn_sinf(u1),
              r2 * __builtin_amdgcn_cosf(u3)};
}

// ---------------------------------------------------------------------------
// Field protocol
// ---------------------------------------------------------------------------
// Fraction of the peak applied field at step n (FP64).  The phase k/N is
// formed with the stored reciprocal of N (within one ulp of the quotient).
__device__ __forceinline__ double wave_at(const LevelDev& L, int64_t n)
{
    int64_t k = n;
    while (k >= L.n_period) k -= L.n_period;
    const double s = static_cast<double>(k) * L.inv_period;
    if (L.wave == 0) return (2 * k <= L.n_period) ? 1.0 - 4.0 * s : 4.0 * s - 3.0;
    if (L.wave == 1) return cospi(2.0 * s);
    return 1.0;
}

// ---------------------------------------------------------------------------
// Effective field and the Landau-Lifshitz right-hand side (Eq. 1 / Ms):
//   H = c_ex * sum_j (m_j - m_i) + H_K (m.u) u + hz z + H_th
//   f = -gamma1 m x H - alpha gamma1 m x (m x H)
// ---------------------------------------------------------------------------
__device__ __forceinline__ V3 eff_field(float c_ex, float hk, V3 m, V3 ex, V3 u, float hz, V3 hth)
{
    const float a = hk * dot3(m, u);
    V3 H;
    H.x = fmaf(c_ex, ex.x, fmaf(a, u.x, hth.x));
    H.y = fmaf(c_ex, ex.y, fmaf(a, u.y, hth.y));
    H.z = fmaf(c_ex, ex.z, fmaf(a, u.z, hth.z + hz));
    return H;
}

__device__ __forceinline__ V3 llg_rhs(float g1, float ag1, V3 m, V3 H)
{
    const V3 t = cross3(m, H);
    const V3 d = cross3(m, t);
    return V3{-fmaf(g1, t.x, ag1 * d.x), -fmaf(g1, t.y, ag1 * d.y), -fmaf(g1, t.z, ag1 * d.z)};
}

__device__ __forceinline__ V3 normalized(V3 p)
{
    const float r = __builtin_amdgcn_rsqf(dot3(p, p));
    return V3{p.x * r, p.y * r, p.z * r};
}

// Sum over the six face neighbours of (m_j - m_i), formed as
// (sum_j m_j) - 6 m_i: five adds in pairs and one fused multiply-add per
// component (the FP32 rounding error is a few 1e-7, against 1e-7 for the
// differences summed one by one).  A missing neighbour is passed as the cell
// itself, so it contributes zero up to that rounding.
__device__ __forceinline__ V3 nb_sum(V3 m, V3 xm, V3 xp, V3 ym, V3 yp, V3 zm, V3 zp)
{
    V3 e;
    e.x = fmaf(-6.0f, m.x, ((xm.x + xp.x) + (ym.x + yp.x)) + (zm.x + zp.x));
    e.y = fmaf(-6.0f, m.y, ((xm.y + xp.y) + (ym.y + yp.y)) + (zm.y + zp.y));
    e.z = fmaf(-6.0f, m.z, ((xm.z + xp.z) + (ym.z + yp.z)) + (zm.z + zp.z));
    return e;
}

// Predictor stage: m' = (m + dt f)/|.|; also q = m + dt/2 f for the corrector.
__device__ __forceinline__ void heun_predict(const LevelDev& L, V3 m, V3 ex, V3 u, float hz, V3 hth,
                                             V3& mp, V3& q)
{
    const V3 H = eff_field(L.c_ex, L.hk, m, ex, u, hz, hth);
    const V3 f = llg_rhs(L.g1, L.ag1, m, H);
    mp = normalized(V3{fmaf(L.dt, f.x, m.x), fmaf(L.dt, f.y, m.y), fmaf(L.dt, f.z, m.z)});
    q = V3{fmaf(L.half_dt, f.x, m.x), fmaf(L.half_dt, f.y, m.y), fmaf(L.half_dt, f.z, m.z)};
}

// Corrector stage: m_{n+1} = (q + dt/2 f(m', H'))/|.|.
__device__ __forceinline__ V3 heun_correct(const LevelDev& L, V3 mp, V3 exp_, V3 u, float hz1, V3 hth,
                                           V3 q)
{
    const V3 H = eff_field(L.c_ex, L.hk, mp, exp_, u, hz1, hth);
    const V3 f = llg_rhs(L.g1, L.ag1, mp, H);
    return normalized(V3{fmaf(L.half_dt, f.x, q.x), fmaf(L.half_dt, f.y, q.y), fmaf(L.half_dt, f.z, q.z)});
}

__device__ __forceinline__ V3 thermal_field(const LevelDev& L, uint64_t seed, uint32_t cell, int64_t n)
{
    const V3 xi = gauss3(philox_cell(seed, static_cast<uint32_t>(L.level_tag), kTagNoise, cell,
                                     static_cast<uint64_t>(n)));
    return V3{L.sigma * xi.x, L.sigma * xi.y, L.sigma * xi.z};
}

// ---------------------------------------------------------------------------
// Online loop accumulation for one instance at step n -> n+1 (FP64).
// ---------------------------------------------------------------------------
// Field where the ordinate crosses zero between steps (linear in H), and the
// ordinate where the field crosses zero.
__device__ inline double cross_field(double h0, double dH, double m0, double m1)
{
    return h0 - m0 * dH / (m1 - m0);
}
__device__ inline double zero_field_ordinate(double h0, double dH, double m0, double m1)
{
    return m0 + (m1 - m0) * (0.0 - h0) / dH;
}

// h0, h1: simulated field (Oe) at steps n and n + 1.  Written with selects
// rather than stores in branches, so that a copy of the accumulators can
// live in registers.
__device__ inline void loop_accumulate_h(AccDev& a, const LevelDev& L, double h0, double h1, double m_new,
                                         double* rec)
{
    const double dH = h1 - h0;
    const double m0 = a.m_prev;
    a.area -= 0.5 * (m0 + m_new) * dH;
    const int change = (m0 > 0.0) != (m_new > 0.0);
    const bool fall = dH < 0.0, rise = dH > 0.0;
    a.ncross_d += fall ? change : 0;
    a.ncross_a += rise ? change : 0;
    // first crossing of the ordinate through zero on each branch
    const bool hit_d = fall && !a.found_d && m0 > 0.0 && m_new <= 0.0;
    const bool hit_a = rise && !a.found_a && m0 < 0.0 && m_new >= 0.0;
    double xf = 0.0;
    if (hit_d || hit_a) xf = cross_field(h0, dH, m0, m_new);
    a.hstar_d = hit_d ? xf : a.hstar_d;
    a.hstar_a = hit_a ? xf : a.hstar_a;
    a.found_d |= hit_d ? 1 : 0;
    a.found_a |= hit_a ? 1 : 0;
    // ordinate where the field crosses zero on each branch
    const bool z_d = fall && !a.found0_d && h0 > 0.0 && h1 <= 0.0;
    const bool z_a = rise && !a.found0_a && h0 < 0.0 && h1 >= 0.0;
    double zf = 0.0;
    if (z_d || z_a) zf = zero_field_ordinate(h0, dH, m0, m_new);
    a.m0_d = z_d ? zf : a.m0_d;
    a.m0_a = z_a ? zf : a.m0_a;
    a.found0_d |= z_d ? 1 : 0;
    a.found0_a |= z_a ? 1 : 0;
    a.m_prev = m_new;
    if (++a.rec_phase == L.record_every) {
        a.rec_phase = 0;
        if (a.rec_idx + 1 < L.n_rec) rec[++a.rec_idx] = m_new;   // never past the record
    }
}

__device__ inline void loop_accumulate(AccDev& a, const LevelDev& L, int64_t n, double m_new, double* rec)
{
    loop_accumulate_h(a, L, L.hz_oe * wave_at(L, n), L.hz_oe * wave_at(L, n + 1), m_new, rec);
}

// Wave-wide FP32 sum (every lane gets the total).
__device__ __forceinline__ float wave_sum(float v);
__device__ __forceinline__ double wave_sum_d(double v);

// Stream plan bookkeeping without device-wide fences.  Tile partials of step
// n go to partials[(n & 1) * ptiles + tile]; the instance's first tile folds
// the partials of step n - 1 into the loop at the start of the launch for
// step n (the kernel boundary makes them visible); a flush kernel folds the
// last step of a run.  Wave 0 of the calling block sums the partials in a
// fixed order, so the loop is bitwise reproducible.
__device__ inline void fold_partials(const InstDev& I, const LevelDev& L, int64_t n, const double* partials,
                                     int ptiles, AccDev* accs, int inst, double* records, int* status)
{
    if (threadIdx.x >= 64) return;
    const double* p = partials + (n & 1) * static_cast<int64_t>(ptiles) + I.tile0;
    double s = 0.0;
    for (int t = static_cast<int>(threadIdx.x); t < I.ntiles; t += 64) s += p[t];
    s = wave_sum_d(s);
    if (threadIdx.x == 0) {
        AccDev a = accs[inst];
        loop_accumulate(a, L, n, s / static_cast<double>(L.ncell), records + I.rec_off);
        accs[inst] = a;
        if (!isfinite(a.m_prev)) atomicOr(status, 1);
    }
}

// Block sum of one FP32 value per thread: FP32 within waves, FP64 across
// waves in wave order.  red holds NT / 64 doubles; thread 0 gets the total.
template <int NT>
__device__ inline double block_sum(float v, double* red)
{
    const float ws = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = static_cast<double>(ws);
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) tot += red[w];
    return tot;
}

// End of a stream-plan block: publish the tile partial; the last block of
// the launch advances the step counter (relaxed atomics: every block read
// the counter before it arrived here).
__device__ inline void stream_block_end(double tot, int64_t n, int tile, int ptiles, double* partials,
                                        bool first_tile, uint32_t* pend, int inst, uint32_t* launch_cnt,
                                        int64_t* steps, int level, int64_t n_steps)
{
    if (threadIdx.x != 0) return;
    partials[(n & 1) * static_cast<int64_t>(ptiles) + tile] = tot;
    if (first_tile) pend[inst] = 1u;
    const uint32_t prev = __hip_atomic_fetch_add(launch_cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
        __hip_atomic_store(launch_cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n + 1 <= n_steps) __hip_atomic_store(&steps[level], n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
// DPP lane move (data-parallel primitive; lanes that receive nothing get 0)
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

// Wave-wide FP32 sum in a fixed order without the LDS crossbar: pairs and
// quads (quad permutes), half rows and rows (mirrors), then rows 0+1 and
// 2+3 (broadcast of lane 15) and all four (broadcast of lane 31); lane 63
// ends with the total, which is returned to every lane.  Called with every
// lane of the wave active.
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_mov<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);          // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);         // row_half_mirror
    v += dpp_mov<0x140>(v);         // row_mirror
    v += dpp_mov<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_mov<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace sllg
