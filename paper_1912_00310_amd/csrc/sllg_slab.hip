// Persistent z-slab plan: several workgroups share one realization and run
// many Heun steps per launch, exchanging only boundary planes.
//
// Workgroup s owns the planes [z0, z0 + nzs) (nzs >= 2) of one instance; all
// of a plane's nx*ny cells are handled by one workgroup, so x-y neighbours are
// always local.  Per step it
//   1. predicts planes z0-1 .. z0+nzs (its own planes plus one halo plane on
//      each side) from m_n in LDS, which holds planes z0-2 .. z0+nzs+1;
//   2. corrects its own planes from m' in LDS and writes m_{n+1} over m_n;
//   3. publishes its first two and last two planes of m_{n+1} (each plane
//      once) into a step-parity exchange buffer, one 32-bit word per
//      component written by one agent-coherent store: a component of a unit
//      vector has |v| < 2, so bit 30 of its FP32 pattern is 0 and carries a
//      tag bit that alternates between successive uses of a buffer;
//   4. polls the words its z neighbours publish for the same step until every
//      tag matches, and puts their values into its LDS halo.
// A word carries its own tag, so no separate flag or store acknowledgement is
// needed: one trip through device memory per step.  The host fills both
// buffers with the opposite tags before each launch.
// Neighbouring workgroups never drift apart by more than one step, so the
// double-buffered exchange has no write-after-read hazard.  The per-step
// partial sums of m_z go to a [slab][step] buffer that a fold kernel turns
// into loops after the launch.  The launch is cooperative (all workgroups
// resident); every wait is bounded and a timeout sets a status bit and ends
// the kernel.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

struct SlabDev {
    int32_t inst;
    int32_t z0, nzs;
    int32_t prev, next;   // workgroup of the slab below / above (-1 at the grid ends)
    int32_t lid;          // slab index in instance order (row of the partials buffer)
    int32_t pad0, pad1;
};

constexpr uint32_t kTagBit = 1u << 30;

// 32-bit exchange word: the FP32 pattern of |v| < 2 with bit 30 as the tag;
// any other value (only after a numerical blow-up, which the loop fold
// reports) is sent as +-1.5
__device__ __forceinline__ void st_word32(uint32_t* p, float v, uint32_t tbit)
{
    const float s = fabsf(v) < 2.0f ? v : copysignf(1.5f, v);
    __hip_atomic_store(p, __float_as_uint(s) | (tbit << 30), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_word32(const uint32_t* p)
{
    return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float word32_val(uint32_t w) { return __uint_as_float(w & ~kTagBit); }

// exchange slot of own plane e (1-based) of a slab of nzs planes: the first
// two planes use slots 0, 1, the last two slots 2, 3 unless already sent
__device__ __forceinline__ int slab_slot(int e, int nzs) { return e <= 2 ? e - 1 : 2 + (e - (nzs - 1)); }
constexpr int kSlabChunk = 1024;   // steps per launch (depth of the partials buffer)

__device__ __forceinline__ void st_word(uint64_t* p, float v, uint32_t tag)
{
    const uint64_t w = static_cast<uint64_t>(__float_as_uint(v)) | (static_cast<uint64_t>(tag) << 32);
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_word(const uint64_t* p)
{
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t word_tag(uint64_t w) { return static_cast<uint32_t>(w >> 32); }
__device__ __forceinline__ float word_val(uint64_t w) { return __uint_as_float(static_cast<uint32_t>(w)); }

// tag of the words published at step st of a launch: tag_base + st + 1,
// tag_base = (launch sequence number mod 2^21) << 11, st < 2048
template <int NT, int K>
__global__ __launch_bounds__(NT) void k_slab(const SlabDev* __restrict__ slabs, const InstDev* __restrict__ insts,
                                             const LevelDev* __restrict__ levels, float* __restrict__ buf0,
                                             float* __restrict__ buf1, const float* __restrict__ axes,
                                             uint64_t* __restrict__ xch64, uint32_t tag_base,
                                             double* __restrict__ partials, int pstride, float* __restrict__ ckpt,
                                             int ckpt_every, int64_t n0, int nsteps, int* __restrict__ status,
                                             uint32_t spin_limit)
{
    extern __shared__ float4 lds_slab[];
    __shared__ double red[NT / 64];
    __shared__ int s_abort;
    __shared__ float s_hz[kSlabChunk + 1];   // applied field of the launch's steps

    const int sid = static_cast<int>(blockIdx.x);
    const SlabDev S = slabs[sid];
    const InstDev I = insts[S.inst];
    const LevelDev& L = levels[I.level];
    const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.ncell;
    const int P = nx * ny;
    const int NPP = NT / P;
    const int tid = threadIdx.x;
    const int c = tid % P, r = tid / P;
    const bool lane_on = r < NPP;
    const int x = c % nx, y = c / nx;
    const int z0 = S.z0, nzs = S.nzs;
    const int NE = nzs + 2;                     // predicted planes
    // one float4 (x, y, z, unused) per cell: one 16-byte LDS access per neighbour
    float4* Mn = lds_slab;                      // (nzs + 4) planes of P cells
    float4* Mp = lds_slab + (nzs + 4) * P;      // (nzs + 2) planes of P cells
    auto f4 = [](float x, float y, float z) { return make_float4(x, y, z, 0.0f); };
    auto v34 = [](float4 v) { return V3{v.x, v.y, v.z}; };
    const int ixm = x > 0 ? c - 1 : c, ixp = x < nx - 1 ? c + 1 : c;
    const int iym = y > 0 ? c - nx : c, iyp = y < ny - 1 ? c + nx : c;
    // exchange slot (3 x P words) of one plane of one slab at a step parity
    (void)tag_base;
    uint32_t* const xch = reinterpret_cast<uint32_t*>(xch64);
    // (the parity stride is formed once: gridDim.x read inside the step loop
    // is a scalar load that waits on the same counter as the LDS accesses)
    const int64_t par_stride = static_cast<int64_t>(gridDim.x) * 4 * 3 * P;
    uint32_t* const xch_par[2] = {xch, xch + par_stride};
    auto xslot = [&](int par, int slab, int slot) {
        return xch_par[par] + (static_cast<int64_t>(slab) * 4 + slot) * 3 * P;
    };
    const int nzs_prev = S.prev >= 0 ? slabs[S.prev].nzs : 0;
    // a launch after an exchange timeout (status bit 2) does nothing: the
    // state is undefined until the host resets it
    if (tid == 0) s_abort = (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) ? 1 : 0;

    for (int st = tid; st <= nsteps; st += NT) s_hz[st] = static_cast<float>(L.hz_amp * wave_at(L, n0 + st));
    // ---- load m_n of planes z0-2 .. z0+nzs+1 (those inside the grid)
    {
        const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
        for (int me = r; me < nzs + 4; me += NPP) {
            const int z = z0 - 2 + me;
            if (!lane_on || z < 0 || z >= nz) continue;
            const int cell = c + P * z;
            Mn[me * P + c] = f4(mi[cell], mi[N + cell], mi[2 * N + cell]);
        }
    }
    __syncthreads();
    if (s_abort) return;

    const bool axes_on = L.has_axes != 0;
    // step constants in vector registers with one plane per thread (a scalar
    // reload inside the step loop waits on the same counter as LDS accesses)
    LevelDev Lv{};
    if constexpr (K == 1) {
        Lv = L;
        Lv.c_ex = vreg(L.c_ex);
        Lv.hk = vreg(L.hk);
        Lv.g1 = vreg(L.g1);
        Lv.ag1 = vreg(L.ag1);
        Lv.dt = vreg(L.dt);
        Lv.half_dt = vreg(L.half_dt);
        Lv.sigma = vreg(L.sigma);
    }
    const LevelDev& Lc = K == 1 ? Lv : L;
    const float* ax = axes + L.axes_off;
    // The thermal field of a step does not depend on m: the field of step
    // n + 1 is drawn while the boundary words of step n are in flight, and the
    // applied field of step n + 1 is the end-of-step field of step n.
    V3 hth[K];
    auto draw = [&](int64_t n) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            const int z = z0 - 1 + e;
            if (!lane_on || e >= NE || z < 0 || z >= nz) continue;
            hth[j] = thermal_field(Lc, I.seed, static_cast<uint32_t>(c + P * z), n);
        }
    };
    draw(n0);
    // the last wave folds the block's m_z sum of the previous step
    const bool folder = tid >= NT - 64;
    for (int st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        const float hz0 = s_hz[st], hz1 = s_hz[st + 1];
        V3 q[K], u[K], mps[K];   // mps: the own cell's m' (also in LDS for the neighbours)
        // ---- 1. predictor on planes z0-1 .. z0+nzs
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            const int z = z0 - 1 + e;
            if (!lane_on || e >= NE || z < 0 || z >= nz) continue;
            const int me = e + 1;
            const float4* pl = Mn + me * P;
            const V3 m = v34(pl[c]);
            const V3 ex = nb_sum(m, v34(pl[ixm]), v34(pl[ixp]), v34(pl[iym]), v34(pl[iyp]),
                                 z > 0 ? v34(pl[c - P]) : m, z < nz - 1 ? v34(pl[c + P]) : m);
            const int cell = c + P * z;
            u[j] = axes_on ? V3{ax[cell], ax[N + cell], ax[2 * N + cell]} : V3{L.ux, L.uy, L.uz};
            V3 mp;
            heun_predict(Lc, m, ex, u[j], hz0, hth[j], mp, q[j]);
            Mp[e * P + c] = f4(mp.x, mp.y, mp.z);
            mps[j] = mp;
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0 && e >= 1 && e <= nzs) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N);
                cp[cell] = m.x;
                cp[N + cell] = m.y;
                cp[2 * N + cell] = m.z;
            }
        }
        __syncthreads();
        // ---- 2. corrector on own planes; m_{n+1} replaces m_n in LDS and
        //         the boundary planes go out as tagged words
        float msum = 0.0f;
        const int par = static_cast<int>((n + 1) & 1);
        const uint32_t tbit = static_cast<uint32_t>((n + 1) >> 1) & 1u;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            if (!lane_on || e < 1 || e > nzs) continue;
            const int z = z0 - 1 + e;
            const float4* pl = Mp + e * P;
            const V3 mp = mps[j];
            const V3 ex = nb_sum(mp, v34(pl[ixm]), v34(pl[ixp]), v34(pl[iym]), v34(pl[iyp]),
                                 z > 0 ? v34(pl[c - P]) : mp, z < nz - 1 ? v34(pl[c + P]) : mp);
            const V3 mnew = heun_correct(Lc, mp, ex, u[j], hz1, hth[j], q[j]);
            const int me = e + 1;
            Mn[me * P + c] = f4(mnew.x, mnew.y, mnew.z);
            msum += mnew.z;
            // the first two and the last two planes, each once
            if (e <= 2 || e >= nzs - 1) {
                uint32_t* d = xslot(par, sid, slab_slot(e, nzs));
                st_word32(d + c, mnew.x, tbit);
                st_word32(d + P + c, mnew.y, tbit);
                st_word32(d + 2 * P + c, mnew.z, tbit);
            }
        }
        {
            const float ws = wave_sum(msum);
            if ((tid & 63) == 0) red[tid >> 6] = static_cast<double>(ws);
        }
        if (st + 1 < nsteps) draw(n + 1);
        // ---- 3. halo planes z0-2, z0-1 from the slab below, z0+nzs, z0+nzs+1
        //         from above, once every word carries this step's tag (bounded)
        for (int h = r; h < 4 && lane_on; h += NPP) {
            const int me = h < 2 ? h : nzs + h;   // 0, 1, nzs+2, nzs+3
            const int z = z0 - 2 + me;
            if (z < 0 || z >= nz) continue;
            // below: the last two planes of the previous slab; above: the
            // first two of the next
            const uint32_t* s = h < 2 ? xslot(par, S.prev, slab_slot(nzs_prev - 1 + h, nzs_prev))
                                      : xslot(par, S.next, h - 2);
            uint32_t w0, w1, w2;
            uint32_t spins = 0;
            bool ok = true;
            const uint32_t want = tbit << 30;
            for (;;) {
                w0 = ld_word32(s + c);
                w1 = ld_word32(s + P + c);
                w2 = ld_word32(s + 2 * P + c);
                if ((w0 & kTagBit) == want && (w1 & kTagBit) == want && (w2 & kTagBit) == want) break;
                if (++spins > spin_limit) {
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (!ok) {
                s_abort = 1;
                atomicOr(status, 2);
                break;
            }
            Mn[me * P + c] = f4(word32_val(w0), word32_val(w1), word32_val(w2));
        }
        __syncthreads();
        if (s_abort) return;
        if (folder && tid == NT - 64) {
            double tot = 0.0;
            for (int w = 0; w < NT / 64; ++w) tot += red[w];
            partials[static_cast<int64_t>(S.lid) * pstride + st] = tot;
        }
    }
    // ---- write back own planes at step n0 + nsteps
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    for (int me = 2 + r; me < nzs + 2; me += NPP) {
        if (!lane_on) break;
        const int cell = c + P * (z0 - 2 + me);
        const float4 v = Mn[me * P + c];
        mo[cell] = v.x;
        mo[N + cell] = v.y;
        mo[2 * N + cell] = v.z;
    }
}

// Slab variant without recomputation: the predictor runs on the slab's own
// planes only and the boundary planes of m' are exchanged as well, so a step
// has two trips through device memory (m' after the predictor, m_{n+1} after
// the corrector), each of one plane per side, and half the per-cell work of
// k_slab.  A slab may be a single plane.  Rows of threads without own planes
// poll the neighbours' words while the other rows compute.  One buffer per
// stage suffices: a workgroup writes a stage's slot again only after it has
// received the neighbour's words of the other stage, which the neighbour
// publishes after it has read the slot.
template <int NT, int K>
__global__ __launch_bounds__(NT) void k_slab2(const SlabDev* __restrict__ slabs, const InstDev* __restrict__ insts,
                                              const LevelDev* __restrict__ levels, float* __restrict__ buf0,
                                              float* __restrict__ buf1, const float* __restrict__ axes,
                                              uint64_t* __restrict__ xch, uint32_t tag_base,
                                              double* __restrict__ partials, int pstride, float* __restrict__ ckpt,
                                              int ckpt_every, int64_t n0, int nsteps, int* __restrict__ status,
                                             uint32_t spin_limit)
{
    extern __shared__ float lds[];
    __shared__ double red[NT / 64];
    __shared__ int s_abort;

    const int sid = static_cast<int>(blockIdx.x);
    const SlabDev S = slabs[sid];
    const InstDev I = insts[S.inst];
    const LevelDev& L = levels[I.level];
    const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.ncell;
    const int P = nx * ny;
    const int NPP = NT / P;
    const int tid = threadIdx.x;
    const int c = tid % P, r = tid / P;
    const bool lane_on = r < NPP;
    const int x = c % nx, y = c / nx;
    const int z0 = S.z0, nzs = S.nzs;
    // planes me = 0 .. nzs + 1 hold z0 - 1 .. z0 + nzs (halo, own planes, halo)
    float* Mn = lds;                            // m_n
    float* Mp = lds + (nzs + 2) * 3 * P;        // m'
    const int ixm = x > 0 ? c - 1 : c, ixp = x < nx - 1 ? c + 1 : c;
    const int iym = y > 0 ? c - nx : c, iyp = y < ny - 1 ? c + nx : c;
    // exchange slot (3 x P words): stage 0 = m', 1 = m_{n+1}; slot 0 = first own plane, 1 = last
    auto xslot = [&](int stage, int slab, int slot) {
        return xch + ((static_cast<int64_t>(stage) * gridDim.x + slab) * 2 + slot) * 3 * P;
    };
    // rows that poll the halo below (h = 0) and above (h = 1)
    const int prow0 = nzs % NPP, prow1 = (nzs + 1) % NPP;
    // a launch after an exchange timeout (status bit 2) does nothing: the
    // state is undefined until the host resets it
    if (tid == 0) s_abort = (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) ? 1 : 0;

    {
        const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
        for (int me = r; me < nzs + 2; me += NPP) {
            const int z = z0 - 1 + me;
            if (!lane_on || z < 0 || z >= nz) continue;
            const int cell = c + P * z;
            Mn[(me * 3 + 0) * P + c] = mi[cell];
            Mn[(me * 3 + 1) * P + c] = mi[N + cell];
            Mn[(me * 3 + 2) * P + c] = mi[2 * N + cell];
        }
    }
    __syncthreads();
    if (s_abort) return;

    const bool axes_on = L.has_axes != 0;
    const float* ax = axes + L.axes_off;
    V3 hth[K];
    auto draw = [&](int64_t n) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            if (!lane_on || e >= nzs) continue;
            hth[j] = thermal_field(L, I.seed, static_cast<uint32_t>(c + P * (z0 + e)), n);
        }
    };
    // receive one halo plane of a stage into dst (bounded wait); false on timeout
    auto receive = [&](int stage, int h, float* dst, uint32_t tag) -> bool {
        const int nb = h == 0 ? S.prev : S.next;
        if (nb < 0) return true;
        const uint64_t* src = xslot(stage, nb, h == 0 ? 1 : 0);
        uint64_t w0, w1, w2;
        uint32_t spins = 0;
        for (;;) {
            w0 = ld_word(src + c);
            w1 = ld_word(src + P + c);
            w2 = ld_word(src + 2 * P + c);
            if (word_tag(w0) == tag && word_tag(w1) == tag && word_tag(w2) == tag) break;
            if (++spins > spin_limit) return false;
            __builtin_amdgcn_s_sleep(1);
        }
        dst[c] = word_val(w0);
        dst[P + c] = word_val(w1);
        dst[2 * P + c] = word_val(w2);
        return true;
    };
    auto fail = [&]() {
        s_abort = 1;
        atomicOr(status, 2);
    };
    draw(n0);
    float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n0));
    const bool folder = tid >= NT - 64;
    for (int st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        const float hz0 = hz1;
        hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
        const uint32_t tag = tag_base + static_cast<uint32_t>(st) + 1u;
        V3 q[K], u[K];
        // ---- 1. predictor on own planes; boundary planes of m' go out
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            if (!lane_on || e >= nzs) continue;
            const int z = z0 + e, me = e + 1;
            const float* pl = Mn + me * 3 * P;
            const V3 m = v3(pl[c], pl[P + c], pl[2 * P + c]);
            const float* plm = pl - 3 * P;
            const float* plp = pl + 3 * P;
            const V3 ex = nb_sum(m, v3(pl[ixm], pl[P + ixm], pl[2 * P + ixm]),
                                 v3(pl[ixp], pl[P + ixp], pl[2 * P + ixp]),
                                 v3(pl[iym], pl[P + iym], pl[2 * P + iym]),
                                 v3(pl[iyp], pl[P + iyp], pl[2 * P + iyp]),
                                 z > 0 ? v3(plm[c], plm[P + c], plm[2 * P + c]) : m,
                                 z < nz - 1 ? v3(plp[c], plp[P + c], plp[2 * P + c]) : m);
            const int cell = c + P * z;
            u[j] = axes_on ? V3{ax[cell], ax[N + cell], ax[2 * N + cell]} : V3{L.ux, L.uy, L.uz};
            V3 mp;
            heun_predict(L, m, ex, u[j], hz0, hth[j], mp, q[j]);
            float* o = Mp + me * 3 * P;
            o[c] = mp.x;
            o[P + c] = mp.y;
            o[2 * P + c] = mp.z;
            if (e == 0) {
                uint64_t* d = xslot(0, sid, 0);
                st_word(d + c, mp.x, tag);
                st_word(d + P + c, mp.y, tag);
                st_word(d + 2 * P + c, mp.z, tag);
            }
            if (e == nzs - 1) {
                uint64_t* d = xslot(0, sid, 1);
                st_word(d + c, mp.x, tag);
                st_word(d + P + c, mp.y, tag);
                st_word(d + 2 * P + c, mp.z, tag);
            }
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N);
                cp[cell] = m.x;
                cp[N + cell] = m.y;
                cp[2 * N + cell] = m.z;
            }
        }
        if (lane_on && r == prow0 && !receive(0, 0, Mp, tag)) fail();
        if (lane_on && r == prow1 && !receive(0, 1, Mp + (nzs + 1) * 3 * P, tag)) fail();
        __syncthreads();
        if (s_abort) return;
        // ---- 2. corrector on own planes; boundary planes of m_{n+1} go out
        float msum = 0.0f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            if (!lane_on || e >= nzs) continue;
            const int z = z0 + e, me = e + 1;
            const float* pl = Mp + me * 3 * P;
            const V3 mp = v3(pl[c], pl[P + c], pl[2 * P + c]);
            const float* plm = pl - 3 * P;
            const float* plp = pl + 3 * P;
            const V3 ex = nb_sum(mp, v3(pl[ixm], pl[P + ixm], pl[2 * P + ixm]),
                                 v3(pl[ixp], pl[P + ixp], pl[2 * P + ixp]),
                                 v3(pl[iym], pl[P + iym], pl[2 * P + iym]),
                                 v3(pl[iyp], pl[P + iyp], pl[2 * P + iyp]),
                                 z > 0 ? v3(plm[c], plm[P + c], plm[2 * P + c]) : mp,
                                 z < nz - 1 ? v3(plp[c], plp[P + c], plp[2 * P + c]) : mp);
            const V3 mnew = heun_correct(L, mp, ex, u[j], hz1, hth[j], q[j]);
            float* o = Mn + me * 3 * P;
            o[c] = mnew.x;
            o[P + c] = mnew.y;
            o[2 * P + c] = mnew.z;
            msum += mnew.z;
            if (e == 0) {
                uint64_t* d = xslot(1, sid, 0);
                st_word(d + c, mnew.x, tag);
                st_word(d + P + c, mnew.y, tag);
                st_word(d + 2 * P + c, mnew.z, tag);
            }
            if (e == nzs - 1) {
                uint64_t* d = xslot(1, sid, 1);
                st_word(d + c, mnew.x, tag);
                st_word(d + P + c, mnew.y, tag);
                st_word(d + 2 * P + c, mnew.z, tag);
            }
        }
        {
            const float ws = wave_sum(msum);
            if ((tid & 63) == 0) red[tid >> 6] = static_cast<double>(ws);
        }
        if (st + 1 < nsteps) draw(n + 1);
        if (lane_on && r == prow0 && !receive(1, 0, Mn, tag)) fail();
        if (lane_on && r == prow1 && !receive(1, 1, Mn + (nzs + 1) * 3 * P, tag)) fail();
        __syncthreads();
        if (s_abort) return;
        if (folder && tid == NT - 64) {
            double tot = 0.0;
            for (int w = 0; w < NT / 64; ++w) tot += red[w];
            partials[static_cast<int64_t>(S.lid) * pstride + st] = tot;
        }
    }
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    for (int me = 1 + r; me <= nzs; me += NPP) {
        if (!lane_on) break;
        const int cell = c + P * (z0 - 1 + me);
        mo[cell] = Mn[(me * 3 + 0) * P + c];
        mo[N + cell] = Mn[(me * 3 + 1) * P + c];
        mo[2 * N + cell] = Mn[(me * 3 + 2) * P + c];
    }
}

// Fold the per-step slab partials of one launch into the loops, one block
// per instance, with no sequential pass over the steps: every thread sums
// the slabs of its steps in slab order and evaluates the field (into LDS);
// then each thread takes a contiguous run of steps and forms its part of the
// area, its zero-crossing counts, its first crossings and its records; block
// reductions combine them (area in a fixed order, so it is reproducible) and
// thread 0 applies the first crossing of the launch with the same formulas
// as the per-step accumulation.
template <int NT>
__global__ __launch_bounds__(NT) void k_fold_slabs(const InstDev* __restrict__ insts, int inst0,
                                                   const int32_t* __restrict__ islab,
                                                   const LevelDev* __restrict__ levels,
                                                   const double* __restrict__ partials, int pstride, int64_t n0,
                                                   int nsteps, AccDev* __restrict__ accs,
                                                   double* __restrict__ records, int* __restrict__ status)
{
    __shared__ double mz[kSlabChunk];
    __shared__ double hh[kSlabChunk + 1];
    __shared__ double red[NT / 64];
    __shared__ int cnt[2];
    __shared__ int first[4];   // first falling crossing, rising crossing, falling H = 0, rising H = 0
    const int k = static_cast<int>(blockIdx.x);
    const int inst = inst0 + k;
    const int tid = static_cast<int>(threadIdx.x);
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    const int s0 = islab[2 * k], ns = islab[2 * k + 1];   // level-relative first slab, count
    const double ncell = static_cast<double>(L.ncell);
    if (tid < 4) first[tid] = INT_MAX;
    if (tid < 2) cnt[tid] = 0;
    for (int st = tid; st <= nsteps; st += NT) {
        hh[st] = L.hz_oe * wave_at(L, n0 + st);
        if (st == nsteps) continue;
        double v = 0.0;
        for (int s = 0; s < ns; ++s) v += partials[static_cast<int64_t>(s0 + s) * pstride + st];
        mz[st] = v / ncell;
    }
    __syncthreads();
    const AccDev a0 = accs[inst];
    double* rec = records + I.rec_off;
    const int per = (nsteps + NT - 1) / NT;
    double area = 0.0;
    int cd = 0, ca = 0;
    int f[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    for (int st = tid * per; st < min(nsteps, (tid + 1) * per); ++st) {
        const double m0 = st == 0 ? a0.m_prev : mz[st - 1], m1 = mz[st];
        const double h0 = hh[st], h1 = hh[st + 1], dH = h1 - h0;
        area += 0.5 * (m0 + m1) * dH;
        const int change = (m0 > 0.0) != (m1 > 0.0);
        if (dH < 0.0) {
            cd += change;
            if (m0 > 0.0 && m1 <= 0.0) f[0] = min(f[0], st);
            if (h0 > 0.0 && h1 <= 0.0) f[2] = min(f[2], st);
        } else if (dH > 0.0) {
            ca += change;
            if (m0 < 0.0 && m1 >= 0.0) f[1] = min(f[1], st);
            if (h0 < 0.0 && h1 >= 0.0) f[3] = min(f[3], st);
        }
        const int q = a0.rec_phase + st + 1;
        if (q % L.record_every == 0) {
            const int64_t idx = a0.rec_idx + q / L.record_every;
            if (idx < L.n_rec) rec[idx] = m1;
        }
    }
    area = wave_sum_d(area);
    if ((tid & 63) == 0) red[tid >> 6] = area;
    if (cd) atomicAdd(&cnt[0], cd);
    if (ca) atomicAdd(&cnt[1], ca);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (f[i] != INT_MAX) atomicMin(&first[i], f[i]);
    __syncthreads();
    if (tid != 0) return;
    AccDev a = a0;
    double tot = 0.0;
    for (int w = 0; w < NT / 64; ++w) tot += red[w];
    a.area -= tot;
    a.ncross_d += cnt[0];
    a.ncross_a += cnt[1];
    auto at = [&](int st, double& m0, double& m1, double& h0, double& dH) {
        m0 = st == 0 ? a0.m_prev : mz[st - 1];
        m1 = mz[st];
        h0 = hh[st];
        dH = hh[st + 1] - h0;
    };
    double m0, m1, h0, dH;
    if (!a.found_d && first[0] != INT_MAX) {
        at(first[0], m0, m1, h0, dH);
        a.found_d = 1;
        a.hstar_d = cross_field(h0, dH, m0, m1);
    }
    if (!a.found_a && first[1] != INT_MAX) {
        at(first[1], m0, m1, h0, dH);
        a.found_a = 1;
        a.hstar_a = cross_field(h0, dH, m0, m1);
    }
    if (!a.found0_d && first[2] != INT_MAX) {
        at(first[2], m0, m1, h0, dH);
        a.found0_d = 1;
        a.m0_d = zero_field_ordinate(h0, dH, m0, m1);
    }
    if (!a.found0_a && first[3] != INT_MAX) {
        at(first[3], m0, m1, h0, dH);
        a.found0_a = 1;
        a.m0_a = zero_field_ordinate(h0, dH, m0, m1);
    }
    if (nsteps > 0) a.m_prev = mz[nsteps - 1];
    const int q = a0.rec_phase + nsteps;
    a.rec_phase = q % L.record_every;
    a.rec_idx = static_cast<int32_t>(min<int64_t>(a0.rec_idx + q / L.record_every, L.n_rec - 1));
    accs[inst] = a;
    if (!isfinite(a.m_prev)) atomicOr(status, 1);
}

}  // namespace sllg
