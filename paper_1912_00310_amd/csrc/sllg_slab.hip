// Persistent z-slab plan: several workgroups share one realization and run
// many Heun steps per launch, exchanging only boundary planes.
//
// Workgroup s owns the planes [z0, z0 + nzs) (nzs >= 2) of one instance; all
// of a plane's nx*ny cells are handled by one workgroup, so x-y neighbours are
// always local.  Per step it
//   1. predicts planes z0-1 .. z0+nzs (its own planes plus one halo plane on
//      each side) from m_n in LDS, which holds planes z0-2 .. z0+nzs+1;
//   2. corrects its own planes from m' in LDS and writes m_{n+1} over m_n;
//   3. publishes its first two and last two planes of m_{n+1} into a
//      step-parity exchange buffer with agent-coherent stores, waits for the
//      stores, then publishes its step count in a flag;
//   4. waits for the flags of its z neighbours and copies their boundary
//      planes into its LDS halo.
// Neighbouring workgroups therefore never drift apart by more than one step,
// and the double-buffered exchange has no write-after-read hazard.  The
// per-step partial sums of m_z go to a [workgroup][step] buffer that a fold
// kernel turns into loops after the launch.  The launch is cooperative (all
// workgroups resident); every wait is bounded and a timeout sets a status
// bit and ends the kernel.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

struct SlabDev {
    int32_t inst;
    int32_t z0, nzs;
    int32_t prev, next;   // slab below / above (-1 at the grid ends)
    int32_t slab0;        // first slab of the instance
    int32_t pad0, pad1;
};

__device__ __forceinline__ void st_agent(float* p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float* p)
{
    return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT, int K>
__global__ __launch_bounds__(NT) void k_slab(const SlabDev* __restrict__ slabs, const InstDev* __restrict__ insts,
                                             const LevelDev* __restrict__ levels, float* __restrict__ buf0,
                                             float* __restrict__ buf1, const float* __restrict__ axes,
                                             float* __restrict__ xch, uint32_t* __restrict__ flags,
                                             double* __restrict__ partials, int pstride, float* __restrict__ ckpt,
                                             int ckpt_every, int64_t n0, int nsteps, int* __restrict__ status)
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
    const int NE = nzs + 2;                     // predicted planes
    float* Mn = lds;                            // (nzs + 4) planes x 3 x P
    float* Mp = lds + (nzs + 4) * 3 * P;        // (nzs + 2) planes x 3 x P
    auto mn = [&](int me, int k) -> float& { return Mn[(me * 3 + k) * P + c]; };
    const int ixm = x > 0 ? c - 1 : c, ixp = x < nx - 1 ? c + 1 : c;
    const int iym = y > 0 ? c - nx : c, iyp = y < ny - 1 ? c + nx : c;
    // exchange slot of one plane of one slab at a step parity
    const int64_t XS = 4LL * 3 * P;
    auto xslot = [&](int par, int slab, int slot) {
        return xch + (static_cast<int64_t>(par) * gridDim.x + slab) * XS + static_cast<int64_t>(slot) * 3 * P;
    };
    if (tid == 0) s_abort = 0;

    // ---- load m_n of planes z0-2 .. z0+nzs+1 (those inside the grid)
    {
        const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
        for (int me = r; me < nzs + 4; me += NPP) {
            const int z = z0 - 2 + me;
            if (!lane_on || z < 0 || z >= nz) continue;
            const int cell = c + P * z;
            mn(me, 0) = mi[cell];
            mn(me, 1) = mi[N + cell];
            mn(me, 2) = mi[2 * N + cell];
        }
    }
    __syncthreads();

    const bool axes_on = L.has_axes != 0;
    const float* ax = axes + L.axes_off;
    for (int st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        const float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n));
        const float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
        V3 q[K], hth[K], u[K];
        // ---- 1. predictor on planes z0-1 .. z0+nzs
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            const int z = z0 - 1 + e;
            if (!lane_on || e >= NE || z < 0 || z >= nz) continue;
            const int me = e + 1;
            const V3 m = v3(mn(me, 0), mn(me, 1), mn(me, 2));
            const float* pl = Mn + me * 3 * P;
            const V3 ex = nb_sum(m, v3(pl[ixm], pl[P + ixm], pl[2 * P + ixm]),
                                 v3(pl[ixp], pl[P + ixp], pl[2 * P + ixp]),
                                 v3(pl[iym], pl[P + iym], pl[2 * P + iym]),
                                 v3(pl[iyp], pl[P + iyp], pl[2 * P + iyp]),
                                 z > 0 ? v3(mn(me - 1, 0), mn(me - 1, 1), mn(me - 1, 2)) : m,
                                 z < nz - 1 ? v3(mn(me + 1, 0), mn(me + 1, 1), mn(me + 1, 2)) : m);
            const int cell = c + P * z;
            u[j] = axes_on ? V3{ax[cell], ax[N + cell], ax[2 * N + cell]} : V3{L.ux, L.uy, L.uz};
            hth[j] = thermal_field(L, I.seed, static_cast<uint32_t>(cell), n);
            V3 mp;
            heun_predict(L, m, ex, u[j], hz0, hth[j], mp, q[j]);
            float* o = Mp + e * 3 * P;
            o[c] = mp.x;
            o[P + c] = mp.y;
            o[2 * P + c] = mp.z;
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0 && e >= 1 && e <= nzs) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N);
                cp[cell] = m.x;
                cp[N + cell] = m.y;
                cp[2 * N + cell] = m.z;
            }
        }
        __syncthreads();
        // ---- 2. corrector on own planes; m_{n+1} replaces m_n in LDS
        float msum = 0.0f;
        const int par = static_cast<int>((n + 1) & 1);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = r + j * NPP;
            if (!lane_on || e < 1 || e > nzs) continue;
            const int z = z0 - 1 + e;
            const float* pl = Mp + e * 3 * P;
            const V3 mp = v3(pl[c], pl[P + c], pl[2 * P + c]);
            const float* plm = Mp + (e - 1) * 3 * P;
            const float* plp = Mp + (e + 1) * 3 * P;
            const V3 ex = nb_sum(mp, v3(pl[ixm], pl[P + ixm], pl[2 * P + ixm]),
                                 v3(pl[ixp], pl[P + ixp], pl[2 * P + ixp]),
                                 v3(pl[iym], pl[P + iym], pl[2 * P + iym]),
                                 v3(pl[iyp], pl[P + iyp], pl[2 * P + iyp]),
                                 z > 0 ? v3(plm[c], plm[P + c], plm[2 * P + c]) : mp,
                                 z < nz - 1 ? v3(plp[c], plp[P + c], plp[2 * P + c]) : mp);
            const V3 mnew = heun_correct(L, mp, ex, u[j], hz1, hth[j], q[j]);
            const int me = e + 1;
            mn(me, 0) = mnew.x;
            mn(me, 1) = mnew.y;
            mn(me, 2) = mnew.z;
            msum += mnew.z;
            // boundary planes for the neighbours: slots 0, 1 = first two, 2, 3 = last two
            if (e <= 2) {
                float* d = xslot(par, sid, e - 1);
                st_agent(d + c, mnew.x);
                st_agent(d + P + c, mnew.y);
                st_agent(d + 2 * P + c, mnew.z);
            }
            if (e >= nzs - 1) {
                float* d = xslot(par, sid, 2 + (e - (nzs - 1)));
                st_agent(d + c, mnew.x);
                st_agent(d + P + c, mnew.y);
                st_agent(d + 2 * P + c, mnew.z);
            }
        }
        const double tot = block_sum<NT>(msum, red);   // contains a barrier
        if (tid == 0) partials[static_cast<int64_t>(sid) * pstride + st] = tot;
        // ---- 3. publish: every thread's exchange stores complete, then the flag
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            const uint32_t want = static_cast<uint32_t>(n + 1);
            __hip_atomic_store(&flags[sid], want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // ---- 4. wait for the z neighbours (bounded)
            for (int k = 0; k < 2; ++k) {
                const int nb = k == 0 ? S.prev : S.next;
                if (nb < 0) continue;
                uint32_t spins = 0;
                while (static_cast<int32_t>(__hip_atomic_load(&flags[nb], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) - want) < 0) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > (1u << 20)) {
                        s_abort = 1;
                        atomicOr(status, 2);
                        break;
                    }
                }
            }
        }
        __syncthreads();
        if (s_abort) return;
        // halo planes z0-2, z0-1 from the slab below; z0+nzs, z0+nzs+1 from above
        for (int h = r; h < 4; h += NPP) {
            if (!lane_on) break;
            const int me = h < 2 ? h : nzs + h;   // 0, 1, nzs+2, nzs+3
            const int z = z0 - 2 + me;
            if (z < 0 || z >= nz) continue;
            const float* s = h < 2 ? xslot(par, S.prev, 2 + h) : xslot(par, S.next, h - 2);
            mn(me, 0) = ld_agent(s + c);
            mn(me, 1) = ld_agent(s + P + c);
            mn(me, 2) = ld_agent(s + 2 * P + c);
        }
        __syncthreads();
    }
    // ---- write back own planes at step n0 + nsteps
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    for (int me = 2 + r; me < nzs + 2; me += NPP) {
        if (!lane_on) break;
        const int cell = c + P * (z0 - 2 + me);
        mo[cell] = mn(me, 0);
        mo[N + cell] = mn(me, 1);
        mo[2 * N + cell] = mn(me, 2);
    }
}

// Fold the per-step slab partials of one launch into the loops, one wave per
// instance: lanes sum the slabs of a step in a fixed order, lane 0 folds.
__global__ void k_fold_slabs(const InstDev* __restrict__ insts, int inst0, const int32_t* __restrict__ islab,
                             const LevelDev* __restrict__ levels,
                             const double* __restrict__ partials, int pstride, int64_t n0, int nsteps,
                             AccDev* __restrict__ accs, double* __restrict__ records, int* __restrict__ status)
{
    const int k = static_cast<int>(blockIdx.x);
    const int inst = inst0 + k;
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    const int s0 = islab[2 * k], ns = islab[2 * k + 1];   // level-relative first slab, count
    AccDev a;
    if (threadIdx.x == 0) a = accs[inst];
    for (int st = 0; st < nsteps; ++st) {
        double v = 0.0;
        for (int s = static_cast<int>(threadIdx.x); s < ns; s += 64)
            v += partials[static_cast<int64_t>(s0 + s) * pstride + st];
        v = wave_sum_d(v);
        if (threadIdx.x == 0) loop_accumulate(a, L, n0 + st, v / static_cast<double>(L.ncell), records + I.rec_off);
    }
    if (threadIdx.x == 0) {
        accs[inst] = a;
        if (!isfinite(a.m_prev)) atomicOr(status, 1);
    }
}

}  // namespace sllg
