// gfx950 kernels of the stochastic-LLG hysteresis-loop library.
//
//   k_init           every cell to +z, loop accumulators and record 0
//   k_axes           per-cell easy axes in a uniform cone (Philox, axis tag)
//   k_resident       LDS-resident persistent kernel: each workgroup owns whole
//                    instances (state double-buffered in LDS), runs many Heun
//                    steps per launch and reduces the loop every step
//   k_stream         one fused Heun step per launch over x-y tiles marching in
//                    z; the predictor is recomputed on a one-cell halo so that
//                    no intermediate leaves the workgroup
//   k_philox_probe   raw Philox words and normals for tests
//
// State in global memory is structure-of-arrays per instance (planes mx, my,
// mz of ncell floats); the state at step n lives in buffer n & 1.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

// ---------------------------------------------------------------------------
__global__ void k_init(const InstDev* __restrict__ insts, const LevelDev* __restrict__ levels,
                       int ninst, float* __restrict__ buf0, AccDev* __restrict__ accs,
                       double* __restrict__ records)
{
    const int inst = blockIdx.y;
    if (inst >= ninst) return;
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    float* m = buf0 + I.state_off;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < L.ncell; c += gridDim.x * blockDim.x) {
        m[c] = 0.0f;
        m[L.ncell + c] = 0.0f;
        m[2 * L.ncell + c] = 1.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        AccDev a{};
        a.m_prev = 1.0;
        accs[inst] = a;
        records[I.rec_off] = 1.0;
    }
}

__global__ void k_axes(const LevelDev* __restrict__ levels, int level, uint64_t axis_seed,
                       float one_minus_cos_max, float rx0, float rx1, float rx2, float ry0, float ry1,
                       float ry2, float rz0, float rz1, float rz2, float* __restrict__ axes)
{
    const LevelDev& L = levels[level];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= L.ncell) return;
    const U4 w = philox_cell(axis_seed, static_cast<uint32_t>(L.level_tag), kTagAxis,
                             static_cast<uint32_t>(c), 0);
    // 1 - cos(theta) is uniform on [0, 1 - cos(theta_max)]; sin from it without cancellation
    const float omc = unit_open(w.a) * one_minus_cos_max;
    const float ct = 1.0f - omc;
    const float st = sqrtf(omc * (2.0f - omc));
    const float ph = unit_open(w.b);
    const float vx = st * __builtin_amdgcn_cosf(ph), vy = st * __builtin_amdgcn_sinf(ph), vz = ct;
    // rows of the rotation taking +z to the level axis
    float* u = axes + L.axes_off;
    u[c] = fmaf(rx0, vx, fmaf(rx1, vy, rx2 * vz));
    u[L.ncell + c] = fmaf(ry0, vx, fmaf(ry1, vy, ry2 * vz));
    u[2 * L.ncell + c] = fmaf(rz0, vx, fmaf(rz1, vy, rz2 * vz));
}

__device__ __forceinline__ V3 load_axis(const LevelDev& L, const float* __restrict__ axes, int c)
{
    if (!L.has_axes) return V3{L.ux, L.uy, L.uz};
    const float* u = axes + L.axes_off;
    return V3{u[c], u[L.ncell + c], u[2 * L.ncell + c]};
}

// ---------------------------------------------------------------------------
// Resident plan.
//
// LDS holds two array-of-structs copies of the workgroup's state (A = m_n,
// B = m'), 12 bytes per cell each, the chunk sums of m_z of even and odd
// steps, the loop accumulators of the slots and a ring of applied fields per
// slot.  A wave owns up to CPW chunks of 64 consecutive cells of one instance
// (chunk j of the workgroup belongs to wave j % NW).  Per step: predictor
// A -> B, barrier, corrector B -> A with a wave sum of m_z per chunk,
// barrier.  One thread per slot, in the last wave, folds a step's chunk sums
// (FP64, fixed order) into the loop during the next step and computes the
// applied field two steps ahead, so this work is off the critical path when
// the last wave owns fewer chunks than the others (the planner leaves it
// without chunks where it can).  Everything that does not change with the
// step (the level, seed and cell of each owned chunk, the LDS offsets of the
// cell and its neighbours, the easy axis, the slot data of the folding
// thread) is loaded once before the step loop, and checkpoints are found by
// a countdown, so a step has no global loads, no FP64 and no integer
// division on the critical path of the waves that own cells.
// ---------------------------------------------------------------------------
// With NW <= 8 the workgroup has NW more waves: wave NW + w draws the
// thermal field of step n + 1 for the cells of wave w into an LDS buffer
// (two step parities) while the cell waves predict step n, so Philox and
// Box-Muller leave the cell waves' chain.
template <int NW>
constexpr bool kNoiseWaves = NW <= 8;
template <int NW>
constexpr int kResThreads = (kNoiseWaves<NW> ? 2 : 1) * NW * 64;

template <int NW, int CPW>
__global__ __launch_bounds__(kResThreads<NW>) void k_resident(
    const GroupDev* __restrict__ groups, const SlotDev* __restrict__ slots,
    const ChunkDev* __restrict__ chunks, const InstDev* __restrict__ insts,
    const LevelDev* __restrict__ levels, float* __restrict__ buf0, float* __restrict__ buf1,
    const float* __restrict__ axes, double* __restrict__ records, AccDev* __restrict__ accs,
    float* __restrict__ ckpt, int ckpt_every, int64_t n0, int64_t nsteps, int* __restrict__ status)
{
    extern __shared__ float lds[];
    const GroupDev G = groups[blockIdx.x];
    constexpr bool NP = kNoiseWaves<NW>;
    float* A = lds;
    float* B = lds + 3 * G.ncells;
    // thermal field of even and odd steps (noise waves only)
    float* T = B + 3 * G.ncells;
    // chunk sums of even and odd steps
    const int pstride = (G.nchunks + 3) & ~3;
    float* part = T + (NP ? 6 * G.ncells : 0);
    AccDev* acc = reinterpret_cast<AccDev*>(part + 2 * pstride + 4);
    // applied field (FP32) per slot for steps n + 1 .. n + 2, a ring of four
    float* s_hz = reinterpret_cast<float*>(acc + G.nslots);

    const int lane = threadIdx.x & 63;
    const int w_id = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool noise_wave = NP && w_id >= NW;
    const int wave = noise_wave ? w_id - NW : w_id;   // the cell wave whose chunks this wave serves

    // ---- per owned chunk: step-invariant data
    const LevelDev* Lk[CPW];   // wave-uniform
    int slot[CPW];             // wave-uniform
    uint64_t seed[CPW];        // wave-uniform
    int64_t ck_off[CPW];       // wave-uniform: float offset of the instance's checkpoint 0
    bool has[CPW];             // wave-uniform: the chunk exists
    // per lane: the cell index, and the float offset of the cell in A / B
    // (bits 0-15) with the existing neighbours (bits 16-21: x-1, x+1, y-1,
    // y+1, z-1, z+1) and a valid flag (bit 31)
    int cell[CPW];
    uint32_t pk[CPW];
    V3 u[CPW];
    // the step constants of each chunk's level, held in vector registers
    LevelDev Lc[CPW];
    int sy[CPW], sz[CPW];
    const float* min_ = (n0 & 1) ? buf1 : buf0;
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        const int j = wave + k * NW;
        has[k] = j < G.nchunks;
        Lk[k] = levels;
        slot[k] = 0;
        seed[k] = 0;
        ck_off[k] = 0;
        cell[k] = 0;
        pk[k] = 0u;
        u[k] = V3{0.0f, 0.0f, 1.0f};
        Lc[k] = LevelDev{};
        sy[k] = sz[k] = 0;
        if (!has[k]) continue;
        const ChunkDev ch = chunks[G.chunk0 + j];
        const InstDev I = insts[ch.inst];
        const LevelDev& L = levels[I.level];
        const SlotDev S = slots[G.slot0 + ch.slot];
        Lk[k] = &levels[I.level];
        // (with two chunks per wave the registers are needed elsewhere)
        auto keep = [](float x) { return CPW == 1 ? vreg(x) : x; };
        Lc[k].c_ex = keep(L.c_ex);
        Lc[k].hk = keep(L.hk);
        Lc[k].g1 = keep(L.g1);
        Lc[k].ag1 = keep(L.ag1);
        Lc[k].dt = keep(L.dt);
        Lc[k].half_dt = keep(L.half_dt);
        sy[k] = __float_as_int(keep(__int_as_float(3 * L.nx)));
        sz[k] = __float_as_int(keep(__int_as_float(3 * L.nx * L.ny)));
        slot[k] = ch.slot;
        seed[k] = I.seed;
        ck_off[k] = I.ckpt_off;
        const int c = ch.c0 + lane;
        if (c >= L.ncell) continue;
        cell[k] = c;
        const int x = c % L.nx, y = (c / L.nx) % L.ny, z = c / (L.nx * L.ny);
        const int own = 3 * (S.lds_off + c);
        pk[k] = static_cast<uint32_t>(own) | (x > 0 ? 1u << 16 : 0u) | (x < L.nx - 1 ? 1u << 17 : 0u) |
                (y > 0 ? 1u << 18 : 0u) | (y < L.ny - 1 ? 1u << 19 : 0u) | (z > 0 ? 1u << 20 : 0u) |
                (z < L.nz - 1 ? 1u << 21 : 0u) | 0x80000000u;
        if (noise_wave) {
            // the thermal field of the first step
            const V3 h = thermal_field(L, seed[k], static_cast<uint32_t>(c), n0);
            float* t = T + (n0 & 1) * 3 * G.ncells + own;
            t[0] = h.x;
            t[1] = h.y;
            t[2] = h.z;
            continue;
        }
        u[k] = load_axis(L, axes, c);
        const float* src = min_ + I.state_off;
        A[own] = src[c];
        A[own + 1] = src[L.ncell + c];
        A[own + 2] = src[2 * L.ncell + c];
    }
    // neighbour sum over the six face neighbours read from an AoS LDS copy
    auto stencil = [&](const float* M, uint32_t p, int sy, int sz, V3 m) {
        const int o = static_cast<int>(p & 0xFFFFu);
        auto at = [&](int i) { return v3(M[i], M[i + 1], M[i + 2]); };
        return nb_sum(m, at((p & (1u << 16)) ? o - 3 : o), at((p & (1u << 17)) ? o + 3 : o),
                      at((p & (1u << 18)) ? o - sy : o), at((p & (1u << 19)) ? o + sy : o),
                      at((p & (1u << 20)) ? o - sz : o), at((p & (1u << 21)) ? o + sz : o));
    };

    // ---- the folding thread of each slot, in the last wave (a group has at
    // most NW * CPW <= 64 chunks, so at most one slot per thread)
    const int fs = static_cast<int>(threadIdx.x) - (NW - 1) * 64;
    const bool folder = fs >= 0 && fs < G.nslots;
    // the folding thread's level by value: the fields the fold reads stay in
    // registers (a per-thread pointer would be a vector load every step)
    LevelDev Lf{};
    int f_chunk0 = 0, f_nchunks = 0;
    double f_inv_ncell = 0.0;
    double H0 = 0.0, H1 = 0.0, H2 = 0.0;   // applied field (Oe) at steps n - 1, n, n + 1 of step n
    double* f_rec = records;
    int f_inst = 0;
    if (folder) {
        const SlotDev S = slots[G.slot0 + fs];
        const InstDev I = insts[S.inst];
        Lf = levels[I.level];
        f_inst = S.inst;
        f_chunk0 = S.chunk0;
        f_nchunks = S.nchunks;
        f_inv_ncell = 1.0 / static_cast<double>(Lf.ncell);
        f_rec = records + I.rec_off;
        H1 = Lf.hz_oe * wave_at(Lf, n0);
        const double w = wave_at(Lf, n0 + 1);
        H2 = Lf.hz_oe * w;
        s_hz[4 * fs + ((n0 + 1) & 3)] = static_cast<float>(Lf.hz_amp * w);
        acc[fs] = accs[S.inst];
    }
    // the folding thread's accumulators: in registers when the workgroup has
    // at most 512 threads, else in LDS
    constexpr bool kAccReg = CPW == 1 && kResThreads<NW> <= 512;
    AccDev a_reg{};
    if (kAccReg && folder) a_reg = acc[fs];
    AccDev& a = [&]() -> AccDev& {
        if constexpr (kAccReg) return a_reg;
        else return acc[fs];
    }();
    // The folding thread splits its work over the two phases of step n:
    // while the other waves predict, the loop ordinate of step n (from the
    // chunk sums of step n - 1, in a fixed order) and the applied field of
    // step n + 2 for the correctors of step n + 1; while they correct, the
    // FP64 loop update of step n - 1 -> n.  H0, H1, H2 hold the applied field
    // (Oe) at steps n - 1, n, n + 1.
    double m_fold = 0.0, H3 = 0.0;
    auto ordinate = [&](int64_t m) {
        const float* p = part + (m & 1) * pstride + f_chunk0;
        double sum = 0.0;
        for (int j = 0; j < f_nchunks; ++j) sum += static_cast<double>(p[j]);
        m_fold = sum * f_inv_ncell;
    };
    auto field_ahead = [&](int64_t n) {
        const double w = wave_at(Lf, n + 2);
        s_hz[4 * fs + ((n + 2) & 3)] = static_cast<float>(Lf.hz_amp * w);
        H3 = Lf.hz_oe * w;
    };

    // applied field (FP32) at the current step of each owned chunk
    float hz[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k)
        hz[k] = has[k] ? static_cast<float>(Lk[k]->hz_amp * wave_at(*Lk[k], n0)) : 0.0f;
    // next checkpointed step (a multiple of ckpt_every) and its index
    const bool do_ckpt = ckpt != nullptr && ckpt_every > 0;
    int64_t ck_idx = do_ckpt ? (n0 + ckpt_every - 1) / ckpt_every : 0;
    int64_t ck_next = do_ckpt ? ck_idx * ckpt_every : -1;
    __syncthreads();

    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        const bool ck_now = n == ck_next;
        V3 q[CPW], hth[CPW];
        // ---- loop ordinate of the previous step, field ahead
        if (folder) {
            if (st > 0) ordinate(n - 1);
            field_ahead(n);
        }
        // ---- noise waves: the thermal field of step n + 1 (the buffer of
        //      that parity was last read by the predictor of step n - 1)
        if (noise_wave && st + 1 < nsteps) {
#pragma unroll
            for (int k = 0; k < CPW; ++k) {
                if (!has[k] || !(pk[k] & 0x80000000u)) continue;
                const V3 h = thermal_field(*Lk[k], seed[k], static_cast<uint32_t>(cell[k]), n + 1);
                float* t = T + ((n + 1) & 1) * 3 * G.ncells + static_cast<int>(pk[k] & 0xFFFFu);
                t[0] = h.x;
                t[1] = h.y;
                t[2] = h.z;
            }
        }
        // ---- predictor: A -> B
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            q[k] = hth[k] = V3{0.0f, 0.0f, 0.0f};
            if (noise_wave || !has[k] || !(pk[k] & 0x80000000u)) continue;
            const int own = static_cast<int>(pk[k] & 0xFFFFu);
            const V3 m = v3(A[own], A[own + 1], A[own + 2]);
            if (ck_now) {
                const int N = Lk[k]->ncell;
                float* cp = ckpt + ck_off[k] + ck_idx * 3 * N;
                cp[cell[k]] = m.x;
                cp[N + cell[k]] = m.y;
                cp[2 * N + cell[k]] = m.z;
            }
            const V3 ex = stencil(A, pk[k], sy[k], sz[k], m);
            if (NP) {
                const float* t = T + (n & 1) * 3 * G.ncells + own;
                hth[k] = v3(t[0], t[1], t[2]);
            } else {
                hth[k] = thermal_field(*Lk[k], seed[k], static_cast<uint32_t>(cell[k]), n);
            }
            V3 mp;
            heun_predict(Lc[k], m, ex, u[k], hz[k], hth[k], mp, q[k]);
            B[own] = mp.x;
            B[own + 1] = mp.y;
            B[own + 2] = mp.z;
        }
        __syncthreads();
        // ---- loop update of the previous step
        if (folder) {
            if (st > 0) loop_accumulate_h(a, Lf, H0, H1, m_fold, f_rec);
            H0 = H1;
            H1 = H2;
            H2 = H3;
        }
        // ---- corrector: B -> A, wave sums of m_z per chunk
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            if (noise_wave || !has[k]) continue;
            const float hz1 = s_hz[4 * slot[k] + ((n + 1) & 3)];
            float mz = 0.0f;
            if (pk[k] & 0x80000000u) {
                const int own = static_cast<int>(pk[k] & 0xFFFFu);
                const V3 mp = v3(B[own], B[own + 1], B[own + 2]);
                const V3 ex = stencil(B, pk[k], sy[k], sz[k], mp);
                const V3 mn = heun_correct(Lc[k], mp, ex, u[k], hz1, hth[k], q[k]);
                A[own] = mn.x;
                A[own + 1] = mn.y;
                A[own + 2] = mn.z;
                mz = mn.z;
            }
            hz[k] = hz1;
            const float ps = wave_sum(mz);
            if (lane == 0) part[(n & 1) * pstride + wave + k * NW] = ps;
        }
        __syncthreads();
        if (ck_now) {
            ck_next += ckpt_every;
            ++ck_idx;
        }
        // the next predictor only reads A, the next corrector writes A after a barrier
    }
    if (folder && nsteps > 0) {
        ordinate(n0 + nsteps - 1);
        loop_accumulate_h(a, Lf, H0, H1, m_fold, f_rec);
    }
    __syncthreads();
    // write back state (buffer (n0 + nsteps) & 1) and accumulators
    float* mout = ((n0 + nsteps) & 1) ? buf1 : buf0;
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        if (noise_wave || !has[k] || !(pk[k] & 0x80000000u)) continue;
        const int j = wave + k * NW;
        const ChunkDev ch = chunks[G.chunk0 + j];
        const int N = Lk[k]->ncell;
        const int own = static_cast<int>(pk[k] & 0xFFFFu);
        float* d = mout + insts[ch.inst].state_off;
        d[cell[k]] = A[own];
        d[N + cell[k]] = A[own + 1];
        d[2 * N + cell[k]] = A[own + 2];
    }
    if (folder) {
        accs[f_inst] = a;
        if (!isfinite(a.m_prev)) atomicOr(status, 1);
    }
}

// ---------------------------------------------------------------------------
// Stream plan: one Heun step per launch.
//
// A workgroup of TX*TY*PZ threads owns an x-y window (at most TX x TY cells)
// of one instance and a z range, and marches through it PZ planes at a time.
// LDS rings hold m_n on the window plus a two-cell x-y border (predictor
// neighbours), m' on the window plus a one-cell border (corrector
// neighbours) and q, H_th of the window cells.  The predictor runs on the
// window, on its one-cell x-y ring and on one plane above and below, so the
// corrector needs nothing from other workgroups.  Each workgroup writes an
// FP64 partial of sum m_z; the last workgroup of an instance folds the
// partials in tile order into the loop, and the last workgroup of the launch
// advances the step counters.
// ---------------------------------------------------------------------------
template <int TX, int TY, int PZ>
__global__ __launch_bounds__(TX* TY* PZ) void k_stream(
    const TileDev* __restrict__ tiles, const InstDev* __restrict__ insts,
    const LevelDev* __restrict__ levels, float* __restrict__ buf0, float* __restrict__ buf1,
    const float* __restrict__ axes, int64_t* __restrict__ steps, int tile_base, int ptiles,
    double* __restrict__ partials, uint32_t* __restrict__ pend, uint32_t* __restrict__ launch_cnt,
    double* __restrict__ records, AccDev* __restrict__ accs, float* __restrict__ ckpt, int ckpt_every,
    int* __restrict__ status)
{
    constexpr int NT = TX * TY * PZ;
    constexpr int TXY = TX * TY;
    constexpr int R2W = TX + 4, R2 = (TX + 4) * (TY + 4);
    constexpr int R1W = TX + 2, R1 = (TX + 2) * (TY + 2);
    constexpr int NS = PZ + 2, NQ = PZ + 1;
    __shared__ float Mn[NS][3][R2];
    __shared__ float Mp[NS][3][R1];
    __shared__ float QH[NQ][6][TXY];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const int tile = tile_base + static_cast<int>(blockIdx.x);
    const TileDev T = tiles[tile];
    const InstDev I = insts[T.inst];
    const LevelDev L = levels[I.level];
    const int64_t n = steps[I.level];
    const bool first_tile = tile == I.tile0;
    if (first_tile && pend[T.inst]) {
        fold_partials(I, L, n - 1, partials, ptiles, accs, T.inst, records, status);
        if (tid == 0) pend[T.inst] = 0u;
    }

    if (n < L.n_steps) {
        const float* __restrict__ mi = ((n & 1) ? buf1 : buf0) + I.state_off;
        float* __restrict__ mo = ((n & 1) ? buf0 : buf1) + I.state_off;
        const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.ncell;
        const int x0 = T.x0, y0 = T.y0, z0 = T.z0, nxt = T.nxt, nyt = T.nyt;
        const int zc_end = z0 + T.nzt;
        const int pz0 = max(z0 - 1, 0), pz1 = min(zc_end, nz - 1);
        const int tx = tid % TX, ty = (tid / TX) % TY, dz = tid / TXY;
        const bool inside = tx < nxt && ty < nyt;
        const int gx = x0 + tx, gy = y0 + ty;
        const float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n));
        const float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
        const bool ring = (x0 > 0) || (x0 + nxt < nx) || (y0 > 0) || (y0 + nyt < ny);
        const int nring = ring ? 2 * (nxt + 2) + 2 * nyt : 0;
        const bool do_ckpt = (ckpt != nullptr) && ckpt_every > 0 && (n % ckpt_every) == 0;

        auto load_plane = [&](int z) {
            const int s = z % NS;
            for (int idx = tid; idx < R2; idx += NT) {
                const int lx = idx % R2W, ly = idx / R2W;
                const int x = x0 - 2 + lx, y = y0 - 2 + ly;
                if (x >= 0 && x < nx && y >= 0 && y < ny) {
                    const int c = x + nx * (y + ny * z);
                    Mn[s][0][idx] = mi[c];
                    Mn[s][1][idx] = mi[N + c];
                    Mn[s][2][idx] = mi[2 * N + c];
                }
            }
        };

        // predictor for grid cell (x, y, z) inside R1; returns m', q, H_th
        auto predict = [&](int x, int y, int z, V3& mp, V3& q, V3& hth) {
            const int i2 = (y - y0 + 2) * R2W + (x - x0 + 2);
            const int s = z % NS;
            const int sm = (z > 0 ? z - 1 : z) % NS, sp = (z < nz - 1 ? z + 1 : z) % NS;
            const int ixm = x > 0 ? i2 - 1 : i2, ixp = x < nx - 1 ? i2 + 1 : i2;
            const int iym = y > 0 ? i2 - R2W : i2, iyp = y < ny - 1 ? i2 + R2W : i2;
            const V3 m = v3(Mn[s][0][i2], Mn[s][1][i2], Mn[s][2][i2]);
            const V3 ex = nb_sum(m, v3(Mn[s][0][ixm], Mn[s][1][ixm], Mn[s][2][ixm]),
                                 v3(Mn[s][0][ixp], Mn[s][1][ixp], Mn[s][2][ixp]),
                                 v3(Mn[s][0][iym], Mn[s][1][iym], Mn[s][2][iym]),
                                 v3(Mn[s][0][iyp], Mn[s][1][iyp], Mn[s][2][iyp]),
                                 v3(Mn[sm][0][i2], Mn[sm][1][i2], Mn[sm][2][i2]),
                                 v3(Mn[sp][0][i2], Mn[sp][1][i2], Mn[sp][2][i2]));
            const int c = x + nx * (y + ny * z);
            hth = thermal_field(L, I.seed, static_cast<uint32_t>(c), n);
            heun_predict(L, m, ex, load_axis(L, axes, c), hz0, hth, mp, q);
        };

        if (pz0 - 1 >= 0) load_plane(pz0 - 1);
        load_plane(pz0);
        float msum = 0.0f;
        const int zload_max = min(pz1 + 1, nz - 1);
        for (int p = pz0; p <= zc_end; p += PZ) {
            for (int z = p + 1; z <= p + PZ && z <= zload_max; ++z) load_plane(z);
            __syncthreads();
            // predictor on the window cells of planes p .. p+PZ-1
            const int pp = p + dz;
            if (pp <= pz1 && inside) {
                V3 mp, q, hth;
                predict(gx, gy, pp, mp, q, hth);
                const int i1 = (ty + 1) * R1W + (tx + 1);
                const int s = pp % NS;
                Mp[s][0][i1] = mp.x;
                Mp[s][1][i1] = mp.y;
                Mp[s][2][i1] = mp.z;
                if (pp >= z0 && pp < zc_end) {
                    const int sq = pp % NQ, t = tx + TX * ty;
                    QH[sq][0][t] = q.x;
                    QH[sq][1][t] = q.y;
                    QH[sq][2][t] = q.z;
                    QH[sq][3][t] = hth.x;
                    QH[sq][4][t] = hth.y;
                    QH[sq][5][t] = hth.z;
                }
            }
            // predictor on the one-cell x-y ring of the window planes
            for (int item = tid; item < nring * PZ; item += NT) {
                const int pr = p + item / nring;
                if (pr > pz1 || pr < z0 || pr >= zc_end) continue;
                int r = item % nring, x, y;
                if (r < nxt + 2) {
                    x = x0 - 1 + r;
                    y = y0 - 1;
                } else if ((r -= nxt + 2) < nxt + 2) {
                    x = x0 - 1 + r;
                    y = y0 + nyt;
                } else if ((r -= nxt + 2) < nyt) {
                    x = x0 - 1;
                    y = y0 + r;
                } else {
                    x = x0 + nxt;
                    y = y0 + (r - nyt);
                }
                if (x < 0 || x >= nx || y < 0 || y >= ny) continue;
                V3 mp, q, hth;
                predict(x, y, pr, mp, q, hth);
                const int i1 = (y - y0 + 1) * R1W + (x - x0 + 1);
                const int s = pr % NS;
                Mp[s][0][i1] = mp.x;
                Mp[s][1][i1] = mp.y;
                Mp[s][2][i1] = mp.z;
            }
            __syncthreads();
            // corrector on planes p-1 .. p+PZ-2
            const int c = p - 1 + dz;
            if (c >= z0 && c < zc_end && inside) {
                const int i1 = (ty + 1) * R1W + (tx + 1);
                const int s = c % NS;
                const int sm = (c > 0 ? c - 1 : c) % NS, sp = (c < nz - 1 ? c + 1 : c) % NS;
                const int ixm = gx > 0 ? i1 - 1 : i1, ixp = gx < nx - 1 ? i1 + 1 : i1;
                const int iym = gy > 0 ? i1 - R1W : i1, iyp = gy < ny - 1 ? i1 + R1W : i1;
                const V3 mp = v3(Mp[s][0][i1], Mp[s][1][i1], Mp[s][2][i1]);
                const V3 ex = nb_sum(mp, v3(Mp[s][0][ixm], Mp[s][1][ixm], Mp[s][2][ixm]),
                                     v3(Mp[s][0][ixp], Mp[s][1][ixp], Mp[s][2][ixp]),
                                     v3(Mp[s][0][iym], Mp[s][1][iym], Mp[s][2][iym]),
                                     v3(Mp[s][0][iyp], Mp[s][1][iyp], Mp[s][2][iyp]),
                                     v3(Mp[sm][0][i1], Mp[sm][1][i1], Mp[sm][2][i1]),
                                     v3(Mp[sp][0][i1], Mp[sp][1][i1], Mp[sp][2][i1]));
                const int sq = c % NQ, t = tx + TX * ty;
                const V3 q = v3(QH[sq][0][t], QH[sq][1][t], QH[sq][2][t]);
                const V3 hth = v3(QH[sq][3][t], QH[sq][4][t], QH[sq][5][t]);
                const int cell = gx + nx * (gy + ny * c);
                const V3 mn = heun_correct(L, mp, ex, load_axis(L, axes, cell), hz1, hth, q);
                mo[cell] = mn.x;
                mo[N + cell] = mn.y;
                mo[2 * N + cell] = mn.z;
                msum += mn.z;
                if (do_ckpt) {
                    const int i2 = (ty + 2) * R2W + (tx + 2);
                    float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * N;
                    cp[cell] = Mn[c % NS][0][i2];
                    cp[N + cell] = Mn[c % NS][1][i2];
                    cp[2 * N + cell] = Mn[c % NS][2][i2];
                }
            }
        }
        const double tot = block_sum<TX * TY * PZ>(msum, red);
        stream_block_end(tot, n, tile, ptiles, partials, first_tile, pend, T.inst, launch_cnt, steps, I.level,
                         L.n_steps);
    }
}

// Fold the last pending step of every instance of a stream-plan level.
__global__ void k_flush(const InstDev* __restrict__ insts, int inst0, const LevelDev* __restrict__ levels,
                        const int64_t* __restrict__ steps, const double* __restrict__ partials, int ptiles,
                        uint32_t* __restrict__ pend, AccDev* __restrict__ accs, double* __restrict__ records,
                        int* __restrict__ status)
{
    const int inst = inst0 + static_cast<int>(blockIdx.x);
    const InstDev I = insts[inst];
    if (!pend[inst]) return;
    const LevelDev& L = levels[I.level];
    fold_partials(I, L, steps[I.level] - 1, partials, ptiles, accs, inst, records, status);
    if (threadIdx.x == 0) pend[inst] = 0u;
}

// ---------------------------------------------------------------------------
__global__ void k_philox_probe(uint64_t seed, uint32_t level, uint32_t tag,
                               const uint32_t* __restrict__ cells, const uint64_t* __restrict__ steps,
                               int n, uint32_t* __restrict__ raw, float* __restrict__ normals)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const U4 w = philox_cell(seed, level, tag, cells[k], steps[k]);
    raw[4 * k] = w.a;
    raw[4 * k + 1] = w.b;
    raw[4 * k + 2] = w.c;
    raw[4 * k + 3] = w.d;
    const V3 g = gauss3(w);
    normals[3 * k] = g.x;
    normals[3 * k + 1] = g.y;
    normals[3 * k + 2] = g.z;
}

}  // namespace sllg
