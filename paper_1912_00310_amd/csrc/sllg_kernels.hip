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
// B = m'), 12 bytes per cell each, followed by one float per chunk for the
// loop reduction and the slots' loop accumulators.  A wave owns up to CPW
// chunks of 64 consecutive cells of one instance (chunk j of the workgroup
// belongs to wave j % NW).  Per step: predictor A -> B, barrier, corrector
// B -> A with a wave sum of m_z per chunk, barrier, one thread per slot folds
// the chunk sums (FP64, fixed order) into the loop.
// ---------------------------------------------------------------------------
template <int NW, int CPW>
__global__ __launch_bounds__(NW * 64) void k_resident(
    const GroupDev* __restrict__ groups, const SlotDev* __restrict__ slots,
    const ChunkDev* __restrict__ chunks, const InstDev* __restrict__ insts,
    const LevelDev* __restrict__ levels, float* __restrict__ buf0, float* __restrict__ buf1,
    const float* __restrict__ axes, double* __restrict__ records, AccDev* __restrict__ accs,
    float* __restrict__ ckpt, int ckpt_every, int64_t n0, int64_t nsteps, int* __restrict__ status)
{
    extern __shared__ float lds[];
    const GroupDev G = groups[blockIdx.x];
    float* A = lds;
    float* B = lds + 3 * G.ncells;
    float* part = B + 3 * G.ncells;
    AccDev* acc = reinterpret_cast<AccDev*>(part + ((G.nchunks + 3) & ~3) + 4);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // packed lane coordinates per owned chunk: x | y << 10 | z << 20 | valid << 31
    uint32_t info[CPW];
    const float* min_ = (n0 & 1) ? buf1 : buf0;
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        info[k] = 0u;
        const int j = wave + k * NW;
        if (j < G.nchunks) {
            const ChunkDev ch = chunks[G.chunk0 + j];
            const LevelDev& L = levels[insts[ch.inst].level];
            const int c = ch.c0 + lane;
            if (c < L.ncell) {
                const int x = c % L.nx, y = (c / L.nx) % L.ny, z = c / (L.nx * L.ny);
                info[k] = static_cast<uint32_t>(x) | (static_cast<uint32_t>(y) << 10) |
                          (static_cast<uint32_t>(z) << 20) | 0x80000000u;
                const SlotDev S = slots[G.slot0 + ch.slot];
                const float* src = min_ + insts[ch.inst].state_off;
                float* d = A + 3 * (S.lds_off + c);
                d[0] = src[c];
                d[1] = src[L.ncell + c];
                d[2] = src[2 * L.ncell + c];
            }
        }
    }
    for (int s = threadIdx.x; s < G.nslots; s += blockDim.x) acc[s] = accs[slots[G.slot0 + s].inst];
    __syncthreads();

    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        V3 q[CPW], hth[CPW];
        // ---- predictor: A -> B
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            const int j = wave + k * NW;
            if (j >= G.nchunks) continue;
            const ChunkDev ch = chunks[G.chunk0 + j];
            const InstDev I = insts[ch.inst];
            const LevelDev& L = levels[I.level];
            const SlotDev S = slots[G.slot0 + ch.slot];
            if (!(info[k] & 0x80000000u)) continue;
            const int c = ch.c0 + lane;
            const int x = info[k] & 1023, y = (info[k] >> 10) & 1023, z = (info[k] >> 20) & 1023;
            const int sy = L.nx, sz = L.nx * L.ny;
            const float* a = A + 3 * S.lds_off;
            const int ixm = (x > 0) ? c - 1 : c, ixp = (x < L.nx - 1) ? c + 1 : c;
            const int iym = (y > 0) ? c - sy : c, iyp = (y < L.ny - 1) ? c + sy : c;
            const int izm = (z > 0) ? c - sz : c, izp = (z < L.nz - 1) ? c + sz : c;
            const V3 m = v3(a[3 * c], a[3 * c + 1], a[3 * c + 2]);
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * L.ncell;
                cp[c] = m.x;
                cp[L.ncell + c] = m.y;
                cp[2 * L.ncell + c] = m.z;
            }
            const V3 ex = nb_sum(m, v3(a[3 * ixm], a[3 * ixm + 1], a[3 * ixm + 2]),
                                 v3(a[3 * ixp], a[3 * ixp + 1], a[3 * ixp + 2]),
                                 v3(a[3 * iym], a[3 * iym + 1], a[3 * iym + 2]),
                                 v3(a[3 * iyp], a[3 * iyp + 1], a[3 * iyp + 2]),
                                 v3(a[3 * izm], a[3 * izm + 1], a[3 * izm + 2]),
                                 v3(a[3 * izp], a[3 * izp + 1], a[3 * izp + 2]));
            const float hz = static_cast<float>(L.hz_amp * wave_at(L, n));
            hth[k] = thermal_field(L, I.seed, static_cast<uint32_t>(c), n);
            V3 mp;
            heun_predict(L, m, ex, load_axis(L, axes, c), hz, hth[k], mp, q[k]);
            float* b = B + 3 * (S.lds_off + c);
            b[0] = mp.x;
            b[1] = mp.y;
            b[2] = mp.z;
        }
        __syncthreads();
        // ---- corrector: B -> A, wave sums of m_z per chunk
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            const int j = wave + k * NW;
            if (j >= G.nchunks) continue;
            const ChunkDev ch = chunks[G.chunk0 + j];
            const InstDev I = insts[ch.inst];
            const LevelDev& L = levels[I.level];
            const SlotDev S = slots[G.slot0 + ch.slot];
            float mz = 0.0f;
            if (info[k] & 0x80000000u) {
                const int c = ch.c0 + lane;
                const int x = info[k] & 1023, y = (info[k] >> 10) & 1023, z = (info[k] >> 20) & 1023;
                const int sy = L.nx, sz = L.nx * L.ny;
                const float* b = B + 3 * S.lds_off;
                const int ixm = (x > 0) ? c - 1 : c, ixp = (x < L.nx - 1) ? c + 1 : c;
                const int iym = (y > 0) ? c - sy : c, iyp = (y < L.ny - 1) ? c + sy : c;
                const int izm = (z > 0) ? c - sz : c, izp = (z < L.nz - 1) ? c + sz : c;
                const V3 mp = v3(b[3 * c], b[3 * c + 1], b[3 * c + 2]);
                const V3 ex = nb_sum(mp, v3(b[3 * ixm], b[3 * ixm + 1], b[3 * ixm + 2]),
                                     v3(b[3 * ixp], b[3 * ixp + 1], b[3 * ixp + 2]),
                                     v3(b[3 * iym], b[3 * iym + 1], b[3 * iym + 2]),
                                     v3(b[3 * iyp], b[3 * iyp + 1], b[3 * iyp + 2]),
                                     v3(b[3 * izm], b[3 * izm + 1], b[3 * izm + 2]),
                                     v3(b[3 * izp], b[3 * izp + 1], b[3 * izp + 2]));
                const float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
                const V3 mn = heun_correct(L, mp, ex, load_axis(L, axes, c), hz1, hth[k], q[k]);
                float* a = A + 3 * (S.lds_off + c);
                a[0] = mn.x;
                a[1] = mn.y;
                a[2] = mn.z;
                mz = mn.z;
            }
            const float ps = wave_sum(mz);
            if (lane == 0) part[j] = ps;
        }
        __syncthreads();
        // ---- loop reduction, one thread per slot, fixed order
        for (int s = threadIdx.x; s < G.nslots; s += blockDim.x) {
            const SlotDev S = slots[G.slot0 + s];
            const InstDev I = insts[S.inst];
            const LevelDev& L = levels[I.level];
            double sum = 0.0;
            for (int j = 0; j < S.nchunks; ++j) sum += static_cast<double>(part[S.chunk0 + j]);
            loop_accumulate(acc[s], L, n, sum / static_cast<double>(L.ncell), records + I.rec_off);
        }
        // the next predictor only reads A, the next corrector writes A after a barrier
    }
    __syncthreads();
    // write back state (buffer (n0 + nsteps) & 1) and accumulators
    float* mout = ((n0 + nsteps) & 1) ? buf1 : buf0;
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        const int j = wave + k * NW;
        if (j >= G.nchunks) continue;
        const ChunkDev ch = chunks[G.chunk0 + j];
        const LevelDev& L = levels[insts[ch.inst].level];
        const SlotDev S = slots[G.slot0 + ch.slot];
        if (!(info[k] & 0x80000000u)) continue;
        const int c = ch.c0 + lane;
        const float* a = A + 3 * (S.lds_off + c);
        float* d = mout + insts[ch.inst].state_off;
        d[c] = a[0];
        d[L.ncell + c] = a[1];
        d[2 * L.ncell + c] = a[2];
    }
    for (int s = threadIdx.x; s < G.nslots; s += blockDim.x) {
        const AccDev a = acc[s];
        accs[slots[G.slot0 + s].inst] = a;
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
