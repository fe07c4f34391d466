// Streamed Heun step over full-width tiles (one launch per step).
//
// A workgroup of NT threads owns the rows [y0, y0 + ny_t) of every x of one
// instance over the z range [z0, z0 + nz_t).  Threads form TR = NT / nx rows
// of nx lanes; thread (x, r) owns the cells (x, py0 + r + j*TR), j < K, of
// the predicted rows [py0, py1) = the window plus one ring row on each side
// that is inside the grid.  The workgroup marches in z with m_n of planes
// p-1, p, p+1 in an LDS ring; at plane p it
//   1. predicts plane p (neighbours from the ring, noise in registers),
//   2. corrects plane p - 1 (x-y neighbours of m' from LDS, z neighbours from
//      the thread's own m' of planes p - 2 and p in registers), storing m_{n+1},
//   3. publishes m'(p) and stores the prefetched plane p + 2 in the ring slot
//      of plane p - 1, between two barriers,
// while the global loads of plane p + 3 are in flight.  Every predicted cell
// costs one thread slot, so the recomputed ring rows are spread evenly over
// the waves.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

// Barrier for LDS traffic only: waits for this wave's LDS operations, not for
// its global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int NT, int K>
__global__ __launch_bounds__(NT) void k_rows(
    const TileDev* __restrict__ tiles, const InstDev* __restrict__ insts,
    const LevelDev* __restrict__ levels, float* __restrict__ buf0, float* __restrict__ buf1,
    const float* __restrict__ axes, int64_t* __restrict__ steps, int tile_base, int ptiles,
    double* __restrict__ partials, uint32_t* __restrict__ pend, uint32_t* __restrict__ launch_cnt,
    double* __restrict__ records, AccDev* __restrict__ accs, float* __restrict__ ckpt, int ckpt_every,
    int* __restrict__ status)
{
    // LDS: a ring of three planes of m_n (predicted rows plus one row above and
    // below) and one plane of m' (predicted rows); structure of arrays.
    constexpr int MN = (K + 2) * NT;
    constexpr int MP = K * NT;
    __shared__ float Mn[3][3][MN];
    __shared__ float Mp[3][MP];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const int tile = tile_base + static_cast<int>(blockIdx.x);
    const TileDev T = tiles[tile];
    const InstDev I = insts[T.inst];
    const LevelDev& L = levels[I.level];
    const int64_t n = steps[I.level];
    const bool first_tile = tile == I.tile0;
    if (first_tile && pend[T.inst]) {
        fold_partials(I, L, n - 1, partials, ptiles, accs, T.inst, records, status);
        if (tid == 0) pend[T.inst] = 0u;
    }

    if (n < L.n_steps) {
        const float* __restrict__ mi = ((n & 1) ? buf1 : buf0) + I.state_off;
        float* __restrict__ mo = ((n & 1) ? buf0 : buf1) + I.state_off;
        const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.ncell, nxy = nx * ny;
        const int TR = NT / nx;
        const int x = tid % nx, r = tid / nx;
        const bool lane_on = r < TR;
        const int y0 = T.y0, yend = T.y0 + T.nyt;   // window rows
        const int z0 = T.z0, zend = T.z0 + T.nzt;   // window planes
        const int py0 = max(y0 - 1, 0), py1 = min(yend + 1, ny);
        const int pz0 = max(z0 - 1, 0), pz1 = min(zend, nz - 1);
        const float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n));
        const float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
        const bool do_ckpt = (ckpt != nullptr) && ckpt_every > 0 && (n % ckpt_every) == 0;
        float* cp = do_ckpt ? ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N) : nullptr;
        const bool axes_on = L.has_axes != 0;
        const float* ax = axes + L.axes_off;

        int yy[K];
        bool on[K], win[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            yy[j] = py0 + r + j * TR;
            on[j] = lane_on && yy[j] < py1;
            win[j] = on[j] && yy[j] >= y0 && yy[j] < yend;
        }
        auto mn_at = [&](int y) { return (y - py0 + 1) * nx + x; };
        auto mp_at = [&](int y) { return (y - py0) * nx + x; };
        auto ld = [&](int y, int z) -> V3 {
            const int c = x + nx * y + nxy * z;
            return V3{mi[c], mi[N + c], mi[2 * N + c]};
        };
        auto st_mn = [&](int s, int i, V3 v) {
            Mn[s][0][i] = v.x;
            Mn[s][1][i] = v.y;
            Mn[s][2][i] = v.z;
        };
        auto ld_mn = [&](int s, int i) { return v3(Mn[s][0][i], Mn[s][1][i], Mn[s][2][i]); };
        // extra m_n rows py0 - 1 and py1 are loaded by the first thread row
        const bool ex_lo = lane_on && r == 0 && py0 - 1 >= 0;
        const bool ex_hi = lane_on && r == 0 && py1 < ny;
        // a plane is fetched into registers one iteration ahead and stored to
        // the LDS ring after the compute of that iteration
        auto fetch = [&](int z, V3* pre, V3& pl, V3& ph) {
            const int zc = min(z, nz - 1);
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (on[j]) pre[j] = ld(yy[j], zc);
            if (ex_lo) pl = ld(py0 - 1, zc);
            if (ex_hi) ph = ld(py1, zc);
        };
        auto store = [&](int z, const V3* pre, V3 pl, V3 ph) {
            const int s = z % 3;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (on[j]) st_mn(s, mn_at(yy[j]), pre[j]);
            if (ex_lo) st_mn(s, mn_at(py0 - 1), pl);
            if (ex_hi) st_mn(s, mn_at(py1), ph);
        };

        V3 pre[K], pl = V3{0, 0, 0}, ph = V3{0, 0, 0};
        V3 mpm2[K], mpm1[K];          // m' at planes p-2, p-1 (own cells)
        V3 qm1[K], hm1[K], um1[K];    // q, H_th and axis of plane p-1
        float msum = 0.0f;

        // ---- prologue: planes pz0 - 1 .. pz0 + 1 into the ring
        for (int z = pz0 - 1; z <= pz0 + 1; ++z) {
            if (z < 0 || z >= nz) continue;
            fetch(z, pre, pl, ph);
            store(z, pre, pl, ph);
        }
        fetch(pz0 + 2, pre, pl, ph);
        lds_barrier();

        for (int p = pz0; p <= pz1 + 1; ++p) {
            const bool predict = p <= pz1;
            const bool halo_plane = p < z0 || p >= zend;
            const int s0 = p % 3, sm = (p + 2) % 3, sp = (p + 1) % 3;
            V3 mpn[K], qn[K], hn[K], un[K];
            // ---- 1. predictor at plane p
            if (predict) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if (!on[j] || (halo_plane && !win[j])) continue;
                    const int y = yy[j];
                    const int i = mn_at(y);
                    const int ixm = x > 0 ? i - 1 : i, ixp = x < nx - 1 ? i + 1 : i;
                    const int iym = y > 0 ? i - nx : i, iyp = y < ny - 1 ? i + nx : i;
                    const V3 m = ld_mn(s0, i);
                    const V3 ex = nb_sum(m, ld_mn(s0, ixm), ld_mn(s0, ixp), ld_mn(s0, iym), ld_mn(s0, iyp),
                                         p > 0 ? ld_mn(sm, i) : m, p < nz - 1 ? ld_mn(sp, i) : m);
                    const int c = x + nx * y + nxy * p;
                    un[j] = axes_on ? V3{ax[c], ax[N + c], ax[2 * N + c]} : V3{L.ux, L.uy, L.uz};
                    hn[j] = thermal_field(L, I.seed, static_cast<uint32_t>(c), n);
                    heun_predict(L, m, ex, un[j], hz0, hn[j], mpn[j], qn[j]);
                }
            }
            // ---- 2. corrector at plane c = p - 1
            const int cz = p - 1;
            if (cz >= z0 && cz < zend) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if (!win[j]) continue;
                    const int y = yy[j];
                    const int i = mp_at(y);
                    const int ixm = x > 0 ? i - 1 : i, ixp = x < nx - 1 ? i + 1 : i;
                    const int iym = y > 0 ? i - nx : i, iyp = y < ny - 1 ? i + nx : i;
                    const V3 mpc = mpm1[j];
                    const V3 zmn = cz > 0 ? mpm2[j] : mpc;
                    const V3 zpn = predict ? mpn[j] : mpc;   // no plane above the grid top
                    const V3 ex = nb_sum(mpc, v3(Mp[0][ixm], Mp[1][ixm], Mp[2][ixm]),
                                         v3(Mp[0][ixp], Mp[1][ixp], Mp[2][ixp]),
                                         v3(Mp[0][iym], Mp[1][iym], Mp[2][iym]),
                                         v3(Mp[0][iyp], Mp[1][iyp], Mp[2][iyp]), zmn, zpn);
                    const V3 mn1 = heun_correct(L, mpc, ex, um1[j], hz1, hm1[j], qm1[j]);
                    const int c = x + nx * y + nxy * cz;
                    mo[c] = mn1.x;
                    mo[N + c] = mn1.y;
                    mo[2 * N + c] = mn1.z;
                    msum += mn1.z;
                    if (do_ckpt) {
                        const V3 m0 = ld_mn(sm, mn_at(y));   // m_n at plane p - 1
                        cp[c] = m0.x;
                        cp[N + c] = m0.y;
                        cp[2 * N + c] = m0.z;
                    }
                }
            }
            lds_barrier();
            if (p > pz1) break;
            // ---- 3. publish m'(p); plane p + 2 replaces p - 1 in the ring
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (!on[j]) continue;
                if (!(halo_plane && !win[j])) {
                    const int i = mp_at(yy[j]);
                    Mp[0][i] = mpn[j].x;
                    Mp[1][i] = mpn[j].y;
                    Mp[2][i] = mpn[j].z;
                }
                mpm2[j] = mpm1[j];
                mpm1[j] = mpn[j];
                qm1[j] = qn[j];
                hm1[j] = hn[j];
                um1[j] = un[j];
            }
            if (p + 2 < nz) store(p + 2, pre, pl, ph);
            fetch(p + 3, pre, pl, ph);
            lds_barrier();
        }

        const double tot = block_sum<NT>(msum, red);
        stream_block_end(tot, n, tile, ptiles, partials, first_tile, pend, T.inst, launch_cnt, steps, I.level,
                         L.n_steps);
    }
}

}  // namespace sllg
