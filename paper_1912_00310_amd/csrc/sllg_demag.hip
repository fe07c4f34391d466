// Heun step with the magnetostatic (demagnetising) field, for levels of up to
// 1024 cells: one workgroup per realization, the state and the tensor table in
// LDS for a launch of many steps.
//
// Beyond the paper, which leaves magnetostatics out (shape anisotropy is
// folded into K; material paragraph and closing discussion).  The field on
// cell i is Hd_i = sum_j T(r_i - r_j) m_j with T = -Ms N the demagnetising
// tensor of two uniformly magnetised cubes.  The host tabulates T in one of
// two forms (six planes xx yy zz xy xz yz):
//   - wide: every offset of the grid, in rows of wx >= 2nx-1 and planes of
//     wy >= 2ny-1 rows (2nz-1 planes), offset index
//     ((dz+nz-1) wy + dy+ny-1) wx + dx+nx-1, used when it fits the LDS: the
//     index of a pair is base(i) - base(j) with base(j) stored beside m_j,
//     one subtraction per pair.  The host pads wx and wy so that the 64
//     lanes of a wave, which read the table at 64 different offsets, spread
//     over the LDS banks;
//   - octant: the offsets with dx, dy, dz >= 0 only (one per cell), for the
//     larger grids: N is even in every component of the offset on its
//     diagonal, N_xy odd in dx and dy (even in dz), N_xz odd in dx and dz,
//     N_yz odd in dy and dz, and the kernel restores the signs.
//
// The sum is direct, split over S groups of threads: thread s*N + i sums the
// cells of chunk s for cell i (m_j and base(j) are one LDS broadcast, the
// table reads run over consecutive cells), the partial sums meet in LDS and
// the owner thread i (s = 0) adds them in chunk order and takes the Heun
// stage.  While the owners take their stages the other threads are idle:
// there, helper threads in waves without owners draw the next step's thermal
// field (kept in LDS for the owners) and fold the previous step into the
// loop accumulators, so neither lies on the owners' path.  S depends only on the cell count, so the summation order, and hence
// every state, is fixed by the level.  Hd is added to the thermal field (both
// enter the effective field as plain additive terms), so the per-cell Heun
// functions are those of every other kernel; the field is recomputed for m'
// in the corrector.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

constexpr int kDemagMaxThreads = 1024;
constexpr int kDemagMaxCells = 1024;

// Chunks of the direct sum for a level of n cells: about 1024/n, at most 16,
// every chunk non-empty.  Threads of the workgroup: chunks x n, rounded up to
// whole waves.
__host__ __device__ constexpr int demag_chunk_len(int n)
{
    const int s0 = n >= kDemagMaxThreads ? 1 : (kDemagMaxThreads / n > 16 ? 16 : kDemagMaxThreads / n);
    return (n + s0 - 1) / s0;
}
__host__ __device__ constexpr int demag_chunks(int n) { return (n + demag_chunk_len(n) - 1) / demag_chunk_len(n); }
__host__ __device__ constexpr int demag_block(int n) { return (demag_chunks(n) * n + 63) / 64 * 64; }

__device__ __forceinline__ float sgnf(int d) { return static_cast<float>((d > 0) - (d < 0)); }

// Partial field on cell i from cells j0 .. j1-1 of the state S (xyz of m_j
// and base(j) in w), wide table.
__device__ __forceinline__ V3 demag_partial_wide(const float4* __restrict__ S, const float* __restrict__ Tt,
                                                 int W, int base, int j0, int j1)
{
    V3 h = V3{0.0f, 0.0f, 0.0f};
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const float4 mj = S[j];
        const int o = base - __float_as_int(mj.w);
        const float txx = Tt[o], tyy = Tt[W + o], tzz = Tt[2 * W + o];
        const float txy = Tt[3 * W + o], txz = Tt[4 * W + o], tyz = Tt[5 * W + o];
        h.x = fmaf(txx, mj.x, fmaf(txy, mj.y, fmaf(txz, mj.z, h.x)));
        h.y = fmaf(txy, mj.x, fmaf(tyy, mj.y, fmaf(tyz, mj.z, h.y)));
        h.z = fmaf(txz, mj.x, fmaf(tyz, mj.y, fmaf(tzz, mj.z, h.z)));
    }
    return h;
}

// The same with the octant table: the offset's magnitudes index the table
// and its signs those of the off-diagonal terms.
__device__ __forceinline__ V3 demag_partial_octant(const float4* __restrict__ S, const float* __restrict__ Tt,
                                                   int x, int y, int z, int nx, int ny, int N, int j0, int j1)
{
    V3 h = V3{0.0f, 0.0f, 0.0f};
    int xj = j0 % nx, yj = (j0 / nx) % ny, zj = j0 / (nx * ny);
    int dy = y - yj, dz = z - zj;
    int rowo = nx * (abs(dy) + ny * abs(dz));
    float syz = sgnf(dy) * sgnf(dz), sy = sgnf(dy), sz = sgnf(dz);
    for (int j = j0; j < j1; ++j) {
        const int dx = x - xj;
        const int o = rowo + abs(dx);
        const float sx = sgnf(dx);
        const float txx = Tt[o], tyy = Tt[N + o], tzz = Tt[2 * N + o];
        const float txy = sx * sy * Tt[3 * N + o], txz = sx * sz * Tt[4 * N + o], tyz = syz * Tt[5 * N + o];
        const float4 mj = S[j];
        h.x = fmaf(txx, mj.x, fmaf(txy, mj.y, fmaf(txz, mj.z, h.x)));
        h.y = fmaf(txy, mj.x, fmaf(tyy, mj.y, fmaf(tyz, mj.z, h.y)));
        h.z = fmaf(txz, mj.x, fmaf(tyz, mj.y, fmaf(tzz, mj.z, h.z)));
        if (++xj == nx) {
            xj = 0;
            if (++yj == ny) {
                yj = 0;
                ++zj;
                dz = z - zj;
                sz = sgnf(dz);
            }
            dy = y - yj;
            sy = sgnf(dy);
            syz = sy * sz;
            rowo = nx * (abs(dy) + ny * abs(dz));
        }
    }
    return h;
}

// Static LDS of k_demag; the table is dynamic (6 planes of W floats).
constexpr size_t kDemagStaticLds = 2 * sizeof(float4) * kDemagMaxCells + 3 * sizeof(float) * kDemagMaxThreads +
                                   3 * sizeof(float) * kDemagMaxCells + 8 * (kDemagMaxThreads / 64) + 128;

// wide != 0: the table holds every offset (W = wx wy (2nz-1) of them, rows of
// wx, planes of wy rows); else the octant table (W = N).
__global__ __launch_bounds__(kDemagMaxThreads) void k_demag(const InstDev* __restrict__ insts, int inst0,
                                                           const LevelDev* __restrict__ levels,
                                                           float* __restrict__ buf0, float* __restrict__ buf1,
                                                           const float* __restrict__ axes,
                                                           const float* __restrict__ demag, int wide, int W,
                                                           int wx, int wy,
                                                           double* __restrict__ records, AccDev* __restrict__ accs,
                                                           float* __restrict__ ckpt, int ckpt_every, int64_t n0,
                                                           int64_t nsteps, int* __restrict__ status)
{
    extern __shared__ float Tt[];                 // tensor planes xx yy zz xy xz yz of W floats
    __shared__ float4 A[kDemagMaxCells];          // m_n (xyz) and base(j) (w)
    __shared__ float4 B[kDemagMaxCells];          // m'
    __shared__ float P[3 * kDemagMaxThreads];     // partial sums of chunks 1 .. S-1
    __shared__ float HT[3 * kDemagMaxCells];      // thermal field of the step (drawn by the helpers)
    __shared__ double red[kDemagMaxThreads / 64];
    __shared__ AccDev acc;                        // the loop accumulators (thread 0)
    const int inst = inst0 + static_cast<int>(blockIdx.x);
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    const int N = L.ncell, nx = L.nx, ny = L.ny, nz = L.nz;
    const int tid = static_cast<int>(threadIdx.x), nthr = static_cast<int>(blockDim.x);
    const int clen = demag_chunk_len(N), S = demag_chunks(N);
    const int s = tid / N, i = tid - s * N;
    const bool sums = s < S;                 // computes a partial sum
    const bool on = tid < N;                 // owns cell i
    const int j0 = sums ? s * clen : 0, j1 = sums ? min(N, j0 + clen) : 0;
    const int x = sums ? i % nx : 0, y = sums ? (i / nx) % ny : 0, z = sums ? i / (nx * ny) : 0;
    // index of the cell in the wide offset grid: offset (i - j) = base(i) - base(j) + centre
    // helpers: the threads from the first wave boundary after the owners on,
    // one per cell, if the workgroup has that many; thread d0 also folds
    const int d0 = (N + 63) / 64 * 64;
    const bool helpers = d0 + N <= nthr;
    const bool drawer = helpers && tid >= d0 && tid < d0 + N;
    const int di = tid - d0;   // the drawer's cell
    const int basej = (z * wy + y) * wx + x;
    const int basei = ((z + nz - 1) * wy + y + ny - 1) * wx + x + nx - 1;
    const float* T = demag + L.demag_off;
    for (int k = tid; k < 6 * W; k += nthr) Tt[k] = T[k];
    const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
    V3 m = V3{0.0f, 0.0f, 0.0f};
    V3 u = V3{L.ux, L.uy, L.uz};
    const float wbits = __int_as_float(basej);
    if (on) {
        m = V3{mi[i], mi[N + i], mi[2 * N + i]};
        if (L.has_axes) u = V3{axes[L.axes_off + i], axes[L.axes_off + N + i], axes[L.axes_off + 2 * N + i]};
        A[i] = make_float4(m.x, m.y, m.z, wbits);
    }
    if (tid == 0) acc = accs[inst];
    double* rec = records + I.rec_off;
    // the exchange neighbours are recomputed from (x, y, z) at each use
    // (fewer live registers across the Heun stages)
    auto nb = [&](const float4* St, V3 c) {
        const int ixm = x > 0 ? i - 1 : i, ixp = x < nx - 1 ? i + 1 : i;
        const int iym = y > 0 ? i - nx : i, iyp = y < ny - 1 ? i + nx : i;
        const int izm = z > 0 ? i - nx * ny : i, izp = z < nz - 1 ? i + nx * ny : i;
        const float4 a = St[ixm], b = St[ixp], c2 = St[iym], d = St[iyp], e = St[izm], f = St[izp];
        return nb_sum(c, V3{a.x, a.y, a.z}, V3{b.x, b.y, b.z}, V3{c2.x, c2.y, c2.z}, V3{d.x, d.y, d.z},
                      V3{e.x, e.y, e.z}, V3{f.x, f.y, f.z});
    };
    // partial sum of the thread's chunk over the state St; chunks 1 .. S-1
    // park theirs in P, the owner keeps chunk 0's in registers
    auto partial = [&](const float4* St) {
        V3 h = V3{0.0f, 0.0f, 0.0f};
        if (sums)
            h = wide ? demag_partial_wide(St, Tt, W, basei, j0, j1)
                     : demag_partial_octant(St, Tt, x, y, z, nx, ny, N, j0, j1);
        if (sums && s > 0) {
            const int p = (s - 1) * N + i;
            P[p] = h.x;
            P[(S - 1) * N + p] = h.y;
            P[2 * (S - 1) * N + p] = h.z;
        }
        return h;
    };
    // the owner's total: chunk 0, then chunks 1 .. S-1 in order
    auto total = [&](V3 h) {
        for (int c = 1; c < S; ++c) {
            const int p = (c - 1) * N + i;
            h.x += P[p];
            h.y += P[(S - 1) * N + p];
            h.z += P[2 * (S - 1) * N + p];
        }
        return h;
    };
    auto draw = [&](int64_t n) {
        const V3 h = thermal_field(L, I.seed, static_cast<uint32_t>(di), n);
        HT[di] = h.x;
        HT[N + di] = h.y;
        HT[2 * N + di] = h.z;
    };
    // the loop value of step n from the wave partial sums in red
    auto fold = [&](int64_t n) {
        double tot = 0.0;
        for (int k = 0; k < nthr / 64; ++k) tot += red[k];
        loop_accumulate(acc, L, n, tot / static_cast<double>(N), rec);
    };
    if (drawer) draw(n0);
    float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n0));
    __syncthreads();
    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        const float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
        V3 mp = V3{0.0f, 0.0f, 0.0f}, q = V3{0.0f, 0.0f, 0.0f}, hth = V3{0.0f, 0.0f, 0.0f};
        V3 hd = partial(A);
        __syncthreads();
        if (on) {
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N);
                cp[i] = m.x;
                cp[N + i] = m.y;
                cp[2 * N + i] = m.z;
            }
            hth = helpers ? V3{HT[i], HT[N + i], HT[2 * N + i]} : thermal_field(L, I.seed, static_cast<uint32_t>(i), n);
            hd = total(hd);
            heun_predict(L, m, nb(A, m), u, hz0, V3{hth.x + hd.x, hth.y + hd.y, hth.z + hd.z}, mp, q);
            B[i] = make_float4(mp.x, mp.y, mp.z, wbits);
        }
        // the previous step's loop value, off the owners' path (red is next
        // written after the corrector)
        if (helpers && tid == d0 && st > 0) fold(n - 1);
        __syncthreads();
        hd = partial(B);
        __syncthreads();
        float mz = 0.0f;
        if (on) {
            hd = total(hd);
            m = heun_correct(L, mp, nb(B, mp), u, hz1, V3{hth.x + hd.x, hth.y + hd.y, hth.z + hd.z}, q);
            // nobody reads m_n after the first barrier of the step
            A[i] = make_float4(m.x, m.y, m.z, wbits);
            mz = m.z;
        }
        // the next step's thermal field (the owners hold this step's in
        // registers since the predictor)
        if (drawer && st + 1 < nsteps) draw(n + 1);
        // block sum over whole waves (its barrier also ends the step: A
        // holds m_{n+1}; the next partial sums overwrite P only after it)
        const float ws = wave_sum(mz);
        if ((tid & 63) == 0) red[tid >> 6] = static_cast<double>(ws);
        __syncthreads();
        hz0 = hz1;
        if (!helpers) {
            if (tid == 0) fold(n);
            __syncthreads();
        }
    }
    if (helpers) {
        if (tid == d0 && nsteps > 0) fold(n0 + nsteps - 1);
        __syncthreads();
    }
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    if (on) {
        mo[i] = m.x;
        mo[N + i] = m.y;
        mo[2 * N + i] = m.z;
    }
    if (tid == 0) {
        accs[inst] = acc;
        if (!isfinite(acc.m_prev)) atomicOr(status, 1);
    }
}

}  // namespace sllg
