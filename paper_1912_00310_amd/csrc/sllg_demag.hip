// Heun step with the magnetostatic (demagnetising) field, for levels of up to
// 1024 cells: one workgroup per realization, one cell per thread, the state in
// LDS for a launch of many steps.
//
// Beyond the paper, which leaves magnetostatics out (shape anisotropy is
// folded into K; material paragraph and closing discussion).  The field on
// cell i is Hd_i = sum_j T(r_i - r_j) m_j with T = -Ms N the demagnetising
// tensor of two uniformly magnetised cubes, tabulated by the host for every
// offset between two cells of the grid (8 floats per offset: xx yy zz xy |
// xz yz 0 0).  The sum is direct: every thread walks all cells, the m_j reads
// are LDS broadcasts (all lanes read the same cell) and the tensor reads come
// from the cached table.  Hd is added to the thermal field (both enter the
// effective field as plain additive terms), so the per-cell Heun functions
// are those of every other kernel; the field is recomputed for m' in the
// corrector.
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

template <int NT>
__device__ __forceinline__ V3 demag_sum(const float* __restrict__ S, const float4* __restrict__ T, int x, int y,
                                        int z, int nx, int ny, int nz, int N)
{
    const int wx = 2 * nx - 1, wy = 2 * ny - 1;
    V3 h = V3{0.0f, 0.0f, 0.0f};
    int j = 0;
    for (int zj = 0; zj < nz; ++zj)
        for (int yj = 0; yj < ny; ++yj) {
            // offset index of (x - xj, y - yj, z - zj) for xj = 0; it falls by
            // one per step in xj
            int o = ((z - zj + nz - 1) * wy + (y - yj + ny - 1)) * wx + x + nx - 1;
            for (int xj = 0; xj < nx; ++xj, ++j, --o) {
                const float4 a = T[2 * o], b = T[2 * o + 1];   // xx yy zz xy | xz yz
                const float mx = S[j], my = S[N + j], mz = S[2 * N + j];
                h.x = fmaf(a.x, mx, fmaf(a.w, my, fmaf(b.x, mz, h.x)));
                h.y = fmaf(a.w, mx, fmaf(a.y, my, fmaf(b.y, mz, h.y)));
                h.z = fmaf(b.x, mx, fmaf(b.y, my, fmaf(a.z, mz, h.z)));
            }
        }
    return h;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_demag(const InstDev* __restrict__ insts, int inst0,
                                              const LevelDev* __restrict__ levels, float* __restrict__ buf0,
                                              float* __restrict__ buf1, const float* __restrict__ axes,
                                              const float* __restrict__ demag, double* __restrict__ records,
                                              AccDev* __restrict__ accs, float* __restrict__ ckpt, int ckpt_every,
                                              int64_t n0, int64_t nsteps, int* __restrict__ status)
{
    __shared__ float A[3 * NT];    // m_n, planes x | y | z of N cells
    __shared__ float B[3 * NT];    // m'
    __shared__ double red[NT / 64];
    const int inst = inst0 + static_cast<int>(blockIdx.x);
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    const int N = L.ncell, nx = L.nx, ny = L.ny, nz = L.nz;
    const int i = static_cast<int>(threadIdx.x);
    const bool on = i < N;
    const int x = on ? i % nx : 0, y = on ? (i / nx) % ny : 0, z = on ? i / (nx * ny) : 0;
    const int ixm = x > 0 ? i - 1 : i, ixp = x < nx - 1 ? i + 1 : i;
    const int iym = y > 0 ? i - nx : i, iyp = y < ny - 1 ? i + nx : i;
    const int izm = z > 0 ? i - nx * ny : i, izp = z < nz - 1 ? i + nx * ny : i;
    const float4* T = reinterpret_cast<const float4*>(demag + L.demag_off);
    const float* mi = ((n0 & 1) ? buf1 : buf0) + I.state_off;
    V3 m = V3{0.0f, 0.0f, 0.0f};
    V3 u = V3{L.ux, L.uy, L.uz};
    if (on) {
        m = V3{mi[i], mi[N + i], mi[2 * N + i]};
        if (L.has_axes) u = V3{axes[L.axes_off + i], axes[L.axes_off + N + i], axes[L.axes_off + 2 * N + i]};
        A[i] = m.x;
        A[N + i] = m.y;
        A[2 * N + i] = m.z;
    }
    AccDev a{};
    if (i == 0) a = accs[inst];
    double* rec = records + I.rec_off;
    auto nb = [&](const float* S, V3 c) {
        return nb_sum(c, V3{S[ixm], S[N + ixm], S[2 * N + ixm]}, V3{S[ixp], S[N + ixp], S[2 * N + ixp]},
                      V3{S[iym], S[N + iym], S[2 * N + iym]}, V3{S[iyp], S[N + iyp], S[2 * N + iyp]},
                      V3{S[izm], S[N + izm], S[2 * N + izm]}, V3{S[izp], S[N + izp], S[2 * N + izp]});
    };
    double w = wave_at(L, n0);
    float hz0 = static_cast<float>(L.hz_amp * w);
    double H0 = L.hz_oe * w;
    __syncthreads();
    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t n = n0 + st;
        w = wave_at(L, n + 1);
        const float hz1 = static_cast<float>(L.hz_amp * w);
        const double H1 = L.hz_oe * w;
        V3 mp = V3{0.0f, 0.0f, 0.0f}, q = V3{0.0f, 0.0f, 0.0f}, hth = V3{0.0f, 0.0f, 0.0f};
        if (on) {
            if (ckpt != nullptr && ckpt_every > 0 && (n % ckpt_every) == 0) {
                float* cp = ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N);
                cp[i] = m.x;
                cp[N + i] = m.y;
                cp[2 * N + i] = m.z;
            }
            hth = thermal_field(L, I.seed, static_cast<uint32_t>(i), n);
            const V3 hd = demag_sum<NT>(A, T, x, y, z, nx, ny, nz, N);
            heun_predict(L, m, nb(A, m), u, hz0, V3{hth.x + hd.x, hth.y + hd.y, hth.z + hd.z}, mp, q);
            B[i] = mp.x;
            B[N + i] = mp.y;
            B[2 * N + i] = mp.z;
        }
        __syncthreads();
        float mz = 0.0f;
        if (on) {
            const V3 hd = demag_sum<NT>(B, T, x, y, z, nx, ny, nz, N);
            m = heun_correct(L, mp, nb(B, mp), u, hz1, V3{hth.x + hd.x, hth.y + hd.y, hth.z + hd.z}, q);
            // nobody reads m_n after the first barrier of the step
            A[i] = m.x;
            A[N + i] = m.y;
            A[2 * N + i] = m.z;
            mz = m.z;
        }
        // block sum (its barrier also ends the step: A holds m_{n+1})
        const double tot = block_sum<NT>(mz, red);
        if (i == 0) loop_accumulate_h(a, L, H0, H1, tot / static_cast<double>(N), rec);
        hz0 = hz1;
        H0 = H1;
        __syncthreads();
    }
    float* mo = (((n0 + nsteps) & 1) ? buf1 : buf0) + I.state_off;
    if (on) {
        mo[i] = m.x;
        mo[N + i] = m.y;
        mo[2 * N + i] = m.z;
    }
    if (i == 0) {
        accs[inst] = a;
        if (!isfinite(a.m_prev)) atomicOr(status, 1);
    }
}

}  // namespace sllg
