// Streamed Heun step (one launch per step) with the vertical neighbours in
// registers.
//
// A workgroup owns the rows [y0, y0 + nyt) of every x of one instance over
// the planes [z0, z0 + nzt).  It predicts the window plus one ring row on
// each side that lies inside the grid (rows [py0, py1)); the cells of that
// region are dealt to the threads in row-major order, K per thread, and a
// thread keeps its cells' z-columns in registers: m_n of planes p, p+1 and
// p+2 (the load of p+3 is issued during plane p), the easy axes of p-1, p and
// p+1, q and H_th of the plane before, m' of planes p, p-1 and p-2, and the
// extra rows (below) of planes p+1 .. p+3.  The three-plane columns rotate by
// renaming and the LDS buffers alternate, so the plane loop is unrolled six
// times.  LDS holds only x-y planes, one 16-byte slot per cell: m_n of planes
// p and p - 1 (the predicted rows plus the rows py0 - 1 and py1, which the
// first 2*nx threads load three planes ahead) and m' of planes p and p - 1;
// every buffer is written once per plane and read by other threads only
// until the next barrier, so one barrier per plane suffices, and a thread
// reads its own column's previous plane back from LDS.  Global accesses are
// buffer instructions with 32-bit offsets.  At plane p the workgroup
//   1. writes m_n(p) to LDS and waits at the barrier,
//   2. predicts plane p from LDS (x-y) and registers (z),
//   3. writes m'(p) to the other LDS buffer, and the extra rows of plane
//      p + 1 into the m_n buffer of plane p - 1,
//   4. corrects plane p - 1 from m'(p - 1) in LDS (x-y) and registers (z),
//      storing m_{n+1},
//   5. issues the loads of the extra rows of plane p + 4, of plane p + 3 and
//      of the axes of plane p + 2.
// The planes z0 - 1 and z0 + nzt are predicted for the window cells only
// (their m' is needed only as a vertical neighbour).  Workgroups are dealt to
// the XCDs so that each XCD runs a contiguous part of the tile list.
//
// Built with SLLG_LDS_CHECK defined (a debug build of the library, never the
// product), every LDS slot also carries in its fourth word the plane it
// stands for: the slots are filled with an impossible tag at the start, each
// write stores its plane, and each read of a neighbour or of the plane below
// compares the tag with the plane it expects.  A mismatch (a slot read
// before the write of its plane, or a write that never came) sets bit 2
// (value 4) of the status word; the arithmetic is unchanged.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

// third descriptor word of a raw (unformatted) buffer resource on gfx9
constexpr int kBufDword3 = 0x00020000;

#ifdef SLLG_LDS_CHECK
constexpr bool kLdsCheck = true;
#else
constexpr bool kLdsCheck = false;
#endif
constexpr int kLdsPoison = static_cast<int>(0x80000000u);   // tag of a slot never written

template <int NT, int K, bool AXES>
__global__ __launch_bounds__(NT) void k_rows2(
    const TileDev* __restrict__ tiles, const InstDev* __restrict__ insts,
    const LevelDev* __restrict__ levels, float* __restrict__ buf0, float* __restrict__ buf1,
    const float* __restrict__ axes, int64_t* __restrict__ steps, int tile_base, int ptiles,
    double* __restrict__ partials, uint32_t* __restrict__ pend, uint32_t* __restrict__ launch_cnt,
    double* __restrict__ records, AccDev* __restrict__ accs, float* __restrict__ ckpt, int ckpt_every,
    int* __restrict__ status)
{
    extern __shared__ float4 lds_rows2[];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    // Workgroups go to the 8 XCDs round-robin by block index; block b runs
    // tile start(b % 8) + b / 8, so that each XCD takes a contiguous run of
    // the tile list (neighbouring y windows of one z range), whose shared
    // rows then come from that XCD's L2.  A bijection for any grid size.
    const int tile = [] {
        const int nb = static_cast<int>(gridDim.x), b = static_cast<int>(blockIdx.x);
        const int x = b % 8;
        return x * (nb / 8) + min(x, nb % 8) + b / 8;
    }() + tile_base;
    const TileDev T = tiles[tile];
    const InstDev I = insts[T.inst];
    const LevelDev& L = levels[I.level];
    const int64_t n = steps[I.level];
    const bool first_tile = tile == I.tile0;
    if (first_tile && pend[T.inst]) {
        fold_partials(I, L, n - 1, partials, ptiles, accs, T.inst, records, status);
        if (tid == 0) pend[T.inst] = 0u;
    }
    if (n >= L.n_steps) return;

    const float* __restrict__ mi = ((n & 1) ? buf1 : buf0) + I.state_off;
    float* __restrict__ mo = ((n & 1) ? buf0 : buf1) + I.state_off;
    const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.ncell, nxy = nx * ny;
    const int y0 = T.y0, yend = T.y0 + T.nyt;
    const int z0 = T.z0, zend = T.z0 + T.nzt;
    const int py0 = max(y0 - 1, 0), py1 = min(yend + 1, ny);
    const int pz0 = max(z0 - 1, 0), pz1 = min(zend, nz - 1);
    const int LC = (py1 - py0 + 2) * nx;   // LDS cells of an m_n plane (rows py0 - 1 .. py1)
    const int PC = (py1 - py0) * nx;       // predicted cells
    // cells in 16-byte slots (x, y, z, unused): one LDS access per neighbour
    // Buffer (p - pz0) & 1 of each pair holds plane p.  With one cell per
    // thread the buffers sit at fixed strides (an m_n plane holds at most
    // 2 NT cells: the host refuses tiles with more), so that with the plane
    // loop unrolled six times every LDS access is a per-thread offset plus an
    // immediate; with two cells per thread they are packed.
    constexpr bool FIXED = K == 1;
    const int SN = FIXED ? 2 * NT : LC;        // stride of the m_n buffers (cells)
    const int SP = FIXED ? NT : PC;            // stride of the m' buffers
    float4* const Mn0 = lds_rows2;             // [2][SN]: m_n of planes p and p - 1
    float4* const Mp0 = lds_rows2 + 2 * SN;    // [2][SP]: m' of planes p and p - 1
    bool lds_bad = false;                      // debug build: a slot read with the wrong tag
    if constexpr (kLdsCheck) {
        for (int i = tid; i < 2 * SN + 2 * SP; i += NT) lds_rows2[i] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(kLdsPoison));
        __syncthreads();
    }
    const float hz0 = static_cast<float>(L.hz_amp * wave_at(L, n));
    const float hz1 = static_cast<float>(L.hz_amp * wave_at(L, n + 1));
    const bool do_ckpt = (ckpt != nullptr) && ckpt_every > 0 && (n % ckpt_every) == 0;
    float* cp = do_ckpt ? ckpt + I.ckpt_off + (n / ckpt_every) * 3 * static_cast<int64_t>(N) : nullptr;
    const float* ax = axes + L.axes_off;
    const V3 u0 = V3{L.ux, L.uy, L.uz};
    // The step constants, in vector registers with one cell per thread (a
    // scalar reload inside the loop waits on the same counter as the plane's
    // LDS reads); with two cells per thread the registers are needed elsewhere.
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

    // own cells: index ii in the predicted region (the m' plane index; the
    // m_n LDS index is ii + nx, the plane index ii + py0 nx) and which x-y
    // neighbours exist (bits: x-1, x+1, y-1, y+1); neighbours outside the
    // grid are replaced by the cell itself
    int ii[K], edge[K];
    bool on[K], win[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int i = tid + j * NT;
        on[j] = i < PC;
        ii[j] = on[j] ? i : 0;
        const int y = py0 + ii[j] / nx, x = ii[j] - (y - py0) * nx;
        win[j] = on[j] && y >= y0 && y < yend;
        edge[j] = (x > 0 ? 1 : 0) | (x < nx - 1 ? 2 : 0) | (y > 0 ? 4 : 0) | (y < ny - 1 ? 8 : 0);
    }
    const int gofs = py0 * nx;   // plane index of predicted-region index 0
    // the rows py0 - 1 and py1 (when inside the grid) are loaded by threads
    // [0, nx) and [nx, 2 nx)
    const bool ex_lo = tid < nx && py0 > 0;
    const bool ex_hi = tid >= nx && tid < 2 * nx && py1 < ny;
    const bool ex = ex_lo || ex_hi;
    const int ex_x = ex_lo ? tid : tid - nx;
    const int ex_gc = ex ? ex_x + nx * (ex_lo ? py0 - 1 : py1) : 0;
    const int ex_li = ex_lo ? ex_x : (py1 - py0 + 1) * nx + ex_x;

    // global accesses as buffer instructions over one instance's planes: a
    // 32-bit lane byte offset plus a wave-uniform plane byte offset, so no
    // per-lane 64-bit address arithmetic (out-of-range offsets read 0)
    const uint32_t region = 12u * static_cast<uint32_t>(N);   // bytes of mx | my | mz
    const __amdgpu_buffer_rsrc_t r_in = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(mi), 0, region, kBufDword3);
    const __amdgpu_buffer_rsrc_t r_out = __builtin_amdgcn_make_buffer_rsrc(mo, 0, region, kBufDword3);
    const __amdgpu_buffer_rsrc_t r_ax = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(ax), 0, region, kBufDword3);
    const __amdgpu_buffer_rsrc_t r_ck = __builtin_amdgcn_make_buffer_rsrc(do_ckpt ? cp : mo, 0, region, kBufDword3);
    auto plane_ofs = [&](int z) { return static_cast<uint32_t>(min(z, nz - 1)) * static_cast<uint32_t>(nxy) * 4u; };
    // (plane z given within the grid: a second clamp would be merged with the
    // caller's into a vector min3, and a vector plane offset turns each load
    // into a loop over distinct values)
    auto ldc = [&](int z, uint32_t off) -> V3 {
        const uint32_t pz = static_cast<uint32_t>(z) * static_cast<uint32_t>(nxy) * 4u;
        return V3{__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_in, off, pz, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_in, off, pz + 4u * N, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_in, off, pz + 8u * N, 0))};
    };
    auto lduc = [&](int z, uint32_t off) -> V3 {
        const uint32_t pz = static_cast<uint32_t>(z) * static_cast<uint32_t>(nxy) * 4u;
        return V3{__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_ax, off, pz, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_ax, off, pz + 4u * N, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_ax, off, pz + 8u * N, 0))};
    };
    auto ld = [&](int z, uint32_t off) -> V3 {
        const uint32_t pz = plane_ofs(z);
        return V3{__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_in, off, pz, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_in, off, pz + 4u * N, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_in, off, pz + 8u * N, 0))};
    };
    auto ldu = [&](int z, uint32_t off) -> V3 {
        const uint32_t pz = plane_ofs(z);
        return V3{__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_ax, off, pz, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_ax, off, pz + 4u * N, 0)),
                  __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r_ax, off, pz + 8u * N, 0))};
    };
    auto st3 = [&](__amdgpu_buffer_rsrc_t r, int z, uint32_t off, V3 v) {
        const uint32_t pz = plane_ofs(z);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v.x), r, off, pz, 0);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v.y), r, off, pz + 4u * N, 0);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v.z), r, off, pz + 8u * N, 0);
    };
    uint32_t gb[K];   // byte offset of each own cell within a plane
#pragma unroll
    for (int j = 0; j < K; ++j) gb[j] = static_cast<uint32_t>(ii[j] + gofs) * 4u;
    const uint32_t ex_gb = static_cast<uint32_t>(ex_gc) * 4u;
    // a cell to LDS: x, y, z of its 16-byte slot (one 12-byte store; the
    // fourth word is never read)
    // (the debug build also writes the plane tag into the fourth word)
    auto put = [](float4* slot, V3 v, int plane) {
        float* q = static_cast<float*>(__builtin_assume_aligned(slot, 16));
        q[0] = v.x;
        q[1] = v.y;
        q[2] = v.z;
        if constexpr (kLdsCheck) q[3] = __int_as_float(plane);
        (void)plane;
    };
    // a slot's cell, read as the cell of the given plane
    auto rd = [&](const float4* slot, int plane) {
        const float4 v = *slot;
        if constexpr (kLdsCheck) lds_bad = lds_bad || __float_as_int(v.w) != plane;
        (void)plane;
        return V3{v.x, v.y, v.z};
    };

    auto xm = [&](int i, int e) { return (e & 1) ? i - 1 : i; };
    auto xp = [&](int i, int e) { return (e & 2) ? i + 1 : i; };
    auto ym = [&](int i, int e) { return (e & 4) ? i - nx : i; };
    auto yp = [&](int i, int e) { return (e & 8) ? i + nx : i; };

    // The z-columns rotate with period 3 (m_n of p, p+1, p+2; axes of p-1, p,
    // p+1; q and H_th of the plane before): the plane loop is unrolled six
    // times and slot (p - pz0) % 3 of each array is renamed, not copied.
    V3 M[3][K];          // m_n: slot PH = plane p, PH+1 = p+1, PH+2 = p+2
    V3 U[3][K];          // axes: slot PH = plane p-1, PH+1 = p, PH+2 = p+1
    V3 Q[3][K], HT[3][K];   // q, H_th: slot PH = plane p, PH+2 = plane p-1
    V3 MP[3][K];         // m' (own cells): slot PH = plane p, PH+2 = p-1, PH+1 = p-2
#pragma unroll
    for (int j = 0; j < K; ++j) {
#pragma unroll
        for (int k = 0; k < 3; ++k) M[k][j] = U[k][j] = Q[k][j] = HT[k][j] = V3{0, 0, 0};
        MP[0][j] = MP[1][j] = MP[2][j] = V3{0, 0, 0};
        if (on[j]) {
            // plane pz0 - 1 of the own column, the lower neighbour of the
            // first plane; at the bottom of the grid plane 0 itself, so that
            // the missing neighbour is the cell (no select in the loop)
            put(&Mn0[SN + ii[j] + nx], ld(max(pz0 - 1, 0), gb[j]), pz0 - 1);
        }
        M[0][j] = ld(pz0, gb[j]);
        M[1][j] = ld(pz0 + 1, gb[j]);
        M[2][j] = ld(pz0 + 2, gb[j]);
        if (AXES) {
            U[1][j] = ldu(pz0, gb[j]);
            U[2][j] = ldu(pz0 + 1, gb[j]);
        }
    }
    // the extra rows of plane p go to LDS during plane p - 1 (below), loaded
    // at the end of plane p - 3; those of the first plane here
    if (ex) put(&Mn0[ex_li], ld(pz0, ex_gb), pz0);
    // extra rows of the planes p + 1, p + 2, p + 3 (slot PH holds p + 1)
    V3 E[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) E[k] = ld(min(pz0 + 1 + k, pz1), ex_gb);

    float msum = 0.0f;
    const int zlast = min(pz1 + 1, nz - 1);    // the last plane of m_n the tile reads
    const int plast = zend == nz ? nz : pz1;   // the last plane holds only a corrector when zend = nz
    auto plane = [&](auto phase, const int p) {
        constexpr int PH = decltype(phase)::value % 3;
        constexpr int P1 = (PH + 1) % 3, P2 = (PH + 2) % 3;
        constexpr int b = decltype(phase)::value & 1;   // buffer of plane p
        const bool predict = p <= pz1;
        const bool halo_plane = p < z0 || p >= zend;
        float4* Mn = Mn0 + b * SN;
        const float4* Mo = Mn0 + (b ^ 1) * SN;                      // m_n of plane p - 1
        float4* Mp = Mp0 + b * SP;
        const float4* Mq = Mp0 + (b ^ 1) * SP;                      // m' of plane p - 1
        // ---- 1. m_n(p) to LDS
        if (predict) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (!on[j]) continue;
                put(&Mn[ii[j] + nx], M[PH][j], p);
            }
        }
        lds_barrier();
        // ---- 2. predictor at plane p; 3. m'(p) to LDS
        // (a cell that is not predicted here is not corrected from this plane
        // either, so its m', q and H_th slots are left as they are)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!predict || !on[j] || (halo_plane && !win[j])) continue;
            const V3 m = M[PH][j];
            const int l = ii[j] + nx, e = edge[j];
            const uint32_t cell = static_cast<uint32_t>((ii[j] + gofs) + nxy * p);
            V3 exs;
            if constexpr (K == 1) {
                // the LDS reads are issued, then the noise is drawn while they
                // are in flight (with two cells per thread the values held
                // meanwhile would spill)
                const V3 n_xm = rd(&Mn[xm(l, e)], p), n_xp = rd(&Mn[xp(l, e)], p);
                const V3 n_ym = rd(&Mn[ym(l, e)], p), n_yp = rd(&Mn[yp(l, e)], p);
                // (below plane 0 the buffer holds plane 0; above nz - 1 the
                // clamped load of M[P1] holds plane nz - 1: the cell itself)
                const V3 n_zm = rd(&Mo[l], p - 1);
                HT[PH][j] = thermal_field(Lc, I.seed, cell, n);
                exs = nb_sum(m, n_xm, n_xp, n_ym, n_yp, n_zm, M[P1][j]);
            } else {
                exs = nb_sum(m, rd(&Mn[xm(l, e)], p), rd(&Mn[xp(l, e)], p), rd(&Mn[ym(l, e)], p),
                             rd(&Mn[yp(l, e)], p), rd(&Mo[l], p - 1), M[P1][j]);
                HT[PH][j] = thermal_field(Lc, I.seed, cell, n);
            }
            heun_predict(Lc, m, exs, AXES ? U[P1][j] : u0, hz0, HT[PH][j], MP[PH][j], Q[PH][j]);
            put(&Mp[ii[j]], MP[PH][j], p);
        }
        // ---- the extra rows of plane p + 1 into the m_n buffer of plane
        //      p - 1, whose extra rows nobody reads after the barrier above.
        //      (Before the corrector's stores, so that the wait for the load
        //      does not include them; the empty asm uses the loaded values in
        //      every wave, so that the wait is taken here whichever lanes store.)
        asm volatile("" ::"v"(E[PH].x), "v"(E[PH].y), "v"(E[PH].z));
        if (ex && p + 1 <= pz1) put(&Mn0[(b ^ 1) * SN + ex_li], E[PH], p + 1);
        // ---- 4. corrector at plane p - 1
        const int cz = p - 1;
        if (cz >= z0 && cz < zend) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (!win[j]) continue;
                const int i = ii[j], e = edge[j];
                const V3 mpc = MP[P2][j];   // the own cell's m'(p - 1), also in LDS for the neighbours
                const V3 exs = nb_sum(mpc, rd(&Mq[xm(i, e)], cz), rd(&Mq[xp(i, e)], cz), rd(&Mq[ym(i, e)], cz),
                                      rd(&Mq[yp(i, e)], cz), cz > 0 ? MP[P1][j] : mpc, predict ? MP[PH][j] : mpc);
                const V3 mn1 = heun_correct(Lc, mpc, exs, AXES ? U[PH][j] : u0, hz1, HT[P2][j], Q[P2][j]);
                st3(r_out, cz, gb[j], mn1);
                msum += mn1.z;
                if (do_ckpt) st3(r_ck, cz, gb[j], rd(&Mo[ii[j] + nx], cz));
            }
        }
        // ---- 5. loads of the extra rows of plane p + 4 into their slot of
        //         plane p + 1, of plane p + 3 into the slot of plane p and of
        //         the axes of plane p + 2 into the slot of plane p - 1
        E[PH] = ldc(min(p + 4, pz1), ex_gb);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            // The loads are unconditional, so that the compiler can count the
            // memory operations in flight exactly and wait only for the ones a
            // value needs: past the last plane a tile uses they repeat that
            // plane (a cache hit), and lanes without a cell read at offset 0.
            M[PH][j] = ldc(min(p + 3, zlast), gb[j]);
            if (AXES) U[PH][j] = lduc(min(p + 2, pz1), gb[j]);
        }
    };
    // the first loads complete before the loop, so that the wait counts in
    // the loop follow its own loads only
    __builtin_amdgcn_s_waitcnt(0);
    // Whole groups of six planes (the register slots rotate with period 3,
    // the LDS buffers with period 2), so that the loop has one path per trip
    // and the wait counts of the loads stay exact: a plane past plast
    // predicts and corrects nothing (p > pz1 and p - 1 >= zend), and its
    // loads repeat the last plane.
    for (int p = pz0; p <= plast; p += 6) {
        plane(std::integral_constant<int, 0>{}, p);
        plane(std::integral_constant<int, 1>{}, p + 1);
        plane(std::integral_constant<int, 2>{}, p + 2);
        plane(std::integral_constant<int, 3>{}, p + 3);
        plane(std::integral_constant<int, 4>{}, p + 4);
        plane(std::integral_constant<int, 5>{}, p + 5);
    }

    if constexpr (kLdsCheck)
        if (lds_bad) atomicOr(status, 4);
    const double tot = block_sum<NT>(msum, red);
    stream_block_end(tot, n, tile, ptiles, partials, first_tile, pend, T.inst, launch_cnt, steps, I.level,
                     L.n_steps);
}

}  // namespace sllg
