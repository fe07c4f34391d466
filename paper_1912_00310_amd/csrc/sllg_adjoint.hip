// Discrete adjoint of the Heun stochastic-LLG step under fixed noise.
//
// One workgroup per realization, one cell per thread (levels up to 1024
// cells).  The sweep is replayed backwards in segments of ckpt_every steps:
// each segment is first recomputed forward from its checkpoint with the same
// per-cell arithmetic as the forward kernels (so the replay is bit-identical)
// and taped to global memory (m_n, m', xi per cell and step); then the
// segment is walked in reverse.  Two losses are carried together:
//   L_l = sum_n w[l][n] * mbar_n,   mbar_n = (1/N) sum_i m_z,i(n)
// (loop area and coercive field of the ensemble-mean loop, weights from the
// host).  For one step, with lambda = dL/dm_{n+1}:
//   q-bar  = (I - m_{n+1} m_{n+1}^T) lambda / |q|
//   f'-bar = f-bar = dt/2 q-bar,  m-bar = q-bar
//   H'-bar = gamma1 m' x f'-bar - alpha gamma1 m' x (m' x f'-bar)
//   m'-bar = (df/dm)^T f'-bar + c_ex sum_j (H'-bar_j - H'-bar_i) + H_K u (u.H'-bar)
//   p-bar  = (I - m' m'^T) m'-bar / |p|;  m-bar += p-bar;  f-bar += dt p-bar
//   H-bar  and m-bar as for the primed stage, then lambda_n = m-bar + dL/dm_n.
// (df/dm)^T v = -gamma1 H x v - alpha gamma1 ((m x H) x v + H x (v x m)).
// Parameter partials per loss, accumulated in FP64: c_ex (H-bar . exchange sum),
// H_K ((m.u)(u.H-bar)), gamma1 (f-bar . f / gamma1), alpha with gamma1 held
// (f-bar . -gamma1 m x (m x H)), sigma (H-bar . xi).
#include <hip/hip_runtime.h>

#include "sllg_device.hpp"
#include "sllg_types.hpp"

namespace sllg {

__device__ __forceinline__ V3 add3(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 scale3(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }

// (I - n n^T) v / len
__device__ __forceinline__ V3 unit_T(V3 nrm, float inv_len, V3 v)
{
    const float d = dot3(nrm, v);
    return V3{(v.x - nrm.x * d) * inv_len, (v.y - nrm.y * d) * inv_len, (v.z - nrm.z * d) * inv_len};
}

// (df/dH)^T v
__device__ __forceinline__ V3 rhs_dH_T(float g1, float ag1, V3 m, V3 v)
{
    const V3 a = cross3(m, v);
    const V3 b = cross3(m, a);
    return V3{g1 * a.x - ag1 * b.x, g1 * a.y - ag1 * b.y, g1 * a.z - ag1 * b.z};
}

// (df/dm)^T v with H fixed
__device__ __forceinline__ V3 rhs_dm_T(float g1, float ag1, V3 m, V3 H, V3 v)
{
    const V3 t1 = cross3(H, v);
    const V3 t2 = cross3(cross3(m, H), v);
    const V3 t3 = cross3(H, cross3(v, m));
    return V3{-g1 * t1.x - ag1 * (t2.x + t3.x), -g1 * t1.y - ag1 * (t2.y + t3.y),
              -g1 * t1.z - ag1 * (t2.z + t3.z)};
}

// Workgroups of up to 256 cells get NT more threads: thread NT + i draws the
// thermal field of cell i for the next replay step into LDS while the cell
// threads step the current one.
template <int NT>
constexpr int kAdjThreads = NT <= 256 ? 2 * NT : NT;

template <int NT>
__global__ __launch_bounds__(kAdjThreads<NT>) void k_adjoint(const InstDev* __restrict__ insts, int inst0,
                                                const LevelDev* __restrict__ levels,
                                                const float* __restrict__ axes,
                                                const float* __restrict__ ckpt, int ckpt_every,
                                                float* __restrict__ tape, const double* __restrict__ w,
                                                double* __restrict__ grads)
{
    // m_n and m' by step parity: the replay uses parity 0; the reverse walk
    // writes the tape of step n - 1 into the other parity while step n works,
    // so a reverse step needs two barriers
    __shared__ float AA[2][3][NT];
    __shared__ float BB[2][3][NT];
    __shared__ float HB[2][2][3][NT];   // H'-bar, H-bar per loss
    __shared__ double red[NT / 64][10];
    __shared__ float XI[2][3][NT];      // replay noise by step parity (noise threads)
    // per segment: the applied field of steps nA .. nB and the loss weights
    // of steps nA .. nB divided by N (FP32, dynamic, ckpt_every + 1 of each)
    extern __shared__ float seg_tab[];

    const int inst = inst0 + static_cast<int>(blockIdx.x);
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    const int N = L.ncell, nx = L.nx, ny = L.ny, nz = L.nz;
    constexpr bool NP = kAdjThreads<NT> > NT;
    const bool noise_thread = NP && static_cast<int>(threadIdx.x) >= NT;
    const int i = noise_thread ? static_cast<int>(threadIdx.x) - NT : static_cast<int>(threadIdx.x);
    const bool on = i < N && !noise_thread;
    const bool draws = noise_thread && i < N;
    auto draw = [&](int64_t n) {
        const V3 xi = gauss3(philox_cell(I.seed, static_cast<uint32_t>(L.level_tag), kTagNoise,
                                         static_cast<uint32_t>(i), static_cast<uint64_t>(n)));
        XI[n & 1][0][i] = xi.x;
        XI[n & 1][1][i] = xi.y;
        XI[n & 1][2][i] = xi.z;
    };
    const int64_t NS = L.n_steps;
    const int64_t K = ckpt_every;
    const int64_t nseg = (NS + K - 1) / K;
    float* tp = tape + static_cast<int64_t>(blockIdx.x) * K * 9 * N;

    float* s_w0 = seg_tab;                   // weights of loss 0 over N
    float* s_w1 = seg_tab + (K + 1);         // weights of loss 1 over N
    float* s_hz = seg_tab + 2 * (K + 1);
    // step constants in vector registers (a scalar reload inside the step
    // loops would wait on the same counter as the LDS reads)
    const float c_ex = vreg(L.c_ex), hk = vreg(L.hk), g1 = vreg(L.g1), ag1 = vreg(L.ag1);
    const float dt = vreg(L.dt), half_dt = vreg(L.half_dt), sigma = vreg(L.sigma);
    const float inv_g1 = vreg(1.0f / L.g1);
    LevelDev Lc{};
    Lc.c_ex = c_ex;
    Lc.hk = hk;
    Lc.g1 = g1;
    Lc.ag1 = ag1;
    Lc.dt = dt;
    Lc.half_dt = half_dt;

    int ixm = i, ixp = i, iym = i, iyp = i, izm = i, izp = i;
    V3 u = V3{L.ux, L.uy, L.uz};
    if (on) {
        const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        ixm = x > 0 ? i - 1 : i;
        ixp = x < nx - 1 ? i + 1 : i;
        iym = y > 0 ? i - nx : i;
        iyp = y < ny - 1 ? i + nx : i;
        izm = z > 0 ? i - nx * ny : i;
        izp = z < nz - 1 ? i + nx * ny : i;
        if (L.has_axes) {
            const float* a = axes + L.axes_off;
            u = V3{a[i], a[N + i], a[2 * N + i]};
        }
    }
    auto nb = [&](float (*S)[NT], V3 m) {
        return nb_sum(m, v3(S[0][ixm], S[1][ixm], S[2][ixm]), v3(S[0][ixp], S[1][ixp], S[2][ixp]),
                      v3(S[0][iym], S[1][iym], S[2][iym]), v3(S[0][iyp], S[1][iyp], S[2][iyp]),
                      v3(S[0][izm], S[1][izm], S[2][izm]), v3(S[0][izp], S[1][izp], S[2][izp]));
    };
    auto put = [&](float (*S)[NT], V3 v) {
        S[0][i] = v.x;
        S[1][i] = v.y;
        S[2][i] = v.z;
    };

    V3 lam[2];
    for (int l = 0; l < 2; ++l) lam[l] = V3{0.0f, 0.0f, static_cast<float>(w[l * (NS + 1) + NS] / N)};
    double g[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};

    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int64_t nA = seg * K, nB = min(nA + K, NS);
        // ---- the segment's applied fields and loss weights, in parallel
        __syncthreads();
        for (int k = i; k <= nB - nA; k += NT) {
            s_hz[k] = static_cast<float>(L.hz_amp * wave_at(L, nA + k));
            s_w0[k] = static_cast<float>(w[nA + k] / N);
            s_w1[k] = static_cast<float>(w[(NS + 1) + nA + k] / N);
        }
        // ---- forward replay of the segment from its checkpoint
        float (*A)[NT] = AA[0];
        float (*B)[NT] = BB[0];
        V3 m = V3{0, 0, 0};
        if (on) {
            const float* c = ckpt + I.ckpt_off + seg * 3 * static_cast<int64_t>(N);
            m = V3{c[i], c[N + i], c[2 * N + i]};
            put(A, m);
        }
        if (draws) draw(nA);
        __syncthreads();
        for (int64_t n = nA; n < nB; ++n) {
            float* t = tp + (n - nA) * 9 * N;
            V3 q, hth, mp;
            // the noise of step n + 1 (its buffer was last read before the
            // previous step's second barrier)
            if (draws && n + 1 < nB) draw(n + 1);
            if (on) {
                const float hz0 = s_hz[n - nA];
                V3 xi;
                if (NP) {
                    xi = V3{XI[n & 1][0][i], XI[n & 1][1][i], XI[n & 1][2][i]};
                } else {
                    xi = gauss3(philox_cell(I.seed, static_cast<uint32_t>(L.level_tag), kTagNoise,
                                            static_cast<uint32_t>(i), static_cast<uint64_t>(n)));
                }
                hth = V3{sigma * xi.x, sigma * xi.y, sigma * xi.z};
                heun_predict(Lc, m, nb(A, m), u, hz0, hth, mp, q);
                put(B, mp);
                t[i] = m.x;
                t[N + i] = m.y;
                t[2 * N + i] = m.z;
                t[3 * N + i] = mp.x;
                t[4 * N + i] = mp.y;
                t[5 * N + i] = mp.z;
                t[6 * N + i] = xi.x;
                t[7 * N + i] = xi.y;
                t[8 * N + i] = xi.z;
            }
            __syncthreads();
            if (on) {
                const float hz1 = s_hz[n + 1 - nA];
                m = heun_correct(Lc, mp, nb(B, mp), u, hz1, hth, q);
                put(A, m);
            }
            __syncthreads();
        }
        // the tape of the segment's last step in LDS and registers, the step
        // before it in registers: each reverse step puts the tape of the step
        // before it into the other parity and loads the one before that
        auto load_tape = [&](int64_t n, V3& a, V3& b, V3& c) {
            const float* t = tp + (n - nA) * 9 * N;
            a = V3{t[i], t[N + i], t[2 * N + i]};
            b = V3{t[3 * N + i], t[4 * N + i], t[5 * N + i]};
            c = V3{t[6 * N + i], t[7 * N + i], t[8 * N + i]};
        };
        V3 cm = V3{0, 0, 0}, cp = V3{0, 0, 0}, cx = V3{0, 0, 0};   // step n
        V3 tm = V3{0, 0, 0}, tp_ = V3{0, 0, 0}, tx = V3{0, 0, 0};  // step n - 1
        if (on) {
            load_tape(nB - 1, cm, cp, cx);
            put(AA[(nB - 1) & 1], cm);
            put(BB[(nB - 1) & 1], cp);
            if (nB - 1 > nA) load_tape(nB - 2, tm, tp_, tx);
        }
        __syncthreads();
        // ---- reverse walk of the segment
        for (int64_t n = nB - 1; n >= nA; --n) {
            const V3 mm = cm, mp = cp, xi = cx;
            float (*A)[NT] = AA[n & 1];
            float (*B)[NT] = BB[n & 1];
            V3 ex, exq, H, f, Hp, fp, mn, mpb[2], mb[2], fb[2];
            float ip = 0.f, iq = 0.f;
            if (on) {
                const float hz0 = s_hz[n - nA];
                const float hz1 = s_hz[n + 1 - nA];
                const V3 hth = V3{sigma * xi.x, sigma * xi.y, sigma * xi.z};
                ex = nb(A, mm);
                H = eff_field(c_ex, hk, mm, ex, u, hz0, hth);
                f = llg_rhs(g1, ag1, mm, H);
                const V3 pv = V3{fmaf(dt, f.x, mm.x), fmaf(dt, f.y, mm.y), fmaf(dt, f.z, mm.z)};
                ip = __builtin_amdgcn_rsqf(dot3(pv, pv));
                exq = nb(B, mp);
                Hp = eff_field(c_ex, hk, mp, exq, u, hz1, hth);
                fp = llg_rhs(g1, ag1, mp, Hp);
                // q as the forward step forms it: (m + dt/2 f) + dt/2 f'
                const V3 q0 = V3{fmaf(half_dt, f.x, mm.x), fmaf(half_dt, f.y, mm.y), fmaf(half_dt, f.z, mm.z)};
                const V3 qv = V3{fmaf(half_dt, fp.x, q0.x), fmaf(half_dt, fp.y, q0.y), fmaf(half_dt, fp.z, q0.z)};
                iq = __builtin_amdgcn_rsqf(dot3(qv, qv));
                mn = scale3(iq, qv);
                const V3 mxH = cross3(mp, Hp);
                const V3 dmp = cross3(mp, mxH);
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const V3 qb = unit_T(mn, iq, lam[l]);
                    mb[l] = qb;
                    const V3 fpb = scale3(half_dt, qb);
                    fb[l] = fpb;
                    const V3 hpb = rhs_dH_T(g1, ag1, mp, fpb);
                    mpb[l] = rhs_dm_T(g1, ag1, mp, Hp, fpb);
                    g[l][2] += static_cast<double>(dot3(fpb, fp) * inv_g1);
                    g[l][3] += static_cast<double>(-g1 * dot3(fpb, dmp));
                    HB[l][0][0][i] = hpb.x;
                    HB[l][0][1][i] = hpb.y;
                    HB[l][0][2][i] = hpb.z;
                }
                if (n > nA) {
                    put(AA[(n - 1) & 1], tm);
                    put(BB[(n - 1) & 1], tp_);
                    cm = tm;
                    cp = tp_;
                    cx = tx;
                    if (n - 1 > nA) load_tape(n - 2, tm, tp_, tx);
                }
            }
            __syncthreads();
            if (on) {
                const V3 mxH = cross3(mm, H);
                const V3 dm = cross3(mm, mxH);
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    float (*S)[NT] = HB[l][0];
                    const V3 hpb = v3(S[0][i], S[1][i], S[2][i]);
                    const V3 d = nb(S, hpb);
                    const float uh = dot3(u, hpb);
                    V3 v = mpb[l];
                    v.x = fmaf(c_ex, d.x, fmaf(hk * uh, u.x, v.x));
                    v.y = fmaf(c_ex, d.y, fmaf(hk * uh, u.y, v.y));
                    v.z = fmaf(c_ex, d.z, fmaf(hk * uh, u.z, v.z));
                    g[l][0] += static_cast<double>(dot3(hpb, exq));
                    g[l][1] += static_cast<double>(dot3(mp, u) * uh);
                    g[l][4] += static_cast<double>(dot3(hpb, xi));
                    const V3 pb = unit_T(mp, ip, v);
                    mb[l] = add3(mb[l], pb);
                    fb[l] = V3{fmaf(dt, pb.x, fb[l].x), fmaf(dt, pb.y, fb[l].y), fmaf(dt, pb.z, fb[l].z)};
                    const V3 hb = rhs_dH_T(g1, ag1, mm, fb[l]);
                    mb[l] = add3(mb[l], rhs_dm_T(g1, ag1, mm, H, fb[l]));
                    g[l][2] += static_cast<double>(dot3(fb[l], f) * inv_g1);
                    g[l][3] += static_cast<double>(-g1 * dot3(fb[l], dm));
                    HB[l][1][0][i] = hb.x;
                    HB[l][1][1][i] = hb.y;
                    HB[l][1][2][i] = hb.z;
                }
            }
            __syncthreads();
            if (on) {
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    float (*S)[NT] = HB[l][1];
                    const V3 hb = v3(S[0][i], S[1][i], S[2][i]);
                    const V3 d = nb(S, hb);
                    const float uh = dot3(u, hb);
                    V3 v = mb[l];
                    v.x = fmaf(c_ex, d.x, fmaf(hk * uh, u.x, v.x));
                    v.y = fmaf(c_ex, d.y, fmaf(hk * uh, u.y, v.y));
                    v.z = fmaf(c_ex, d.z, fmaf(hk * uh, u.z, v.z));
                    g[l][0] += static_cast<double>(dot3(hb, ex));
                    g[l][1] += static_cast<double>(dot3(mm, u) * uh);
                    g[l][4] += static_cast<double>(dot3(hb, xi));
                    v.z += (l == 0 ? s_w0 : s_w1)[n - nA];
                    lam[l] = v;
                }
            }
            // no barrier: the next step reads m_n, m' of the other parity
            // (written before this step's first barrier), writes the first
            // H-bar buffers (last read before this step's second barrier) and
            // writes the second ones only after its own first barrier
        }
    }
    // ---- FP64 block reduction in fixed order (cell threads)
    const int lane = i & 63, wv = i >> 6;
    if (!noise_thread) {
        for (int l = 0; l < 2; ++l)
            for (int k = 0; k < 5; ++k) {
                const double s = wave_sum_d(g[l][k]);
                if (lane == 0) red[wv][l * 5 + k] = s;
            }
    }
    __syncthreads();
    if (!noise_thread && i < 10) {
        double s = 0.0;
        for (int k = 0; k < NT / 64; ++k) s += red[k][i];
        grads[static_cast<int64_t>(inst) * 10 + i] = s;
    }
}

}  // namespace sllg
