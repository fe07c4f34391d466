// Discrete adjoint of the Heun stochastic-LLG step under fixed noise.
//
// One workgroup per realization, one cell per thread (levels up to 1024
// cells), or two cells per thread for levels of up to 1536 cells.  The sweep is replayed backwards in segments of ckpt_every steps:
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
// threads step the current one.  With KC > 1 every thread owns the cells
// tid + k NT (k < KC) and draws their noise itself (levels of more than 1024
// cells, up to NT KC).
template <int NT, int KC>
constexpr bool kAdjNoiseThreads = KC == 1 && NT <= 256;
template <int NT, int KC = 1>
constexpr int kAdjThreads = kAdjNoiseThreads<NT, KC> ? 2 * NT : NT;

template <int NT, int KC>
__global__ __launch_bounds__((kAdjThreads<NT, KC>)) void k_adjoint(const InstDev* __restrict__ insts, int inst0,
                                                                 const LevelDev* __restrict__ levels,
                                                                 const float* __restrict__ axes,
                                                                 const float* __restrict__ ckpt, int ckpt_every,
                                                                 float* __restrict__ tape,
                                                                 const double* __restrict__ w,
                                                                 double* __restrict__ grads)
{
    constexpr int NC = NT * KC;   // cells a workgroup holds
    constexpr bool NP = kAdjNoiseThreads<NT, KC>;
    // m_n and m' by step parity: the replay uses parity 0; the reverse walk
    // writes the tape of step n - 1 into the other parity while step n works,
    // so a reverse step needs two barriers
    __shared__ float AA[2][3][NC];
    __shared__ float BB[2][3][NC];
    __shared__ float HB[2][2][3][NC];   // H'-bar, H-bar per loss
    __shared__ double red[NT / 64][10];
    __shared__ float XI[2][3][NP ? NT : 1];   // replay noise by step parity (noise threads)
    // per segment: the applied field of steps nA .. nB and the loss weights
    // of steps nA .. nB divided by N (FP32, dynamic, ckpt_every + 1 of each)
    extern __shared__ float seg_tab[];

    const int inst = inst0 + static_cast<int>(blockIdx.x);
    const InstDev I = insts[inst];
    const LevelDev& L = levels[I.level];
    const int N = L.ncell, nx = L.nx, ny = L.ny, nz = L.nz;
    const bool noise_thread = NP && static_cast<int>(threadIdx.x) >= NT;
    const int t = noise_thread ? static_cast<int>(threadIdx.x) - NT : static_cast<int>(threadIdx.x);
    const bool draws = noise_thread && t < N;
    auto draw = [&](int64_t n) {
        const V3 xi = gauss3(philox_cell(I.seed, static_cast<uint32_t>(L.level_tag), kTagNoise,
                                         static_cast<uint32_t>(t), static_cast<uint64_t>(n)));
        XI[n & 1][0][t] = xi.x;
        XI[n & 1][1][t] = xi.y;
        XI[n & 1][2][t] = xi.z;
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

    // the thread's cells
    int ci[KC], ixm[KC], ixp[KC], iym[KC], iyp[KC], izm[KC], izp[KC];
    bool on[KC];
    V3 u[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int i = t + k * NT;
        ci[k] = i;
        on[k] = i < N && !noise_thread;
        ixm[k] = ixp[k] = iym[k] = iyp[k] = izm[k] = izp[k] = i;
        u[k] = V3{L.ux, L.uy, L.uz};
        if (on[k]) {
            const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
            ixm[k] = x > 0 ? i - 1 : i;
            ixp[k] = x < nx - 1 ? i + 1 : i;
            iym[k] = y > 0 ? i - nx : i;
            iyp[k] = y < ny - 1 ? i + nx : i;
            izm[k] = z > 0 ? i - nx * ny : i;
            izp[k] = z < nz - 1 ? i + nx * ny : i;
            if (L.has_axes) {
                const float* a = axes + L.axes_off;
                u[k] = V3{a[i], a[N + i], a[2 * N + i]};
            }
        }
    }
    auto nb = [&](float (*S)[NC], V3 m, int k) {
        return nb_sum(m, v3(S[0][ixm[k]], S[1][ixm[k]], S[2][ixm[k]]), v3(S[0][ixp[k]], S[1][ixp[k]], S[2][ixp[k]]),
                      v3(S[0][iym[k]], S[1][iym[k]], S[2][iym[k]]), v3(S[0][iyp[k]], S[1][iyp[k]], S[2][iyp[k]]),
                      v3(S[0][izm[k]], S[1][izm[k]], S[2][izm[k]]), v3(S[0][izp[k]], S[1][izp[k]], S[2][izp[k]]));
    };
    auto put = [&](float (*S)[NC], int i, V3 v) {
        S[0][i] = v.x;
        S[1][i] = v.y;
        S[2][i] = v.z;
    };

    V3 lam[KC][2];
#pragma unroll
    for (int k = 0; k < KC; ++k)
        for (int l = 0; l < 2; ++l) lam[k][l] = V3{0.0f, 0.0f, static_cast<float>(w[l * (NS + 1) + NS] / N)};
    double g[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};

    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int64_t nA = seg * K, nB = min(nA + K, NS);
        // ---- the segment's applied fields and loss weights, in parallel
        __syncthreads();
        for (int k = t; k <= nB - nA; k += NT) {
            s_hz[k] = static_cast<float>(L.hz_amp * wave_at(L, nA + k));
            s_w0[k] = static_cast<float>(w[nA + k] / N);
            s_w1[k] = static_cast<float>(w[(NS + 1) + nA + k] / N);
        }
        // ---- forward replay of the segment from its checkpoint
        float (*A)[NC] = AA[0];
        float (*B)[NC] = BB[0];
        V3 m[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            m[k] = V3{0, 0, 0};
            if (on[k]) {
                const float* c = ckpt + I.ckpt_off + seg * 3 * static_cast<int64_t>(N);
                m[k] = V3{c[ci[k]], c[N + ci[k]], c[2 * N + ci[k]]};
                put(A, ci[k], m[k]);
            }
        }
        if (draws) draw(nA);
        __syncthreads();
        for (int64_t n = nA; n < nB; ++n) {
            float* tn = tp + (n - nA) * 9 * N;
            V3 q[KC], hth[KC], mp[KC];
            // the noise of step n + 1 (its buffer was last read before the
            // previous step's second barrier)
            if (draws && n + 1 < nB) draw(n + 1);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if (!on[k]) continue;
                const int i = ci[k];
                const float hz0 = s_hz[n - nA];
                V3 xi;
                if (NP) {
                    xi = V3{XI[n & 1][0][i], XI[n & 1][1][i], XI[n & 1][2][i]};
                } else {
                    xi = gauss3(philox_cell(I.seed, static_cast<uint32_t>(L.level_tag), kTagNoise,
                                            static_cast<uint32_t>(i), static_cast<uint64_t>(n)));
                }
                hth[k] = V3{sigma * xi.x, sigma * xi.y, sigma * xi.z};
                heun_predict(Lc, m[k], nb(A, m[k], k), u[k], hz0, hth[k], mp[k], q[k]);
                put(B, i, mp[k]);
                tn[i] = m[k].x;
                tn[N + i] = m[k].y;
                tn[2 * N + i] = m[k].z;
                tn[3 * N + i] = mp[k].x;
                tn[4 * N + i] = mp[k].y;
                tn[5 * N + i] = mp[k].z;
                tn[6 * N + i] = xi.x;
                tn[7 * N + i] = xi.y;
                tn[8 * N + i] = xi.z;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if (!on[k]) continue;
                const float hz1 = s_hz[n + 1 - nA];
                m[k] = heun_correct(Lc, mp[k], nb(B, mp[k], k), u[k], hz1, hth[k], q[k]);
                put(A, ci[k], m[k]);
            }
            __syncthreads();
        }
        // the tape of the segment's last step in LDS and registers, the step
        // before it in registers: each reverse step puts the tape of the step
        // before it into the other parity and loads the one before that
        auto load_tape = [&](int64_t n, int i, V3& a, V3& b, V3& c) {
            const float* tt = tp + (n - nA) * 9 * N;
            a = V3{tt[i], tt[N + i], tt[2 * N + i]};
            b = V3{tt[3 * N + i], tt[4 * N + i], tt[5 * N + i]};
            c = V3{tt[6 * N + i], tt[7 * N + i], tt[8 * N + i]};
        };
        V3 cm[KC], cp[KC], cx[KC];   // step n
        V3 tm[KC], tq[KC], tx[KC];   // step n - 1
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            cm[k] = cp[k] = cx[k] = tm[k] = tq[k] = tx[k] = V3{0, 0, 0};
            if (on[k]) {
                load_tape(nB - 1, ci[k], cm[k], cp[k], cx[k]);
                put(AA[(nB - 1) & 1], ci[k], cm[k]);
                put(BB[(nB - 1) & 1], ci[k], cp[k]);
                if (nB - 1 > nA) load_tape(nB - 2, ci[k], tm[k], tq[k], tx[k]);
            }
        }
        __syncthreads();
        // ---- reverse walk of the segment
        for (int64_t n = nB - 1; n >= nA; --n) {
            float (*A)[NC] = AA[n & 1];
            float (*B)[NC] = BB[n & 1];
            V3 mm[KC], mpk[KC], xik[KC], ex[KC], exq[KC], H[KC], f[KC], mpb[KC][2], mb[KC][2], fb[KC][2];
            float ip[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                mm[k] = cm[k];
                mpk[k] = cp[k];
                xik[k] = cx[k];
                ip[k] = 0.f;
                if (!on[k]) continue;
                const V3 mpc = mpk[k];
                const float hz0 = s_hz[n - nA];
                const float hz1 = s_hz[n + 1 - nA];
                const V3 hth = V3{sigma * xik[k].x, sigma * xik[k].y, sigma * xik[k].z};
                ex[k] = nb(A, mm[k], k);
                H[k] = eff_field(c_ex, hk, mm[k], ex[k], u[k], hz0, hth);
                f[k] = llg_rhs(g1, ag1, mm[k], H[k]);
                const V3 pv = V3{fmaf(dt, f[k].x, mm[k].x), fmaf(dt, f[k].y, mm[k].y), fmaf(dt, f[k].z, mm[k].z)};
                ip[k] = __builtin_amdgcn_rsqf(dot3(pv, pv));
                exq[k] = nb(B, mpc, k);
                const V3 Hp = eff_field(c_ex, hk, mpc, exq[k], u[k], hz1, hth);
                const V3 fp = llg_rhs(g1, ag1, mpc, Hp);
                // q as the forward step forms it: (m + dt/2 f) + dt/2 f'
                const V3 q0 = V3{fmaf(half_dt, f[k].x, mm[k].x), fmaf(half_dt, f[k].y, mm[k].y),
                                 fmaf(half_dt, f[k].z, mm[k].z)};
                const V3 qv = V3{fmaf(half_dt, fp.x, q0.x), fmaf(half_dt, fp.y, q0.y), fmaf(half_dt, fp.z, q0.z)};
                const float iq = __builtin_amdgcn_rsqf(dot3(qv, qv));
                const V3 mn = scale3(iq, qv);
                const V3 mxH = cross3(mpc, Hp);
                const V3 dmp = cross3(mpc, mxH);
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const V3 qb = unit_T(mn, iq, lam[k][l]);
                    mb[k][l] = qb;
                    const V3 fpb = scale3(half_dt, qb);
                    fb[k][l] = fpb;
                    const V3 hpb = rhs_dH_T(g1, ag1, mpc, fpb);
                    mpb[k][l] = rhs_dm_T(g1, ag1, mpc, Hp, fpb);
                    g[l][2] += static_cast<double>(dot3(fpb, fp) * inv_g1);
                    g[l][3] += static_cast<double>(-g1 * dot3(fpb, dmp));
                    HB[l][0][0][ci[k]] = hpb.x;
                    HB[l][0][1][ci[k]] = hpb.y;
                    HB[l][0][2][ci[k]] = hpb.z;
                }
                if (n > nA) {
                    put(AA[(n - 1) & 1], ci[k], tm[k]);
                    put(BB[(n - 1) & 1], ci[k], tq[k]);
                    cm[k] = tm[k];
                    cp[k] = tq[k];
                    cx[k] = tx[k];
                    if (n - 1 > nA) load_tape(n - 2, ci[k], tm[k], tq[k], tx[k]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if (!on[k]) continue;
                const V3 mxH = cross3(mm[k], H[k]);
                const V3 dm = cross3(mm[k], mxH);
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    float (*S)[NC] = HB[l][0];
                    const V3 hpb = v3(S[0][ci[k]], S[1][ci[k]], S[2][ci[k]]);
                    const V3 d = nb(S, hpb, k);
                    const float uh = dot3(u[k], hpb);
                    V3 v = mpb[k][l];
                    v.x = fmaf(c_ex, d.x, fmaf(hk * uh, u[k].x, v.x));
                    v.y = fmaf(c_ex, d.y, fmaf(hk * uh, u[k].y, v.y));
                    v.z = fmaf(c_ex, d.z, fmaf(hk * uh, u[k].z, v.z));
                    g[l][0] += static_cast<double>(dot3(hpb, exq[k]));
                    g[l][1] += static_cast<double>(dot3(mpk[k], u[k]) * uh);
                    g[l][4] += static_cast<double>(dot3(hpb, xik[k]));
                    const V3 pb = unit_T(mpk[k], ip[k], v);
                    mb[k][l] = add3(mb[k][l], pb);
                    fb[k][l] = V3{fmaf(dt, pb.x, fb[k][l].x), fmaf(dt, pb.y, fb[k][l].y), fmaf(dt, pb.z, fb[k][l].z)};
                    const V3 hb = rhs_dH_T(g1, ag1, mm[k], fb[k][l]);
                    mb[k][l] = add3(mb[k][l], rhs_dm_T(g1, ag1, mm[k], H[k], fb[k][l]));
                    g[l][2] += static_cast<double>(dot3(fb[k][l], f[k]) * inv_g1);
                    g[l][3] += static_cast<double>(-g1 * dot3(fb[k][l], dm));
                    HB[l][1][0][ci[k]] = hb.x;
                    HB[l][1][1][ci[k]] = hb.y;
                    HB[l][1][2][ci[k]] = hb.z;
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if (!on[k]) continue;
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    float (*S)[NC] = HB[l][1];
                    const V3 hb = v3(S[0][ci[k]], S[1][ci[k]], S[2][ci[k]]);
                    const V3 d = nb(S, hb, k);
                    const float uh = dot3(u[k], hb);
                    V3 v = mb[k][l];
                    v.x = fmaf(c_ex, d.x, fmaf(hk * uh, u[k].x, v.x));
                    v.y = fmaf(c_ex, d.y, fmaf(hk * uh, u[k].y, v.y));
                    v.z = fmaf(c_ex, d.z, fmaf(hk * uh, u[k].z, v.z));
                    g[l][0] += static_cast<double>(dot3(hb, ex[k]));
                    g[l][1] += static_cast<double>(dot3(mm[k], u[k]) * uh);
                    g[l][4] += static_cast<double>(dot3(hb, xik[k]));
                    v.z += (l == 0 ? s_w0 : s_w1)[n - nA];
                    lam[k][l] = v;
                }
            }
            // no barrier: the next step reads m_n, m' of the other parity
            // (written before this step's first barrier), writes the first
            // H-bar buffers (last read before this step's second barrier) and
            // writes the second ones only after its own first barrier
        }
    }
    // ---- FP64 block reduction in fixed order (cell threads)
    const int lane = t & 63, wv = t >> 6;
    if (!noise_thread) {
        for (int l = 0; l < 2; ++l)
            for (int k = 0; k < 5; ++k) {
                const double sum = wave_sum_d(g[l][k]);
                if (lane == 0) red[wv][l * 5 + k] = sum;
            }
    }
    __syncthreads();
    if (!noise_thread && t < 10) {
        double sum = 0.0;
        for (int k = 0; k < NT / 64; ++k) sum += red[k][t];
        grads[static_cast<int64_t>(inst) * 10 + t] = sum;
    }
}

}  // namespace sllg
