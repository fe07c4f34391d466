/*
 * FP64 CPU oracle for the stochastic Landau-Lifshitz-Gilbert hysteresis-loop
 * path of Behbahani, Plumer and Saika-Voivod, "Coarse-graining in
 * micromagnetic simulations of dynamic hysteresis loops" (arXiv:1912.00310).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  It shares no code with the product library
 * and may only be built and called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.
 *
 * Everything is IEEE double.  State layout is array-of-structs: m[3*i + c]
 * for cell i = x + nx*(y + ny*z), component c in {x, y, z}.
 *
 * What is computed (paper section / equation in brackets):
 *   - Philox4x32-10 counter RNG (Salmon, Moraes, Dror, Shaw, SC'11) and the
 *     Box-Muller transform (Box and Muller 1958) for the Brown thermal field
 *     [text under Eq. 1, "stochastic thermal field"];
 *   - the effective field: 6-neighbour exchange with free boundaries,
 *     uniaxial anisotropy, swept Zeeman field along z, thermal field
 *     [material paragraph; Eq. 1];
 *   - the Landau-Lifshitz form of the LLG equation [Eq. 1] stepped by the
 *     Heun predictor-corrector with the noise held over both stages and |m|
 *     renormalised after each stage;
 *   - the loop ordinate m_H = mean over cells of m_z [text after Eq. 1];
 *   - loop area, coercive field and remanence [loop-area paragraph, Fig. 2];
 *   - the discrete adjoint of the Heun step under fixed noise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Level description: every FP64 constant one grid needs. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t level_tag;     /* enters the RNG counter */
    double c_ex;           /* A/m: 2A/(mu0 Ms a^2) */
    double hk;             /* A/m: 2K/(mu0 Ms) */
    double gamma1;         /* m/(A s): gamma0/(1+alpha^2) */
    double alpha;
    double sigma;          /* A/m: thermal-field standard deviation per component */
    double dt;             /* s */
    double hz_amp;         /* A/m: peak applied field */
    int64_t n_period;      /* steps per field cycle */
    int32_t wave;          /* 0 triangle, 1 cosine, 2 constant */
    double axis[3];        /* easy axis (unit) */
    double cone_deg;       /* > 0: per-cell axes in a uniform cone about axis */
    uint64_t axis_seed;
    double demag_ms;       /* A/m: Ms of the magnetostatic field; 0 = none */
} orc_level;

enum { ORC_TAG_NOISE = 1, ORC_TAG_AXIS = 2 };

/* ------------------------------------------------------------------------ */
/* Philox: one round structure, instantiated for 32- and 64-bit words.       */
/* Each round multiplies counter words 0 and 2 by the round multipliers,     */
/* takes high halves xor the other two words and the key, keeps low halves,  */
/* then adds the Weyl increments to the key.                                 */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX4_10(NAME, U, UW, BITS, M0, M1, W0, W1)                     \
    void NAME(const U ctr[4], const U key[2], U out[4])                       \
    {                                                                         \
        U c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];                 \
        U k0 = key[0], k1 = key[1];                                           \
        for (int r = 0; r < 10; ++r) {                                        \
            UW p0 = (UW)(M0) * (UW)c0;                                        \
            UW p1 = (UW)(M1) * (UW)c2;                                        \
            U hi0 = (U)(p0 >> (BITS)), lo0 = (U)p0;                           \
            U hi1 = (U)(p1 >> (BITS)), lo1 = (U)p1;                           \
            U n0 = hi1 ^ c1 ^ k0;                                             \
            U n2 = hi0 ^ c3 ^ k1;                                             \
            c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;                             \
            k0 = (U)(k0 + (U)(W0));                                           \
            k1 = (U)(k1 + (U)(W1));                                           \
        }                                                                     \
        out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;                   \
    }

ORC_PHILOX4_10(orc_philox4x32_10, uint32_t, uint64_t, 32,
               0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
ORC_PHILOX4_10(orc_philox4x64_10, uint64_t, unsigned __int128, 64,
               0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
               0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* Counter layout: key = seed (low, high words); counter = (cell, step low,
 * step bits 32..47 | level << 16 | tag << 24, 0). */
void orc_philox_cell(uint64_t seed, uint32_t level, uint32_t tag,
                     uint32_t cell, uint64_t step, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {cell, (uint32_t)step,
                       ((uint32_t)(step >> 32) & 0xFFFFu) | ((level & 0xFFu) << 16) |
                           ((tag & 0xFFu) << 24),
                       0u};
    orc_philox4x32_10(ctr, key, out);
}

/* 23-bit uniform on (0,1): u = (2*(x >> 9) + 1) * 2^-24, exact in FP32. */
static double uniform23(uint32_t x)
{
    return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0);
}

void orc_uniforms(uint64_t seed, uint32_t level, uint32_t tag, uint32_t cell,
                  uint64_t step, double u[4])
{
    uint32_t r[4];
    orc_philox_cell(seed, level, tag, cell, step, r);
    for (int k = 0; k < 4; ++k) u[k] = uniform23(r[k]);
}

/* Box-Muller: (u0,u1) -> two normals, (u2,u3) -> one (cosine branch). */
void orc_normals(uint64_t seed, uint32_t level, uint32_t cell, uint64_t step,
                 double xi[3])
{
    double u[4];
    orc_uniforms(seed, level, ORC_TAG_NOISE, cell, step, u);
    double r0 = sqrt(-2.0 * log(u[0]));
    double r2 = sqrt(-2.0 * log(u[2]));
    xi[0] = r0 * cos(2.0 * M_PI * u[1]);
    xi[1] = r0 * sin(2.0 * M_PI * u[1]);
    xi[2] = r2 * cos(2.0 * M_PI * u[3]);
}

/* Per-cell easy axes: cos(theta) uniform in [cos(theta_max), 1], phi uniform,
 * drawn about +z and then rotated so that +z lands on the level's axis. */
void orc_make_axes(const orc_level* L, double* u)
{
    int64_t n = (int64_t)L->nx * L->ny * L->nz;
    double e[3] = {L->axis[0], L->axis[1], L->axis[2]};
    double en = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    for (int c = 0; c < 3; ++c) e[c] /= en;
    /* rotation matrix R with R z = e (Rodrigues about z x e) */
    double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double s = sqrt(e[0] * e[0] + e[1] * e[1]); /* |z x e| */
    if (s > 0.0) {
        double k[3] = {-e[1] / s, e[0] / s, 0.0}; /* unit z x e */
        double ct = e[2], st = s;
        double K[3][3] = {{0, -k[2], k[1]}, {k[2], 0, -k[0]}, {-k[1], k[0], 0}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double kk = 0.0;
                for (int l = 0; l < 3; ++l) kk += K[i][l] * K[l][j];
                R[i][j] = (i == j ? 1.0 : 0.0) + st * K[i][j] + (1.0 - ct) * kk;
            }
    } else if (e[2] < 0.0) {
        R[1][1] = -1.0; R[2][2] = -1.0; /* pi about x */
    }
    double cmin = cos(L->cone_deg * M_PI / 180.0);
    for (int64_t i = 0; i < n; ++i) {
        double v[3];
        if (L->cone_deg > 0.0) {
            double r[4];
            orc_uniforms(L->axis_seed, (uint32_t)L->level_tag, ORC_TAG_AXIS,
                         (uint32_t)i, 0, r);
            double ctheta = 1.0 - r[0] * (1.0 - cmin);
            double stheta = sqrt(fmax(0.0, 1.0 - ctheta * ctheta));
            double phi = 2.0 * M_PI * r[1];
            v[0] = stheta * cos(phi);
            v[1] = stheta * sin(phi);
            v[2] = ctheta;
        } else {
            v[0] = 0.0; v[1] = 0.0; v[2] = 1.0;
        }
        for (int c = 0; c < 3; ++c)
            u[3 * i + c] = R[c][0] * v[0] + R[c][1] * v[1] + R[c][2] * v[2];
    }
}

/* Applied field along z at step n, A/m.  Triangle: +peak -> -peak -> +peak
 * over one period at constant rate; cosine: peak*cos(2 pi n/N). */
double orc_applied_field(const orc_level* L, int64_t n)
{
    int64_t N = L->n_period;
    int64_t k = n % N;
    double s = (double)k / (double)N;
    double v;
    switch (L->wave) {
    case 0: v = (2 * k <= N) ? 1.0 - 4.0 * s : 4.0 * s - 3.0; break;
    case 1: v = cos(2.0 * M_PI * s); break;
    default: v = 1.0; break;
    }
    return L->hz_amp * v;
}

/* ------------------------------------------------------------------------ */
/* Effective field and the right-hand side of Eq. (1)                        */
/* ------------------------------------------------------------------------ */

static const double* axis_of(const orc_level* L, const double* u, int64_t i)
{
    return u ? u + 3 * i : L->axis;
}

/* Sum over existing face neighbours of (v_j - v_i); free boundaries. */
static void neighbour_diff(const orc_level* L, const double* v, int x, int y,
                           int z, double out[3])
{
    int64_t nx = L->nx, ny = L->ny, nz = L->nz;
    int64_t i = x + nx * (y + ny * z);
    out[0] = out[1] = out[2] = 0.0;
    int64_t nb[6];
    int cnt = 0;
    if (x > 0) nb[cnt++] = i - 1;
    if (x < nx - 1) nb[cnt++] = i + 1;
    if (y > 0) nb[cnt++] = i - nx;
    if (y < ny - 1) nb[cnt++] = i + nx;
    if (z > 0) nb[cnt++] = i - nx * ny;
    if (z < nz - 1) nb[cnt++] = i + nx * ny;
    for (int k = 0; k < cnt; ++k)
        for (int c = 0; c < 3; ++c) out[c] += v[3 * nb[k] + c] - v[3 * i + c];
}

/* Grids of at least this many cells spread their per-cell loops over the
 * OpenMP threads (each cell is computed independently, so the result does not
 * depend on the thread count).  Inside a parallel region over realizations
 * these loops run on the calling thread only (no nested parallelism).
 * Smaller grids never enter a parallel region (even an inactive one costs
 * about a microsecond, more than a single cell's step). */
#define ORC_CELL_PAR 65536

/* for (int64_t VAR = 0; VAR < N; ++VAR) { BODY }, over the threads when BIG */
#ifdef _OPENMP
#define ORC_LOOP(BIG, N, VAR, ...)                                            \
    do {                                                                      \
        if (BIG) {                                                            \
            _Pragma("omp parallel for schedule(static)")                      \
            for (int64_t VAR = 0; VAR < (N); ++VAR) { __VA_ARGS__ }           \
        } else {                                                              \
            for (int64_t VAR = 0; VAR < (N); ++VAR) { __VA_ARGS__ }           \
        }                                                                     \
    } while (0)
#else
#define ORC_LOOP(BIG, N, VAR, ...)                                            \
    do { for (int64_t VAR = 0; VAR < (N); ++VAR) { __VA_ARGS__ } } while (0)
#endif

/* ------------------------------------------------------------------------ */
/* Magnetostatic (demagnetising) field of uniformly magnetised cubic cells     */
/* ------------------------------------------------------------------------ */
/* Beyond the paper (it leaves magnetostatics out and folds shape anisotropy
 * into K, material paragraph and closing discussion).  The field of cell j on
 * cell i, averaged over cell i, is -Ms N(r_i - r_j) m_j with N the demagnetising
 * tensor of two cubes (Newell, Williams and Dunlop, J. Geophys. Res. 98, 9551
 * (1993)): N_xx = -(1/(4 pi V)) D2x D2y D2z f and N_xy = -(1/(4 pi V)) D2 D2
 * D2 g, where D2 is the second difference (h(s + a) - 2 h(s) + h(s - a)) in
 * each coordinate and f, g are Newell's closed-form double integrals below.
 * Lengths are in units of the cell edge (V = 1).  Long double: the 27 terms
 * of the stencil cancel to ~r^-3 from values ~r^2. */
typedef long double ld;

static ld newell_f(ld x, ld y, ld z)
{
    x = fabsl(x); y = fabsl(y); z = fabsl(z);
    ld x2 = x * x, y2 = y * y, z2 = z * z;
    ld R = sqrtl(x2 + y2 + z2);
    ld r = (2 * x2 - y2 - z2) * R / 6;
    if (y > 0 && x2 + z2 > 0) r += y / 2 * (z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (z > 0 && x2 + y2 > 0) r += z / 2 * (y2 - x2) * asinhl(z / sqrtl(x2 + y2));
    if (x > 0 && y > 0 && z > 0) r -= x * y * z * atanl(y * z / (x * R));
    return r;
}

static ld newell_g(ld x, ld y, ld z)
{
    ld sg = ((x < 0) != (y < 0)) ? -1 : 1;
    x = fabsl(x); y = fabsl(y); z = fabsl(z);
    ld x2 = x * x, y2 = y * y, z2 = z * z;
    ld R = sqrtl(x2 + y2 + z2);
    ld r = -x * y * R / 3;
    if (x > 0 && y > 0 && z > 0) r += x * y * z * asinhl(z / sqrtl(x2 + y2));
    if (y > 0 && y2 + z2 > 0 && x > 0) r += y / 6 * (3 * z2 - y2) * asinhl(x / sqrtl(y2 + z2));
    if (x > 0 && x2 + z2 > 0 && y > 0) r += x / 6 * (3 * z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (z > 0 && x > 0 && y > 0) r -= z * z2 / 6 * atanl(x * y / (z * R));
    if (z > 0 && y > 0 && x > 0) r -= z * y2 / 2 * atanl(x * z / (y * R));
    if (z > 0 && x > 0 && y > 0) r -= z * x2 / 2 * atanl(y * z / (x * R));
    return sg * r;
}

/* -(1/4pi) sum over the 27-point stencil with weights (1, -2, 1)^3 */
static ld newell_stencil(ld (*fn)(ld, ld, ld), ld X, ld Y, ld Z)
{
    static const ld w[3] = {1, -2, 1};
    ld acc = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                acc += w[i] * w[j] * w[k] * fn(X + i - 1, Y + j - 1, Z + k - 1);
    return -acc / (4 * (ld)M_PI);
}

/* The tensor for integer offsets (X, Y, Z) in cell edges: out = xx, yy, zz,
 * xy, xz, yz (symmetric). */
void orc_newell(int X, int Y, int Z, double out[6])
{
    out[0] = (double)newell_stencil(newell_f, X, Y, Z);
    out[1] = (double)newell_stencil(newell_f, Y, X, Z);
    out[2] = (double)newell_stencil(newell_f, Z, Y, X);
    out[3] = (double)newell_stencil(newell_g, X, Y, Z);
    out[4] = (double)newell_stencil(newell_g, X, Z, Y);
    out[5] = (double)newell_stencil(newell_g, Y, Z, X);
}

/* Table of N for every offset between two cells of the grid:
 * T[6 * (((dz + nz - 1) * (2 ny - 1) + dy + ny - 1) * (2 nx - 1) + dx + nx - 1) + c]. */
void orc_demag_tensor(const orc_level* L, double* T)
{
    int64_t wx = 2 * L->nx - 1, wy = 2 * L->ny - 1, wz = 2 * L->nz - 1;
    for (int64_t k = 0; k < wz; ++k)
        for (int64_t j = 0; j < wy; ++j)
            for (int64_t i = 0; i < wx; ++i)
                orc_newell((int)(i - L->nx + 1), (int)(j - L->ny + 1), (int)(k - L->nz + 1),
                           T + 6 * ((k * wy + j) * wx + i));
}

static double* demag_table(const orc_level* L)
{
    if (L->demag_ms == 0.0) return NULL;
    int64_t n = (2 * (int64_t)L->nx - 1) * (2 * L->ny - 1) * (2 * L->nz - 1);
    double* T = (double*)malloc(sizeof(double) * 6 * (size_t)n);
    if (T) orc_demag_tensor(L, T);
    return T;
}

/* Hd_i = -Ms sum_j N(r_i - r_j) m_j, a plain double sum over all cells */
static void demag_field(const orc_level* L, const double* T, const double* m, double* Hd)
{
    int64_t nx = L->nx, ny = L->ny, nz = L->nz, N = nx * ny * nz;
    int64_t wx = 2 * nx - 1, wy = 2 * ny - 1;
    ORC_LOOP(N >= ORC_CELL_PAR, N, i,
        int64_t xi = i % nx, yi = (i / nx) % ny, zi = i / (nx * ny);
        double h[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            int64_t xj = j % nx, yj = (j / nx) % ny, zj = j / (nx * ny);
            const double* t = T + 6 * (((zi - zj + nz - 1) * wy + yi - yj + ny - 1) * wx + xi - xj + nx - 1);
            const double* v = m + 3 * j;
            h[0] += t[0] * v[0] + t[3] * v[1] + t[4] * v[2];
            h[1] += t[3] * v[0] + t[1] * v[1] + t[5] * v[2];
            h[2] += t[4] * v[0] + t[5] * v[1] + t[2] * v[2];
        }
        for (int c = 0; c < 3; ++c) Hd[3 * i + c] = -L->demag_ms * h[c];
    );
}

static void effective_field_t(const orc_level* L, const double* u, const double* m,
                              double hz, const double* hth, double* H, const double* T);

void orc_effective_field(const orc_level* L, const double* u, const double* m,
                         double hz, const double* hth, double* H)
{
    double* T = demag_table(L);
    effective_field_t(L, u, m, hz, hth, H, T);
    free(T);
}

static void effective_field_t(const orc_level* L, const double* u, const double* m,
                              double hz, const double* hth, double* H, const double* T)
{
    const int big = (int64_t)L->nx * L->ny * L->nz >= ORC_CELL_PAR;
    ORC_LOOP(big, L->nz, zz,
        const int z = (int)zz;
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                int64_t i = x + (int64_t)L->nx * (y + (int64_t)L->ny * z);
                double ex[3];
                neighbour_diff(L, m, x, y, z, ex);
                const double* a = axis_of(L, u, i);
                const double* mi = m + 3 * i;
                double d = mi[0] * a[0] + mi[1] * a[1] + mi[2] * a[2];
                for (int c = 0; c < 3; ++c)
                    H[3 * i + c] = L->c_ex * ex[c] + L->hk * d * a[c] +
                                   (hth ? hth[3 * i + c] : 0.0);
                H[3 * i + 2] += hz;
            }
    );
    if (T) {
        int64_t N = (int64_t)L->nx * L->ny * L->nz;
        double* Hd = (double*)malloc(sizeof(double) * 3 * (size_t)N);
        if (!Hd) return;
        demag_field(L, T, m, Hd);
        for (int64_t k = 0; k < 3 * N; ++k) H[k] += Hd[k];
        free(Hd);
    }
}

static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Eq. (1) divided by Ms: f = -gamma1 m x H - alpha gamma1 m x (m x H). */
static void llg_rhs(const orc_level* L, const double m[3], const double H[3],
                    double f[3])
{
    double mxH[3], mxmxH[3];
    cross(m, H, mxH);
    cross(m, mxH, mxmxH);
    for (int c = 0; c < 3; ++c)
        f[c] = -L->gamma1 * mxH[c] - L->alpha * L->gamma1 * mxmxH[c];
}

/* Thermal field sigma*xi for every cell at step n. */
static void thermal_field(const orc_level* L, uint64_t seed, int64_t n,
                          double* hth, double* xi_out)
{
    int64_t N = (int64_t)L->nx * L->ny * L->nz;
    ORC_LOOP(N >= ORC_CELL_PAR, N, i,
        double xi[3] = {0.0, 0.0, 0.0};
        if (L->sigma != 0.0 || xi_out)
            orc_normals(seed, (uint32_t)L->level_tag, (uint32_t)i, (uint64_t)n, xi);
        for (int c = 0; c < 3; ++c) {
            hth[3 * i + c] = L->sigma * xi[c];
            if (xi_out) xi_out[3 * i + c] = xi[c];
        }
    );
}

/* Scratch for one step of one grid. */
typedef struct {
    double *hth, *xi, *H, *f, *mp, *Hp, *fp, *pn, *qn;
    double* demag;   /* tensor table when the level has magnetostatics */
} step_ws;

static int ws_alloc(step_ws* w, const orc_level* L)
{
    int64_t N = (int64_t)L->nx * L->ny * L->nz;
    double* blk = (double*)malloc(sizeof(double) * (size_t)(3 * N * 7 + 2 * N));
    if (!blk) return -1;
    w->demag = demag_table(L);
    if (L->demag_ms != 0.0 && !w->demag) { free(blk); return -1; }
    w->hth = blk;
    w->xi = blk + 3 * N;
    w->H = blk + 6 * N;
    w->f = blk + 9 * N;
    w->mp = blk + 12 * N;
    w->Hp = blk + 15 * N;
    w->fp = blk + 18 * N;
    w->pn = blk + 21 * N;
    w->qn = blk + 22 * N;
    return 0;
}

static void ws_free(step_ws* w) { free(w->hth); free(w->demag); }

/* One Heun step n -> n+1.  Predictor with the field at t_n, corrector with
 * the field at t_{n+1}; the same thermal field in both stages; |m| = 1 is
 * restored after each stage.  Fills the workspace with every intermediate. */
static void heun_step_ws(const orc_level* L, const double* u, uint64_t seed,
                         int64_t n, const double* m, double* m_out, step_ws* w)
{
    int64_t N = (int64_t)L->nx * L->ny * L->nz;
    double hz0 = orc_applied_field(L, n);
    double hz1 = orc_applied_field(L, n + 1);
    thermal_field(L, seed, n, w->hth, w->xi);
    effective_field_t(L, u, m, hz0, w->hth, w->H, w->demag);
    const int big = N >= ORC_CELL_PAR;
    ORC_LOOP(big, N, i,
        llg_rhs(L, m + 3 * i, w->H + 3 * i, w->f + 3 * i);
        double p[3];
        for (int c = 0; c < 3; ++c) p[c] = m[3 * i + c] + L->dt * w->f[3 * i + c];
        double pn = sqrt(dot3(p, p));
        w->pn[i] = pn;
        for (int c = 0; c < 3; ++c) w->mp[3 * i + c] = p[c] / pn;
    );
    effective_field_t(L, u, w->mp, hz1, w->hth, w->Hp, w->demag);
    ORC_LOOP(big, N, i,
        llg_rhs(L, w->mp + 3 * i, w->Hp + 3 * i, w->fp + 3 * i);
        double q[3];
        for (int c = 0; c < 3; ++c)
            q[c] = m[3 * i + c] + 0.5 * L->dt * (w->f[3 * i + c] + w->fp[3 * i + c]);
        double qn = sqrt(dot3(q, q));
        w->qn[i] = qn;
        for (int c = 0; c < 3; ++c) m_out[3 * i + c] = q[c] / qn;
    );
}

int orc_heun_step(const orc_level* L, const double* u, uint64_t seed, int64_t n,
                  const double* m, double* m_out)
{
    step_ws w;
    if (ws_alloc(&w, L)) return -1;
    heun_step_ws(L, u, seed, n, m, m_out, &w);
    ws_free(&w);
    return 0;
}

static double mean_mz(const double* m, int64_t N)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += m[3 * i + 2];
    return s / (double)N;
}

/* Reduced energy e = E/(mu0 Ms V) for a constant applied field hz along z:
 * e = -sum m.H_app - (hk/2) sum (m.u)^2 + (c_ex/2) sum_<ij> |m_i - m_j|^2
 *     (+ (Ms/2) sum_ij m_i . N(r_i - r_j) m_j with magnetostatics). */
double orc_energy(const orc_level* L, const double* u, const double* m, double hz)
{
    int64_t nx = L->nx, ny = L->ny, nz = L->nz;
    double e = 0.0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = x + nx * (y + ny * z);
                const double* a = axis_of(L, u, i);
                const double* mi = m + 3 * i;
                double d = dot3(mi, a);
                e += -mi[2] * hz - 0.5 * L->hk * d * d;
                int64_t nb[3];
                int cnt = 0;
                if (x < nx - 1) nb[cnt++] = i + 1;
                if (y < ny - 1) nb[cnt++] = i + nx;
                if (z < nz - 1) nb[cnt++] = i + nx * ny;
                for (int k = 0; k < cnt; ++k) {
                    double dd = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        double df = mi[c] - m[3 * nb[k] + c];
                        dd += df * df;
                    }
                    e += 0.5 * L->c_ex * dd;
                }
            }
    if (L->demag_ms != 0.0) {
        /* magnetostatic self-energy e = -(1/2) sum_i m_i . Hd_i */
        int64_t N = nx * ny * nz;
        double* T = demag_table(L);
        double* Hd = (double*)malloc(sizeof(double) * 3 * (size_t)N);
        if (!T || !Hd) { free(T); free(Hd); return NAN; }
        demag_field(L, T, m, Hd);
        for (int64_t i = 0; i < N; ++i) e -= 0.5 * dot3(m + 3 * i, Hd + 3 * i);
        free(T);
        free(Hd);
    }
    return e;
}

/* Run steps n0 .. n0+nsteps-1 of one realization in place.  mbar (optional,
 * nsteps+1 entries) receives the loop ordinate before the first and after
 * every step. */
int orc_run(const orc_level* L, const double* u, uint64_t seed, int64_t n0,
            int64_t nsteps, double* m, double* mbar)
{
    int64_t N = (int64_t)L->nx * L->ny * L->nz;
    step_ws w;
    if (ws_alloc(&w, L)) return -1;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)(3 * N));
    if (!tmp) { ws_free(&w); return -1; }
    if (mbar) mbar[0] = mean_mz(m, N);
    for (int64_t s = 0; s < nsteps; ++s) {
        heun_step_ws(L, u, seed, n0 + s, m, tmp, &w);
        memcpy(m, tmp, sizeof(double) * (size_t)(3 * N));
        if (mbar) mbar[s + 1] = mean_mz(m, N);
    }
    free(tmp);
    ws_free(&w);
    return 0;
}

/* Many realizations from the all-+z state.  With at least as many
 * realizations as threads, one thread per realization; with fewer, the
 * realizations run one after another and each step's cell loops use all
 * threads.  Either way every realization's arithmetic is the same.
 * mbar: nreal x (nsteps+1); m_final (optional): nreal x 3N. */
int orc_run_batch(const orc_level* L, const double* u, const uint64_t* seeds,
                  int32_t nreal, int64_t nsteps, double* mbar, double* m_final,
                  int32_t nthreads)
{
    int64_t N = (int64_t)L->nx * L->ny * L->nz;
    int err = 0;
    int per_real = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    per_real = nreal >= omp_get_max_threads() || N < ORC_CELL_PAR;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err) if (per_real)
#endif
    for (int32_t r = 0; r < nreal; ++r) {
        double* m = (double*)malloc(sizeof(double) * (size_t)(3 * N));
        if (!m) { err |= 1; continue; }
        for (int64_t i = 0; i < N; ++i) {
            m[3 * i] = 0.0; m[3 * i + 1] = 0.0; m[3 * i + 2] = 1.0;
        }
        err |= orc_run(L, u, seeds[r], 0, nsteps, m,
                       mbar ? mbar + (int64_t)r * (nsteps + 1) : NULL);
        if (m_final) memcpy(m_final + (int64_t)r * 3 * N, m, sizeof(double) * (size_t)(3 * N));
        free(m);
    }
    return err ? -1 : 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Loop analytics                                                             */
/* ------------------------------------------------------------------------ */
/* out[0]  S   = -sum 1/2 (m_k + m_{k+1}) (H_{k+1} - H_k)   (trapezoid)
 * out[1]  H* on the descending branch: first k with H falling and
 *         m_k > 0 >= m_{k+1}, linear interpolation   (NaN if none)
 * out[2]  H* on the ascending branch: first k with H rising and
 *         m_k < 0 <= m_{k+1}                           (NaN if none)
 * out[3]  Hc = (H*_asc - H*_desc)/2
 * out[4]  Mr = (m(H=0 falling) - m(H=0 rising))/2, linear interpolation
 * out[5]  sign changes of m on falling segments
 * out[6]  sign changes of m on rising segments
 * out[7]  k of the selected falling crossing (-1 if none)
 * out[8]  k of the selected rising crossing (-1 if none)
 * out[9]  m at H = 0 on the falling branch, out[10] on the rising branch */
void orc_loop_stats(const double* H, const double* m, int64_t npts, double* out)
{
    double S = 0.0;
    double hd = NAN, ha = NAN, md0 = NAN, ma0 = NAN;
    int64_t kd = -1, ka = -1, nd = 0, na = 0;
    for (int64_t k = 0; k + 1 < npts; ++k) {
        double dH = H[k + 1] - H[k];
        S -= 0.5 * (m[k] + m[k + 1]) * dH;
        int change = (m[k] > 0.0) != (m[k + 1] > 0.0);
        if (dH < 0.0) {
            nd += change;
            if (kd < 0 && m[k] > 0.0 && m[k + 1] <= 0.0) {
                kd = k;
                hd = H[k] - m[k] * dH / (m[k + 1] - m[k]);
            }
            if (isnan(md0) && H[k] > 0.0 && H[k + 1] <= 0.0)
                md0 = m[k] + (m[k + 1] - m[k]) * (0.0 - H[k]) / dH;
        } else if (dH > 0.0) {
            na += change;
            if (ka < 0 && m[k] < 0.0 && m[k + 1] >= 0.0) {
                ka = k;
                ha = H[k] - m[k] * dH / (m[k + 1] - m[k]);
            }
            if (isnan(ma0) && H[k] < 0.0 && H[k + 1] >= 0.0)
                ma0 = m[k] + (m[k + 1] - m[k]) * (0.0 - H[k]) / dH;
        }
    }
    out[0] = S;
    out[1] = hd;
    out[2] = ha;
    out[3] = 0.5 * (ha - hd);
    out[4] = 0.5 * (md0 - ma0);
    out[5] = (double)nd;
    out[6] = (double)na;
    out[7] = (double)kd;
    out[8] = (double)ka;
    out[9] = md0;
    out[10] = ma0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the Heun step under fixed noise                        */
/* ------------------------------------------------------------------------ */
/* Loss L = sum_n w[n] * mbar_n for each of nloss weight vectors w
 * (each nsteps+1 long, row-major nloss x (nsteps+1)).  Returns in g
 * (nloss x 5) dL/d(c_ex, hk, gamma1, alpha, sigma), where alpha is the
 * factor that multiplies the damping term of Eq. (1) with gamma1 held
 * fixed.  The whole trajectory is stored (plain, not checkpointed). */

/* v -> (df/dm)^T v for f = -g1 m x H - a g1 m x (m x H), H fixed */
static void rhs_dm_T(double g1, double a, const double m[3], const double H[3],
                     const double v[3], double o[3])
{
    double t1[3], mxH[3], t2[3], vxm[3], t3[3];
    cross(H, v, t1);
    cross(m, H, mxH);
    cross(mxH, v, t2);
    cross(v, m, vxm);
    cross(H, vxm, t3);
    for (int c = 0; c < 3; ++c) o[c] = -g1 * t1[c] - a * g1 * (t2[c] + t3[c]);
}

/* v -> (df/dH)^T v = g1 m x v - a g1 m x (m x v) */
static void rhs_dH_T(double g1, double a, const double m[3], const double v[3],
                     double o[3])
{
    double mxv[3], mxmxv[3];
    cross(m, v, mxv);
    cross(m, mxv, mxmxv);
    for (int c = 0; c < 3; ++c) o[c] = g1 * mxv[c] - a * g1 * mxmxv[c];
}

/* (I - n n^T) v / len */
static void unit_T(const double n[3], double len, const double v[3], double o[3])
{
    double d = dot3(n, v);
    for (int c = 0; c < 3; ++c) o[c] = (v[c] - n[c] * d) / len;
}

int orc_adjoint(const orc_level* L, const double* u, uint64_t seed,
                int64_t nsteps, const double* w, int32_t nloss, double* g,
                double* mbar)
{
    int64_t N = (int64_t)L->nx * L->ny * L->nz;
    if (L->demag_ms != 0.0) return -2;   /* the adjoint has no magnetostatic term */
    size_t st = (size_t)(3 * N);
    double* traj = (double*)malloc(sizeof(double) * st * (size_t)(nsteps + 1));
    double* lam = (double*)malloc(sizeof(double) * st * (size_t)nloss);
    double* mb = (double*)malloc(sizeof(double) * st);
    double* Hb = (double*)malloc(sizeof(double) * st);
    double* tmp = (double*)malloc(sizeof(double) * st);
    double* ex = (double*)malloc(sizeof(double) * st);
    step_ws ws;
    if (!traj || !lam || !mb || !Hb || !tmp || !ex || ws_alloc(&ws, L)) {
        free(traj); free(lam); free(mb); free(Hb); free(tmp); free(ex);
        return -1;
    }
    const double* ua = u;
    /* forward, storing every state */
    for (int64_t i = 0; i < N; ++i) {
        traj[3 * i] = 0.0; traj[3 * i + 1] = 0.0; traj[3 * i + 2] = 1.0;
    }
    if (mbar) mbar[0] = mean_mz(traj, N);
    for (int64_t n = 0; n < nsteps; ++n) {
        heun_step_ws(L, ua, seed, n, traj + st * n, traj + st * (n + 1), &ws);
        if (mbar) mbar[n + 1] = mean_mz(traj + st * (n + 1), N);
    }
    for (int l = 0; l < nloss * 5; ++l) g[l] = 0.0;
    /* terminal source */
    for (int l = 0; l < nloss; ++l) {
        memset(lam + st * l, 0, sizeof(double) * st);
        for (int64_t i = 0; i < N; ++i)
            lam[st * l + 3 * i + 2] = w[(int64_t)l * (nsteps + 1) + nsteps] / (double)N;
    }
    const double g1 = L->gamma1, al = L->alpha, dt = L->dt;
    for (int64_t n = nsteps - 1; n >= 0; --n) {
        const double* m = traj + st * n;
        const double* mn = traj + st * (n + 1);
        /* recompute every intermediate of step n */
        heun_step_ws(L, ua, seed, n, m, tmp, &ws);
        for (int l = 0; l < nloss; ++l) {
            double* lm = lam + st * l;
            double* gl = g + 5 * l;
            double* fb = ex; /* reuse as dL/df */
            /* through m_{n+1} = q/|q| and q = m + dt/2 (f + f') */
            for (int64_t i = 0; i < N; ++i) {
                double qb[3], fpb[3], t[3];
                unit_T(mn + 3 * i, ws.qn[i], lm + 3 * i, qb);
                for (int c = 0; c < 3; ++c) {
                    mb[3 * i + c] = qb[c];
                    fb[3 * i + c] = 0.5 * dt * qb[c];
                    fpb[c] = 0.5 * dt * qb[c];
                }
                /* f' = F(m', H') */
                const double* mp = ws.mp + 3 * i;
                const double* Hp = ws.Hp + 3 * i;
                rhs_dH_T(g1, al, mp, fpb, Hb + 3 * i);
                rhs_dm_T(g1, al, mp, Hp, fpb, t);
                for (int c = 0; c < 3; ++c) tmp[3 * i + c] = t[c]; /* dL/dm' so far */
                double mxH[3], mxmxH[3];
                cross(mp, Hp, mxH);
                cross(mp, mxH, mxmxH);
                gl[2] += dot3(fpb, ws.fp + 3 * i) / g1;
                gl[3] += -g1 * dot3(fpb, mxmxH);
            }
            /* through H' = c_ex E(m') + hk (m'.u)u + hz + sigma xi */
            for (int z = 0; z < L->nz; ++z)
                for (int y = 0; y < L->ny; ++y)
                    for (int x = 0; x < L->nx; ++x) {
                        int64_t i = x + (int64_t)L->nx * (y + (int64_t)L->ny * z);
                        double d[3], e[3];
                        const double* a = axis_of(L, ua, i);
                        neighbour_diff(L, Hb, x, y, z, d);
                        neighbour_diff(L, ws.mp, x, y, z, e);
                        double uHb = dot3(a, Hb + 3 * i);
                        for (int c = 0; c < 3; ++c)
                            tmp[3 * i + c] += L->c_ex * d[c] + L->hk * uHb * a[c];
                        gl[0] += dot3(Hb + 3 * i, e);
                        gl[1] += dot3(ws.mp + 3 * i, a) * uHb;
                        gl[4] += dot3(Hb + 3 * i, ws.xi + 3 * i);
                    }
            /* through m' = p/|p|, p = m + dt f; then f = F(m, H) */
            for (int64_t i = 0; i < N; ++i) {
                double pb[3], t[3];
                unit_T(ws.mp + 3 * i, ws.pn[i], tmp + 3 * i, pb);
                for (int c = 0; c < 3; ++c) {
                    mb[3 * i + c] += pb[c];
                    fb[3 * i + c] += dt * pb[c];
                }
                const double* mi = m + 3 * i;
                const double* Hi = ws.H + 3 * i;
                rhs_dH_T(g1, al, mi, fb + 3 * i, Hb + 3 * i);
                rhs_dm_T(g1, al, mi, Hi, fb + 3 * i, t);
                for (int c = 0; c < 3; ++c) mb[3 * i + c] += t[c];
                double mxH[3], mxmxH[3];
                cross(mi, Hi, mxH);
                cross(mi, mxH, mxmxH);
                gl[2] += dot3(fb + 3 * i, ws.f + 3 * i) / g1;
                gl[3] += -g1 * dot3(fb + 3 * i, mxmxH);
            }
            /* through H = c_ex E(m) + hk (m.u)u + hz + sigma xi */
            for (int z = 0; z < L->nz; ++z)
                for (int y = 0; y < L->ny; ++y)
                    for (int x = 0; x < L->nx; ++x) {
                        int64_t i = x + (int64_t)L->nx * (y + (int64_t)L->ny * z);
                        double d[3], e[3];
                        const double* a = axis_of(L, ua, i);
                        neighbour_diff(L, Hb, x, y, z, d);
                        neighbour_diff(L, m, x, y, z, e);
                        double uHb = dot3(a, Hb + 3 * i);
                        for (int c = 0; c < 3; ++c)
                            mb[3 * i + c] += L->c_ex * d[c] + L->hk * uHb * a[c];
                        gl[0] += dot3(Hb + 3 * i, e);
                        gl[1] += dot3(m + 3 * i, a) * uHb;
                        gl[4] += dot3(Hb + 3 * i, ws.xi + 3 * i);
                    }
            /* lambda_n = dL/dm_n including the source at step n */
            double src = w[(int64_t)l * (nsteps + 1) + n] / (double)N;
            for (int64_t i = 0; i < N; ++i) {
                lm[3 * i] = mb[3 * i];
                lm[3 * i + 1] = mb[3 * i + 1];
                lm[3 * i + 2] = mb[3 * i + 2] + src;
            }
        }
    }
    ws_free(&ws);
    free(traj); free(lam); free(mb); free(Hb); free(tmp); free(ex);
    return 0;
}

/* Adjoint over many realizations (one thread each); g sums over them.
 * mbar (optional): nreal x (nsteps+1). */
int orc_adjoint_batch(const orc_level* L, const double* u, const uint64_t* seeds, int32_t nreal,
                      int64_t nsteps, const double* w, int32_t nloss, double* g,
                      double* mbar, int32_t nthreads)
{
    double* gr = (double*)calloc((size_t)nreal * (size_t)nloss * 5, sizeof(double));
    if (!gr) return -1;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
#endif
    for (int32_t r = 0; r < nreal; ++r)
        err |= orc_adjoint(L, u, seeds[r], nsteps, w, nloss, gr + (size_t)r * nloss * 5,
                           mbar ? mbar + (int64_t)r * (nsteps + 1) : NULL);
    for (int l = 0; l < nloss * 5; ++l) g[l] = 0.0;
    for (int32_t r = 0; r < nreal; ++r)
        for (int l = 0; l < nloss * 5; ++l) g[l] += gr[(size_t)r * nloss * 5 + l];
    free(gr);
    return err ? -1 : 0;
}
