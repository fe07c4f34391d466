/* Drives every entry point of the FP64 oracle on small ragged grids, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure: tests/test_sanitizers.py compiles and runs it).  The
 * oracle's source is included whole so that its static helpers are
 * instrumented too.  Exit status 0 when every call returned 0 and every
 * result is finite. */
#include "../../oracle/sllg_oracle.c"

#include <stdio.h>

static int bad = 0;

static void expect(int ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        bad = 1;
    }
}

static int finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* A level with the constants of the 2x6x14 rod at b = 4 on a given grid. */
static orc_level level(int nx, int ny, int nz, double cone, double demag_ms, int wave)
{
    orc_level L;
    memset(&L, 0, sizeof L);
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.level_tag = 1;
    L.c_ex = 2103299.370380639;
    L.hk = 12846.918612797526;
    L.gamma1 = 218978.33941853608;
    L.alpha = 0.1;
    L.sigma = 5826835.2526868945;
    L.dt = 5e-15;
    L.hz_amp = 58013.64621444088;
    L.n_period = 400;
    L.wave = wave;
    L.axis[2] = 1.0;
    L.cone_deg = cone;
    L.axis_seed = 3;
    L.demag_ms = demag_ms;
    return L;
}

static void exercise(int nx, int ny, int nz, double cone, double demag_ms, int wave)
{
    orc_level L = level(nx, ny, nz, cone, demag_ms, wave);
    const int64_t N = (int64_t)nx * ny * nz, S = 60;
    double* u = malloc(sizeof(double) * 3 * N);
    double* m = malloc(sizeof(double) * 3 * N);
    double* H = malloc(sizeof(double) * 3 * N);
    double* mbar = malloc(sizeof(double) * 3 * (S + 1));
    double* mfin = malloc(sizeof(double) * 3 * 3 * N);
    double* w = calloc(2 * (S + 1), sizeof(double));
    double g[10], gb[10], stats[16];
    uint64_t seeds[3] = {1, 2, 3};
    orc_make_axes(&L, u);
    expect(finite_all(u, 3 * N), "axes");
    for (int64_t i = 0; i < N; ++i) {
        m[3 * i] = 0.6;
        m[3 * i + 1] = 0.0;
        m[3 * i + 2] = 0.8;
    }
    double* hth = calloc(3 * N, sizeof(double));
    hth[0] = 1e3;
    orc_effective_field(&L, u, m, 1000.0, hth, H);
    free(hth);
    expect(finite_all(H, 3 * N), "effective field");
    expect(isfinite(orc_energy(&L, u, m, 1000.0)), "energy");
    expect(orc_run(&L, u, 7, 0, S, m, mbar) == 0 && finite_all(mbar, S + 1), "run");
    expect(orc_run_batch(&L, u, seeds, 3, S, mbar, mfin, 2) == 0 && finite_all(mfin, 9 * N), "run_batch");
    double* Hs = malloc(sizeof(double) * (S + 1));
    for (int64_t n = 0; n <= S; ++n) Hs[n] = orc_applied_field(&L, n) / (1000.0 / (4.0 * M_PI));
    orc_loop_stats(Hs, mbar, S + 1, stats);
    for (int64_t n = 0; n <= S; ++n) {
        w[n] = 1.0 / (S + 1);
        w[S + 1 + n] = (n == S) ? 1.0 : 0.0;
    }
    if (demag_ms == 0.0) {
        expect(orc_adjoint(&L, u, 7, S, w, 2, g, NULL) == 0 && finite_all(g, 10), "adjoint");
        expect(orc_adjoint_batch(&L, u, seeds, 3, S, w, 2, gb, NULL, 2) == 0 && finite_all(gb, 10),
               "adjoint_batch");
    } else {
        expect(orc_adjoint(&L, u, 7, S, w, 2, g, NULL) == -2, "adjoint refuses magnetostatics");
        const int64_t nt = (int64_t)(2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1) * 6;
        double* T = malloc(sizeof(double) * nt);
        orc_demag_tensor(&L, T);
        expect(finite_all(T, nt), "demag tensor");
        free(T);
    }
    free(Hs);
    free(u);
    free(m);
    free(H);
    free(mbar);
    free(mfin);
    free(w);
}

/* A grid of 64k cells with one realization: the cell loops run in
 * parallel (the path for grids larger than the realization count). */
static void exercise_cell_parallel(void)
{
    orc_level L = level(64, 32, 32, 5.0, 0.0, 0);
    const int64_t N = 64 * 32 * 32, S = 2;
    double* u = malloc(sizeof(double) * 3 * N);
    double* mbar = malloc(sizeof(double) * (S + 1));
    double* mfin = malloc(sizeof(double) * 3 * N);
    uint64_t seed = 11;
    orc_make_axes(&L, u);
    expect(orc_run_batch(&L, u, &seed, 1, S, mbar, mfin, 2) == 0 && finite_all(mfin, 3 * N),
           "run_batch over cells");
    free(u);
    free(mbar);
    free(mfin);
}

int main(void)
{
    double nw[6];
    orc_newell(1, 2, 0, nw);
    expect(finite_all(nw, 6), "newell");
    uint32_t words[4];
    orc_philox_cell(5, 1, ORC_TAG_NOISE, 3, 9, words);
    double un[4];
    orc_uniforms(5, 1, ORC_TAG_NOISE, 3, 9, un);
    expect(finite_all(un, 4), "uniforms");
    exercise(1, 1, 1, 0.0, 0.0, 0);
    exercise(3, 2, 5, 5.0, 0.0, 1);
    exercise(2, 6, 14, 10.0, 0.0, 0);
    exercise(3, 2, 5, 5.0, 480000.0, 1);
    exercise(1, 3, 7, 0.0, 480000.0, 2);
    exercise_cell_parallel();
    if (!bad) printf("oracle driver: all calls clean\n");
    return bad;
}
