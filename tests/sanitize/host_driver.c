/* Drives the host side of libsllg that runs without a GPU (argument
 * validation, the level compiler, the workspace layout, the error paths of
 * sllg_init) for a build whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py compiles and runs it).
 * Exit status 0 when every call answered as the header says. */
#include <stdio.h>
#include <string.h>

#include "../../include/sllg.h"

static int bad = 0;

static void expect(int ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s (%s)\n", what, sllg_last_error());
        bad = 1;
    }
}

static sllg_material material(void)
{
    sllg_material m;
    memset(&m, 0, sizeof m);
    m.a0_m = 0.839e-9;
    m.Ms0 = 480e3;
    m.A0 = 0.98e-11;
    m.K0 = 1.0e4;
    m.T_K = 310.0;
    m.Tc_K = 858.0;
    m.delta = 0.511;
    m.easy_axis[2] = 1.0;
    m.Hmax_Oe = 1000.0;
    m.sweep_Oe_per_ns = 2.0e4;
    m.wave = SLLG_WAVE_TRIANGLE;
    m.n_cycles = 1;
    m.scale_AK = 1;
    m.scale_H = 1;
    m.ms_scale = 1.0;
    return m;
}

static sllg_level level(int nx, int ny, int nz, double b, int n_real, double cone)
{
    sllg_level l;
    memset(&l, 0, sizeof l);
    l.nx = nx;
    l.ny = ny;
    l.nz = nz;
    l.b = b;
    l.n_real = n_real;
    l.seed_base = 1;
    l.alpha = 0.1;
    l.dt_s = 5e-15;
    l.cone_deg = cone;
    l.axis_seed = 7;
    l.record_every = 1;
    return l;
}

int main(void)
{
    sllg_material m = material();
    sllg_level rod = level(2, 6, 14, 4.0, 64, 5.0);
    size_t ws = sllg_workspace_bytes(&m, &rod, 1, 256);
    expect(ws > 0 && (ws & 255) == 0, "workspace of the rod with checkpoints");

    /* the four-level batch, uneven sizes and record intervals */
    sllg_level four[4] = {level(8, 24, 56, 1.0, 256, 0.0), level(4, 12, 28, 2.0, 256, 0.0),
                          level(2, 6, 14, 4.0, 256, 0.0), level(1, 3, 7, 8.0, 256, 0.0)};
    for (int i = 0; i < 4; ++i) four[i].record_every = 100;
    expect(sllg_workspace_bytes(&m, four, 4, 0) > 0, "workspace of the four-level batch");

    /* the block with per-cell axes */
    sllg_level block = level(128, 128, 512, 2.0, 1, 10.0);
    expect(sllg_workspace_bytes(&m, &block, 1, 0) > (size_t)128 * 128 * 512 * 36, "workspace of the block");

    /* magnetostatics up to its cell limit, refused beyond it */
    m.demag = 1;
    sllg_level small = level(8, 8, 16, 4.0, 4, 0.0);
    expect(sllg_workspace_bytes(&m, &small, 1, 0) > 0, "workspace with magnetostatics");
    sllg_level big = level(8, 8, 17, 4.0, 4, 0.0);
    expect(sllg_workspace_bytes(&m, &big, 1, 0) == 0, "magnetostatics beyond 1024 cells refused");
    m.demag = 0;

    /* invalid levels: every one refused with 0 bytes */
    sllg_level bad_levels[5] = {level(0, 6, 14, 4.0, 1, 0.0), level(2, 6, 14, 0.5, 1, 0.0),
                                level(2, 6, 14, 4.0, 0, 0.0), level(2, 6, 14, 4.0, 1, 95.0),
                                level(5000, 1, 1, 4.0, 1, 0.0)};
    for (int i = 0; i < 5; ++i) expect(sllg_workspace_bytes(&m, &bad_levels[i], 1, 0) == 0, "invalid level");
    expect(sllg_workspace_bytes(&m, &rod, 1, -1) == 0, "negative checkpoint interval");
    expect(sllg_workspace_bytes(NULL, &rod, 1, 0) == 0, "no material");

    /* sllg_init error paths that return before any device call */
    sllg_ctx* ctx = (sllg_ctx*)1;
    expect(sllg_init(&m, &rod, 1, 256, NULL, ws, NULL, &ctx) == SLLG_E_WORKSPACE && ctx == NULL,
           "init without a workspace");
    expect(sllg_init(&m, &rod, 1, 256, (void*)(uintptr_t)4096, 256, NULL, &ctx) == SLLG_E_WORKSPACE,
           "init with a workspace too small");
    expect(sllg_init(&m, &rod, 1, 256, (void*)(uintptr_t)4100, ws, NULL, &ctx) == SLLG_E_WORKSPACE,
           "init with a misaligned workspace");
    expect(sllg_init(&m, &bad_levels[0], 1, 0, (void*)(uintptr_t)4096, ws, NULL, &ctx) == SLLG_E_INVAL,
           "init with an invalid level");
    expect(sllg_init(&m, &rod, 1, 0, NULL, ws, NULL, NULL) == SLLG_E_INVAL, "init without an output pointer");
    expect(strlen(sllg_last_error()) > 0, "error message");
    expect(sllg_set_options(SLLG_OPT_NO_TUNE) == SLLG_OK && sllg_set_options(0) == SLLG_OK, "options");
    sllg_free(NULL);
    if (!bad) printf("host driver: all calls clean\n");
    return bad;
}
