/*
 * sllg.h - C ABI of the MI355X stochastic-LLG hysteresis-loop library.
 *
 * The library integrates the stochastic Landau-Lifshitz-Gilbert equation
 * (Eq. 1 of Behbahani, Plumer, Saika-Voivod, arXiv:1912.00310) on 3-D grids
 * of cubic macrospin cells of edge b*a0, with
 *   - 6-neighbour exchange, free boundaries (material paragraph: A0, J_eff),
 *   - uniaxial anisotropy along z or per-cell axes in a cone ("5 degree
 *     dispersion", material paragraph),
 *   - an applied field along z swept in time (protocol paragraph, SR = 4 Hmax f),
 *   - Brown's stochastic thermal field (text under Eq. 1),
 * stepped by the Heun predictor-corrector, and reduces the mean z-component of
 * the cells' unit magnetisation into dynamic hysteresis loops every step
 * (the loop ordinate m_H defined after Eq. 1).  Cell parameters follow the
 * modified Grinstein-Koch rule: A(b) = zeta A0, K(b) = zeta^3 K0 (Eqs. 8-9),
 * H(b) = zeta H0 (Eq. 10), loops rescaled by 1 - delta(1 - zeta) (Eq. 13),
 * zeta = t/b + 1 - t, and optionally alpha scaled with the sweep rate so that
 * SR/alpha is fixed (Eq. 14 discussion).
 *
 * Conventions
 *   - Every function returns an int status: SLLG_OK (0) or a negative
 *     SLLG_E_* code; sllg_last_error() gives a thread-local message.
 *   - Device memory is owned by the caller: one workspace of
 *     sllg_workspace_bytes() bytes (256-byte aligned) passed to sllg_init().
 *     The library never allocates or frees device memory.
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the default stream).  sllg_run_* return without waiting;
 *     sllg_sync, sllg_loop, sllg_grad and sllg_get_state synchronise that
 *     stream and report failures of the kernels enqueued before them.
 *   - Host arrays are owned by the caller.  A context is not thread safe.
 *   - SI units inside; fields in the loop outputs are in Oe.
 */
#ifndef SLLG_H
#define SLLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SLLG_OK = 0,
    SLLG_E_INVAL = -1,      /* bad argument (dims, b < 1, dt <= 0, alpha < 0, T < 0, ...) */
    SLLG_E_WORKSPACE = -2,  /* workspace missing, misaligned or too small                   */
    SLLG_E_CAPACITY = -3,   /* host output array too small; *n_out holds the size needed     */
    SLLG_E_STATE = -4,      /* call-order error (e.g. grad without checkpoints)              */
    SLLG_E_HIP = -5,        /* HIP runtime error, or a slab-plan exchange wait that gave up;
                               text in sllg_last_error()                                    */
    SLLG_E_NUMERIC = -6     /* a loop ordinate (mean m_z of a realization) became non-finite:
                               the magnetisation blew up (e.g. a time step far too large).
                               |m| itself is renormalised every stage and not checked     */
};

/* Process-wide options, read by every later sllg_init (sllg_set_options). */
enum {
    SLLG_OPT_NO_TUNE = 1,   /* no timing at init: streamed levels keep the default tile
                               shape and the slab plan is not tried; pin shapes afterwards
                               with sllg_set_stream_shape / sllg_set_slab_shape           */
    SLLG_OPT_NO_SLAB = 2,   /* init never picks the slab plan (plan 3) on its own          */
    SLLG_OPT_NO_GRAPH = 4,  /* streamed steps are launched one by one, not replayed from
                               HIP graphs of 128 launches                                   */
    SLLG_OPT_VERBOSE = 8    /* the tuners print every candidate's time to stderr           */
};

enum { SLLG_WAVE_TRIANGLE = 0, SLLG_WAVE_COSINE = 1, SLLG_WAVE_CONSTANT = 2 };

/* Base (b = 1) material and field protocol.  Defaults quoted are the paper's. */
typedef struct {
    double a0_m;            /* cubic unit-cell edge, 0.839e-9 m                         */
    double Ms0;             /* saturation magnetisation, 480e3 A/m                       */
    double A0;              /* exchange stiffness, 0.98e-11 J/m                          */
    double K0;              /* uniaxial anisotropy, 1e4 J/m^3                            */
    double T_K;             /* temperature, 310 K                                        */
    double Tc_K;            /* <= 0: 1.44 a0 A0/k_B; the paper prints 858 K              */
    double delta;           /* Eq. (13) weight, 0.511                                    */
    double easy_axis[3];    /* anisotropy axis (normalised by the library)               */
    double Hmax_Oe;         /* physical field amplitude                                  */
    double sweep_Oe_per_ns; /* SR; one cycle lasts 4 Hmax/SR                              */
    int32_t wave;           /* SLLG_WAVE_*; both start at +Hmax                           */
    int32_t n_cycles;       /* field cycles per sweep (>= 1)                              */
    int32_t scale_AK;       /* apply A = zeta A0, K = zeta^3 K0                          */
    int32_t scale_H;        /* apply H_sim = zeta H_phys and m_phys = (1-delta(1-zeta)) m */
    double ms_scale;        /* Ms = ms_scale * Ms0 (not rescaled with b); 1 by default   */
    double sr_ref_Oe_per_ns;/* > 0: alpha = alpha_ref * SR / SR_ref for every level      */
    double alpha_ref;
    int32_t demag;          /* != 0: add the magnetostatic field of the cells, -Ms sum_j
                               N(r_i - r_j) m_j with N the demagnetising tensor of two
                               uniformly magnetised cubes (beyond the paper, which folds
                               shape anisotropy into K); every level then runs on plan 5,
                               a direct sum over the cells, and may hold at most 1024
                               cells; sllg_grad refuses such levels                      */
} sllg_material;

/* One coarse-graining level: a grid and its realizations. */
typedef struct {
    int32_t nx, ny, nz;     /* cells; cell index i = x + nx*(y + ny*z)                    */
    double b;               /* cell edge in units of a0 (>= 1)                            */
    int32_t n_real;         /* independent realizations (>= 1)                            */
    uint64_t seed_base;     /* realization r draws from seed_base + r                     */
    double alpha;           /* Gilbert damping (ignored if sr_ref_Oe_per_ns > 0)          */
    double dt_s;            /* time step; <= 0 picks the largest whole fs <= 5 fs within
                               0.15 sqrt(1+alpha^2)/(gamma0 (12 c_ex + H_K + H_max))     */
    double cone_deg;        /* > 0: per-cell easy axes uniform in a cone of this angle    */
    uint64_t axis_seed;     /* Philox key for the per-cell axes                           */
    int32_t record_every;   /* keep the loop ordinate every k steps (area and the online
                               crossings still use every step); >= 1                      */
} sllg_level;

/* Loop statistics.  *_sim are in simulation units (Oe of the simulated field,
 * unit-vector magnetisation); *_phys apply H/zeta and the Eq. (13) factor.
 * Hc is half the distance between the first zero crossing on the falling
 * branch and the first on the rising branch (linear interpolation); NaN when
 * a branch never crosses zero.  S is -closed integral of m dH (trapezoid, every
 * step).  S_se and Hc_se are one standard error over realizations (NaN for
 * a single realization). */
typedef struct {
    double S_sim, S_phys;
    double Hc_desc, Hc_asc;     /* crossing fields, Oe (sim)                      */
    double Hc_sim, Hc_phys;
    double Mr_sim, Mr_phys;     /* (m(H=0, falling) - m(H=0, rising))/2           */
    double S_se, Hc_se;         /* standard errors of S_sim and Hc_sim            */
    int32_t n_cross_desc, n_cross_asc; /* sign changes of m on each branch        */
    int32_t n_real;             /* realizations the statistics cover              */
} sllg_loop_stats;

typedef struct sllg_ctx sllg_ctx;

/* Bytes of device workspace a context needs.  ckpt_every > 0 reserves a
 * checkpoint of every instance every ckpt_every steps (needed by sllg_grad). */
size_t sllg_workspace_bytes(const sllg_material* mat, const sllg_level* levels,
                            int32_t n_levels, int32_t ckpt_every);

/* Compile every level's parameters (FP64 on the host: zeta, A, K, Ms, c_ex =
 * 2A/(mu0 Ms a^2), H_K = 2K/(mu0 Ms), gamma1 = mu0 gamma_e/(1+alpha^2),
 * sigma = sqrt(2 alpha k_B T/(gamma0 mu0 Ms V dt)), dt, steps per sweep),
 * lay the state, loop records and checkpoints out in d_workspace, choose an
 * execution plan for every level (tuned on first use of a shape) and set every
 * cell to +z at step 0.  The workspace must stay valid until sllg_free(). */
int sllg_init(const sllg_material* mat, const sllg_level* levels, int32_t n_levels,
              int32_t ckpt_every, void* d_workspace, size_t ws_bytes,
              void* hip_stream, sllg_ctx** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * sllg_init, but the workspace is a device array of 64 MiB inside the
 * library (one per GPU, held until the process ends) instead of the
 * caller's.  Neither this call nor the calls on the context it returns
 * allocate device memory: the tuners are off (default tile shapes, the slab
 * plan is only used if sllg_set_slab_shape asks for it) and streamed steps
 * are launched one by one instead of from HIP graphs.  A workload needing
 * more than 64 MiB (sllg_workspace_bytes) gives SLLG_E_WORKSPACE.  One live
 * context per GPU: while one holds the array, another sllg_init_static on
 * that GPU gives SLLG_E_STATE; sllg_free releases it.  The array keeps the
 * last context's contents; initialisation clears everything a sweep reads
 * before writing.  Calls from several threads on one GPU race. */
int sllg_init_static(const sllg_material* mat, const sllg_level* levels, int32_t n_levels,
                     int32_t ckpt_every, void* hip_stream, sllg_ctx** out);

/* Enqueue the remaining steps of the sweep for every level and realization.
 * Asynchronous: failures inside kernels (the device status word: a
 * non-finite loop ordinate, a slab exchange that timed out) are reported by
 * the next call that synchronises (sllg_sync, sllg_loop, sllg_grad,
 * sllg_get_state).  After an exchange timeout the remaining slab launches of
 * the run do nothing and the state is undefined until sllg_reset. */
int sllg_run_sweep(sllg_ctx* ctx);

/* Enqueue at most nsteps further steps (levels stop at their own sweep end).
 * Asynchronous, as sllg_run_sweep. */
int sllg_run_steps(sllg_ctx* ctx, int64_t nsteps);

/* Wait for the context's stream and report the device status word:
 * SLLG_E_HIP if a slab exchange wait gave up, SLLG_E_NUMERIC if a loop
 * ordinate became non-finite, else SLLG_OK.  A debug build of the library
 * (compiled with SLLG_LDS_CHECK; libsllg_ldscheck.so) also gives SLLG_E_HIP
 * when the streamed full-width-row kernel read an LDS neighbour slot that
 * had not been written for the plane it stands for. */
int sllg_sync(sllg_ctx* ctx);

/* Reset every level to step 0 (all cells +z, loops cleared, device status
 * word cleared). */
int sllg_reset(sllg_ctx* ctx);

/* Copy one loop to the host and analyse it.  real = -1 gives the ensemble
 * mean loop (statistics of the mean loop, standard errors over realizations).
 * H_Oe and mH (either may be NULL) receive the simulated field and loop
 * ordinate at every recorded step, up to cap entries; *n_out gets the count.
 * Synchronises the stream. */
int sllg_loop(sllg_ctx* ctx, int32_t level, int32_t real, double* H_Oe, double* mH,
              int64_t cap, int64_t* n_out, sllg_loop_stats* stats);

/* Gradients, by the discrete adjoint of the Heun step under the same noise,
 * of the ensemble-mean loop area S_sim (g_area) and of the coercive field
 * Hc_sim of the ensemble-mean loop (g_hc) with respect to
 * (K, A, alpha, ms_scale), K and A being the level's simulated values.
 * Needs a completed sweep run with ckpt_every > 0 and record_every == 1,
 * and a level of at most 1536 cells (one workgroup per realization; two
 * cells per thread above 1024), without magnetostatics.  One segment of
 * ckpt_every steps has its applied field and loss weights in LDS: the
 * largest ckpt_every allowed shrinks with the level (11065 up to 256 cells,
 * 9501 up to 512, 5351 up to 1024, 1282 up to 1536); beyond that
 * SLLG_E_INVAL.  g_hc is NaN when the mean loop has no crossing on a
 * branch.  FP64 accumulation; synchronises the stream. */
int sllg_grad(sllg_ctx* ctx, int32_t level, double g_area[4], double g_hc[4]);

/* Set the process-wide SLLG_OPT_* flags that later sllg_init calls use
 * (existing contexts keep theirs).  SLLG_E_INVAL for unknown bits. */
int sllg_set_options(int32_t flags);

/* Polls of one exchange word a slab-plan workgroup makes before it gives up
 * (default 2^20, each poll followed by a short sleep).  A wait that gives up
 * sets the status word, ends every workgroup of the launch and makes the
 * following slab launches return at once; sllg_sync then reports SLLG_E_HIP.
 * 0 makes every wait that does not find its words at the first poll give up
 * (for testing the error path; every kernel still exits normally). */
int sllg_set_spin_limit(sllg_ctx* ctx, uint32_t polls);

/* Thread-local text of the last error. */
const char* sllg_last_error(void);

/* Release the context (never the caller's workspace or stream). */
void sllg_free(sllg_ctx* ctx);

/* ---- introspection used by tests and the benchmark ---------------------- */

/* Compiled constants of a level: out[0..15] = zeta, A, K, Ms, a, c_ex, hk,
 * gamma1, alpha, sigma, dt, hscale, cM, n_steps, hz_amp (A/m) and the plan
 * code 100000*plan + 1000*kernel shape + z planes per tile or slab. */
int sllg_level_params(const sllg_ctx* ctx, int32_t level, double out[16]);

/* Name of the kernel (template shape and tiling) that steps a level, as a
 * NUL-terminated string of at most cap bytes. */
int sllg_level_kernel(const sllg_ctx* ctx, int32_t level, char* name, int32_t cap);

/* Current step index of a level. */
int64_t sllg_level_step(const sllg_ctx* ctx, int32_t level);

/* Copy one realization's magnetisation (host, 3*ncell floats, planes
 * mx | my | mz) after synchronising the stream. */
int sllg_get_state(sllg_ctx* ctx, int32_t level, int32_t real, float* host_m);

/* Overwrite one realization's magnetisation from the host (3*ncell floats,
 * planes mx | my | mz; vectors are used as given). */
int sllg_set_state(sllg_ctx* ctx, int32_t level, int32_t real, const float* host_m);

/* Checkpoint and resume of a sweep (the counter-based noise needs only the
 * step index, so no generator state is kept).  sllg_save_state waits for the
 * context's stream and copies everything a sweep carries from one step to
 * the next into host memory: every level's step index, both magnetisation
 * buffers, the FP64 loop accumulators and crossing state, the loop records,
 * the adjoint checkpoints and the device status word.  *need receives the
 * snapshot's size; with host == NULL only the size is returned; cap < *need
 * gives SLLG_E_INVAL; a context whose status word reports a failure is not
 * saved (its error is returned).  The caller owns the buffer; the format is
 * private to this library version.  sllg_load_state puts a snapshot into a
 * context created from the same material, levels and checkpoint interval
 * (grids, seeds, compiled constants and buffer sizes must match, else
 * SLLG_E_INVAL and the context is unchanged); plans and tile shapes may
 * differ, since they all give the same bits.  Continuing from a loaded
 * snapshot gives the states and loops of the uninterrupted run bit for bit.
 * Both synchronise the stream. */
int sllg_save_state(sllg_ctx* ctx, void* host, size_t cap, size_t* need);
int sllg_load_state(sllg_ctx* ctx, const void* host, size_t size);

/* Execution plan of a level: 0 = automatic, 1 = LDS-resident persistent
 * kernel, 2 = one fused launch per step over tiles, 3 = persistent
 * cooperative launch in which every workgroup owns a z-slab of one
 * realization for up to 1024 steps and trades boundary planes with its two
 * neighbours through device memory each step, 4 = single-cell levels only
 * (the single-macrospin limit): one realization per quad of lanes for up to 2^20
 * steps per launch (automatic when every level of the context is a single
 * cell), 5 = with magnetostatics (material demag != 0; the only plan such a
 * level can use): one workgroup per realization, the field summed directly
 * over the cells.  Plans 1-4 give bit-identical states.  Changing the plan is allowed
 * between runs.  Returns SLLG_E_INVAL if the plan cannot hold the level
 * (plan 3: more slabs than can be co-resident, or a slab thicker than the
 * workgroup's LDS holds; plan 4: more than one cell). */
int sllg_set_plan(sllg_ctx* ctx, int32_t level, int32_t plan);

/* Slab plan (3) with a given kernel: kind 0 recomputes the halo predictor
 * and exchanges two boundary planes per side once per step (slabs of at
 * least 2 planes); kind 1 exchanges one boundary plane per side after each
 * Heun stage (slabs of at least 1 plane).  threads and cells_per_thread
 * name the instantiation, planes the slab thickness (the z extent is split
 * into slabs of planes or planes + 1).  Both kinds give the same states as
 * the other plans.  Returns SLLG_E_INVAL if no such kernel exists or it
 * cannot hold the level; the previous plan is then kept. */
int sllg_set_slab_shape(sllg_ctx* ctx, int32_t level, int32_t kind, int32_t threads, int32_t cells_per_thread,
                        int32_t planes);

/* Streamed plan (2) with a given tile kernel and z planes per tile: kind 0
 * = x-y window (a, b threads, c z planes per thread block), kind 1 = full-width
 * rows with an LDS ring of m_n planes (a threads, b cells per thread, c = 1),
 * kind 2 = full-width rows with the z-columns in registers (a threads, b
 * cells per thread, c = 1).  All kernels give the same states.  Returns
 * SLLG_E_INVAL if no such kernel exists or the tiling does not fit. */
int sllg_set_stream_shape(sllg_ctx* ctx, int32_t level, int32_t kind, int32_t a, int32_t b, int32_t c,
                          int32_t planes);

/* Device Philox4x32-10 of the thermal-noise stream: for k < n, the four raw
 * words for (seed, level, tag, cells[k], steps[k]) and the three normals the
 * kernels derive from them.  d_scratch: >= 40*n bytes of device memory.
 * Synchronises the stream. */
int sllg_philox_probe(uint64_t seed, uint32_t level, uint32_t tag, const uint32_t* cells,
                      const uint64_t* steps, int32_t n, uint32_t* raw, float* normals,
                      void* d_scratch, void* hip_stream);

/* Per-cell easy axes of a level as the kernels use them (host, 3*ncell floats,
 * planes ux | uy | uz).  Synchronises the stream. */
int sllg_get_axes(sllg_ctx* ctx, int32_t level, float* host_u);

/* Timing of the dominant kernel (the streamed step kernel if a level uses
 * it, else the resident kernel).  sllg_set_timing(ctx, k) with k > 0 brackets
 * every k-th launch unit (one launch, or one replay of a graph of streamed
 * launches) with HIP events on the context stream; k = 0 switches it off.
 * sllg_kernel_time returns the mean time per kernel launch over the timed
 * units in milliseconds, the number of launches covered, and the mean
 * cell-updates per launch (launches of many steps may differ in length);
 * a launch of the slab plan (3) counts as one launch per step it covers.  It synchronises the stream and restarts
 * the count. */
int sllg_set_timing(sllg_ctx* ctx, int32_t every);
int sllg_kernel_time(sllg_ctx* ctx, double* mean_ms, int64_t* launches, int64_t* cells_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* SLLG_H */
