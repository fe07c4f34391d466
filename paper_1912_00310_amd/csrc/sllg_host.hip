// Host runtime and C ABI of the stochastic-LLG hysteresis-loop library.
//
//   - parameter compiler: the modified Grinstein-Koch rule per level (FP64)
//   - workspace layout: every device buffer carved from the caller's block
//   - planner: LDS-resident groups or streamed tiles per level, with a small
//     timing-based tuner for the tile shape
//   - launch sequencing on the caller's stream, optional HIP graphs
//   - loop analytics (FP64) and the adjoint driver
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sllg.h"
#include "sllg_types.hpp"

// The kernels are compiled in this translation unit (one shared library).
#include "sllg_kernels.hip"
#include "sllg_rows.hip"
#include "sllg_adjoint.hip"
#include "sllg_slab.hip"
#include "sllg_rows2.hip"
#include "sllg_lanes.hip"
#include "sllg_demag.hip"

using namespace sllg;

// Device workspace of sllg_init_static, for callers that cannot allocate
// device memory.  In host code `scratch` is only a handle: its device
// address (one copy per GPU) comes from hipGetSymbolAddress and is kept per
// device below.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(SLLG_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                          \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kKB = 1.380649e-23;
constexpr double kGammaE = 1.76e11;
constexpr double kGamma0 = kMu0 * kGammaE;
constexpr double kOe = 1000.0 / (4.0 * kPi);   // A/m per Oe

constexpr int kPlanAuto = 0, kPlanResident = 1, kPlanStream = 2, kPlanSlab = 3, kPlanLanes = 4, kPlanDemag = 5;
static_assert(kSlabChunk < 2048, "slab exchange tags hold the step of a launch in 11 bits");

// Compiled FP64 constants of one level.
struct LevelHost {
    sllg_level in;
    double t, zeta, A, K, Ms, a, V, alpha, dt, c_ex, hk, gamma1, sigma, hscale, cM, hz_amp;
    int64_t n_period, n_steps, n_rec;
    int inst0, ninst;
    int64_t ncell;
    int64_t axes_off;     // float offset in the axes buffer (-1: uniform axis)
    int plan;             // kPlanResident / kPlanStream in use
    int forced;           // plan fixed by sllg_set_plan
    // stream plan
    int shape;            // index into kShapes
    int tz;
    int tile0, ntiles;
    // slab plan
    int slab_kernel;      // index into kSlabKernels
    int slab_tz;
    int slab0, nslab;     // slab table range
    int64_t xch_off;      // word offset of the level's exchange buffer
    int64_t demag_off = -1;   // float offset of the demagnetising-tensor table
    int64_t step;         // host view of the step index
};

// Slab kernels.  kind 0: k_slab<nt, k> (halo predictor recomputed, one
// exchange per step, slabs of >= 2 planes); kind 1: k_slab2<nt, k> (m' and
// m_{n+1} exchanged, slabs of >= 1 plane).
struct SlabKernel {
    int kind, nt, k;
};
const SlabKernel kSlabKernels[] = {{0, 192, 4},  {0, 384, 2},  {0, 384, 3},  {0, 576, 2},  {0, 768, 1},
                                   {0, 768, 2},  {0, 1024, 1}, {0, 1024, 2}, {1, 192, 2},  {1, 384, 1},
                                   {1, 576, 1},  {1, 768, 1},  {1, 1024, 1}, {1, 384, 2},  {1, 768, 2},
                                   {1, 1024, 2}};
constexpr int kNumSlabKernels = sizeof(kSlabKernels) / sizeof(kSlabKernels[0]);

bool slab_eligible(const sllg_level& L) { return L.nx * L.ny <= 1024 && L.nz >= 4; }

// Stream-plan tile shapes.  kind 0: k_stream<tx, ty, pz> (x-y window with a
// recomputed ring); kind 1: k_rows<tx = threads, ty = cells per thread>
// (full-width tiles, needs nx <= threads); kind 2: k_rows2<tx = threads,
// ty = cells per thread> (full-width tiles, z-columns in registers).
struct Shape {
    int kind, tx, ty, pz;
};
const Shape kShapes[] = {{0, 64, 8, 1},  {0, 32, 16, 1}, {0, 64, 16, 1}, {0, 32, 8, 2},
                         {0, 8, 24, 4},  {0, 8, 24, 2},  {0, 8, 24, 1},  {0, 16, 16, 2},
                         {0, 4, 12, 8},  {1, 192, 1, 1}, {1, 256, 1, 1}, {1, 256, 2, 1},
                         {1, 512, 1, 1}, {1, 512, 2, 1}, {1, 1024, 1, 1}, {1, 256, 4, 1},
                         {2, 1024, 2, 1}, {2, 1024, 1, 1}, {2, 768, 2, 1}, {2, 512, 2, 1},
                         {2, 256, 2, 1},  {2, 256, 1, 1},  {2, 192, 1, 1}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
const int kTzChoices[] = {1, 2, 4, 8, 16, 32, 64};

struct ResidentKernel {
    int nw, cpw;
};
// At most 32 chunks of 64 cells per workgroup: the step-invariant per-chunk
// data of up to two chunks per wave stays in registers.  The planner takes
// the first kernel whose last wave owns no chunk (it folds the loop), else
// the first that holds every chunk.
const ResidentKernel kResKernels[] = {{2, 1}, {4, 1}, {8, 1}, {16, 1}, {16, 2}};
constexpr int kResMaxChunks = 32;

// Layout of the workspace (byte offsets).
struct Layout {
    size_t levels, insts, accs, steps, status, inst_cnt, launch_cnt, partials, tiles, groups, slots,
        chunks, buf0, buf1, axes, records, ckpt, tape, lam, weights, grads, slabs, xch, spart, islab,
        demag, total;
    int64_t state_floats, axes_floats, rec_doubles, ckpt_floats, tape_floats, lam_floats,
        max_tiles, max_groups, max_chunks, max_w, ninst_total, max_slabs, xch_words, demag_floats;
};

// The demagnetising-tensor table of a grid holds every cell offset when its
// six planes fit the LDS beside the kernel's state (wide), else the offsets
// with non-negative components only (one per cell).
//
// Row and plane strides of the wide table: at least 2nx - 1 and 2ny - 1,
// padded so that the table reads of a wave (lane i reads offset base(i) -
// base(j), every lane a different address) fall on as few addresses per LDS
// bank as the budget allows.  The cost model follows k_demag's threads
// (thread s N + i sums chunk s for cell i): for every wave and a few steps j
// of the chunk loop, the largest number of distinct addresses on one of 32
// banks of 4 bytes, for each half-wave of 32 lanes.  (This rule ranked the
// measured strides of the 2x6x14 rod in their order of speed; a 64-lane rule
// over 32 or 64 banks did not.)
struct WideDims {
    int wx, wy;
};
WideDims demag_wide_dims(const sllg_level& L)
{
    const int nx = L.nx, ny = L.ny, nz = L.nz, N = nx * ny * nz;
    const WideDims tight{2 * nx - 1, 2 * ny - 1};
    // chosen once per grid shape (the search takes some milliseconds)
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, WideDims> cache;
    const auto key = std::make_tuple(nx, ny, nz);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    auto fits = [&](int wx, int wy) {
        return 6 * sizeof(float) * (size_t)wx * wy * (2 * nz - 1) + kDemagStaticLds <= 160 * 1024;
    };
    const int clen = demag_chunk_len(N), S = demag_chunks(N), waves = demag_block(N) / 64;
    auto cost = [&](int wx, int wy) {
        int64_t c = 0;
        std::vector<int> addr(32), hits;
        for (int w = 0; w < waves; ++w)
            for (int k = 0; k < clen; k += std::max(1, clen / 4))
                for (int half = 0; half < 2; ++half) {
                    int na = 0;
                    for (int l = 32 * half; l < 32 * half + 32; ++l) {
                        const int t = 64 * w + l, s = t / N, i = t - s * N;
                        const int j = s * clen + k;
                        if (s >= S || j >= N || (j >= (s + 1) * clen)) continue;
                        const int bi = ((i / (nx * ny)) * wy + (i / nx) % ny) * wx + i % nx;
                        const int bj = ((j / (nx * ny)) * wy + (j / nx) % ny) * wx + j % nx;
                        addr[na++] = bi - bj;
                    }
                    std::sort(addr.begin(), addr.begin() + na);
                    na = (int)(std::unique(addr.begin(), addr.begin() + na) - addr.begin());
                    hits.assign(32, 0);
                    int worst = 0;
                    for (int a = 0; a < na; ++a) worst = std::max(worst, ++hits[((addr[a] % 32) + 32) % 32]);
                    c += worst;
                }
        return c;
    };
    WideDims best = tight;
    if (N > kDemagMaxCells || !fits(tight.wx, tight.wy)) {
        std::lock_guard<std::mutex> g(mu);
        cache[key] = best;
        return best;
    }
    int64_t best_c = cost(tight.wx, tight.wy);
    for (int wx = tight.wx; wx <= tight.wx + 8; ++wx)
        for (int wy = tight.wy; wy <= tight.wy + 24; ++wy) {
            if (!fits(wx, wy)) continue;
            const int64_t c = cost(wx, wy);
            if (c < best_c || (c == best_c && wx * wy < best.wx * best.wy)) {
                best_c = c;
                best = WideDims{wx, wy};
            }
        }
    std::lock_guard<std::mutex> g(mu);
    cache[key] = best;
    return best;
}
int64_t demag_wide_offsets(const sllg_level& L)
{
    const WideDims d = demag_wide_dims(L);
    return (int64_t)d.wx * d.wy * (2 * L.nz - 1);
}
bool demag_is_wide(const sllg_level& L)
{
    return 6 * sizeof(float) * (size_t)(2 * L.nx - 1) * (2 * L.ny - 1) * (2 * L.nz - 1) + kDemagStaticLds <=
           160 * 1024;
}
int64_t demag_table_offsets(const sllg_level& L)
{
    return demag_is_wide(L) ? demag_wide_offsets(L) : (int64_t)L.nx * L.ny * L.nz;
}
int64_t demag_table_floats(const sllg_level& L) { return 6 * demag_table_offsets(L); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Row windows [y0, y0 + nyt) of a full-width tile with R predicted rows
// (the window plus one ring row on each side inside the grid).
std::vector<std::pair<int, int>> row_windows(int ny, int R)
{
    std::vector<std::pair<int, int>> w;
    if (R < 3 && ny > R) return w;
    int y0 = 0;
    while (y0 < ny) {
        int nyt = R - (y0 > 0 ? 1 : 0);               // rows left after the upper ring
        if (y0 + nyt >= ny) nyt = ny - y0;              // last window: no lower ring
        else nyt -= 1;                                   // keep a row for the lower ring
        w.push_back({y0, nyt});
        y0 += nyt;
    }
    return w;
}

// Predicted rows a full-width tile holds (kinds 1 and 2).
int shape_rows(const sllg_level& L, const Shape& s)
{
    return s.kind == 1 ? (s.tx / L.nx) * s.ty : (s.tx * s.ty) / L.nx;
}

// Dynamic LDS of a k_rows2 tile: two m_n planes (predicted rows + 2) and
// two m' planes (predicted rows), one float4 per cell.  With one cell per
// thread the planes sit at fixed strides: 2 tx cells for m_n, tx for m'.
size_t rows2_lds(const sllg_level& L, const Shape& s)
{
    if (s.ty == 1) return 16 * (size_t)6 * s.tx;
    const int R = std::min(shape_rows(L, s), L.ny);
    return 16 * (size_t)(2 * (R + 2) + 2 * R) * L.nx;
}

// Cells of an m_n plane of a k_rows2 tile (predicted rows + 2).
int64_t rows2_plane_cells(const sllg_level& L, const Shape& s)
{
    return (int64_t)(std::min(shape_rows(L, s), L.ny) + 2) * L.nx;
}

bool shape_fits(const sllg_level& L, const Shape& s)
{
    if (s.kind == 0) return true;
    if (L.nx > s.tx) return false;
    const int R = shape_rows(L, s);
    if (s.kind == 2) {
        if (R < L.ny && 2 * L.nx > s.tx) return false;   // the two extra rows need 2 nx threads
        if (rows2_lds(L, s) > 160 * 1024 - 1024) return false;
        if (s.ty == 1 && rows2_plane_cells(L, s) > 2 * s.tx) return false;   // the fixed m_n stride
    }
    return !row_windows(L.ny, R).empty();
}

int64_t tiles_for(const sllg_level& L, const Shape& s, int tz)
{
    if (s.kind >= 1) {
        if (!shape_fits(L, s)) return 0;
        return (int64_t)row_windows(L.ny, shape_rows(L, s)).size() * ceil_div(L.nz, tz);
    }
    return ceil_div(L.nx, s.tx) * ceil_div(L.ny, s.ty) * ceil_div(L.nz, tz);
}

int64_t max_tiles_for(const sllg_level& L)
{
    int64_t m = 0;
    for (const Shape& s : kShapes)
        for (int tz : kTzChoices) m = std::max(m, tiles_for(L, s, tz));
    return m;
}

}  // namespace

struct sllg_ctx {
    sllg_material mat{};
    std::vector<LevelHost> lv;
    int ckpt_every = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay{};
    // device views
    LevelDev* d_levels = nullptr;
    InstDev* d_insts = nullptr;
    AccDev* d_accs = nullptr;
    int64_t* d_steps = nullptr;
    int* d_status = nullptr;
    uint32_t* d_inst_cnt = nullptr;
    uint32_t* d_launch_cnt = nullptr;
    double* d_partials = nullptr;
    TileDev* d_tiles = nullptr;
    GroupDev* d_groups = nullptr;
    SlotDev* d_slots = nullptr;
    ChunkDev* d_chunks = nullptr;
    float* d_buf0 = nullptr;
    float* d_buf1 = nullptr;
    float* d_axes = nullptr;
    double* d_records = nullptr;
    float* d_ckpt = nullptr;
    float* d_tape = nullptr;
    float* d_lam = nullptr;
    double* d_weights = nullptr;
    double* d_grads = nullptr;
    SlabDev* d_slabs = nullptr;
    uint64_t* d_xch = nullptr;
    uint32_t slab_seq = 0;        // slab launches so far (exchange tags)
    double* d_spart = nullptr;
    int32_t* d_islab = nullptr;   // per instance: first slab (level-relative), then slab count
    float* d_demag = nullptr;     // demagnetising-tensor tables of the levels (magnetostatics)
    std::vector<SlabDev> h_slabs;
    std::vector<int32_t> h_islab;
    // host mirrors
    std::vector<LevelDev> h_levels;
    std::vector<InstDev> h_insts;
    std::vector<TileDev> h_tiles;
    // resident sets: levels advanced together by one launch sequence
    struct ResSet {
        std::vector<int> levels;
        int group0 = 0, ngroups = 0;
        int nw = 1, cpw = 1;
        size_t lds = 0;
    };
    std::vector<ResSet> res_sets;
    std::vector<GroupDev> h_groups;
    std::vector<SlotDev> h_slots;
    std::vector<ChunkDev> h_chunks;
    // timing of the dominant kernel
    int timing = 0;              // 0 off, k: time every k-th launch unit of the dominant kernel
    int64_t unit_counter = 0;
    std::vector<int64_t> ev_launches;   // kernel launches inside each timed event pair
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int64_t timed_cells = 0;            // cell-updates inside the timed event pairs
    int max_lds = 65536;
    int num_cus = 256;
    // HIP graphs of kGraphSteps stream launches per level (the stream kernel
    // reads its step index from device memory, so one graph serves any step)
    bool use_graph = true;
    // polls of one exchange word before a slab workgroup gives up (bounded
    // waits; sllg_set_spin_limit)
    uint32_t spin_limit = 1u << 20;
    int static_dev = -1;          // device whose static workspace this context holds (sllg_init_static)
    hipStream_t cap_stream = nullptr;
    std::map<int, hipGraphExec_t> graphs;
};

namespace {

// ---------------------------------------------------------------------------
// Parameter compiler (modified Grinstein-Koch rule).
// ---------------------------------------------------------------------------
int validate(const sllg_material* m, const sllg_level* L, int n)
{
    if (!m || !L || n < 1 || n > 255) return fail(SLLG_E_INVAL, "need 1..255 levels and a material");
    if (!(m->a0_m > 0) || !(m->Ms0 > 0) || !(m->A0 >= 0) || !(m->K0 >= 0) || !(m->T_K >= 0))
        return fail(SLLG_E_INVAL, "material: a0, Ms0 > 0; A0, K0, T >= 0 required");
    if (!(m->Hmax_Oe >= 0) || !(m->sweep_Oe_per_ns > 0) || m->n_cycles < 1)
        return fail(SLLG_E_INVAL, "protocol: Hmax >= 0, sweep rate > 0, n_cycles >= 1 required");
    if (m->wave < 0 || m->wave > 2) return fail(SLLG_E_INVAL, "unknown waveform %d", m->wave);
    double an = std::sqrt(m->easy_axis[0] * m->easy_axis[0] + m->easy_axis[1] * m->easy_axis[1] +
                          m->easy_axis[2] * m->easy_axis[2]);
    if (!(an > 0) || !std::isfinite(an)) return fail(SLLG_E_INVAL, "easy axis must be non-zero");
    if (!(m->ms_scale > 0)) return fail(SLLG_E_INVAL, "ms_scale must be > 0");
    if (m->sr_ref_Oe_per_ns > 0 && !(m->alpha_ref >= 0))
        return fail(SLLG_E_INVAL, "alpha_ref must be >= 0");
    for (int i = 0; i < n; ++i) {
        const sllg_level& l = L[i];
        if (l.nx < 1 || l.ny < 1 || l.nz < 1 || l.nx > 4096 || l.ny > 4096 || l.nz > 4096 ||
            (int64_t)l.nx * l.ny * l.nz > (1 << 26))
            return fail(SLLG_E_INVAL, "level %d: dims must be 1..4096 and at most 2^26 cells", i);
        if (!(l.b >= 1.0)) return fail(SLLG_E_INVAL, "level %d: b must be >= 1", i);
        if (l.n_real < 1) return fail(SLLG_E_INVAL, "level %d: n_real must be >= 1", i);
        if (!(l.alpha >= 0) && !(m->sr_ref_Oe_per_ns > 0))
            return fail(SLLG_E_INVAL, "level %d: alpha must be >= 0", i);
        if (l.dt_s < 0 || !std::isfinite(l.dt_s)) return fail(SLLG_E_INVAL, "level %d: dt must be >= 0", i);
        if (!(l.cone_deg >= 0) || l.cone_deg >= 90) return fail(SLLG_E_INVAL, "level %d: cone in [0, 90)", i);
        if (l.record_every < 1) return fail(SLLG_E_INVAL, "level %d: record_every must be >= 1", i);
        if (m->demag && (int64_t)l.nx * l.ny * l.nz > kDemagMaxCells)
            return fail(SLLG_E_INVAL, "level %d: magnetostatics holds at most 1024 cells per realization", i);
    }
    return SLLG_OK;
}

// ---------------------------------------------------------------------------
// Demagnetising tensor of two uniformly magnetised cubes of unit edge whose
// centres are (X, Y, Z) edges apart (Newell, Williams and Dunlop, J. Geophys.
// Res. 98, 9551 (1993)): N_xx is -1/(4 pi) times the second differences (step
// 1, weights 1 -2 1) in x, y and z of their function f(x, y, z), N_xy the same
// of g(x, y, z); the other components permute the arguments.  Long double:
// the differences cancel to ~r^-3 from terms ~r^2.
// ---------------------------------------------------------------------------
using ldbl = long double;

ldbl asinh_ratio(ldbl a, ldbl b2)   // asinh(a / sqrt(b2)) for a >= 0, b2 > 0
{
    return std::log((a + std::sqrt(a * a + b2)) / std::sqrt(b2));
}

ldbl nwl_f(ldbl x, ldbl y, ldbl z)
{
    x = std::fabs(x);
    y = std::fabs(y);
    z = std::fabs(z);
    const ldbl xx = x * x, yy = y * y, zz = z * z, R = std::sqrt(xx + yy + zz);
    ldbl v = (2 * xx - yy - zz) * R / 6;
    if (y > 0 && xx + zz > 0) v += y * (zz - xx) / 2 * asinh_ratio(y, xx + zz);
    if (z > 0 && xx + yy > 0) v += z * (yy - xx) / 2 * asinh_ratio(z, xx + yy);
    if (x > 0 && y > 0 && z > 0) v -= x * y * z * std::atan2(y * z, x * R);
    return v;
}

ldbl nwl_g(ldbl x, ldbl y, ldbl z)
{
    const ldbl sign = (x < 0) == (y < 0) ? 1 : -1;   // odd in x and in y
    x = std::fabs(x);
    y = std::fabs(y);
    z = std::fabs(z);
    const ldbl xx = x * x, yy = y * y, zz = z * z, R = std::sqrt(xx + yy + zz);
    ldbl v = -x * y * R / 3;
    if (x > 0 && y > 0) {
        if (z > 0) {
            v += x * y * z * asinh_ratio(z, xx + yy);
            v -= z * zz / 6 * std::atan2(x * y, z * R);
            v -= z * yy / 2 * std::atan2(x * z, y * R);
            v -= z * xx / 2 * std::atan2(y * z, x * R);
        }
        v += y * (3 * zz - yy) / 6 * asinh_ratio(x, yy + zz);
        v += x * (3 * zz - xx) / 6 * asinh_ratio(y, xx + zz);
    }
    return sign * v;
}

template <class F>
ldbl second_differences(F fn, ldbl X, ldbl Y, ldbl Z)
{
    auto dz = [&](ldbl x, ldbl y) { return fn(x, y, Z + 1) - 2 * fn(x, y, Z) + fn(x, y, Z - 1); };
    auto dy = [&](ldbl x) { return dz(x, Y + 1) - 2 * dz(x, Y) + dz(x, Y - 1); };
    return -(dy(X + 1) - 2 * dy(X) + dy(X - 1)) / (4 * (ldbl)kPi);
}

// -Ms N of an nx x ny x nz grid as six planes (xx yy zz xy xz yz) of the
// table's offsets: every offset (wide; index ((dz + nz-1) wy + dy + ny-1) wx
// + dx + nx-1 with the strides of demag_wide_dims; the padding entries are
// zero and never read), or those with dx, dy, dz >= 0 (octant; index
// dx + nx (dy + ny dz)), from which the kernel takes the others by the
// parities of N: the diagonal is even in each component, N_xy odd in dx and
// dy, N_xz in dx and dz, N_yz in dy and dz.
void demag_table(const sllg_level& L, double Ms, std::vector<float>& out)
{
    const bool wide = demag_is_wide(L);
    const WideDims d = demag_wide_dims(L);
    const int ex = wide ? d.wx : L.nx, ey = wide ? d.wy : L.ny, ez = wide ? 2 * L.nz - 1 : L.nz;
    const int cx = wide ? L.nx - 1 : 0, cy = wide ? L.ny - 1 : 0, cz = wide ? L.nz - 1 : 0;
    const size_t n = (size_t)ex * ey * ez;
    out.assign(6 * n, 0.0f);
    for (int k = 0; k < ez; ++k)
        for (int j = 0; j < ey; ++j)
            for (int i = 0; i < ex; ++i) {
                if (i - cx > L.nx - 1 || j - cy > L.ny - 1) continue;   // padding
                const ldbl X = i - cx, Y = j - cy, Z = k - cz;
                const size_t o = ((size_t)k * ey + j) * ex + i;
                out[o] = (float)(-Ms * second_differences(nwl_f, X, Y, Z));
                out[n + o] = (float)(-Ms * second_differences(nwl_f, Y, X, Z));
                out[2 * n + o] = (float)(-Ms * second_differences(nwl_f, Z, Y, X));
                out[3 * n + o] = (float)(-Ms * second_differences(nwl_g, X, Y, Z));
                out[4 * n + o] = (float)(-Ms * second_differences(nwl_g, X, Z, Y));
                out[5 * n + o] = (float)(-Ms * second_differences(nwl_g, Y, Z, X));
            }
}

void compile_level(const sllg_material& m, const sllg_level& in, LevelHost& o)
{
    o.in = in;
    const double Tc = m.Tc_K > 0 ? m.Tc_K : 1.44 * m.a0_m * m.A0 / kKB;
    o.t = m.T_K / Tc;
    o.zeta = o.t / in.b + 1.0 - o.t;                      // text after Eq. (11)
    o.A = m.scale_AK ? o.zeta * m.A0 : m.A0;              // Eq. (8)
    o.K = m.scale_AK ? o.zeta * o.zeta * o.zeta * m.K0 : m.K0;   // Eq. (9)
    o.hscale = m.scale_H ? o.zeta : 1.0;                  // Eq. (10)
    o.cM = m.scale_H ? 1.0 - m.delta * (1.0 - o.zeta) : 1.0;     // Eq. (13)
    o.Ms = m.ms_scale * m.Ms0;
    o.a = in.b * m.a0_m;
    o.V = o.a * o.a * o.a;
    o.alpha = m.sr_ref_Oe_per_ns > 0 ? m.alpha_ref * m.sweep_Oe_per_ns / m.sr_ref_Oe_per_ns : in.alpha;
    o.c_ex = 2.0 * o.A / (kMu0 * o.Ms * o.a * o.a);
    o.hk = 2.0 * o.K / (kMu0 * o.Ms);
    o.hz_amp = o.hscale * m.Hmax_Oe * kOe;
    if (in.dt_s > 0) {
        o.dt = in.dt_s;
    } else {
        const double bound = 0.15 * std::sqrt(1.0 + o.alpha * o.alpha) /
                             (kGamma0 * (12.0 * o.c_ex + o.hk + o.hz_amp));
        double fs = std::floor(bound / 1e-15);
        fs = std::max(1.0, std::min(5.0, fs));
        o.dt = fs * 1e-15;
    }
    o.gamma1 = kGamma0 / (1.0 + o.alpha * o.alpha);
    o.sigma = std::sqrt(2.0 * o.alpha * kKB * m.T_K / (kGamma0 * kMu0 * o.Ms * o.V * o.dt));
    const double period = 4.0 * m.Hmax_Oe / (m.sweep_Oe_per_ns * 1e9);
    o.n_period = std::max<int64_t>(1, (int64_t)std::llround(period / o.dt));
    o.n_steps = o.n_period * m.n_cycles;
    o.n_rec = o.n_steps / in.record_every + 1;
    o.ncell = (int64_t)in.nx * in.ny * in.nz;
}

LevelDev to_dev(const sllg_material& m, const LevelHost& h, int tag)
{
    LevelDev d{};
    d.c_ex = (float)h.c_ex;
    d.hk = (float)h.hk;
    d.g1 = (float)h.gamma1;
    d.ag1 = (float)(h.alpha * h.gamma1);
    d.sigma = (float)h.sigma;
    d.dt = (float)h.dt;
    d.half_dt = (float)(0.5 * h.dt);
    const double an = std::sqrt(m.easy_axis[0] * m.easy_axis[0] + m.easy_axis[1] * m.easy_axis[1] +
                                m.easy_axis[2] * m.easy_axis[2]);
    d.ux = (float)(m.easy_axis[0] / an);
    d.uy = (float)(m.easy_axis[1] / an);
    d.uz = (float)(m.easy_axis[2] / an);
    d.hz_amp = h.hz_amp;
    d.hz_oe = h.hz_amp / kOe;
    d.n_period = h.n_period;
    d.n_steps = h.n_steps;
    d.inv_period = 1.0 / (double)h.n_period;
    d.wave = m.wave;
    d.level_tag = tag;
    d.record_every = h.in.record_every;
    d.ncell = (int32_t)h.ncell;
    d.nx = h.in.nx;
    d.ny = h.in.ny;
    d.nz = h.in.nz;
    d.has_axes = h.axes_off >= 0 ? 1 : 0;
    d.axes_off = h.axes_off >= 0 ? h.axes_off : 0;
    d.n_rec = h.n_rec;
    d.demag_off = h.demag_off >= 0 ? h.demag_off : 0;
    return d;
}

int resident_fits(const LevelHost& h, int max_lds)
{
    // two AoS copies of the state plus per-chunk and per-slot bookkeeping
    const int64_t chunks = ceil_div(h.ncell, 64);
    const int64_t bytes = 24 * h.ncell + 8 * chunks + 64 + (int64_t)sizeof(AccDev) + 16;
    return bytes <= max_lds && chunks <= kResMaxChunks;
}

Layout make_layout(const sllg_material& m, const std::vector<LevelHost>& lv, int ckpt_every)
{
    Layout L{};
    int64_t ninst = 0, state = 0, axes = 0, rec = 0, ckpt = 0, tiles = 0, chunks = 0, tape = 0, lam = 0,
            maxw = 0;
    for (const LevelHost& h : lv) {
        ninst += h.in.n_real;
        state += 3 * h.ncell * h.in.n_real;
        if (h.in.cone_deg > 0) axes += 3 * h.ncell;
        rec += h.n_rec * h.in.n_real;
        if (ckpt_every > 0) {
            const int64_t nck = ceil_div(h.n_steps, ckpt_every);
            ckpt += nck * 3 * h.ncell * h.in.n_real;
            tape = std::max<int64_t>(tape, (int64_t)ckpt_every * 9 * h.ncell * h.in.n_real);
            lam = std::max<int64_t>(lam, 6 * h.ncell * h.in.n_real);
            maxw = std::max<int64_t>(maxw, h.n_steps + 1);
        }
        tiles += max_tiles_for(h.in) * h.in.n_real;
        chunks += ceil_div(h.ncell, 64) * h.in.n_real;
        if (slab_eligible(h.in)) {
            const int64_t ns = (int64_t)h.in.nz * h.in.n_real;   // one-plane slabs at most
            L.max_slabs += ns;
            L.xch_words += 2 * ns * 12 * (int64_t)h.in.nx * h.in.ny;
        }
        if (m.demag) L.demag_floats += demag_table_floats(h.in);
    }
    L.ninst_total = ninst;
    L.state_floats = state;
    L.axes_floats = axes;
    L.rec_doubles = rec;
    L.ckpt_floats = ckpt;
    L.tape_floats = tape;
    L.lam_floats = lam;
    L.max_tiles = tiles;
    L.max_chunks = chunks;
    L.max_groups = ninst;
    L.max_w = maxw;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.levels = take(sizeof(LevelDev) * lv.size());
    L.insts = take(sizeof(InstDev) * ninst);
    L.accs = take(sizeof(AccDev) * ninst);
    L.steps = take(sizeof(int64_t) * lv.size());
    L.status = take(sizeof(int) * 4);
    L.inst_cnt = take(sizeof(uint32_t) * ninst);
    L.launch_cnt = take(sizeof(uint32_t) * (lv.size() + 1));
    L.partials = take(sizeof(double) * 2 * tiles);   // two step parities
    L.tiles = take(sizeof(TileDev) * tiles);
    L.groups = take(sizeof(GroupDev) * ninst);
    L.slots = take(sizeof(SlotDev) * ninst);
    L.chunks = take(sizeof(ChunkDev) * chunks);
    L.buf0 = take(sizeof(float) * state);
    L.buf1 = take(sizeof(float) * state);
    L.axes = take(sizeof(float) * axes);
    L.records = take(sizeof(double) * rec);
    L.ckpt = take(sizeof(float) * ckpt);
    L.tape = take(sizeof(float) * tape);
    L.lam = take(sizeof(float) * lam);
    L.weights = take(sizeof(double) * 2 * maxw);
    L.grads = take(sizeof(double) * 10 * ninst);
    L.slabs = take(sizeof(SlabDev) * L.max_slabs);
    L.xch = take(sizeof(uint64_t) * L.xch_words);
    L.spart = take(sizeof(double) * L.max_slabs * kSlabChunk);
    L.islab = take(sizeof(int32_t) * 2 * ninst);
    L.demag = take(sizeof(float) * L.demag_floats);
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------
void build_tiles(sllg_ctx* C, LevelHost& h)
{
    const Shape s = kShapes[h.shape];
    h.tile0 = (int)C->h_tiles.size();
    for (int r = 0; r < h.ninst; ++r) {
        InstDev& I = C->h_insts[h.inst0 + r];
        I.tile0 = (int)C->h_tiles.size();
        if (s.kind >= 1) {
            const auto rows = row_windows(h.in.ny, shape_rows(h.in, s));
            for (int z0 = 0; z0 < h.in.nz; z0 += h.tz)
                for (const auto& w : rows) {
                    TileDev t{};
                    t.inst = h.inst0 + r;
                    t.x0 = 0;
                    t.y0 = (int16_t)w.first;
                    t.z0 = (int16_t)z0;
                    t.nxt = (int16_t)h.in.nx;
                    t.nyt = (int16_t)w.second;
                    t.nzt = (int16_t)std::min(h.tz, h.in.nz - z0);
                    C->h_tiles.push_back(t);
                }
            I.ntiles = (int)C->h_tiles.size() - I.tile0;
            continue;
        }
        for (int z0 = 0; z0 < h.in.nz; z0 += h.tz)
            for (int y0 = 0; y0 < h.in.ny; y0 += s.ty)
                for (int x0 = 0; x0 < h.in.nx; x0 += s.tx) {
                    TileDev t{};
                    t.inst = h.inst0 + r;
                    t.x0 = (int16_t)x0;
                    t.y0 = (int16_t)y0;
                    t.z0 = (int16_t)z0;
                    t.nxt = (int16_t)std::min(s.tx, h.in.nx - x0);
                    t.nyt = (int16_t)std::min(s.ty, h.in.ny - y0);
                    t.nzt = (int16_t)std::min(h.tz, h.in.nz - z0);
                    C->h_tiles.push_back(t);
                }
        I.ntiles = (int)C->h_tiles.size() - I.tile0;
    }
    h.ntiles = (int)C->h_tiles.size() - h.tile0;
}

// Default stream shape: whole x-y planes when they fit a shape, else the
// widest x tile; z ranges long enough to amortise the two halo planes while
// keeping several workgroups per compute unit.
void default_stream_shape(const sllg_ctx* C, LevelHost& h)
{
    int best = -1;
    // full-width rows kernel: the fewest threads that hold a whole plane, else 1024 x 2
    for (int i = 0; i < kNumShapes; ++i) {
        const Shape& s = kShapes[i];
        if (s.kind != 1 || !shape_fits(h.in, s)) continue;
        if ((s.tx / h.in.nx) * s.ty >= h.in.ny) {
            if (best < 0 || s.tx * s.ty < kShapes[best].tx * kShapes[best].ty) best = i;
        }
    }
    if (best < 0)
        for (int i = 0; i < kNumShapes; ++i)
            if (kShapes[i].kind == 1 && kShapes[i].tx == 512 && kShapes[i].ty == 2 && shape_fits(h.in, kShapes[i]))
                best = i;
    if (best < 0) best = 0;
    h.shape = best;
    const Shape s = kShapes[best];
    const int64_t xy = tiles_for(h.in, s, h.in.nz) * h.ninst;
    int tz = 64;
    while (tz > 1 && xy * ceil_div(h.in.nz, tz) < 2LL * C->num_cus) tz /= 2;
    h.tz = s.kind == 0 ? std::max(tz, std::min(s.pz, h.in.nz)) : tz;
}

// Group instances of resident levels with equal sweep length.
int build_resident(sllg_ctx* C)
{
    C->res_sets.clear();
    C->h_groups.clear();
    C->h_slots.clear();
    C->h_chunks.clear();
    std::map<int64_t, std::vector<int>> by_len;
    for (int l = 0; l < (int)C->lv.size(); ++l)
        if (C->lv[l].plan == kPlanResident) by_len[C->lv[l].n_steps * 1000003 + C->lv[l].step].push_back(l);
    for (auto& kv : by_len) {
        sllg_ctx::ResSet rs;
        rs.levels = kv.second;
        // instances, largest first
        std::vector<int> inst;
        int64_t total = 0;
        for (int l : rs.levels)
            for (int r = 0; r < C->lv[l].ninst; ++r) {
                inst.push_back(C->lv[l].inst0 + r);
                total++;
            }
        std::stable_sort(inst.begin(), inst.end(), [&](int a, int b) {
            return C->lv[C->h_insts[a].level].ncell > C->lv[C->h_insts[b].level].ncell;
        });
        // Instances go, largest first, to the group with the fewest chunks so
        // far (ties to the lowest index).  Number of groups: one instance per
        // group up to two per CU, else pack (more groups while a group would
        // exceed the chunk or LDS limit).  Between one and two instances per
        // CU, one group per CU is taken instead when the extra instances fit
        // beside others without any group outgrowing the largest instance:
        // a step then costs what the largest instance costs alone, without
        // two workgroups sharing a CU.
        std::vector<std::vector<int>> members;
        int64_t max_chunks = 0, max_lds = 0, max_cells = 0;
        auto pack = [&](int ngr) {
            members.assign(ngr, {});
            std::vector<int64_t> load(ngr, 0), lds(ngr, 0);
            for (size_t k = 0; k < inst.size(); ++k) {
                int g = 0;
                for (int q = 1; q < ngr; ++q)
                    if (load[q] < load[g]) g = q;
                const LevelHost& h = C->lv[C->h_insts[inst[k]].level];
                members[g].push_back(inst[k]);
                load[g] += ceil_div(h.ncell, 64);
                lds[g] += 24 * h.ncell;
            }
            max_chunks = max_lds = max_cells = 0;
            for (int g = 0; g < ngr; ++g) {
                max_chunks = std::max(max_chunks, load[g]);
                max_cells = std::max(max_cells, lds[g] / 24);
                max_lds = std::max<int64_t>(max_lds, lds[g] + 8 * load[g] + 48 +
                                                         (int64_t)(sizeof(AccDev) + 16) * members[g].size());
            }
        };
        int ng = (int)std::min<int64_t>(total, 2LL * C->num_cus);
        if (total > 2LL * C->num_cus) ng = C->num_cus;
        bool packed = false;
        if (total > C->num_cus && total <= 2LL * C->num_cus) {
            const int64_t largest = ceil_div(C->lv[C->h_insts[inst[0]].level].ncell, 64);
            pack(C->num_cus);
            if (max_chunks <= largest && max_lds <= C->max_lds) {
                ng = C->num_cus;
                packed = true;
            }
        }
        while (!packed) {
            pack(ng);
            if ((max_chunks <= kResMaxChunks && max_lds <= C->max_lds) || ng >= total) break;
            ng = (int)std::min<int64_t>(total, 2LL * ng);
        }
        if (max_lds > C->max_lds)
            return fail(SLLG_E_INVAL, "resident plan: %lld bytes of LDS per workgroup exceed %d",
                        (long long)max_lds, C->max_lds);
        int pick = -1;
        const int nk = (int)(sizeof(kResKernels) / sizeof(kResKernels[0]));
        for (int i = 0; i < nk && pick < 0; ++i)
            if (kResKernels[i].cpw == 1 && kResKernels[i].nw > max_chunks) pick = i;
        for (int i = 0; i < nk && pick < 0; ++i)
            if (kResKernels[i].nw * kResKernels[i].cpw >= max_chunks) pick = i;
        if (pick < 0) return fail(SLLG_E_INVAL, "resident plan: %lld chunks per workgroup", (long long)max_chunks);
        rs.nw = kResKernels[pick].nw;
        rs.cpw = kResKernels[pick].cpw;
        rs.group0 = (int)C->h_groups.size();
        rs.ngroups = ng;
        for (int g = 0; g < ng; ++g) {
            GroupDev G{};
            G.slot0 = (int)C->h_slots.size();
            G.chunk0 = (int)C->h_chunks.size();
            int cells = 0, nch = 0;
            for (size_t s = 0; s < members[g].size(); ++s) {
                const int ii = members[g][s];
                const LevelHost& h = C->lv[C->h_insts[ii].level];
                SlotDev S{};
                S.inst = ii;
                S.lds_off = cells;
                S.chunk0 = nch;
                S.nchunks = (int)ceil_div(h.ncell, 64);
                for (int k = 0; k < S.nchunks; ++k) {
                    ChunkDev ch{};
                    ch.inst = ii;
                    ch.slot = (int)s;
                    ch.c0 = 64 * k;
                    C->h_chunks.push_back(ch);
                }
                cells += (int)h.ncell;
                nch += S.nchunks;
                C->h_slots.push_back(S);
            }
            G.nslots = (int)members[g].size();
            G.nchunks = nch;
            G.ncells = cells;
            C->h_groups.push_back(G);
        }
        rs.lds = (size_t)max_lds + 64;
        // kernels with noise waves (NW <= 8, at most 7 chunks) also hold the
        // thermal field of two steps: 24 bytes per cell
        if (rs.nw <= 8) rs.lds += (size_t)(24 * max_cells);
        C->res_sets.push_back(rs);
    }
    return SLLG_OK;
}

int upload_tables(sllg_ctx* C)
{
    if ((int64_t)C->h_tiles.size() > C->lay.max_tiles ||
        (int64_t)C->h_chunks.size() > C->lay.max_chunks ||
        (int64_t)C->h_groups.size() > C->lay.max_groups)
        return fail(SLLG_E_WORKSPACE, "plan tables exceed the reserved workspace");
    for (size_t l = 0; l < C->lv.size(); ++l) C->h_levels[l] = to_dev(C->mat, C->lv[l], (int)l);
    HIP_OK(hipMemcpyAsync(C->d_levels, C->h_levels.data(), sizeof(LevelDev) * C->h_levels.size(),
                          hipMemcpyHostToDevice, C->stream));
    HIP_OK(hipMemcpyAsync(C->d_insts, C->h_insts.data(), sizeof(InstDev) * C->h_insts.size(),
                          hipMemcpyHostToDevice, C->stream));
    if (!C->h_tiles.empty())
        HIP_OK(hipMemcpyAsync(C->d_tiles, C->h_tiles.data(), sizeof(TileDev) * C->h_tiles.size(),
                              hipMemcpyHostToDevice, C->stream));
    if (!C->h_groups.empty()) {
        HIP_OK(hipMemcpyAsync(C->d_groups, C->h_groups.data(), sizeof(GroupDev) * C->h_groups.size(),
                              hipMemcpyHostToDevice, C->stream));
        HIP_OK(hipMemcpyAsync(C->d_slots, C->h_slots.data(), sizeof(SlotDev) * C->h_slots.size(),
                              hipMemcpyHostToDevice, C->stream));
        HIP_OK(hipMemcpyAsync(C->d_chunks, C->h_chunks.data(), sizeof(ChunkDev) * C->h_chunks.size(),
                              hipMemcpyHostToDevice, C->stream));
    }
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

// Slabs of every instance of a slab-plan level: nz split into runs of
// slab_tz or slab_tz + 1 planes (each at least 2).  Workgroups are handed to
// the 8 XCDs round-robin by block index, so the slabs of one instance are
// placed at block indices of one residue mod 8 where the counts allow: their
// exchanges then stay within one XCD.  The order only affects speed.
constexpr int kXcds = 8;

// Slabs per instance: ceil(nz / tz), but never a slab thinner than the kernel
// allows (two planes for kind 0, one for kind 1); every slab then has at most
// tz + 1 planes.
int slab_count(const LevelHost& h)
{
    const int minp = kSlabKernels[h.slab_kernel].kind == 0 ? 2 : 1;
    const int tz = std::max(minp, h.slab_tz);
    return std::max(1, std::min((h.in.nz + tz - 1) / tz, h.in.nz / minp));
}

void build_slabs(sllg_ctx* C, LevelHost& h)
{
    h.slab0 = (int)C->h_slabs.size();
    const int nz = h.in.nz;
    const int nsl = slab_count(h);
    const int base = nz / nsl, extra = nz % nsl;
    const int total = nsl * h.ninst;
    // lid = r * nsl + k  ->  block index
    std::vector<std::vector<int>> bins(kXcds);
    for (int r = 0; r < h.ninst; ++r)
        for (int k = nsl - 1; k >= 0; --k) bins[r % kXcds].push_back(r * nsl + k);   // popped from the back
    std::vector<int> block_of(total);
    for (int b = 0; b < total; ++b) {
        int pick = b % kXcds;
        if (bins[pick].empty())
            pick = (int)(std::max_element(bins.begin(), bins.end(),
                                          [](const std::vector<int>& a, const std::vector<int>& c) {
                                              return a.size() < c.size();
                                          }) - bins.begin());
        block_of[bins[pick].back()] = b;
        bins[pick].pop_back();
    }
    std::vector<SlabDev> tab(total);
    for (int r = 0; r < h.ninst; ++r) {
        C->h_islab[2 * (h.inst0 + r)] = r * nsl;
        C->h_islab[2 * (h.inst0 + r) + 1] = nsl;
        int z0 = 0;
        for (int k = 0; k < nsl; ++k) {
            const int lid = r * nsl + k;
            SlabDev d{};
            d.inst = h.inst0 + r;
            d.z0 = z0;
            d.nzs = base + (k < extra ? 1 : 0);
            d.prev = k > 0 ? block_of[lid - 1] : -1;
            d.next = k + 1 < nsl ? block_of[lid + 1] : -1;
            d.lid = lid;
            z0 += d.nzs;
            tab[block_of[lid]] = d;
        }
    }
    C->h_slabs.insert(C->h_slabs.end(), tab.begin(), tab.end());
    h.nslab = total;
}

int replan(sllg_ctx* C)
{
    C->h_tiles.clear();
    C->h_slabs.clear();
    int64_t xo = 0;
    for (LevelHost& h : C->lv) {
        if (h.plan == kPlanStream) build_tiles(C, h);
        if (h.plan == kPlanSlab) {
            build_slabs(C, h);
            h.xch_off = xo;
            xo += 2LL * h.nslab * 12 * h.in.nx * h.in.ny;
        }
    }
    if ((int64_t)C->h_slabs.size() > C->lay.max_slabs || xo > C->lay.xch_words)
        return fail(SLLG_E_WORKSPACE, "slab tables exceed the reserved workspace");
    if (!C->h_slabs.empty()) {
        HIP_OK(hipMemcpyAsync(C->d_slabs, C->h_slabs.data(), sizeof(SlabDev) * C->h_slabs.size(),
                              hipMemcpyHostToDevice, C->stream));
        HIP_OK(hipMemcpyAsync(C->d_islab, C->h_islab.data(), sizeof(int32_t) * C->h_islab.size(),
                              hipMemcpyHostToDevice, C->stream));
    }
    int rc = build_resident(C);
    if (rc) return rc;
    for (const auto& g : C->graphs) (void)hipGraphExecDestroy(g.second);
    C->graphs.clear();
    return upload_tables(C);
}

// ---------------------------------------------------------------------------
// Launching
// ---------------------------------------------------------------------------
template <int NW, int CPW>
hipError_t launch_res(sllg_ctx* C, const sllg_ctx::ResSet& rs, int64_t n0, int64_t ns)
{
    const size_t lds = rs.lds;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_resident<NW, CPW>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_resident<NW, CPW>), dim3(rs.ngroups), dim3(kResThreads<NW>), lds, C->stream,
                       C->d_groups + rs.group0, C->d_slots, C->d_chunks, C->d_insts, C->d_levels,
                       C->d_buf0, C->d_buf1, C->d_axes, C->d_records, C->d_accs, C->d_ckpt,
                       C->ckpt_every, n0, ns, C->d_status);
    return hipGetLastError();
}

hipError_t dispatch_res(sllg_ctx* C, const sllg_ctx::ResSet& rs, int64_t n0, int64_t ns)
{
    switch (rs.nw * 100 + rs.cpw) {
    case 201: return launch_res<2, 1>(C, rs, n0, ns);
    case 401: return launch_res<4, 1>(C, rs, n0, ns);
    case 801: return launch_res<8, 1>(C, rs, n0, ns);
    case 1601: return launch_res<16, 1>(C, rs, n0, ns);
    case 1602: return launch_res<16, 2>(C, rs, n0, ns);
    default: return hipErrorInvalidValue;
    }
}

// Single-cell levels [l0, l1) (consecutive, the same sweep position): one
// quad of lanes per realization (four stepping waves and a loop wave per 64),
// ns steps.
hipError_t dispatch_lanes(sllg_ctx* C, int l0, int l1, int64_t n0, int64_t ns)
{
    const int i0 = C->lv[l0].inst0;
    const int ni = C->lv[l1 - 1].inst0 + C->lv[l1 - 1].ninst - i0;
    hipLaunchKernelGGL(k_lanes, dim3((unsigned)ceil_div(ni, kLanesThreads)), dim3(5 * 64), 0, C->stream,
                       C->d_insts, i0, ni, C->d_levels, C->d_buf0, C->d_buf1, C->d_axes, C->d_records, C->d_accs,
                       C->d_ckpt, C->ckpt_every, n0, ns, C->d_status);
    return hipGetLastError();
}

// Levels with magnetostatics: one workgroup per realization (chunks x cells
// threads), ns steps.
hipError_t dispatch_demag(sllg_ctx* C, int level, int64_t n0, int64_t ns)
{
    const LevelHost& h = C->lv[level];
    const int W = (int)demag_table_offsets(h.in);
    const size_t lds = 6 * sizeof(float) * (size_t)W;
    const WideDims d = demag_wide_dims(h.in);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_demag), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k_demag, dim3((unsigned)h.ninst), dim3((unsigned)demag_block((int)h.ncell)), lds, C->stream,
                       C->d_insts, h.inst0, C->d_levels, C->d_buf0, C->d_buf1, C->d_axes, C->d_demag,
                       demag_is_wide(h.in) ? 1 : 0, W, d.wx, d.wy, C->d_records, C->d_accs, C->d_ckpt, C->ckpt_every, n0, ns,
                       C->d_status);
    return hipGetLastError();
}

template <int TX, int TY, int PZ>
hipError_t launch_stream_t(sllg_ctx* C, int level)
{
    const LevelHost& h = C->lv[level];
    hipLaunchKernelGGL((k_stream<TX, TY, PZ>), dim3(h.ntiles), dim3(TX * TY * PZ), 0, C->stream,
                       C->d_tiles, C->d_insts, C->d_levels, C->d_buf0, C->d_buf1, C->d_axes,
                       C->d_steps, h.tile0, (int)C->lay.max_tiles, C->d_partials, C->d_inst_cnt,
                       C->d_launch_cnt + level, C->d_records, C->d_accs, C->d_ckpt, C->ckpt_every,
                       C->d_status);
    return hipGetLastError();
}

template <int NT, int K>
hipError_t launch_rows_t(sllg_ctx* C, int level)
{
    const LevelHost& h = C->lv[level];
    hipLaunchKernelGGL((k_rows<NT, K>), dim3(h.ntiles), dim3(NT), 0, C->stream, C->d_tiles, C->d_insts,
                       C->d_levels, C->d_buf0, C->d_buf1, C->d_axes, C->d_steps, h.tile0,
                       (int)C->lay.max_tiles, C->d_partials, C->d_inst_cnt, C->d_launch_cnt + level,
                       C->d_records, C->d_accs, C->d_ckpt, C->ckpt_every, C->d_status);
    return hipGetLastError();
}

template <int NT, int K>
hipError_t launch_rows2_t(sllg_ctx* C, int level)
{
    const LevelHost& h = C->lv[level];
    const size_t lds = rows2_lds(h.in, kShapes[h.shape]);
    const bool axes = h.axes_off >= 0;
    const void* fn = axes ? reinterpret_cast<const void*>(&k_rows2<NT, K, true>)
                          : reinterpret_cast<const void*>(&k_rows2<NT, K, false>);
    // raise the dynamic-LDS limit of the instantiation once per size
    static size_t set_lds[2] = {0, 0};
    if (lds > set_lds[axes]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        set_lds[axes] = lds;
    }
    if (axes)
        hipLaunchKernelGGL((k_rows2<NT, K, true>), dim3(h.ntiles), dim3(NT), lds, C->stream, C->d_tiles, C->d_insts,
                           C->d_levels, C->d_buf0, C->d_buf1, C->d_axes, C->d_steps, h.tile0, (int)C->lay.max_tiles,
                           C->d_partials, C->d_inst_cnt, C->d_launch_cnt + level, C->d_records, C->d_accs, C->d_ckpt,
                           C->ckpt_every, C->d_status);
    else
        hipLaunchKernelGGL((k_rows2<NT, K, false>), dim3(h.ntiles), dim3(NT), lds, C->stream, C->d_tiles,
                           C->d_insts, C->d_levels, C->d_buf0, C->d_buf1, C->d_axes, C->d_steps, h.tile0,
                           (int)C->lay.max_tiles, C->d_partials, C->d_inst_cnt, C->d_launch_cnt + level, C->d_records,
                           C->d_accs, C->d_ckpt, C->ckpt_every, C->d_status);
    return hipGetLastError();
}

hipError_t dispatch_stream(sllg_ctx* C, int level)
{
    const Shape s = kShapes[C->lv[level].shape];
    if (s.kind == 2) {
        switch (s.tx * 10 + s.ty) {
        case 10242: return launch_rows2_t<1024, 2>(C, level);
        case 10241: return launch_rows2_t<1024, 1>(C, level);
        case 7682: return launch_rows2_t<768, 2>(C, level);
        case 5122: return launch_rows2_t<512, 2>(C, level);
        case 2562: return launch_rows2_t<256, 2>(C, level);
        case 2561: return launch_rows2_t<256, 1>(C, level);
        case 1921: return launch_rows2_t<192, 1>(C, level);
        default: return hipErrorInvalidValue;
        }
    }
    if (s.kind == 1) {
        switch (s.tx * 10 + s.ty) {
        case 1921: return launch_rows_t<192, 1>(C, level);
        case 2561: return launch_rows_t<256, 1>(C, level);
        case 2562: return launch_rows_t<256, 2>(C, level);
        case 5121: return launch_rows_t<512, 1>(C, level);
        case 5122: return launch_rows_t<512, 2>(C, level);
        case 10241: return launch_rows_t<1024, 1>(C, level);
        case 2564: return launch_rows_t<256, 4>(C, level);
        default: return hipErrorInvalidValue;
        }
    }
    const int key = s.tx * 10000 + s.ty * 10 + s.pz;
    switch (key) {
    case 640081: return launch_stream_t<64, 8, 1>(C, level);
    case 320161: return launch_stream_t<32, 16, 1>(C, level);
    case 640161: return launch_stream_t<64, 16, 1>(C, level);
    case 320082: return launch_stream_t<32, 8, 2>(C, level);
    case 80244: return launch_stream_t<8, 24, 4>(C, level);
    case 80242: return launch_stream_t<8, 24, 2>(C, level);
    case 80241: return launch_stream_t<8, 24, 1>(C, level);
    case 160162: return launch_stream_t<16, 16, 2>(C, level);
    case 40128: return launch_stream_t<4, 12, 8>(C, level);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Slab plan
// ---------------------------------------------------------------------------
int slab_max_planes(const LevelHost& h)
{
    const int nsl = slab_count(h);
    return h.in.nz / nsl + (h.in.nz % nsl ? 1 : 0);
}

size_t slab_lds(const LevelHost& h)
{
    const int mp = slab_max_planes(h);
    // kind 0: one float4 per cell; kind 1: three float planes
    if (kSlabKernels[h.slab_kernel].kind == 0) return 16 * (size_t)(2 * mp + 6) * h.in.nx * h.in.ny;
    return sizeof(float) * (size_t)(2 * mp + 4) * 3 * h.in.nx * h.in.ny;
}

template <int KIND, int NT, int K>
hipError_t launch_slab_t(sllg_ctx* C, int level, int64_t n0, int ns, bool check_only, bool* fits)
{
    const LevelHost& h = C->lv[level];
    // every computed plane must have a thread slot (kind 0: slab + 2 halo planes)
    if (slab_max_planes(h) + (KIND == 0 ? 2 : 0) > K * (NT / (h.in.nx * h.in.ny))) {
        if (fits) *fits = false;
        return check_only ? hipSuccess : hipErrorInvalidConfiguration;
    }
    const size_t lds = slab_lds(h);
    const void* fn = KIND == 0 ? reinterpret_cast<const void*>(&k_slab<NT, K>)
                               : reinterpret_cast<const void*>(&k_slab2<NT, K>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NT, lds);
    if (e != hipSuccess) return e;
    // Every workgroup waits on its neighbours, so all must be resident.  The
    // occupancy query assumes a workgroup's waves spread evenly over the four
    // SIMDs; bound it by the wave slots of the fullest SIMD instead (a
    // workgroup may put ceil(waves / 4) waves on one SIMD).
    hipFuncAttributes fa{};
    e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const int vgpr = std::max(8, (fa.numRegs + 7) / 8 * 8);
    const int per_simd = std::min(8, 512 / vgpr);
    const int waves = NT / 64;
    nb = std::min(nb, per_simd / ((waves + 3) / 4));
    if (fits) *fits = (int64_t)nb * C->num_cus >= h.nslab && nb > 0;
    if (check_only) return hipSuccess;
    if ((int64_t)nb * C->num_cus < h.nslab) return hipErrorCooperativeLaunchTooLarge;
    const SlabDev* slabs = C->d_slabs + h.slab0;
    const InstDev* insts = C->d_insts;
    const LevelDev* levels = C->d_levels;
    float* b0 = C->d_buf0;
    float* b1 = C->d_buf1;
    const float* axes = C->d_axes;
    uint64_t* xch = C->d_xch + h.xch_off;
    // tags of this launch: (sequence mod 2^21) << 11 | step + 1; the buffer is
    // cleared whenever the sequence wraps, so a stale word never matches
    const uint32_t seq = C->slab_seq++ & 0x1FFFFFu;
    if (seq == 0) {
        e = hipMemsetAsync(C->d_xch, 0, sizeof(uint64_t) * (size_t)C->lay.xch_words, C->stream);
        if (e != hipSuccess) return e;
    }
    uint32_t tag_base = seq << 11;
    if (KIND == 0) {
        // 32-bit words, tag bit ((n + 1) >> 1) & 1 in buffer (n + 1) & 1: fill
        // the buffer of each of the launch's first two steps with the other bit
        const size_t half = (size_t)h.nslab * 4 * 3 * h.in.nx * h.in.ny;
        for (int k = 1; k <= 2; ++k) {
            const int64_t m = n0 + k;
            const int par = (int)(m & 1);
            const uint32_t other = (uint32_t)(1 - ((m >> 1) & 1)) << 30;
            e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(reinterpret_cast<uint32_t*>(xch) + par * half),
                                  (int)other, half, C->stream);
            if (e != hipSuccess) return e;
        }
    }
    double* part = C->d_spart + (int64_t)h.slab0 * kSlabChunk;
    int pstride = kSlabChunk;
    float* ckpt = C->d_ckpt;
    int ck = C->ckpt_every;
    int* status = C->d_status;
    uint32_t spin = C->spin_limit;
    void* args[] = {&slabs, &insts, &levels, &b0, &b1, &axes, &xch, &tag_base, &part, &pstride, &ckpt, &ck,
                    &n0, &ns, &status, &spin};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)h.nslab), dim3(NT), args, (unsigned)lds, C->stream);
}

hipError_t dispatch_slab(sllg_ctx* C, int level, int64_t n0, int ns, bool check_only = false,
                         bool* fits = nullptr)
{
    const SlabKernel k = kSlabKernels[C->lv[level].slab_kernel];
    switch (k.kind * 100000 + k.nt * 10 + k.k) {
    case 1924: return launch_slab_t<0, 192, 4>(C, level, n0, ns, check_only, fits);
    case 3842: return launch_slab_t<0, 384, 2>(C, level, n0, ns, check_only, fits);
    case 3843: return launch_slab_t<0, 384, 3>(C, level, n0, ns, check_only, fits);
    case 5762: return launch_slab_t<0, 576, 2>(C, level, n0, ns, check_only, fits);
    case 7681: return launch_slab_t<0, 768, 1>(C, level, n0, ns, check_only, fits);
    case 7682: return launch_slab_t<0, 768, 2>(C, level, n0, ns, check_only, fits);
    case 10241: return launch_slab_t<0, 1024, 1>(C, level, n0, ns, check_only, fits);
    case 10242: return launch_slab_t<0, 1024, 2>(C, level, n0, ns, check_only, fits);
    case 101922: return launch_slab_t<1, 192, 2>(C, level, n0, ns, check_only, fits);
    case 103841: return launch_slab_t<1, 384, 1>(C, level, n0, ns, check_only, fits);
    case 105761: return launch_slab_t<1, 576, 1>(C, level, n0, ns, check_only, fits);
    case 107681: return launch_slab_t<1, 768, 1>(C, level, n0, ns, check_only, fits);
    case 110241: return launch_slab_t<1, 1024, 1>(C, level, n0, ns, check_only, fits);
    case 103842: return launch_slab_t<1, 384, 2>(C, level, n0, ns, check_only, fits);
    case 107682: return launch_slab_t<1, 768, 2>(C, level, n0, ns, check_only, fits);
    case 110242: return launch_slab_t<1, 1024, 2>(C, level, n0, ns, check_only, fits);
    default: return hipErrorInvalidValue;
    }
}

hipError_t fold_slabs(sllg_ctx* C, int level, int64_t n0, int ns)
{
    const LevelHost& h = C->lv[level];
    hipLaunchKernelGGL(k_fold_slabs<256>, dim3((unsigned)h.ninst), dim3(256), 0, C->stream, C->d_insts, h.inst0,
                       C->d_islab + 2 * h.inst0, C->d_levels, C->d_spart + (int64_t)h.slab0 * kSlabChunk,
                       kSlabChunk, n0, ns, C->d_accs, C->d_records, C->d_status);
    return hipGetLastError();
}

hipEvent_t next_event(sllg_ctx* C)
{
    if (C->ev_used == C->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        C->ev_pool.push_back(e);
    }
    return C->ev_pool[C->ev_used++];
}

constexpr int kGraphSteps = 128;

// Fold the last streamed step of every instance of a level into its loop.
hipError_t flush_level(sllg_ctx* C, int level)
{
    const LevelHost& h = C->lv[level];
    hipLaunchKernelGGL(k_flush, dim3((unsigned)h.ninst), dim3(64), 0, C->stream, C->d_insts, h.inst0, C->d_levels,
                       C->d_steps, C->d_partials, (int)C->lay.max_tiles, C->d_inst_cnt, C->d_accs, C->d_records,
                       C->d_status);
    return hipGetLastError();
}

// Graph of kGraphSteps consecutive stream launches of one level.
// A HIP graph of nl streamed launches of a level (cached per level and nl).
int stream_graph(sllg_ctx* C, int level, int nl, hipGraphExec_t* out)
{
    const int key = level * 1024 + nl;
    auto it = C->graphs.find(key);
    if (it != C->graphs.end()) {
        *out = it->second;
        return SLLG_OK;
    }
    if (!C->cap_stream) HIP_OK(hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking));
    hipStream_t user = C->stream;
    C->stream = C->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(C->cap_stream, hipStreamCaptureModeThreadLocal);
    for (int i = 0; i < nl && e == hipSuccess; ++i) e = dispatch_stream(C, level);
    hipError_t e2 = hipStreamEndCapture(C->cap_stream, &g);
    C->stream = user;
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(SLLG_E_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(SLLG_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    C->graphs[key] = x;
    *out = x;
    return SLLG_OK;
}

// Run up to nsteps of every unfinished level.
int run_steps(sllg_ctx* C, int64_t nsteps)
{
    if (nsteps <= 0) return SLLG_OK;
    // stream levels: one launch per step, replayed from a HIP graph in blocks
    for (int l = 0; l < (int)C->lv.size(); ++l) {
        LevelHost& h = C->lv[l];
        if (h.plan != kPlanStream) continue;
        int64_t k = std::min(nsteps, h.n_steps - h.step);
        h.step += k;
        while (k > 0) {
            // one launch unit: a graph of kGraphSteps launches or one launch;
            // every C->timing-th unit is bracketed by events
            // graphs of 128, 64, .., 8 launches; single launches below 8
            int64_t nl = 1;
            if (C->use_graph)
                for (int g = kGraphSteps; g >= 8 && nl == 1; g /= 2)
                    if (k >= g) nl = g;
            const bool graph = nl > 1;
            const bool timed = C->timing > 0 && (C->unit_counter++ % C->timing) == 0;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                e0 = next_event(C);
                e1 = next_event(C);
                if (!e0 || !e1) return fail(SLLG_E_HIP, "event pool");
                HIP_OK(hipEventRecord(e0, C->stream));
            }
            if (graph) {
                hipGraphExec_t g = nullptr;
                int rc = stream_graph(C, l, (int)nl, &g);
                if (rc) return rc;
                HIP_OK(hipGraphLaunch(g, C->stream));
            } else {
                HIP_OK(dispatch_stream(C, l));
            }
            if (timed) {
                HIP_OK(hipEventRecord(e1, C->stream));
                C->ev_launches.push_back(nl);
                C->timed_cells += h.ncell * h.ninst * nl;
            }
            k -= nl;
        }
        HIP_OK(flush_level(C, l));
    }
    // slab levels: chunks of kSlabChunk steps, each folded into the loops
    for (int l = 0; l < (int)C->lv.size(); ++l) {
        LevelHost& h = C->lv[l];
        if (h.plan != kPlanSlab) continue;
        int64_t k = std::min(nsteps, h.n_steps - h.step);
        while (k > 0) {
            const int ns = (int)std::min<int64_t>(k, kSlabChunk);
            const bool timed = C->timing > 0 && (C->unit_counter++ % C->timing) == 0;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                e0 = next_event(C);
                e1 = next_event(C);
                if (!e0 || !e1) return fail(SLLG_E_HIP, "event pool");
                HIP_OK(hipEventRecord(e0, C->stream));
            }
            HIP_OK(dispatch_slab(C, l, h.step, ns));
            if (timed) {
                HIP_OK(hipEventRecord(e1, C->stream));
                C->ev_launches.push_back(ns);   // one launch covers ns steps; report per step
                C->timed_cells += h.ncell * h.ninst * ns;
            }
            HIP_OK(fold_slabs(C, l, h.step, ns));
            h.step += ns;
            k -= ns;
        }
    }
    // levels with magnetostatics: launches of at most 4096 steps
    for (int l = 0; l < (int)C->lv.size(); ++l) {
        LevelHost& h = C->lv[l];
        if (h.plan != kPlanDemag) continue;
        int64_t k = std::min(nsteps, h.n_steps - h.step);
        while (k > 0) {
            const int64_t ns = std::min<int64_t>(k, 4096);
            const bool time_this = C->timing > 0 && (C->unit_counter++ % C->timing) == 0;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (time_this) {
                e0 = next_event(C);
                e1 = next_event(C);
                if (!e0 || !e1) return fail(SLLG_E_HIP, "event pool");
                HIP_OK(hipEventRecord(e0, C->stream));
            }
            HIP_OK(dispatch_demag(C, l, h.step, ns));
            if (time_this) {
                HIP_OK(hipEventRecord(e1, C->stream));
                C->ev_launches.push_back(1);
                C->timed_cells += h.ncell * h.ninst * ns;
            }
            h.step += ns;
            k -= ns;
        }
    }
    // single-cell levels on the lanes plan: runs of consecutive levels at the
    // same sweep position share a launch of at most 2^20 steps
    for (int l0 = 0; l0 < (int)C->lv.size();) {
        if (C->lv[l0].plan != kPlanLanes) {
            ++l0;
            continue;
        }
        int l1 = l0 + 1;
        while (l1 < (int)C->lv.size() && C->lv[l1].plan == kPlanLanes && C->lv[l1].n_steps == C->lv[l0].n_steps &&
               C->lv[l1].step == C->lv[l0].step)
            ++l1;
        LevelHost& h0 = C->lv[l0];
        int64_t k = std::min(nsteps, h0.n_steps - h0.step);
        while (k > 0) {
            const int64_t ns = std::min<int64_t>(k, int64_t(1) << 20);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const bool time_this = C->timing > 0 && !std::any_of(C->lv.begin(), C->lv.end(), [](const LevelHost& x) {
                return x.plan == kPlanStream || x.plan == kPlanSlab;
            });
            if (time_this) {
                e0 = next_event(C);
                e1 = next_event(C);
                if (!e0 || !e1) return fail(SLLG_E_HIP, "event pool");
                HIP_OK(hipEventRecord(e0, C->stream));
            }
            HIP_OK(dispatch_lanes(C, l0, l1, h0.step, ns));
            if (time_this) {
                HIP_OK(hipEventRecord(e1, C->stream));
                C->ev_launches.push_back(1);
                int64_t cells = 0;
                for (int l = l0; l < l1; ++l) cells += C->lv[l].ninst;
                C->timed_cells += cells * ns;
            }
            for (int l = l0; l < l1; ++l) C->lv[l].step += ns;
            k -= ns;
        }
        l0 = l1;
    }
    // resident sets: launches of at most 32768 steps
    for (const auto& rs : C->res_sets) {
        LevelHost& h0 = C->lv[rs.levels[0]];
        int64_t k = std::min(nsteps, h0.n_steps - h0.step);
        while (k > 0) {
            const int64_t ns = std::min<int64_t>(k, 32768);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const bool time_this = C->timing > 0 && !std::any_of(C->lv.begin(), C->lv.end(), [](const LevelHost& x) {
                return x.plan == kPlanStream || x.plan == kPlanSlab;
            });
            if (time_this) {
                e0 = next_event(C);
                e1 = next_event(C);
                HIP_OK(hipEventRecord(e0, C->stream));
            }
            HIP_OK(dispatch_res(C, rs, h0.step, ns));
            if (time_this) {
                HIP_OK(hipEventRecord(e1, C->stream));
                C->ev_launches.push_back(1);
                int64_t cells = 0;
                for (int l : rs.levels) cells += C->lv[l].ncell * C->lv[l].ninst;
                C->timed_cells += cells * ns;
            }
            for (int l : rs.levels) C->lv[l].step += ns;
            k -= ns;
        }
    }
    return SLLG_OK;
}

int reset_state(sllg_ctx* C)
{
    for (LevelHost& h : C->lv) h.step = 0;
    HIP_OK(hipMemsetAsync(C->d_steps, 0, sizeof(int64_t) * C->lv.size(), C->stream));
    HIP_OK(hipMemsetAsync(C->d_status, 0, sizeof(int) * 4, C->stream));
    HIP_OK(hipMemsetAsync(C->d_inst_cnt, 0, sizeof(uint32_t) * C->lay.ninst_total, C->stream));
    HIP_OK(hipMemsetAsync(C->d_launch_cnt, 0, sizeof(uint32_t) * (C->lv.size() + 1), C->stream));
    HIP_OK(hipMemsetAsync(C->d_records, 0, sizeof(double) * C->lay.rec_doubles, C->stream));
    int maxc = 1;
    for (const LevelHost& h : C->lv) maxc = (int)std::max<int64_t>(maxc, h.ncell);
    dim3 grid((unsigned)std::min<int64_t>(ceil_div(maxc, 256), 4096), (unsigned)C->lay.ninst_total);
    hipLaunchKernelGGL(k_init, grid, dim3(256), 0, C->stream, C->d_insts, C->d_levels,
                       (int)C->lay.ninst_total, C->d_buf0, C->d_accs, C->d_records);
    HIP_OK(hipGetLastError());
    return SLLG_OK;
}

// Process-wide options read by sllg_init (sllg_set_options).
int g_options = 0;

// Timing-based choice of the stream tile shape (a few steps per candidate),
// cached per (dims, instances, device) for the process.
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tuned;
std::map<std::tuple<int, int, int, int>, double> g_tuned_ms;                      // best stream ms/step
std::map<std::tuple<int, int, int, int>, std::tuple<int, int, double>> g_tuned_slab;  // kernel, tz, ms/step

int tune_stream(sllg_ctx* C, int level)
{
    LevelHost& h = C->lv[level];
    const auto key = std::make_tuple(h.in.nx, h.in.ny, h.in.nz, h.ninst);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
        h.shape = it->second.first;
        h.tz = it->second.second;
        return SLLG_OK;
    }
    default_stream_shape(C, h);
    std::vector<std::pair<int, int>> cands;
    for (int s = 0; s < kNumShapes; ++s) {
        const Shape& S = kShapes[s];
        if (!shape_fits(h.in, S)) continue;
        // keep shapes whose threads are mostly busy
        double use;
        if (S.kind == 0) {
            use = (double)std::min(S.tx, h.in.nx) * std::min(S.ty, h.in.ny) / (S.tx * S.ty);
        } else if (S.kind == 1) {
            const int TR = S.tx / h.in.nx;
            use = (double)(TR * h.in.nx) / S.tx * std::min(1.0, (double)h.in.ny / (TR * S.ty));
        } else {
            use = (double)std::min(shape_rows(h.in, S), h.in.ny) * h.in.nx / (S.tx * S.ty);
        }
        if (use < 0.5) continue;
        // powers of two, plus the depths whose tile count just fills k waves
        // of one workgroup per CU
        std::vector<int> tzs(std::begin(kTzChoices), std::end(kTzChoices));
        const int64_t xy = tiles_for(h.in, S, h.in.nz) * h.ninst;   // tiles of one z chunk
        for (int k = 1; k <= 4 && xy > 0; ++k) {
            const int64_t chunks = (int64_t)k * C->num_cus / xy;
            if (chunks < 1) continue;
            const int tz = (int)ceil_div(h.in.nz, chunks);
            if (std::find(tzs.begin(), tzs.end(), tz) == tzs.end()) tzs.push_back(tz);
        }
        for (int tz : tzs) {
            if (tz < S.pz || tz > h.in.nz * 2) continue;
            const int64_t nt = tiles_for(h.in, S, tz) * h.ninst;
            if (nt == 0) continue;
            if (nt < C->num_cus / 4 && tz > 1) continue;
            if (nt > C->lay.max_tiles) continue;
            cands.push_back({s, tz});
        }
    }
    if (cands.size() <= 1) {
        g_tuned[key] = {h.shape, h.tz};
        return SLLG_OK;
    }
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    // ms per step of one candidate: warm-up, then the better of `runs` runs
    // of `reps` launches; the step counters are reset afterwards
    auto time_cand = [&](std::pair<int, int> c, int reps, int runs, double* out) -> int {
        h.shape = c.first;
        h.tz = c.second;
        int rc = replan(C);
        if (rc) return rc;
        for (int r = 0; r < 2; ++r) HIP_OK(dispatch_stream(C, level));
        float ms = 1e30f;
        for (int run = 0; run < runs; ++run) {
            HIP_OK(hipEventRecord(e0, C->stream));
            for (int r = 0; r < reps; ++r) HIP_OK(dispatch_stream(C, level));
            HIP_OK(hipEventRecord(e1, C->stream));
            HIP_OK(hipEventSynchronize(e1));
            float t = 0;
            HIP_OK(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        HIP_OK(hipMemsetAsync(C->d_steps, 0, sizeof(int64_t) * C->lv.size(), C->stream));
        HIP_OK(hipMemsetAsync(C->d_inst_cnt, 0, sizeof(uint32_t) * C->lay.ninst_total, C->stream));
        *out = ms / reps;
        return SLLG_OK;
    };
    // every candidate briefly (the better of two runs of 6 launches), then
    // the candidates within 5 % of the best again with runs four times as
    // long, so that shapes a few per cent apart are told apart despite launch
    // jitter
    std::vector<std::pair<double, std::pair<int, int>>> timed;
    for (auto c : cands) {
        double t = 0;
        int rc = time_cand(c, 6, 2, &t);
        if (rc) return rc;
        if (g_options & SLLG_OPT_VERBOSE)
            fprintf(stderr, "tune level %d: shape %d (%d,%d,%d,%d) tz %d tiles %d: %.2f us/step\n", level,
                    c.first, kShapes[c.first].kind, kShapes[c.first].tx, kShapes[c.first].ty,
                    kShapes[c.first].pz, c.second, h.ntiles, 1000.0 * t);
        timed.push_back({t, c});
    }
    std::sort(timed.begin(), timed.end());
    double best_t = timed[0].first;
    std::pair<int, int> best = timed[0].second;
    const double lead = timed[0].first;
    if (timed.size() > 1 && timed[1].first <= 1.05 * lead) {
        best_t = 1e30;
        for (size_t i = 0; i < timed.size() && i < 4 && timed[i].first <= 1.05 * lead; ++i) {
            double t = 0;
            int rc = time_cand(timed[i].second, 24, 3, &t);
            if (rc) return rc;
            if (g_options & SLLG_OPT_VERBOSE)
                fprintf(stderr, "tune level %d: finalist shape %d tz %d: %.2f us/step\n", level,
                        timed[i].second.first, timed[i].second.second, 1000.0 * t);
            if (t < best_t) {
                best_t = t;
                best = timed[i].second;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h.shape = best.first;
    h.tz = best.second;
    g_tuned[key] = best;
    g_tuned_ms[key] = best_t;
    return SLLG_OK;
}

// Timing-based choice of the slab kernel and thickness for a slab-eligible
// level; returns the best ms per step in *best_ms (1e30 if none runs).
int tune_slab(sllg_ctx* C, int level, double* best_ms)
{
    LevelHost& h = C->lv[level];
    const auto key = std::make_tuple(h.in.nx, h.in.ny, h.in.nz, h.ninst);
    *best_ms = 1e30;
    auto it = g_tuned_slab.find(key);
    if (it != g_tuned_slab.end()) {
        h.slab_kernel = std::get<0>(it->second);
        h.slab_tz = std::get<1>(it->second);
        *best_ms = std::get<2>(it->second);
        return SLLG_OK;
    }
    const int P = h.in.nx * h.in.ny;
    const int saved_plan = h.plan;
    const int tzs[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32};
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    int best_k = -1, best_tz = 0;
    // ms per step of the candidate set up in h: the better of `runs` launches
    // of `steps` steps after a short warm-up; false if its bounded waits gave
    // up (the time then means nothing; the status word is cleared)
    auto time_slab = [&](int steps, int runs, float* ms, bool* ok) -> int {
        h.step = 0;
        HIP_OK(dispatch_slab(C, level, 0, 16));
        *ms = 1e30f;
        for (int rep = 0; rep < runs; ++rep) {
            HIP_OK(hipEventRecord(e0, C->stream));
            HIP_OK(dispatch_slab(C, level, 16 + rep * steps, steps));
            HIP_OK(hipEventRecord(e1, C->stream));
            HIP_OK(hipEventSynchronize(e1));
            float t = 0;
            HIP_OK(hipEventElapsedTime(&t, e0, e1));
            *ms = std::min(*ms, t / steps);
        }
        int st[4] = {0, 0, 0, 0};
        HIP_OK(hipMemcpyAsync(st, C->d_status, sizeof(st), hipMemcpyDeviceToHost, C->stream));
        HIP_OK(hipStreamSynchronize(C->stream));
        *ok = !(st[0] & 2);
        if (!*ok) HIP_OK(hipMemsetAsync(C->d_status, 0, sizeof(int) * 4, C->stream));
        return SLLG_OK;
    };
    std::vector<std::tuple<float, int, int>> timed;   // ms per step, kernel, tz
    for (int ki = 0; ki < kNumSlabKernels; ++ki) {
        const int NPP = kSlabKernels[ki].nt / P;
        if (NPP < 1) continue;
        const int cap = kSlabKernels[ki].k * NPP;
        const int halo = kSlabKernels[ki].kind == 0 ? 2 : 0;   // recomputed planes
        const int minp = kSlabKernels[ki].kind == 0 ? 2 : 1;
        for (int tz : tzs) {
            if (tz < minp || tz + 1 + halo > cap || tz > h.in.nz) continue;
            if ((kSlabKernels[ki].k - 1) * NPP >= tz + 1 + halo) continue;   // an idle cell slot per thread
            h.plan = kPlanSlab;
            h.slab_kernel = ki;
            h.slab_tz = tz;
            int rc = replan(C);
            if (rc) return rc;
            bool fits = false;
            if (dispatch_slab(C, level, 0, 1, true, &fits) != hipSuccess || !fits) continue;
            // the better of two launches of 256 steps: shapes a few per cent
            // apart are told apart despite the launch overhead and its jitter
            // (a candidate whose bounded waits gave up is dropped)
            float ms = 0;
            bool ok = false;
            rc = time_slab(256, 2, &ms, &ok);
            if (rc) return rc;
            if (!ok) {
                if (g_options & SLLG_OPT_VERBOSE)
                    fprintf(stderr, "tune level %d: slab kernel %d tz %d dropped (exchange timed out)\n", level,
                            ki, tz);
                continue;
            }
            if (g_options & SLLG_OPT_VERBOSE)
                fprintf(stderr, "tune level %d: slab kernel %d (%d,%d) tz %d slabs %d: %.3f us/step\n", level, ki,
                        kSlabKernels[ki].nt, kSlabKernels[ki].k, tz, h.nslab, 1000.0 * ms);
            timed.push_back(std::make_tuple(ms, ki, tz));
        }
    }
    // the candidates within 5 % of the best again, with launches four times
    // as long
    std::sort(timed.begin(), timed.end());
    if (!timed.empty()) {
        const float lead = std::get<0>(timed[0]);
        const bool close = timed.size() > 1 && std::get<0>(timed[1]) <= 1.05f * lead;
        for (size_t i = 0; i < timed.size() && i < 3; ++i) {
            float ms = std::get<0>(timed[i]);
            if (close) {
                if (ms > 1.05f * lead) break;
                h.plan = kPlanSlab;
                h.slab_kernel = std::get<1>(timed[i]);
                h.slab_tz = std::get<2>(timed[i]);
                int rc = replan(C);
                if (rc) return rc;
                bool ok = false;
                rc = time_slab(1024, 2, &ms, &ok);
                if (rc) return rc;
                if (!ok) continue;
                if (g_options & SLLG_OPT_VERBOSE)
                    fprintf(stderr, "tune level %d: finalist slab kernel %d tz %d: %.3f us/step\n", level,
                            std::get<1>(timed[i]), std::get<2>(timed[i]), 1000.0 * ms);
            }
            if (ms < *best_ms) {
                *best_ms = ms;
                best_k = std::get<1>(timed[i]);
                best_tz = std::get<2>(timed[i]);
            }
            if (!close) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h.plan = saved_plan;
    h.step = 0;
    if (best_k >= 0) {
        h.slab_kernel = best_k;
        h.slab_tz = best_tz;
        g_tuned_slab[key] = std::make_tuple(best_k, best_tz, *best_ms);
    }
    int rc = replan(C);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

// Host-side analytics of one loop (FP64).
struct Stats {
    double S, hd, ha, Hc, Mr, md0, ma0;
    int nd, na, kd, ka;
};

Stats analyse(const std::vector<double>& H, const std::vector<double>& m)
{
    Stats s{};
    s.hd = s.ha = s.md0 = s.ma0 = NAN;
    s.kd = s.ka = -1;
    for (size_t k = 0; k + 1 < H.size(); ++k) {
        const double dH = H[k + 1] - H[k];
        s.S -= 0.5 * (m[k] + m[k + 1]) * dH;
        const int ch = (m[k] > 0.0) != (m[k + 1] > 0.0);
        if (dH < 0) {
            s.nd += ch;
            if (s.kd < 0 && m[k] > 0.0 && m[k + 1] <= 0.0) {
                s.kd = (int)k;
                s.hd = H[k] - m[k] * dH / (m[k + 1] - m[k]);
            }
            if (std::isnan(s.md0) && H[k] > 0.0 && H[k + 1] <= 0.0) s.md0 = m[k] + (m[k + 1] - m[k]) * (-H[k]) / dH;
        } else if (dH > 0) {
            s.na += ch;
            if (s.ka < 0 && m[k] < 0.0 && m[k + 1] >= 0.0) {
                s.ka = (int)k;
                s.ha = H[k] - m[k] * dH / (m[k + 1] - m[k]);
            }
            if (std::isnan(s.ma0) && H[k] < 0.0 && H[k + 1] >= 0.0) s.ma0 = m[k] + (m[k + 1] - m[k]) * (-H[k]) / dH;
        }
    }
    s.Hc = 0.5 * (s.ha - s.hd);
    s.Mr = 0.5 * (s.md0 - s.ma0);
    return s;
}

double wave_host(const LevelHost& h, int wave, int64_t n)
{
    const int64_t N = h.n_period;
    const int64_t k = n % N;
    if (wave == 0) {
        const double s = (double)k * (1.0 / (double)N);
        return (2 * k <= N) ? 1.0 - 4.0 * s : 4.0 * s - 3.0;
    }
    if (wave == 1) return std::cos(2.0 * kPi * ((double)k * (1.0 / (double)N)));
    return 1.0;
}

// Device status word: bit 0 (value 1) a non-finite loop ordinate, bit 1
// (value 2) a slab exchange wait that gave up.  Synchronises the stream.
int check_status(sllg_ctx* C)
{
    int st[4] = {0, 0, 0, 0};
    HIP_OK(hipMemcpyAsync(st, C->d_status, sizeof(st), hipMemcpyDeviceToHost, C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    if (st[0] & 2)
        return fail(SLLG_E_HIP, "slab exchange timed out (a neighbour's boundary words did not arrive); "
                                "the state is undefined until sllg_reset");
    if (st[0] & 1) return fail(SLLG_E_NUMERIC, "non-finite loop ordinate (the magnetisation blew up)");
    if (st[0] & 4)
        return fail(SLLG_E_HIP, "LDS check: a tile read a neighbour slot that was not written for its plane "
                                "(set only by a library built with SLLG_LDS_CHECK)");
    return SLLG_OK;
}

}  // namespace

// ---- snapshots: the state a sweep carries from one step to the next ----
// Layout (host bytes): SnapHead, one SnapLevel per level, the device status
// word (4 ints), the step indices, both state buffers, the loop
// accumulators, the loop records and the checkpoints.  Everything else in the
// workspace is either rebuilt by sllg_init (tables, axes) or empty between
// runs (pending folds, launch counters, exchange words, partial sums).
namespace {
constexpr char kSnapMagic[8] = {'S', 'L', 'L', 'G', 'S', 'N', 'P', '1'};
struct SnapHead {
    char magic[8];
    int32_t nlev, ckpt_every;
    int64_t state_floats, rec_doubles, ckpt_floats, ninst;
};
struct SnapLevel {
    int32_t nx, ny, nz, n_real;
    uint64_t seed_base, axis_seed;
    int64_t n_steps, step;
    double dt, sigma, c_ex, hk, alpha, hz_amp;
};
SnapLevel snap_level(const LevelHost& h)
{
    SnapLevel s{};
    s.nx = h.in.nx;
    s.ny = h.in.ny;
    s.nz = h.in.nz;
    s.n_real = h.in.n_real;
    s.seed_base = h.in.seed_base;
    s.axis_seed = h.in.axis_seed;
    s.n_steps = h.n_steps;
    s.step = h.step;
    s.dt = h.dt;
    s.sigma = h.sigma;
    s.c_ex = h.c_ex;
    s.hk = h.hk;
    s.alpha = h.alpha;
    s.hz_amp = h.hz_amp;
    return s;
}
// the device regions of a snapshot, in order
std::vector<std::pair<void*, size_t>> snap_regions(const sllg_ctx* C)
{
    const Layout& L = C->lay;
    return {{C->d_status, sizeof(int) * 4},
            {C->d_steps, sizeof(int64_t) * C->lv.size()},
            {C->d_buf0, sizeof(float) * (size_t)L.state_floats},
            {C->d_buf1, sizeof(float) * (size_t)L.state_floats},
            {C->d_accs, sizeof(AccDev) * (size_t)L.ninst_total},
            {C->d_records, sizeof(double) * (size_t)L.rec_doubles},
            {C->d_ckpt, sizeof(float) * (size_t)L.ckpt_floats}};
}
size_t snap_bytes(const sllg_ctx* C)
{
    size_t n = sizeof(SnapHead) + sizeof(SnapLevel) * C->lv.size();
    for (const auto& r : snap_regions(C)) n += r.second;
    return n;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* sllg_last_error(void) { return g_err.c_str(); }

int sllg_set_options(int32_t flags)
{
    if (flags & ~(SLLG_OPT_NO_TUNE | SLLG_OPT_NO_SLAB | SLLG_OPT_NO_GRAPH | SLLG_OPT_VERBOSE))
        return fail(SLLG_E_INVAL, "unknown option bits 0x%x", flags);
    g_options = flags;
    return SLLG_OK;
}

int sllg_set_spin_limit(sllg_ctx* C, uint32_t polls)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    C->spin_limit = polls;
    return SLLG_OK;
}

int sllg_sync(sllg_ctx* C)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    return check_status(C);
}

size_t sllg_workspace_bytes(const sllg_material* mat, const sllg_level* levels, int32_t n_levels,
                            int32_t ckpt_every)
{
    if (validate(mat, levels, n_levels) != SLLG_OK || ckpt_every < 0) return 0;
    std::vector<LevelHost> lv(n_levels);
    for (int i = 0; i < n_levels; ++i) compile_level(*mat, levels[i], lv[i]);
    return make_layout(*mat, lv, ckpt_every).total;
}

}  // extern "C"

namespace {

int init_impl(const sllg_material* mat, const sllg_level* levels, int32_t n_levels, int32_t ckpt_every,
              void* d_workspace, size_t ws_bytes, void* hip_stream, int options, sllg_ctx** out)
{
    if (!out) return fail(SLLG_E_INVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(mat, levels, n_levels);
    if (rc) return rc;
    if (ckpt_every < 0) return fail(SLLG_E_INVAL, "ckpt_every must be >= 0");
    sllg_ctx* C = new sllg_ctx();
    C->mat = *mat;
    C->ckpt_every = ckpt_every;
    C->stream = (hipStream_t)hip_stream;
    C->lv.resize(n_levels);
    int inst = 0;
    int64_t axes = 0, state = 0, rec = 0, ckpt = 0;
    for (int i = 0; i < n_levels; ++i) {
        LevelHost& h = C->lv[i];
        compile_level(*mat, levels[i], h);
        if (!(h.dt > 0) || !std::isfinite(h.sigma) || !(h.alpha >= 0)) {
            delete C;
            return fail(SLLG_E_INVAL, "level %d: dt, sigma or alpha not usable", i);
        }
        h.inst0 = inst;
        h.ninst = levels[i].n_real;
        h.axes_off = levels[i].cone_deg > 0 ? axes : -1;
        if (levels[i].cone_deg > 0) axes += 3 * h.ncell;
        h.step = 0;
        h.plan = 0;
        h.forced = 0;
        for (int r = 0; r < h.ninst; ++r) {
            InstDev I{};
            I.level = i;
            I.real = r;
            I.seed = levels[i].seed_base + (uint64_t)r;
            I.state_off = state;
            I.rec_off = rec;
            I.ckpt_off = ckpt;
            state += 3 * h.ncell;
            rec += h.n_rec;
            if (ckpt_every > 0) ckpt += ceil_div(h.n_steps, ckpt_every) * 3 * h.ncell;
            C->h_insts.push_back(I);
        }
        inst += h.ninst;
    }
    C->lay = make_layout(*mat, C->lv, ckpt_every);
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) {
        delete C;
        return fail(SLLG_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    }
    if (ws_bytes < C->lay.total) {
        const size_t need = C->lay.total;
        delete C;
        return fail(SLLG_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    }
    C->ws = (char*)d_workspace;
    C->ws_bytes = ws_bytes;
    const Layout& L = C->lay;
    C->d_levels = (LevelDev*)(C->ws + L.levels);
    C->d_insts = (InstDev*)(C->ws + L.insts);
    C->d_accs = (AccDev*)(C->ws + L.accs);
    C->d_steps = (int64_t*)(C->ws + L.steps);
    C->d_status = (int*)(C->ws + L.status);
    C->d_inst_cnt = (uint32_t*)(C->ws + L.inst_cnt);
    C->d_launch_cnt = (uint32_t*)(C->ws + L.launch_cnt);
    C->d_partials = (double*)(C->ws + L.partials);
    C->d_tiles = (TileDev*)(C->ws + L.tiles);
    C->d_groups = (GroupDev*)(C->ws + L.groups);
    C->d_slots = (SlotDev*)(C->ws + L.slots);
    C->d_chunks = (ChunkDev*)(C->ws + L.chunks);
    C->d_buf0 = (float*)(C->ws + L.buf0);
    C->d_buf1 = (float*)(C->ws + L.buf1);
    C->d_axes = (float*)(C->ws + L.axes);
    C->d_records = (double*)(C->ws + L.records);
    C->d_ckpt = ckpt_every > 0 ? (float*)(C->ws + L.ckpt) : nullptr;
    C->d_tape = (float*)(C->ws + L.tape);
    C->d_lam = (float*)(C->ws + L.lam);
    C->d_weights = (double*)(C->ws + L.weights);
    C->d_grads = (double*)(C->ws + L.grads);
    C->d_slabs = (SlabDev*)(C->ws + L.slabs);
    C->d_xch = (uint64_t*)(C->ws + L.xch);
    C->d_spart = (double*)(C->ws + L.spart);
    C->d_islab = (int32_t*)(C->ws + L.islab);
    C->d_demag = (float*)(C->ws + L.demag);
    C->h_islab.assign(2 * (size_t)L.ninst_total, 0);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        C->max_lds = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
        C->num_cus = prop.multiProcessorCount;
    }
    C->use_graph = !(options & SLLG_OPT_NO_GRAPH);
    C->h_levels.resize(n_levels);
    // a context of single-cell levels only runs one realization per lane;
    // single cells beside bigger levels share the resident launch instead
    bool all_single = true;
    for (const LevelHost& h : C->lv) all_single = all_single && h.ncell == 1;
    for (int i = 0; i < n_levels; ++i) {
        LevelHost& h = C->lv[i];
        h.plan = mat->demag    ? kPlanDemag
                 : all_single ? kPlanLanes
                 : resident_fits(h, C->max_lds) ? kPlanResident
                                                : kPlanStream;
        if (h.plan == kPlanStream) default_stream_shape(C, h);
    }
    // tensor tables of the magnetostatic field (host, long double), once
    if (mat->demag) {
        int64_t off = 0;
        for (int i = 0; i < n_levels; ++i) {
            LevelHost& h = C->lv[i];
            std::vector<float> tab;
            demag_table(h.in, h.Ms, tab);
            h.demag_off = off;
            if (hipMemcpy(C->d_demag + off, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice) !=
                hipSuccess) {
                delete C;
                return fail(SLLG_E_HIP, "demagnetising-tensor upload failed");
            }
            off += (int64_t)tab.size();
        }
    }
    rc = replan(C);
    if (rc) {
        delete C;
        return rc;
    }
    // per-cell axes
    for (int i = 0; i < n_levels; ++i) {
        const LevelHost& h = C->lv[i];
        if (h.axes_off < 0) continue;
        double e[3] = {mat->easy_axis[0], mat->easy_axis[1], mat->easy_axis[2]};
        const double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        for (double& x : e) x /= en;
        // rotation taking +z to e: Rodrigues about z x e
        double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        const double s = std::sqrt(e[0] * e[0] + e[1] * e[1]);
        if (s > 0) {
            const double k0 = -e[1] / s, k1 = e[0] / s, c = e[2];
            const double K[3][3] = {{0, 0, k1}, {0, 0, -k0}, {-k1, k0, 0}};
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    double kk = 0;
                    for (int t = 0; t < 3; ++t) kk += K[r][t] * K[t][q];
                    R[r][q] = (r == q ? 1.0 : 0.0) + s * K[r][q] + (1.0 - c) * kk;
                }
        } else if (e[2] < 0) {
            R[1][1] = -1;
            R[2][2] = -1;
        }
        const float cmax = (float)(1.0 - std::cos(h.in.cone_deg * kPi / 180.0));
        hipLaunchKernelGGL(k_axes, dim3((unsigned)ceil_div(h.ncell, 256)), dim3(256), 0, C->stream,
                           C->d_levels, i, h.in.axis_seed, cmax, (float)R[0][0], (float)R[0][1],
                           (float)R[0][2], (float)R[1][0], (float)R[1][1], (float)R[1][2], (float)R[2][0],
                           (float)R[2][1], (float)R[2][2], C->d_axes);
        if (hipGetLastError() != hipSuccess) {
            delete C;
            return fail(SLLG_E_HIP, "axes kernel launch failed");
        }
    }
    rc = reset_state(C);
    if (rc) {
        delete C;
        return rc;
    }
    // tune stream shapes on first use of a shape, then start from step 0 again
    bool tuned = false;
    for (int i = 0; i < n_levels; ++i)
        if (C->lv[i].plan == kPlanStream && !(options & SLLG_OPT_NO_TUNE)) {
            rc = tune_stream(C, i);
            if (rc) {
                delete C;
                return rc;
            }
            tuned = true;
        }
    for (int i = 0; i < n_levels; ++i) {
        LevelHost& h = C->lv[i];
        if (h.plan != kPlanStream || !slab_eligible(h.in) || (options & (SLLG_OPT_NO_SLAB | SLLG_OPT_NO_TUNE)))
            continue;
        double slab_ms = 1e30;
        rc = tune_slab(C, i, &slab_ms);
        if (rc) {
            delete C;
            return rc;
        }
        const auto key = std::make_tuple(h.in.nx, h.in.ny, h.in.nz, h.ninst);
        const double stream_ms = g_tuned_ms.count(key) ? g_tuned_ms[key] : 1e30;
        if (slab_ms < stream_ms) h.plan = kPlanSlab;
        tuned = true;
    }
    if (tuned) {
        rc = replan(C);
        if (!rc) rc = reset_state(C);
        if (rc) {
            delete C;
            return rc;
        }
    }
    *out = C;
    return SLLG_OK;
}

// Device address of this GPU's static workspace (looked up once per device
// with that device current) and whether a live context holds it.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
bool g_static_busy[kMaxDevices] = {};

}  // namespace

extern "C" {

int sllg_init(const sllg_material* mat, const sllg_level* levels, int32_t n_levels, int32_t ckpt_every,
              void* d_workspace, size_t ws_bytes, void* hip_stream, sllg_ctx** out)
{
    return init_impl(mat, levels, n_levels, ckpt_every, d_workspace, ws_bytes, hip_stream, g_options, out);
}

int sllg_init_static(const sllg_material* mat, const sllg_level* levels, int32_t n_levels, int32_t ckpt_every,
                     void* hip_stream, sllg_ctx** out)
{
    if (!out) return fail(SLLG_E_INVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(mat, levels, n_levels);
    if (rc) return rc;
    if (ckpt_every < 0) return fail(SLLG_E_INVAL, "ckpt_every must be >= 0");
    const size_t need = sllg_workspace_bytes(mat, levels, n_levels, ckpt_every);
    if (need == 0) return SLLG_E_INVAL;
    if (need > kStaticScratchBytes)
        return fail(SLLG_E_WORKSPACE, "needs %zu bytes of workspace; the static workspace holds %zu", need,
                    kStaticScratchBytes);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SLLG_E_INVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SLLG_E_HIP, "static workspace address on device %d: %s", dev, hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    if (g_static_busy[dev])
        return fail(SLLG_E_STATE, "the static workspace of device %d is held by a live context (sllg_free it first)",
                    dev);
    // no tuning (it creates events), no graphs (capture and instantiation
    // allocate): default tile shapes, launches issued one by one
    rc = init_impl(mat, levels, n_levels, ckpt_every, g_static_ptr[dev], kStaticScratchBytes, hip_stream,
                   SLLG_OPT_NO_TUNE | SLLG_OPT_NO_GRAPH, out);
    if (rc) return rc;
    (*out)->static_dev = dev;
    g_static_busy[dev] = true;
    return SLLG_OK;
}

int sllg_run_sweep(sllg_ctx* C)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    int64_t left = 0;
    for (const LevelHost& h : C->lv) left = std::max(left, h.n_steps - h.step);
    return run_steps(C, left);
}

int sllg_run_steps(sllg_ctx* C, int64_t nsteps)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    if (nsteps < 0) return fail(SLLG_E_INVAL, "nsteps must be >= 0");
    return run_steps(C, nsteps);
}

int sllg_reset(sllg_ctx* C)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    int rc = reset_state(C);
    if (rc) return rc;
    return replan(C);
}

int sllg_loop(sllg_ctx* C, int32_t level, int32_t real, double* H_Oe, double* mH, int64_t cap,
              int64_t* n_out, sllg_loop_stats* stats)
{
    if (!C || level < 0 || level >= (int)C->lv.size()) return fail(SLLG_E_INVAL, "bad level");
    const LevelHost& h = C->lv[level];
    if (real < -1 || real >= h.ninst) return fail(SLLG_E_INVAL, "bad realization %d", real);
    int rc = check_status(C);
    if (rc) return rc;
    const int64_t npts = h.step / h.in.record_every + 1;
    if (n_out) *n_out = npts;
    if ((H_Oe || mH) && cap < npts) return fail(SLLG_E_CAPACITY, "need %lld entries", (long long)npts);
    if (!H_Oe && !mH && !stats) return SLLG_OK;
    const int r0 = real < 0 ? 0 : real, r1 = real < 0 ? h.ninst : real + 1;
    // only the points recorded so far
    std::vector<double> rec((size_t)(r1 - r0) * npts);
    std::vector<AccDev> acc(r1 - r0);
    for (int r = r0; r < r1; ++r) {
        const InstDev& I = C->h_insts[h.inst0 + r];
        HIP_OK(hipMemcpyAsync(rec.data() + (size_t)(r - r0) * npts, C->d_records + I.rec_off,
                              sizeof(double) * npts, hipMemcpyDeviceToHost, C->stream));
    }
    HIP_OK(hipMemcpyAsync(acc.data(), C->d_accs + h.inst0 + r0, sizeof(AccDev) * (r1 - r0),
                          hipMemcpyDeviceToHost, C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    std::vector<double> H(npts), m(npts, 0.0);
    const double hz_oe = h.hz_amp / kOe;
    for (int64_t k = 0; k < npts; ++k) H[k] = hz_oe * wave_host(h, C->mat.wave, k * h.in.record_every);
    for (int r = 0; r < r1 - r0; ++r)
        for (int64_t k = 0; k < npts; ++k) m[k] += rec[(size_t)r * npts + k];
    for (int64_t k = 0; k < npts; ++k) m[k] /= (double)(r1 - r0);
    if (H_Oe) std::memcpy(H_Oe, H.data(), sizeof(double) * npts);
    if (mH) std::memcpy(mH, m.data(), sizeof(double) * npts);
    if (stats) {
        const Stats s = analyse(H, m);
        sllg_loop_stats o{};
        // area from the per-step accumulators (exact with decimated records)
        double area = 0;
        for (const AccDev& a : acc) area += a.area;
        o.S_sim = area / (double)acc.size();
        o.S_phys = o.S_sim * h.cM / h.hscale;
        o.Hc_desc = s.hd;
        o.Hc_asc = s.ha;
        o.Hc_sim = s.Hc;
        o.Hc_phys = s.Hc / h.hscale;
        o.Mr_sim = s.Mr;
        o.Mr_phys = s.Mr * h.cM;
        o.n_cross_desc = s.nd;
        o.n_cross_asc = s.na;
        o.n_real = (int)acc.size();
        o.S_se = NAN;
        o.Hc_se = NAN;
        if (acc.size() > 1) {
            double ms = 0, vs = 0;
            std::vector<double> hc;
            for (const AccDev& a : acc) {
                ms += a.area;
                if (a.found_d && a.found_a) hc.push_back(0.5 * (a.hstar_a - a.hstar_d));
            }
            ms /= acc.size();
            for (const AccDev& a : acc) vs += (a.area - ms) * (a.area - ms);
            o.S_se = std::sqrt(vs / (acc.size() - 1) / acc.size());
            if (hc.size() > 1) {
                double mh = 0, vh = 0;
                for (double x : hc) mh += x;
                mh /= hc.size();
                for (double x : hc) vh += (x - mh) * (x - mh);
                o.Hc_se = std::sqrt(vh / (hc.size() - 1) / hc.size());
            }
        }
        *stats = o;
    }
    return SLLG_OK;
}

int sllg_level_params(const sllg_ctx* C, int32_t level, double out[16])
{
    if (!C || level < 0 || level >= (int)C->lv.size() || !out) return fail(SLLG_E_INVAL, "bad level");
    const LevelHost& h = C->lv[level];
    const double v[16] = {h.zeta, h.A, h.K, h.Ms, h.a, h.c_ex, h.hk, h.gamma1, h.alpha, h.sigma, h.dt,
                          h.hscale, h.cM, (double)h.n_steps, h.hz_amp,
                          (double)(h.plan * 100000 + (h.plan == kPlanStream ? h.shape * 1000 + h.tz
                                                      : h.plan == kPlanSlab ? h.slab_kernel * 1000 + h.slab_tz
                                                                            : 0))};
    std::memcpy(out, v, sizeof(v));
    return SLLG_OK;
}

int sllg_level_kernel(const sllg_ctx* C, int32_t level, char* name, int32_t cap)
{
    if (!C || level < 0 || level >= (int)C->lv.size() || !name || cap <= 0) return fail(SLLG_E_INVAL, "bad args");
    const LevelHost& h = C->lv[level];
    char buf[96] = "none";
    if (h.plan == kPlanStream) {
        const Shape& sh = kShapes[h.shape];
        if (sh.kind == 0)
            snprintf(buf, sizeof(buf), "k_stream<%d,%d,%d> tz %d", sh.tx, sh.ty, sh.pz, h.tz);
        else
            snprintf(buf, sizeof(buf), "%s<%d,%d> tz %d", sh.kind == 1 ? "k_rows" : "k_rows2", sh.tx, sh.ty, h.tz);
    } else if (h.plan == kPlanSlab) {
        const SlabKernel& k = kSlabKernels[h.slab_kernel];
        snprintf(buf, sizeof(buf), "%s<%d,%d> tz %d steps/launch %d", k.kind == 0 ? "k_slab" : "k_slab2", k.nt, k.k,
                 h.slab_tz, kSlabChunk);
    } else if (h.plan == kPlanLanes) {
        snprintf(buf, sizeof(buf), "k_lanes<%d>", kLanesThreads);
    } else if (h.plan == kPlanDemag) {
        const WideDims d = demag_wide_dims(h.in);
        if (demag_is_wide(h.in))
            snprintf(buf, sizeof(buf), "k_demag %dx%d wide %dx%d", demag_chunks((int)h.ncell), (int)h.ncell, d.wx,
                     d.wy);
        else
            snprintf(buf, sizeof(buf), "k_demag %dx%d octant", demag_chunks((int)h.ncell), (int)h.ncell);
    } else {
        for (const auto& rs : C->res_sets)
            if (std::find(rs.levels.begin(), rs.levels.end(), level) != rs.levels.end())
                snprintf(buf, sizeof(buf), "k_resident<%d,%d>", rs.nw, rs.cpw);
    }
    snprintf(name, (size_t)cap, "%s", buf);
    return SLLG_OK;
}

int64_t sllg_level_step(const sllg_ctx* C, int32_t level)
{
    if (!C || level < 0 || level >= (int)C->lv.size()) return -1;
    return C->lv[level].step;
}

int sllg_get_state(sllg_ctx* C, int32_t level, int32_t real, float* host_m)
{
    if (!C || level < 0 || level >= (int)C->lv.size() || !host_m) return fail(SLLG_E_INVAL, "bad args");
    const LevelHost& h = C->lv[level];
    if (real < 0 || real >= h.ninst) return fail(SLLG_E_INVAL, "bad realization");
    const InstDev& I = C->h_insts[h.inst0 + real];
    const float* src = ((h.step & 1) ? C->d_buf1 : C->d_buf0) + I.state_off;
    HIP_OK(hipMemcpyAsync(host_m, src, sizeof(float) * 3 * h.ncell, hipMemcpyDeviceToHost, C->stream));
    return check_status(C);
}

int sllg_save_state(sllg_ctx* C, void* host, size_t cap, size_t* need)
{
    if (!C || !need) return fail(SLLG_E_INVAL, "bad args");
    *need = snap_bytes(C);
    if (!host) return SLLG_OK;
    if (cap < *need) return fail(SLLG_E_INVAL, "snapshot buffer of %zu bytes, %zu needed", cap, *need);
    // every enqueued step has finished (and folded) once the stream is idle;
    // a failed run is not saved
    const int rc = check_status(C);
    if (rc) return rc;
    char* p = static_cast<char*>(host);
    SnapHead hd{};
    std::memcpy(hd.magic, kSnapMagic, sizeof(hd.magic));
    hd.nlev = (int32_t)C->lv.size();
    hd.ckpt_every = C->ckpt_every;
    hd.state_floats = C->lay.state_floats;
    hd.rec_doubles = C->lay.rec_doubles;
    hd.ckpt_floats = C->lay.ckpt_floats;
    hd.ninst = C->lay.ninst_total;
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    for (const LevelHost& h : C->lv) {
        const SnapLevel sl = snap_level(h);
        std::memcpy(p, &sl, sizeof(sl));
        p += sizeof(sl);
    }
    for (const auto& r : snap_regions(C)) {
        if (r.second) HIP_OK(hipMemcpyAsync(p, r.first, r.second, hipMemcpyDeviceToHost, C->stream));
        p += r.second;
    }
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

int sllg_load_state(sllg_ctx* C, const void* host, size_t size)
{
    if (!C || !host) return fail(SLLG_E_INVAL, "bad args");
    if (size != snap_bytes(C))
        return fail(SLLG_E_INVAL, "snapshot of %zu bytes; this context's snapshots have %zu", size, snap_bytes(C));
    const char* p = static_cast<const char*>(host);
    SnapHead hd;
    std::memcpy(&hd, p, sizeof(hd));
    p += sizeof(hd);
    if (std::memcmp(hd.magic, kSnapMagic, sizeof(hd.magic)) != 0) return fail(SLLG_E_INVAL, "not a snapshot");
    if (hd.nlev != (int32_t)C->lv.size() || hd.ckpt_every != C->ckpt_every ||
        hd.state_floats != C->lay.state_floats || hd.rec_doubles != C->lay.rec_doubles ||
        hd.ckpt_floats != C->lay.ckpt_floats || hd.ninst != C->lay.ninst_total)
        return fail(SLLG_E_INVAL, "snapshot of another configuration (levels, sizes or checkpoint interval)");
    std::vector<SnapLevel> sl(C->lv.size());
    for (size_t l = 0; l < C->lv.size(); ++l) {
        std::memcpy(&sl[l], p, sizeof(SnapLevel));
        p += sizeof(SnapLevel);
        SnapLevel mine = snap_level(C->lv[l]);
        mine.step = sl[l].step;
        if (std::memcmp(&mine, &sl[l], sizeof(SnapLevel)) != 0)
            return fail(SLLG_E_INVAL, "snapshot of another configuration (level %zu: grid, seeds or constants)", l);
        if (sl[l].step < 0 || sl[l].step > sl[l].n_steps) return fail(SLLG_E_INVAL, "snapshot step out of range");
    }
    // nothing of this context may still be running while its state is replaced
    HIP_OK(hipStreamSynchronize(C->stream));
    for (const auto& r : snap_regions(C)) {
        if (r.second) HIP_OK(hipMemcpyAsync(r.first, p, r.second, hipMemcpyHostToDevice, C->stream));
        p += r.second;
    }
    HIP_OK(hipStreamSynchronize(C->stream));
    for (size_t l = 0; l < C->lv.size(); ++l) C->lv[l].step = sl[l].step;
    return SLLG_OK;
}

int sllg_set_state(sllg_ctx* C, int32_t level, int32_t real, const float* host_m)
{
    if (!C || level < 0 || level >= (int)C->lv.size() || !host_m) return fail(SLLG_E_INVAL, "bad args");
    const LevelHost& h = C->lv[level];
    if (real < 0 || real >= h.ninst) return fail(SLLG_E_INVAL, "bad realization");
    const InstDev& I = C->h_insts[h.inst0 + real];
    float* dst = ((h.step & 1) ? C->d_buf1 : C->d_buf0) + I.state_off;
    HIP_OK(hipMemcpyAsync(dst, host_m, sizeof(float) * 3 * h.ncell, hipMemcpyHostToDevice, C->stream));
    // the loop continues from this state's ordinate
    double mz = 0;
    for (int64_t c = 0; c < h.ncell; ++c) mz += host_m[2 * h.ncell + c];
    mz /= (double)h.ncell;
    AccDev a;
    HIP_OK(hipMemcpyAsync(&a, C->d_accs + h.inst0 + real, sizeof(AccDev), hipMemcpyDeviceToHost, C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    a.m_prev = mz;
    HIP_OK(hipMemcpyAsync(C->d_accs + h.inst0 + real, &a, sizeof(AccDev), hipMemcpyHostToDevice, C->stream));
    if (h.step % h.in.record_every == 0)
        HIP_OK(hipMemcpyAsync(C->d_records + I.rec_off + h.step / h.in.record_every, &mz, sizeof(double),
                              hipMemcpyHostToDevice, C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

int sllg_set_plan(sllg_ctx* C, int32_t level, int32_t plan)
{
    if (!C || level < 0 || level >= (int)C->lv.size()) return fail(SLLG_E_INVAL, "bad level");
    LevelHost& h = C->lv[level];
    // magnetostatics has one plan, and that plan needs the field tables
    if (C->mat.demag && plan != kPlanAuto && plan != kPlanDemag)
        return fail(SLLG_E_INVAL, "a level with magnetostatics runs on plan 5 only");
    if (!C->mat.demag && plan == kPlanDemag) return fail(SLLG_E_INVAL, "plan 5 needs material demag != 0");
    if (C->mat.demag) {
        h.forced = plan == kPlanDemag;
        h.plan = kPlanDemag;
        return replan(C);
    }
    if (plan == kPlanAuto) {
        h.forced = 0;
        bool all_single = true;
        for (const LevelHost& x : C->lv) all_single = all_single && x.ncell == 1;
        plan = all_single ? kPlanLanes : resident_fits(h, C->max_lds) ? kPlanResident : kPlanStream;
    } else if (plan == kPlanResident) {
        if (!resident_fits(h, C->max_lds)) return fail(SLLG_E_INVAL, "level %d does not fit in LDS", level);
        h.forced = 1;
    } else if (plan == kPlanStream) {
        h.forced = 1;
    } else if (plan == kPlanLanes) {
        if (h.ncell != 1) return fail(SLLG_E_INVAL, "level %d is not a single cell (plan 4)", level);
        h.forced = 1;
    } else if (plan == kPlanSlab) {
        if (!slab_eligible(h.in)) return fail(SLLG_E_INVAL, "level %d cannot use slabs (nx*ny <= 1024, nz >= 4)", level);
        auto it = g_tuned_slab.find(std::make_tuple(h.in.nx, h.in.ny, h.in.nz, h.ninst));
        if (it != g_tuned_slab.end()) {
            h.slab_kernel = std::get<0>(it->second);
            h.slab_tz = std::get<1>(it->second);
        } else {
            // the smallest kernel that holds two-plane slabs
            const int P = h.in.nx * h.in.ny;
            h.slab_kernel = -1;
            for (int ki = 0; ki < kNumSlabKernels && h.slab_kernel < 0; ++ki)
                if (kSlabKernels[ki].kind == 0 && kSlabKernels[ki].nt / P >= 1 &&
                    kSlabKernels[ki].k * (kSlabKernels[ki].nt / P) >= 5) {
                    h.slab_kernel = ki;
                    h.slab_tz = 2;
                }
            if (h.slab_kernel < 0) return fail(SLLG_E_INVAL, "no slab kernel for level %d", level);
        }
        h.forced = 1;
    } else {
        return fail(SLLG_E_INVAL, "unknown plan %d", plan);
    }
    h.plan = plan;
    if (plan == kPlanStream) {
        auto it = g_tuned.find(std::make_tuple(h.in.nx, h.in.ny, h.in.nz, h.ninst));
        if (it != g_tuned.end()) {
            h.shape = it->second.first;
            h.tz = it->second.second;
        } else {
            default_stream_shape(C, h);
        }
    }
    int rc = replan(C);
    if (rc) return rc;
    // the stream kernel reads the step index from the device
    for (size_t l = 0; l < C->lv.size(); ++l)
        HIP_OK(hipMemcpyAsync(C->d_steps + l, &C->lv[l].step, sizeof(int64_t), hipMemcpyHostToDevice,
                              C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

int sllg_set_slab_shape(sllg_ctx* C, int32_t level, int32_t kind, int32_t threads, int32_t cells_per_thread,
                        int32_t planes)
{
    if (!C || level < 0 || level >= (int)C->lv.size()) return fail(SLLG_E_INVAL, "bad level");
    if (C->mat.demag) return fail(SLLG_E_INVAL, "a level with magnetostatics runs on plan 5 only");
    LevelHost& h = C->lv[level];
    if (!slab_eligible(h.in)) return fail(SLLG_E_INVAL, "level %d cannot use slabs (nx*ny <= 1024, nz >= 4)", level);
    int ki = -1;
    for (int i = 0; i < kNumSlabKernels; ++i)
        if (kSlabKernels[i].kind == kind && kSlabKernels[i].nt == threads && kSlabKernels[i].k == cells_per_thread)
            ki = i;
    if (ki < 0) return fail(SLLG_E_INVAL, "no slab kernel kind %d <%d,%d>", kind, threads, cells_per_thread);
    if (planes < (kind == 0 ? 2 : 1) || planes > h.in.nz) return fail(SLLG_E_INVAL, "bad slab thickness %d", planes);
    const int saved[4] = {h.plan, h.slab_kernel, h.slab_tz, h.forced};
    h.plan = kPlanSlab;
    h.slab_kernel = ki;
    h.slab_tz = planes;
    h.forced = 1;
    int rc = replan(C);
    bool fits = false;
    if (!rc && (dispatch_slab(C, level, 0, 1, true, &fits) != hipSuccess || !fits)) rc = SLLG_E_INVAL;
    if (rc) {
        h.plan = saved[0];
        h.slab_kernel = saved[1];
        h.slab_tz = saved[2];
        h.forced = saved[3];
        (void)replan(C);
        return fail(SLLG_E_INVAL, "slab kernel kind %d <%d,%d> with %d planes cannot hold level %d", kind, threads,
                    cells_per_thread, planes, level);
    }
    return SLLG_OK;
}

int sllg_set_stream_shape(sllg_ctx* C, int32_t level, int32_t kind, int32_t a, int32_t b, int32_t c,
                          int32_t planes)
{
    if (!C || level < 0 || level >= (int)C->lv.size()) return fail(SLLG_E_INVAL, "bad level");
    if (C->mat.demag) return fail(SLLG_E_INVAL, "a level with magnetostatics runs on plan 5 only");
    LevelHost& h = C->lv[level];
    int si = -1;
    for (int i = 0; i < kNumShapes; ++i)
        if (kShapes[i].kind == kind && kShapes[i].tx == a && kShapes[i].ty == b && kShapes[i].pz == c) si = i;
    if (si < 0) return fail(SLLG_E_INVAL, "no stream kernel kind %d <%d,%d,%d>", kind, a, b, c);
    if (planes < 1 || planes < kShapes[si].pz || !shape_fits(h.in, kShapes[si]) ||
        tiles_for(h.in, kShapes[si], planes) * h.ninst > C->lay.max_tiles)
        return fail(SLLG_E_INVAL, "stream kernel kind %d <%d,%d,%d> with %d planes cannot hold level %d", kind, a, b,
                    c, planes, level);
    h.plan = kPlanStream;
    h.shape = si;
    h.tz = planes;
    h.forced = 1;
    int rc = replan(C);
    if (rc) return rc;
    for (size_t l = 0; l < C->lv.size(); ++l)
        HIP_OK(hipMemcpyAsync(C->d_steps + l, &C->lv[l].step, sizeof(int64_t), hipMemcpyHostToDevice, C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

int sllg_philox_probe(uint64_t seed, uint32_t level, uint32_t tag, const uint32_t* cells,
                      const uint64_t* steps, int32_t n, uint32_t* raw, float* normals, void* d_scratch,
                      void* hip_stream)
{
    if (n < 0 || !cells || !steps || !raw || !normals || !d_scratch) return fail(SLLG_E_INVAL, "bad args");
    if (tag > 255 || level > 255) return fail(SLLG_E_INVAL, "tag and level are 8-bit");
    if (n == 0) return SLLG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    char* p = (char*)d_scratch;
    uint32_t* d_cells = (uint32_t*)p;
    uint64_t* d_steps = (uint64_t*)(p + align256(4 * (size_t)n));
    uint32_t* d_raw = (uint32_t*)((char*)d_steps + align256(8 * (size_t)n));
    float* d_nrm = (float*)((char*)d_raw + align256(16 * (size_t)n));
    HIP_OK(hipMemcpyAsync(d_cells, cells, 4 * (size_t)n, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(d_steps, steps, 8 * (size_t)n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_philox_probe, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, seed, level, tag,
                       d_cells, d_steps, n, d_raw, d_nrm);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(raw, d_raw, 16 * (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(normals, d_nrm, 12 * (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return SLLG_OK;
}

int sllg_get_axes(sllg_ctx* C, int32_t level, float* host_u)
{
    if (!C || level < 0 || level >= (int)C->lv.size() || !host_u) return fail(SLLG_E_INVAL, "bad args");
    const LevelHost& h = C->lv[level];
    if (h.axes_off < 0) {
        const LevelDev& d = C->h_levels[level];
        for (int64_t c = 0; c < h.ncell; ++c) {
            host_u[c] = d.ux;
            host_u[h.ncell + c] = d.uy;
            host_u[2 * h.ncell + c] = d.uz;
        }
        return SLLG_OK;
    }
    HIP_OK(hipMemcpyAsync(host_u, C->d_axes + h.axes_off, sizeof(float) * 3 * h.ncell, hipMemcpyDeviceToHost,
                          C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    return SLLG_OK;
}

int sllg_set_timing(sllg_ctx* C, int32_t on)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    C->timing = on > 0 ? on : 0;
    C->ev_used = 0;
    C->ev_launches.clear();
    C->timed_cells = 0;
    C->unit_counter = 0;
    return SLLG_OK;
}

int sllg_kernel_time(sllg_ctx* C, double* mean_ms, int64_t* launches, int64_t* cells_per_launch)
{
    if (!C) return fail(SLLG_E_INVAL, "null context");
    HIP_OK(hipStreamSynchronize(C->stream));
    double tot = 0;
    int64_t nl = 0;
    const int64_t np = (int64_t)(C->ev_used / 2);
    for (int64_t i = 0; i < np && i < (int64_t)C->ev_launches.size(); ++i) {
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, C->ev_pool[2 * i], C->ev_pool[2 * i + 1]));
        tot += ms;
        nl += C->ev_launches[i];
    }
    if (mean_ms) *mean_ms = nl ? tot / nl : 0.0;
    if (launches) *launches = nl;
    if (cells_per_launch) *cells_per_launch = nl ? C->timed_cells / nl : 0;
    C->ev_used = 0;
    C->ev_launches.clear();
    C->timed_cells = 0;
    return SLLG_OK;
}

int sllg_grad(sllg_ctx* C, int32_t level, double g_area[4], double g_hc[4])
{
    if (!C || level < 0 || level >= (int)C->lv.size() || !g_area || !g_hc)
        return fail(SLLG_E_INVAL, "bad arguments");
    const LevelHost& h = C->lv[level];
    if (C->ckpt_every <= 0 || !C->d_ckpt)
        return fail(SLLG_E_STATE, "sllg_grad needs checkpoints: pass ckpt_every > 0 to sllg_init");
    if (h.in.record_every != 1) return fail(SLLG_E_STATE, "sllg_grad needs record_every == 1");
    if (h.step != h.n_steps) return fail(SLLG_E_STATE, "run the whole sweep before sllg_grad");
    if (h.ncell > 1536) return fail(SLLG_E_INVAL, "the adjoint holds at most 1536 cells per realization");
    if (C->mat.demag) return fail(SLLG_E_STATE, "the adjoint has no magnetostatic term");
    int rc = check_status(C);
    if (rc) return rc;
    const int64_t NS = h.n_steps, R = h.ninst;
    // ensemble-mean loop and the loss weights dL/dmbar_n of one realization
    std::vector<double> rec((size_t)(R * (NS + 1)));
    for (int r = 0; r < R; ++r)
        HIP_OK(hipMemcpyAsync(rec.data() + (size_t)r * (NS + 1), C->d_records + C->h_insts[h.inst0 + r].rec_off,
                              sizeof(double) * (NS + 1), hipMemcpyDeviceToHost, C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    std::vector<double> H(NS + 1), m(NS + 1, 0.0), w(2 * (NS + 1), 0.0);
    const double hz_oe = h.hz_amp / kOe;
    for (int64_t k = 0; k <= NS; ++k) H[k] = hz_oe * wave_host(h, C->mat.wave, k);
    for (int r = 0; r < R; ++r)
        for (int64_t k = 0; k <= NS; ++k) m[k] += rec[(size_t)r * (NS + 1) + k];
    for (int64_t k = 0; k <= NS; ++k) m[k] /= (double)R;
    for (int64_t k = 0; k < NS; ++k) {   // area: S = -sum (m_k + m_{k+1})/2 (H_{k+1} - H_k)
        const double dH = H[k + 1] - H[k];
        w[k] -= 0.5 * dH;
        w[k + 1] -= 0.5 * dH;
    }
    const Stats st = analyse(H, m);
    const bool hc_ok = st.kd >= 0 && st.ka >= 0;
    if (hc_ok) {   // Hc = (H*_asc - H*_desc)/2, H* = H_k - m_k dH/(m_{k+1} - m_k)
        const int ks[2] = {st.kd, st.ka};
        const double sg[2] = {-0.5, 0.5};
        for (int b = 0; b < 2; ++b) {
            const int k = ks[b];
            const double dH = H[k + 1] - H[k], D = m[k + 1] - m[k];
            w[(NS + 1) + k] += sg[b] * (-dH * m[k + 1] / (D * D));
            w[(NS + 1) + k + 1] += sg[b] * (dH * m[k] / (D * D));
        }
    }
    for (double& x : w) x /= (double)R;
    HIP_OK(hipMemcpyAsync(C->d_weights, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, C->stream));
    // threads and cells per thread: one cell per thread up to 1024 cells,
    // two per thread (768 threads) up to 1536
    const int nt = h.ncell <= 64 ? 64 : h.ncell <= 128 ? 128 : h.ncell <= 192 ? 192 : h.ncell <= 256 ? 256
                 : h.ncell <= 512 ? 512 : h.ncell <= 1024 ? 1024 : 768;
    const int kc = h.ncell <= 1024 ? 1 : 2;
    // dynamic LDS: the segment's loss weights and applied field (three FP32
    // per step); static LDS: m_n and m' of two parities, four H-bar planes,
    // replay noise of two parities (noise threads), sums
    const size_t seg_lds = 12 * (size_t)(C->ckpt_every + 1);
    const size_t static_lds = (size_t)nt * kc * (2 * 2 * 3 * 4 + 2 * 2 * 3 * 4) +
                              (kc == 1 && nt <= 256 ? (size_t)nt * 2 * 3 * 4 : 24) + (size_t)(nt / 64) * 10 * 8;
    if (seg_lds + static_lds > (size_t)C->max_lds)
        return fail(SLLG_E_INVAL, "ckpt_every %d too large for the adjoint's LDS (at most %d)", C->ckpt_every,
                    (int)((C->max_lds - static_lds) / 12) - 1);
#define SLLG_ADJ(NT, KC)                                                                                      \
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint<NT, KC>),                              \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)seg_lds);                      \
    hipLaunchKernelGGL((k_adjoint<NT, KC>), dim3((unsigned)R), dim3(kAdjThreads<NT, KC>), seg_lds, C->stream, \
                       C->d_insts, h.inst0,                                                                   \
                       C->d_levels, C->d_axes, C->d_ckpt, C->ckpt_every, C->d_tape, C->d_weights, C->d_grads)
    switch (nt * 10 + kc) {
    case 641: SLLG_ADJ(64, 1); break;
    case 1281: SLLG_ADJ(128, 1); break;
    case 1921: SLLG_ADJ(192, 1); break;
    case 2561: SLLG_ADJ(256, 1); break;
    case 5121: SLLG_ADJ(512, 1); break;
    case 10241: SLLG_ADJ(1024, 1); break;
    default: SLLG_ADJ(768, 2); break;
    }
#undef SLLG_ADJ
    HIP_OK(hipGetLastError());
    std::vector<double> gr((size_t)(10 * R));
    HIP_OK(hipMemcpyAsync(gr.data(), C->d_grads + 10 * h.inst0, sizeof(double) * gr.size(), hipMemcpyDeviceToHost,
                          C->stream));
    HIP_OK(hipStreamSynchronize(C->stream));
    double g[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    for (int r = 0; r < R; ++r)
        for (int l = 0; l < 2; ++l)
            for (int k = 0; k < 5; ++k) g[l][k] += gr[(size_t)r * 10 + l * 5 + k];
    // chain rule from (c_ex, H_K, gamma1, alpha|gamma1, sigma) to (K, A, alpha, ms_scale)
    const double al = h.alpha, Ms = h.Ms;
    for (int l = 0; l < 2; ++l) {
        double* out = l == 0 ? g_area : g_hc;
        const double gc = g[l][0], gk = g[l][1], gg = g[l][2], ga = g[l][3], gs = g[l][4];
        out[0] = gk * 2.0 / (kMu0 * Ms);                              // dH_K/dK
        out[1] = gc * 2.0 / (kMu0 * Ms * h.a * h.a);                  // dc_ex/dA
        out[2] = ga + gg * (-2.0 * al * kGamma0 / ((1.0 + al * al) * (1.0 + al * al))) +
                 (al > 0 ? gs * h.sigma / (2.0 * al) : 0.0);           // gamma1(alpha), sigma(alpha)
        out[3] = C->mat.Ms0 * (-gc * h.c_ex / Ms - gk * h.hk / Ms - gs * h.sigma / (2.0 * Ms));
    }
    if (!hc_ok)
        for (int k = 0; k < 4; ++k) g_hc[k] = NAN;
    return SLLG_OK;
}

void sllg_free(sllg_ctx* C)
{
    if (!C) return;
    if (C->static_dev >= 0) {
        // the static workspace is free for the next context once the
        // context's work on it has finished
        (void)hipStreamSynchronize(C->stream);
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[C->static_dev] = false;
    }
    for (hipEvent_t e : C->ev_pool) (void)hipEventDestroy(e);
    if (C->cap_stream) (void)hipStreamDestroy(C->cap_stream);
    for (const auto& g : C->graphs) (void)hipGraphExecDestroy(g.second);
    delete C;
}

}  // extern "C"
