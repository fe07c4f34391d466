// Types shared by the host runtime and the gfx950 kernels of the stochastic-LLG
// library.  Plain structs of scalars so that one copy lives in device memory
// and is read with scalar loads.
#pragma once
#include <cstdint>

namespace sllg {

// Per-level constants of the step (FP32 for the lanes, FP64 for the loop).
struct LevelDev {
    float c_ex;      // A/m, 2A/(mu0 Ms a^2)
    float hk;        // A/m, 2K/(mu0 Ms)
    float g1;        // gamma0/(1+alpha^2)
    float ag1;       // alpha*gamma1
    float sigma;     // thermal field std-dev per component, A/m
    float dt;        // s
    float half_dt;   // s
    float pad0;
    float ux, uy, uz, pad1;  // uniform easy axis
    double hz_amp;   // peak applied field, A/m (already zeta-scaled)
    double hz_oe;    // the same peak in Oe
    int64_t n_period;        // steps per field cycle
    int64_t n_steps;         // steps per sweep
    double inv_period;       // 1 / n_period
    int32_t wave;            // 0 triangle, 1 cosine, 2 constant
    int32_t level_tag;       // RNG counter field
    int32_t record_every;
    int32_t ncell;
    int32_t nx, ny, nz;
    int32_t has_axes;        // per-cell axes stored at axes_off
    int64_t axes_off;        // float offset of the ux plane in the axes array
    int64_t n_rec;           // recorded points per instance
    int64_t demag_off;       // float offset of the demagnetising-tensor table (magnetostatics)
};

// One instance = one realization of one level.
struct InstDev {
    int32_t level;
    int32_t real;
    uint64_t seed;
    int64_t state_off;   // float offset of the mx plane (my, mz follow, ncell apart)
    int64_t rec_off;     // double offset of the loop record
    int64_t ckpt_off;    // float offset of checkpoint 0 (each 3*ncell floats)
    int32_t tile0;       // stream plan: first tile
    int32_t ntiles;      // stream plan: number of tiles
};

// Online loop accumulators of one instance (FP64).
struct AccDev {
    double area;         // -sum (m_k + m_{k+1})/2 (H_{k+1} - H_k)
    double m_prev;       // loop ordinate at the current step
    double hstar_d, hstar_a;   // first crossing field on the falling / rising branch
    double m0_d, m0_a;         // loop ordinate where H crosses 0 falling / rising
    int32_t ncross_d, ncross_a;
    int32_t found_d, found_a, found0_d, found0_a;
    int32_t rec_phase;   // steps since the last recorded point
    int32_t rec_idx;     // index of the last recorded point
};

// A tile of the stream plan: an x-y window of one instance and a z range.
struct TileDev {
    int32_t inst;
    int16_t x0, y0, z0;
    int16_t nxt, nyt, nzt;
};

// Chunk of 64 cells of one instance for the resident plan.
struct ChunkDev {
    int32_t inst;    // global instance index
    int32_t slot;    // instance slot inside the workgroup
    int32_t c0;      // first cell
    int32_t pad;
};

// Instance slot of a resident workgroup.
struct SlotDev {
    int32_t inst;
    int32_t lds_off;   // cell offset inside the workgroup's LDS state
    int32_t chunk0;    // first chunk of the instance in the workgroup list
    int32_t nchunks;
};

// Resident workgroup: a range of slots and chunks.
struct GroupDev {
    int32_t slot0, nslots;
    int32_t chunk0, nchunks;
    int32_t ncells;      // cells of LDS state (sum over slots)
    int32_t pad;
};

constexpr uint32_t kTagNoise = 1;
constexpr uint32_t kTagAxis = 2;

}  // namespace sllg
