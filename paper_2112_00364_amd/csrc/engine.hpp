// Device-side run layout shared by the kernels and the host engine.
#pragma once

#include "models.hpp"

namespace pcfg {

// Per-run control block in device memory. Kernels read the round and status
// from here, so a fixed launch sequence can be replayed without host input.
struct alignas(128) RunCtl {
    unsigned long long maxkey;       // order-preserving key of max lw this round (0 = none)
    unsigned long long block_steps;  // canonical block executions so far
    double log_z;                    // running normalising-constant estimate
    double m_cur;                    // M of the pending resampling
    double qtot;                     // total grid units of the pending resampling
    uint32_t u;                      // offset word of the pending resampling
    uint32_t round;                  // round the next propagation runs
    int32_t status;                  // SMC_OK / FINISHED / ERR_NAN / DEGENERATE
    uint32_t active;                 // particles not at b_stop after this round's propagation
    uint32_t bad;                    // a NaN or +inf log-weight was produced
    uint32_t deep_count;             // particles handed to the deep-stack pass this round
    // partials of the deep-stack pass (one per deep work-group)
    unsigned long long deep_key[4];
    uint32_t deep_cnt[4];            // active | bad << 31
    uint32_t deep_steps[4];
};
// One particle buffer: block index, real fields (storage precision), int
// fields, and the ClaDS stack (level-major: level k of particle j at k*n + j).
struct ParticleBuf {
    uint8_t* blk;
    void* real[4];
    int32_t* ints[2];
    void* stack;
};

struct RunDev {
    uint64_t seed;
    uint32_t n;
    uint32_t red_tiles;  // reduction / scan tiles of kTileRed particles
    const ModelDev* model;
    RunCtl* ctl;
    ParticleBuf buf[2];  // buf[r & 1] is written by the propagation of round r
    double* lw;
    uint32_t* anc;
    uint32_t* deep_list; // particles whose hidden-lineage stack outgrew the registers
    uint32_t prop_tiles; // propagation tiles of kPropThreads particles
    unsigned long long* part_key;  // per propagation tile: max key
    uint32_t* part_cnt;            // per propagation tile: active count | bad << 31
    uint32_t* part_steps;          // per propagation tile: block steps
    double* part_q;      // per reduction tile: sum of grid units
    double* part_e;      // per reduction tile: sum of exp(lw - M)
    double* prefix;      // per reduction tile: grid units before the tile
};

constexpr int kPropThreads = 256;               // one particle per lane
constexpr int kRedThreads = 256;
constexpr int kRedItems = 4;
constexpr int kTileRed = kRedThreads * kRedItems;  // particles per reduction tile

// Work-group -> (run index, tile index within the run).
struct TileRef {
    uint32_t run, tile;
};

}  // namespace pcfg
