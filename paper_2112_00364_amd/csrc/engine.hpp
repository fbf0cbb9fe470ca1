// Device-side run layout shared by the kernels and the host engine.
#pragma once

#include "models.hpp"

namespace pcfg {

// Per-run control block in device memory. Kernels read the round and status
// from here, so a fixed launch sequence can be replayed without host input.
struct alignas(64) RunCtl {
    unsigned long long maxkey;       // order-preserving key of max lw this round (0 = none yet)
    unsigned long long block_steps;  // canonical block executions so far
    double log_z;                    // running normalising-constant estimate
    double m_cur;                    // M of the pending resampling
    double qtot;                     // total grid units of the pending resampling
    uint32_t u;                      // offset word of the pending resampling
    uint32_t round;                  // round the next propagation runs
    int32_t status;                  // SMC_OK / FINISHED / ERR_NAN / DEGENERATE
    uint32_t active;                 // particles not at b_stop after this round's propagation
    uint32_t bad;                    // a NaN or +inf log-weight was produced
    uint32_t ticket;                 // work-groups done in the reduction
    uint32_t deep_count;             // particles handed to the deep-stack pass this round
    uint32_t pad[3];
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
