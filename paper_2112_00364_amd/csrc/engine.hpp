// Device-side run layout shared by the kernels and the host engine.
#pragma once

#include "models.hpp"

namespace pcfg {

// Per-run control block in device memory. Kernels read the round and status
// from here, so a fixed launch sequence can be replayed without host input.
struct alignas(64) RunCtl {
    unsigned long long maxkey;       // order-preserving key of max lw this round (0 = none)
    unsigned long long block_steps;  // canonical block executions so far
    double log_z;                    // running normalising-constant estimate
    double m_cur;                    // M of the pending resampling (fold-kernel path)
    double qtot;                     // total grid units of the pending resampling (fold-kernel path)
    uint32_t u;                      // offset word of the pending resampling
    uint32_t round;                  // round the next propagation runs
    int32_t status;                  // SMC_OK / FINISHED / ERR_NAN / DEGENERATE
    uint32_t active;                 // particles not at b_stop after this round's propagation
    uint32_t bad;                    // a NaN or +inf log-weight was produced
    uint32_t carry;                  // 1: the last round kept its weights (ESS rule), no gather pending
    unsigned long long seed;         // Philox key of the run (set by init / reset)
    uint32_t resamples;              // rounds that resampled
    uint32_t pad;
};

// One particle buffer: block index, real fields (storage precision), int
// fields, and the ClaDS stack (level-major: level k of particle j at k*n + j).
struct ParticleBuf {
    uint8_t* blk;
    void* real[6];
    int32_t* ints[9];
    void* stack;
};

struct RunDev {
    uint32_t n;
    uint32_t red_tiles;            // reduction / scan tiles of kTileRed particles
    uint32_t prop_tiles;           // propagation tiles of `lanes` particles
    uint32_t fused;                // 1: the reduction and scan fold the partials themselves
    uint32_t ess_t;                // ESS threshold numerator over 2^16 (0: resample every round)
    uint32_t lanes;                // lanes per propagation work-group (128 or 256; smc_set_workgroup)
    const ModelDev* model;
    RunCtl* ctl;
    ParticleBuf buf[2];            // buf[r & 1] is written by the propagation of round r
    double* lw;
    uint32_t* anc;
    void* side_stack;              // ClaDS: per-slot side-lineage stacks (start, rate: FP64; depth: byte)
    struct GroupPartials* groups;  // the propagation's partials, folded into kPartialGroups slots
    double* part_q;                // per reduction tile: sum of grid units
    double* part_e;                // per reduction tile: sum of exp(lw - M)
    unsigned long long* part_q2;   // per reduction tile: sum of squared grid units (lo, hi), ESS rule only
    double* prefix;                // per reduction tile: grid units before the tile (fold-kernel path)
    // block bucketing (optional, single runs): the propagation takes slot
    // perm[i] at position i; the counting sort that fills perm keeps its
    // per-(block, tile) counts and per-block totals here
    uint32_t* perm;
    uint32_t* bucket_hist;         // [kBuckets][red_tiles], block-major
    uint32_t* bucket_total;        // [kBuckets]
};

// Default lanes (= particles) per propagation work-group, by model kind: 128
// for the tree models and the small ones (finer scheduling of divergent
// blocks), 256 for the SEIR model (measured faster). A single run can switch
// to the other size (smc_set_workgroup); batches use the default. The resampling-only entry point
// takes its maxima over tiles of kMaxkeyThreads.
__host__ __device__ constexpr int prop_threads(int kind) { return kind == 4 ? 256 : 128; }
constexpr int kMaxkeyThreads = 256;
constexpr int kRedThreads = 256;
constexpr int kRedItems = 4;
constexpr int kTileRed = kRedThreads * kRedItems;  // particles per reduction tile
// Runs with at most this many reduction tiles (2^20 particles) fold the
// reduction's tile sums inside the scan kernel; larger runs use the
// one-work-group fold kernel.
constexpr uint32_t kMaxFusedRedTiles = 1024;
// A batched run of at most this many particles may be owned by one work-group
// (kRedThreads lanes) for all the rounds of a tick.
constexpr uint32_t kOwnedMaxParticles = 4 * kTileRed;
// Block bucketing sorts slots by their resume block (255 = b_stop) into
// kBuckets keys, over the reduction tiles.
constexpr int kBuckets = 256;
static_assert(kBuckets == kRedThreads, "one bucket per thread of a tile work-group");

// Propagation work-group t folds its partial (max order-key of lw; active
// count and block steps packed in one word) into slot t mod kPartialGroups
// with two device-scope atomics on distinct addresses; the reduction reads
// all slots and the scan clears them for the next round.
constexpr uint32_t kPartialGroups = 256;
struct GroupPartials {
    unsigned long long key[kPartialGroups];     // max order-key (all ones: a NaN or +inf weight)
    unsigned long long counts[kPartialGroups];  // particles not at b_stop | block executions << 32
};

// Work-group -> (run index, tile index within the run).
struct TileRef {
    uint32_t run, tile;
};

}  // namespace pcfg
