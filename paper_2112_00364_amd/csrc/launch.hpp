// Kernel launchers (defined in kernels.hip, used by the host engine).
#pragma once

#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace pcfg {

// batch: one launch over a (run, tile) table of runs of one kind, precision
// and work-group size (128 or 256 lanes)
hipError_t launch_propagate(int kind, int precision, int lanes, const RunDev* runs, const TileRef* tiles,
                            uint32_t n_tiles, hipStream_t st);
// batch: runs owned by one work-group each (ids index runs), all `rounds`
// rounds of a tick in one launch; kinds 0-5
hipError_t launch_owned(int kind, int precision, const RunDev* runs, const uint32_t* ids, uint32_t n_runs,
                        uint32_t rounds, hipStream_t st);
// single run: the run record travels as a kernel argument
hipError_t launch_propagate_one(int kind, int precision, const RunDev& run, hipStream_t st);
hipError_t launch_resample_one(const RunDev& run, const RunDev* run_dev, hipStream_t st, int part);
// block bucketing: fills run.perm for the next propagation (three launches)
hipError_t launch_bucket(const RunDev& run, hipStream_t st);
hipError_t launch_reduce(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, uint32_t n_runs,
                         bool any_unfused, hipStream_t st);
hipError_t launch_scan_anc(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, hipStream_t st);
hipError_t launch_maxkey(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, hipStream_t st);
// resampling alone on a run record whose control block, group slots and tile
// partials sit in caller-provided device memory (no table uploads): prepares
// the control block, then max, reduction (+ fold), scan and ancestors, and
// stores the log Z increment at log_z_out
hipError_t launch_resample_weights_one(const RunDev& run, uint32_t round, uint64_t seed, double* log_z_out,
                                       hipStream_t st);
hipError_t launch_gather(int elem_bytes, const void* src, const uint32_t* anc, void* dst, uint64_t n,
                         uint64_t levels, uint64_t stride, hipStream_t st);
hipError_t launch_selftest_math(int op, const double* in, double* out, uint64_t n, hipStream_t st);
hipError_t launch_selftest_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n,
                                  hipStream_t st);
hipError_t launch_model_setup(ModelDev* m, hipStream_t st);
hipError_t launch_reset(RunDev* run, uint64_t seed, hipStream_t st);

}  // namespace pcfg
