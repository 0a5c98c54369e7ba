// dispatch.h -- launch arguments shared by the host API and the march kernels.
#pragma once

#include "media.h"

namespace vrt {

struct EntryState;  // lane32.h

struct LaunchArgs {
    MediumDev m;
    MedF mf;
    BoundaryDev b;
    TraceDev t;
    RaysDev<double> io64;
    RaysDev<float> io32;
    uint32_t n;
    hipStream_t stream;
    uint32_t *queue;  // FP32_COMP: ray-queue counter (device), zeroed by the launcher
    int num_cu;
    int blocks_per_cu;  // FP32_COMP persistent grid: blocks of 256 lanes per CU (0 = default)
    uint32_t max_blocks;  // FP32_COMP persistent grid: cap on the blocks (0 = none)
    EntryState *entry;    // FP32_COMP: n entry states for media marched from them, or null
};

// FP32_COMP: whether a launch on a medium of this kind runs the entry kernel
// first when given room for the entry states
bool fp32c_pre_entry(int kind);

hipError_t launch_march_fp64(const LaunchArgs &a);
hipError_t launch_march_fp32c(const LaunchArgs &a);
hipError_t launch_paths_fp64(const LaunchArgs &a, double *path, uint64_t cap,
                             uint64_t *n_points);

}  // namespace vrt
