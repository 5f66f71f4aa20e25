// psd_internal.h -- shapes shared between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psd_device.h"

namespace psd {

struct UniformArgs {
    const float* pos;
    int np[3];
    int nc[3];
    double scale[3];           // nc_k / box
    int64_t ntet;              // 6 * np0 * np1 * np2
    double m;                  // mass per tetrahedron
    double out_scale;          // 1 for mass, nc0*nc1*nc2/box^3 for density
    void* out;
    double* mass_sum;          // may be null
    unsigned long long* stats; // may be null
    int grid_limit;            // workgroups launched
};

// Zero-fills the output (unless accumulating) and launches the per-cell clip
// kernel (cell_method) or the cumulative kernel.
hipError_t launch_deposit_uniform(const UniformArgs& P, bool fp64, bool accumulate,
                                  bool cell_method, hipStream_t stream);
hipError_t launch_deposit_cumulative(const UniformArgs& P, bool out_fp64, hipStream_t stream);

}  // namespace psd
