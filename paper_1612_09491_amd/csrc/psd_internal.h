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
    // Octree leaves (null for a plain grid): cell (x,y,z) of this resolution
    // belongs to node (x/B, y/B, z/B) of a side^3 level; leaf_map gives its
    // leaf id or -1, and the mass goes to out[leaf][x%B][y%B][z%B].
    const int* leaf_map;
    const int* level_has_leaf; // skip the launch's work when *level_has_leaf == 0
    int leaf_block;            // B
    int leaf_side;             // 2^level
};

// Zero-fills the output (unless accumulating) and launches the per-cell clip
// kernel (cell_method) or the cumulative kernel.
hipError_t launch_deposit_uniform(const UniformArgs& P, bool fp64, bool accumulate,
                                  bool cell_method, hipStream_t stream);
hipError_t launch_deposit_cumulative(const UniformArgs& P, bool out_fp64, hipStream_t stream);

// ---------------------------------------------------------------------------
// Octree (Section 4)
// ---------------------------------------------------------------------------

struct OctNode {  // same layout as psd_octree_node
    int32_t level, ix, iy, iz;
    int32_t first_child;  // -1 for a leaf
    int32_t leaf_id;      // -1 for an interior node
    int64_t count;
};

struct SubblockBox {  // finest-lattice integer box [lo, hi)
    int64_t lo[3], hi[3];
    int64_t ntets;
};

struct OctreeArgs {
    const float* pos;
    int np[3];
    double box;
    int block;        // cells per leaf side (B)
    int max_level;    // refinements below the root
    int subblock;     // Lagrangian cubes per subblock side
    int ns[3];        // subblocks per axis
    int64_t G;        // finest lattice: B * 2^max_level
    double gscale;    // G / box
    int64_t threshold;
};

struct OctreeWorkspace {
    size_t boxes, dense, work, counts, leafmap, levelflag, bytes;
};

int64_t octree_max_nodes(int max_level);
OctreeWorkspace octree_workspace_layout(const OctreeArgs& A);
// Builds the tree; synchronizes `stream`; counts_host[0..1] = nodes, leaves.
hipError_t launch_build_octree(const OctreeArgs& A, void* ws, OctNode* nodes, int64_t capacity,
                               int64_t* counts_host, hipStream_t stream);
// Deposits into the leaves of `nodes`; asynchronous.
hipError_t launch_deposit_octree(const OctreeArgs& A, const UniformArgs& base, const OctNode* nodes,
                                 int64_t n_nodes, int64_t n_leaf_cells, void* ws, bool accumulate,
                                 hipStream_t stream);

}  // namespace psd
