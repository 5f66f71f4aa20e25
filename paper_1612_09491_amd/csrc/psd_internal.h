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
    // Learned overlap surrogate (packed float32 parameters), or null: when
    // set, tetrahedra with a bbox of 2..8 cells inside a 2x2x2 block go to
    // the network instead of the exact clip.
    const float* surrogate;
};

// Zero-fills the output (unless accumulating) and launches the per-cell clip
// kernel (cell_method) or the cumulative queue kernel.
struct Tuning;
hipError_t launch_deposit_uniform(const UniformArgs& P, bool fp64, bool accumulate,
                                  bool cell_method, const Tuning& tune, void* ws, size_t ws_bytes,
                                  hipStream_t stream);
// ---------------------------------------------------------------------------
// Cumulative deposit over a table of independent boxes (one for a plain grid,
// one per level for an octree, many for a batch), driven by a work queue of
// 64-tetrahedron chunks.
// ---------------------------------------------------------------------------

struct BoxDesc {
    const float* pos;
    int np[3];
    int nc[3];
    double scale[3];           // nc_k / box
    double m;                  // mass per tetrahedron
    double out_scale;          // 1 for mass, cells per unit volume for density
    void* out;                 // float (or double) grid, or leaf blocks
    double* mass_sum;          // may be null
    int64_t ntet;
    int64_t chunk_begin;       // first global chunk of this box
    const int* leaf_map;       // octree level: node -> leaf id (null: plain grid)
    const int* level_has_leaf; // octree level: nothing to do when 0
    int leaf_block;
    int leaf_side;
    int skip_small;            // leave bboxes of 2..8 cells within 2x2x2 to the surrogate
    // per 64-tet chunk, the tets left to this deposit (bit = lane), or null
    const unsigned long long* exact_mask;
};

struct Tuning {
    int cap;            // FP64 entries of the per-wave LDS buffer: 512, 960, 1408 or 2048
                        // (0: chosen from the boxes' cells per Lagrangian spacing)
    int waves_per_cu;   // persistent workgroups per compute unit (0: as many as fit)
    int ordered;        // 1: chunks in decreasing estimated cost
    int work_counters;  // 1: the instrumented kernel, adding work events into stats[8..11]
    int slab;           // 1: the slab form (FP32 cell volumes from cached slab pieces)
};

struct QueueArgs {
    const BoxDesc* boxes;      // device table (null: use box0)
    BoxDesc box0;              // the single box when boxes is null
    int n_boxes;
    int64_t n_chunks;
    const int64_t* order;      // device, global chunk ids in processing order, or null
    unsigned long long* next;  // device work counter, zeroed before the launch
    unsigned long long* stats; // may be null
};

// Workspace bytes of a queued launch over n_chunks chunks and n_boxes boxes.
size_t queue_workspace_bytes(int64_t n_chunks, int n_boxes, bool ordered);
int64_t queue_chunks(const BoxDesc* boxes, int n_boxes);
BoxDesc box_from_uniform(const UniformArgs& P);
// Lays out the workspace, uploads the box table (if n_boxes > 1), orders the
// chunks by estimated cost when asked, and launches the deposit.  `boxes` is
// a host array.
hipError_t launch_queue(const BoxDesc* boxes, int n_boxes, bool out_fp64, const Tuning& tune,
                        void* ws, size_t ws_bytes, unsigned long long* stats, hipStream_t stream);
Tuning default_tuning();
// Wavefronts of the deposit kernel with this buffer that fit one compute unit.
hipError_t queue_resident_waves(int cap, bool out_fp64, int& waves, bool work = false,
                                bool slab = false);

// Number of NaN or infinite values among p[0..n) (a device array), counted
// on `stream` into the device word dcount and returned in host_count;
// synchronizes the stream.
hipError_t count_nonfinite(const float* p, int64_t n, unsigned long long* dcount,
                           hipStream_t stream, unsigned long long& host_count);

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
// Deposits into the leaves of `nodes`; asynchronous.  The workspace holds the
// octree layout followed by a queue workspace of octree_queue_bytes.
size_t octree_queue_bytes(const OctreeArgs& A);
hipError_t launch_deposit_octree(const OctreeArgs& A, const UniformArgs& base, const OctNode* nodes,
                                 int64_t n_nodes, int64_t n_leaf_cells, void* ws, size_t ws_bytes,
                                 bool accumulate, const Tuning& tune, hipStream_t stream);

// Coarse levels: every node's B^3 block, leaves copied, internal nodes as
// 2x2x2 sums (averages for densities) of their children, bottom-up.
hipError_t launch_octree_coarsen(const OctNode* nodes, int64_t n_nodes, int64_t n_leaves, int B,
                                 int max_level, bool density, const float* leaves, float* out,
                                 hipStream_t stream);

// ---------------------------------------------------------------------------
// Snapshot ingest
// ---------------------------------------------------------------------------

size_t reorder_workspace_bytes(int64_t n_slots);
hipError_t launch_reorder_by_id(const int64_t* ids, const float* pos_in, int64_t n, int64_t id_base,
                                int64_t n_slots, float* pos_out, int64_t* check, void* ws,
                                hipStream_t stream);

// ---------------------------------------------------------------------------
// Learned overlap surrogate
// ---------------------------------------------------------------------------

int surrogate_param_count();
size_t example_workspace_bytes(int64_t ntet);
// Eligible tetrahedra of cubes [first_cube, first_cube + n_cubes) with features,
// cell masks and exact fractions, in tetrahedron order; synchronizes `stream`
// and sets *n_out to the number found (entries beyond capacity are dropped).
hipError_t launch_examples(const UniformArgs& P, int64_t first_cube, int64_t n_cubes, int min_cells,
                           float* feat, double* frac, uint8_t* mask, int64_t* tet_id,
                           int64_t capacity, void* ws, int64_t* n_out, hipStream_t stream);
hipError_t launch_exact_fractions(const float* tets, double* frac, int64_t n, hipStream_t stream);
hipError_t launch_surrogate_forward(const float* w, const float* feat, const uint8_t* mask, int64_t n,
                                    float* probs, hipStream_t stream);
hipError_t launch_surrogate_backward(const float* w, const float* feat, const double* frac,
                                     const uint8_t* mask, const int64_t* idx, int64_t n, float* grad,
                                     double* loss, hipStream_t stream);
hipError_t launch_surrogate_adam(float* w, const float* grad, float* m, float* v, int64_t step,
                                 float lr, float beta1, float beta2, float eps, hipStream_t stream);
// Deposits the tetrahedra the exact path leaves to the surrogate (P.surrogate
// set) and, when exact_mask is not null, marks per 64-tet chunk the ones the
// exact path still has to deposit.
hipError_t launch_surrogate_deposit(const UniformArgs& P, bool fp64, unsigned long long* exact_mask,
                                    hipStream_t stream);
// Workspace placement of that mask after `base` bytes, and its size.
inline size_t surrogate_mask_offset(size_t base) { return (base + 255) & ~(size_t)255; }
inline size_t surrogate_mask_bytes(int64_t ntet) { return (size_t)((ntet + 63) / 64) * 8; }

}  // namespace psd
