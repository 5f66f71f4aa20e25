// psd_api.hip -- the C ABI (include/psd.h): argument checks, workspace sizes,
// launches.  No allocation, no state kept between calls.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "psd.h"
#include "psd_internal.h"

namespace {

thread_local char g_detail[256] = "";

psd_status fail(psd_status s, const char* msg)
{
    snprintf(g_detail, sizeof(g_detail), "%s", msg);
    return s;
}

psd_status fail_hip(hipError_t e, const char* where)
{
    snprintf(g_detail, sizeof(g_detail), "%s: %s", where, hipGetErrorString(e));
    return PSD_ERR_HIP;
}

bool particles_ok(const psd_particles* p)
{
    if (!p) return false;
    for (int a = 0; a < 3; ++a)
        if (p->np[a] < 1) return false;
    if (!(p->box > 0.0) || !isfinite(p->box) || !isfinite(p->total_mass)) return false;
    // tetrahedron ids are 64-bit; cube ids must fit the grid arithmetic
    if ((double)p->np[0] * p->np[1] * p->np[2] > 4.0e12) return false;
    return true;
}

bool grid_ok(const int32_t nc[3])
{
    if (!nc) return false;
    for (int a = 0; a < 3; ++a)
        if (nc[a] < 1 || nc[a] > (1 << 20)) return false;
    return (double)nc[0] * nc[1] * nc[2] < 9.0e15;
}

constexpr size_t kUniformWorkspace = 256;

bool octree_params_ok(const psd_octree_params* op)
{
    return op && op->block_cells >= 1 && op->block_cells <= 4096 && op->max_level >= 0 &&
           op->max_level <= 7 && op->subblock >= 1 && op->reserved == 0 && op->threshold >= 0 &&
           ((int64_t)op->block_cells << op->max_level) <= (1 << 20);
}

psd::OctreeArgs octree_args(const float* pos, const psd_particles* p, const psd_octree_params* op)
{
    psd::OctreeArgs A;
    memset(&A, 0, sizeof(A));
    A.pos = pos;
    for (int a = 0; a < 3; ++a) {
        A.np[a] = p->np[a];
        A.ns[a] = (p->np[a] + op->subblock - 1) / op->subblock;
    }
    A.box = p->box;
    A.block = op->block_cells;
    A.max_level = op->max_level;
    A.subblock = op->subblock;
    A.G = (int64_t)op->block_cells << op->max_level;
    A.gscale = (double)A.G / p->box;
    A.threshold = op->threshold;
    return A;
}
constexpr uint32_t kUniformFlags = PSD_OUT_DENSITY | PSD_ACCUMULATE | PSD_PREC_FP64 | PSD_METHOD_CELL;

}  // namespace

extern "C" {

const char* psd_status_string(psd_status s)
{
    switch (s) {
    case PSD_OK: return "PSD_OK";
    case PSD_ERR_ARG: return "PSD_ERR_ARG";
    case PSD_ERR_WORKSPACE: return "PSD_ERR_WORKSPACE";
    case PSD_ERR_CAPACITY: return "PSD_ERR_CAPACITY";
    case PSD_ERR_NONFINITE: return "PSD_ERR_NONFINITE";
    case PSD_ERR_UNSUPPORTED: return "PSD_ERR_UNSUPPORTED";
    case PSD_ERR_HIP: return "PSD_ERR_HIP";
    }
    return "PSD_ERR_UNKNOWN";
}

const char* psd_last_error_detail(void) { return g_detail; }

psd_status psd_uniform_workspace_size(const psd_particles* p, const int32_t nc[3],
                                      const psd_options* opt, size_t* bytes)
{
    if (!bytes) return fail(PSD_ERR_ARG, "bytes is null");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!grid_ok(nc)) return fail(PSD_ERR_ARG, "bad grid size");
    if (opt && (opt->flags & ~kUniformFlags)) return fail(PSD_ERR_UNSUPPORTED, "unknown flags");
    *bytes = kUniformWorkspace;
    return PSD_OK;
}

psd_status psd_deposit_uniform(const float* pos, const psd_particles* p, const int32_t nc[3],
                               void* out, double* mass_sum, const psd_options* opt, void* ws,
                               size_t ws_bytes, void* stream)
{
    if (!pos || !out) return fail(PSD_ERR_ARG, "pos or out is null");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!grid_ok(nc)) return fail(PSD_ERR_ARG, "bad grid size");
    const uint32_t flags = opt ? opt->flags : 0u;
    if (flags & ~kUniformFlags) return fail(PSD_ERR_UNSUPPORTED, "unknown flags");
    if (!ws || ws_bytes < kUniformWorkspace) return fail(PSD_ERR_WORKSPACE, "workspace too small");

    psd::UniformArgs A;
    memset(&A, 0, sizeof(A));
    A.pos = pos;
    for (int a = 0; a < 3; ++a) {
        A.np[a] = p->np[a];
        A.nc[a] = nc[a];
        A.scale[a] = (double)nc[a] / p->box;
    }
    A.ntet = 6 * (int64_t)p->np[0] * p->np[1] * p->np[2];
    A.m = p->total_mass / (6.0 * (double)p->np[0] * (double)p->np[1] * (double)p->np[2]);
    A.out_scale = 1.0;
    if (flags & PSD_OUT_DENSITY)
        A.out_scale = (double)nc[0] * (double)nc[1] * (double)nc[2] / (p->box * p->box * p->box);
    A.out = out;
    A.mass_sum = mass_sum;
    A.stats = opt ? reinterpret_cast<unsigned long long*>(opt->stats) : nullptr;
    A.grid_limit = 256 * 32;
    hipError_t e = psd::launch_deposit_uniform(A, (flags & PSD_PREC_FP64) != 0,
                                               (flags & PSD_ACCUMULATE) != 0,
                                               (flags & PSD_METHOD_CELL) != 0,
                                               reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "deposit_uniform launch");
    return PSD_OK;
}

psd_status psd_octree_workspace_size(const psd_particles* p, const psd_octree_params* op,
                                     size_t* bytes)
{
    if (!bytes) return fail(PSD_ERR_ARG, "bytes is null");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!octree_params_ok(op)) return fail(PSD_ERR_ARG, "bad octree parameters");
    *bytes = psd::octree_workspace_layout(octree_args(nullptr, p, op)).bytes;
    return PSD_OK;
}

psd_status psd_build_octree(const float* pos, const psd_particles* p, const psd_octree_params* op,
                            psd_octree_node* nodes, int64_t capacity, int64_t* n_nodes,
                            int64_t* n_leaves, void* ws, size_t ws_bytes, void* stream)
{
    if (!pos || !n_nodes || !n_leaves) return fail(PSD_ERR_ARG, "null pointer");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!octree_params_ok(op)) return fail(PSD_ERR_ARG, "bad octree parameters");
    if (capacity < 0 || (capacity > 0 && !nodes)) return fail(PSD_ERR_ARG, "bad node array");
    const psd::OctreeArgs A = octree_args(pos, p, op);
    if (!ws || ws_bytes < psd::octree_workspace_layout(A).bytes)
        return fail(PSD_ERR_WORKSPACE, "workspace too small");
    int64_t counts[2] = {0, 0};
    hipError_t e = psd::launch_build_octree(A, ws, reinterpret_cast<psd::OctNode*>(nodes), capacity,
                                            counts, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "build_octree");
    *n_nodes = counts[0];
    *n_leaves = counts[1];
    if (counts[0] > capacity) return fail(PSD_ERR_CAPACITY, "node array too small");
    return PSD_OK;
}

psd_status psd_deposit_octree(const float* pos, const psd_particles* p, const psd_octree_params* op,
                              const psd_octree_node* nodes, int64_t n_nodes, int64_t n_leaves,
                              float* out, double* mass_sum, const psd_options* opt, void* ws,
                              size_t ws_bytes, void* stream)
{
    if (!pos || !nodes || !out) return fail(PSD_ERR_ARG, "null pointer");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!octree_params_ok(op)) return fail(PSD_ERR_ARG, "bad octree parameters");
    if (n_nodes < 1 || n_leaves < 1 || n_leaves > n_nodes ||
        n_nodes > psd::octree_max_nodes(op->max_level))
        return fail(PSD_ERR_ARG, "bad node or leaf count");
    const uint32_t flags = opt ? opt->flags : 0u;
    if (flags & ~(uint32_t)(PSD_OUT_DENSITY | PSD_ACCUMULATE))
        return fail(PSD_ERR_UNSUPPORTED, "octree deposit supports PSD_OUT_DENSITY and PSD_ACCUMULATE");
    const psd::OctreeArgs A = octree_args(pos, p, op);
    if (!ws || ws_bytes < psd::octree_workspace_layout(A).bytes)
        return fail(PSD_ERR_WORKSPACE, "workspace too small");
    psd::UniformArgs U;
    memset(&U, 0, sizeof(U));
    U.pos = pos;
    for (int a = 0; a < 3; ++a) U.np[a] = p->np[a];
    U.ntet = 6 * (int64_t)p->np[0] * p->np[1] * p->np[2];
    U.m = p->total_mass / (6.0 * (double)p->np[0] * (double)p->np[1] * (double)p->np[2]);
    U.out_scale = (flags & PSD_OUT_DENSITY) ? 0.0 : 1.0;  // per level when density
    U.out = out;
    U.mass_sum = mass_sum;
    U.stats = opt ? reinterpret_cast<unsigned long long*>(opt->stats) : nullptr;
    U.grid_limit = 256 * 32;
    const int64_t B = op->block_cells;
    hipError_t e = psd::launch_deposit_octree(A, U, reinterpret_cast<const psd::OctNode*>(nodes),
                                              n_nodes, n_leaves * B * B * B, ws,
                                              (flags & PSD_ACCUMULATE) != 0,
                                              reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "deposit_octree launch");
    return PSD_OK;
}

}  // extern "C"
