// psd_api.hip -- the C ABI (include/psd.h): argument checks, workspace sizes,
// launches.  No allocation, no state kept between calls.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "psd.h"
#include "psd_internal.h"

namespace psd {
hipError_t launch_batched(const psd_box* boxes, int n, double* mass_sums, bool density,
                          bool accumulate, const Tuning& tune, void* ws, size_t ws_bytes,
                          unsigned long long* stats, hipStream_t stream);
size_t batched_ws_bytes(const psd_box* boxes, int n, bool ordered);
hipError_t autotune_batched(const psd_box* boxes, int n, uint32_t flags, void* ws, size_t ws_bytes,
                            hipStream_t stream, const char* cache_path, Tuning& best, double& best_ms);
// psd_surrogate.hip: `steps` backward + Adam steps in one cooperative launch.
hipError_t launch_surrogate_train(float* w, const float* feat, const double* frac, const uint8_t* mask,
                                  const int64_t* order, int64_t n, int64_t batch, int64_t steps,
                                  int64_t step0, const float* lr, float beta1, float beta2, float eps,
                                  float* m, float* v, float* grad, double* losses, hipStream_t stream);
}  // namespace psd

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

psd::Tuning tuning_from(const psd_options* opt)
{
    psd::Tuning t = psd::default_tuning();
    if (opt && opt->tuning) {
        const psd_tuning* u = opt->tuning;
        if (u->lds_cap > 0) t.cap = u->lds_cap;
        if (u->waves_per_cu > 0) t.waves_per_cu = u->waves_per_cu;
        t.ordered = u->ordered ? 1 : 0;
    }
    if (opt && (opt->flags & PSD_WORK_COUNTERS) && opt->stats) t.work_counters = 1;
    if (opt && (opt->flags & PSD_METHOD_SLAB)) t.slab = 1;
    return t;
}

// The per-cell method numbers the cells of a bbox with 32-bit indices; a
// bbox spans at most nc_k + 1 cells per axis.
bool cell_method_fits(const int32_t nc[3])
{
    return ((double)nc[0] + 1.0) * ((double)nc[1] + 1.0) * ((double)nc[2] + 1.0) <= 2147483647.0;
}

bool tuning_ok(const psd_options* opt)
{
    if (!opt || !opt->tuning) return true;
    const psd_tuning* u = opt->tuning;
    return (u->lds_cap == 0 || u->lds_cap == 512 || u->lds_cap == 960 || u->lds_cap == 1024 ||
            u->lds_cap == 1408 ||
            u->lds_cap == 2048) &&
           u->waves_per_cu >= 0 && u->waves_per_cu <= 64 && u->reserved == 0;
}

size_t uniform_ws_bytes(const psd_particles* p, const psd_options* opt)
{
    const int64_t ntet = 6 * (int64_t)p->np[0] * p->np[1] * p->np[2];
    const bool ordered = tuning_from(opt).ordered != 0;
    size_t b = psd::queue_workspace_bytes((ntet + 63) / 64, 1, ordered);
    // with the surrogate: one 64-bit word per 64-tet chunk marking the tets
    // the exact path still deposits
    if (opt && (opt->flags & PSD_SURROGATE)) b = psd::surrogate_mask_offset(b) + psd::surrogate_mask_bytes(ntet);
    return b;
}

// Leaves of at most 1024^3 cells: the kernels index cells within a leaf in
// 32 bits.
bool octree_params_ok(const psd_octree_params* op)
{
    return op && op->block_cells >= 1 && op->block_cells <= 1024 && op->max_level >= 0 &&
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
constexpr uint32_t kUniformFlags = PSD_OUT_DENSITY | PSD_ACCUMULATE | PSD_PREC_FP64 |
                                   PSD_METHOD_CELL | PSD_SURROGATE | PSD_CHECK_FINITE |
                                   PSD_WORK_COUNTERS | PSD_METHOD_SLAB;

// The slab form writes FP32 grids and has no surrogate or counting variant.
bool slab_flags_ok(uint32_t flags)
{
    return !(flags & PSD_METHOD_SLAB) ||
           !(flags & (PSD_PREC_FP64 | PSD_METHOD_CELL | PSD_SURROGATE | PSD_WORK_COUNTERS));
}

// PSD_ERR_NONFINITE when one of the n particles' coordinates is NaN or
// infinite; the device word `scratch` (inside the caller's workspace) holds
// the count.  Synchronizes the stream.
psd_status check_positions(const float* pos, int64_t n_particles, void* scratch,
                           hipStream_t stream, const char* where)
{
    unsigned long long bad = 0;
    const hipError_t e = psd::count_nonfinite(pos, 3 * n_particles,
                                              reinterpret_cast<unsigned long long*>(scratch),
                                              stream, bad);
    if (e != hipSuccess) return fail_hip(e, where);
    if (bad) {
        char msg[128];
        snprintf(msg, sizeof(msg), "%s: %llu position coordinates are NaN or infinite", where, bad);
        return fail(PSD_ERR_NONFINITE, msg);
    }
    return PSD_OK;
}

int64_t particle_count(const psd_particles* p)
{
    return (int64_t)p->np[0] * p->np[1] * p->np[2];
}

}  // namespace

namespace psd {
psd_status set_error(psd_status s, const char* detail) { return fail(s, detail); }
}  // namespace psd

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
    if (opt && !slab_flags_ok(opt->flags))
        return fail(PSD_ERR_UNSUPPORTED, "PSD_METHOD_SLAB writes FP32 grids, without the surrogate, "
                                         "PSD_METHOD_CELL or PSD_WORK_COUNTERS");
    if (opt && (opt->flags & PSD_METHOD_CELL) && !cell_method_fits(nc))
        return fail(PSD_ERR_UNSUPPORTED, "PSD_METHOD_CELL needs (nc0+1)(nc1+1)(nc2+1) < 2^31");
    if (!tuning_ok(opt)) return fail(PSD_ERR_ARG, "bad tuning");
    *bytes = uniform_ws_bytes(p, opt);
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
    if (!slab_flags_ok(flags))
        return fail(PSD_ERR_UNSUPPORTED, "PSD_METHOD_SLAB writes FP32 grids, without the surrogate, "
                                         "PSD_METHOD_CELL or PSD_WORK_COUNTERS");
    if ((flags & PSD_METHOD_CELL) && !cell_method_fits(nc))
        return fail(PSD_ERR_UNSUPPORTED, "PSD_METHOD_CELL needs (nc0+1)(nc1+1)(nc2+1) < 2^31");
    if (!tuning_ok(opt)) return fail(PSD_ERR_ARG, "bad tuning");
    if (!ws || ws_bytes < uniform_ws_bytes(p, opt)) return fail(PSD_ERR_WORKSPACE, "workspace too small");
    if (flags & PSD_SURROGATE) {
        if (flags & PSD_METHOD_CELL)
            return fail(PSD_ERR_UNSUPPORTED, "PSD_SURROGATE needs the default (cumulative) method");
        if (!opt->surrogate) return fail(PSD_ERR_ARG, "PSD_SURROGATE without parameters");
    }
    if (flags & PSD_CHECK_FINITE) {
        // the queue's work counter (offset 0) is free until the deposit starts
        const psd_status s = check_positions(pos, particle_count(p), ws,
                                             reinterpret_cast<hipStream_t>(stream), "deposit_uniform");
        if (s != PSD_OK) return s;
    }

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
    A.surrogate = (flags & PSD_SURROGATE) ? opt->surrogate : nullptr;
    hipError_t e = psd::launch_deposit_uniform(A, (flags & PSD_PREC_FP64) != 0,
                                               (flags & PSD_ACCUMULATE) != 0,
                                               (flags & PSD_METHOD_CELL) != 0, tuning_from(opt), ws,
                                               ws_bytes, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "deposit_uniform launch");
    return PSD_OK;
}

static bool boxes_ok(const psd_box* boxes, int32_t n)
{
    if (!boxes || n < 1 || n > (1 << 20)) return false;
    for (int32_t b = 0; b < n; ++b)
        if (!boxes[b].pos || !boxes[b].out || !particles_ok(&boxes[b].p) || !grid_ok(boxes[b].nc))
            return false;
    return true;
}

static const uint32_t kBatchedFlags =
    PSD_OUT_DENSITY | PSD_ACCUMULATE | PSD_CHECK_FINITE | PSD_WORK_COUNTERS;

psd_status psd_batched_workspace_size(const psd_box* boxes, int32_t n_boxes,
                                      const psd_options* opt, size_t* bytes)
{
    if (!bytes) return fail(PSD_ERR_ARG, "bytes is null");
    if (!boxes_ok(boxes, n_boxes)) return fail(PSD_ERR_ARG, "bad box descriptors");
    if (opt && (opt->flags & ~kBatchedFlags)) return fail(PSD_ERR_UNSUPPORTED, "unsupported flags");
    if (!tuning_ok(opt)) return fail(PSD_ERR_ARG, "bad tuning");
    *bytes = psd::batched_ws_bytes(boxes, n_boxes, tuning_from(opt).ordered != 0);
    return PSD_OK;
}

psd_status psd_deposit_batched(const psd_box* boxes, int32_t n_boxes, double* mass_sums,
                               const psd_options* opt, void* ws, size_t ws_bytes, void* stream)
{
    if (!boxes_ok(boxes, n_boxes)) return fail(PSD_ERR_ARG, "bad box descriptors");
    const uint32_t flags = opt ? opt->flags : 0u;
    if (flags & ~kBatchedFlags) return fail(PSD_ERR_UNSUPPORTED, "unsupported flags");
    if (!tuning_ok(opt)) return fail(PSD_ERR_ARG, "bad tuning");
    const psd::Tuning t = tuning_from(opt);
    if (!ws || ws_bytes < psd::batched_ws_bytes(boxes, n_boxes, t.ordered != 0))
        return fail(PSD_ERR_WORKSPACE, "workspace too small");
    if (flags & PSD_CHECK_FINITE)
        for (int32_t b = 0; b < n_boxes; ++b) {
            const psd_status s = check_positions(boxes[b].pos, particle_count(&boxes[b].p), ws,
                                                 reinterpret_cast<hipStream_t>(stream),
                                                 "deposit_batched");
            if (s != PSD_OK) return s;
        }
    hipError_t e = psd::launch_batched(boxes, n_boxes, mass_sums, (flags & PSD_OUT_DENSITY) != 0,
                                       (flags & PSD_ACCUMULATE) != 0, t, ws, ws_bytes,
                                       opt ? reinterpret_cast<unsigned long long*>(opt->stats) : nullptr,
                                       reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "deposit_batched launch");
    return PSD_OK;
}

psd_status psd_autotune_batched(const psd_box* boxes, int32_t n_boxes, const psd_options* opt,
                                void* ws, size_t ws_bytes, void* stream, const char* cache_path,
                                psd_tuning* best, double* best_ms)
{
    if (!best) return fail(PSD_ERR_ARG, "best is null");
    if (!boxes_ok(boxes, n_boxes)) return fail(PSD_ERR_ARG, "bad box descriptors");
    const uint32_t flags = opt ? opt->flags : 0u;
    if (flags & ~kBatchedFlags) return fail(PSD_ERR_UNSUPPORTED, "unsupported flags");
    if (!ws || ws_bytes < psd::batched_ws_bytes(boxes, n_boxes, true))
        return fail(PSD_ERR_WORKSPACE, "workspace too small (size it for ordered chunks)");
    psd::Tuning t = psd::default_tuning();
    double ms = 0.0;
    hipError_t e = psd::autotune_batched(boxes, n_boxes, flags & PSD_OUT_DENSITY, ws, ws_bytes,
                                         reinterpret_cast<hipStream_t>(stream), cache_path, t, ms);
    if (e != hipSuccess) return fail_hip(e, "autotune_batched");
    best->lds_cap = t.cap;
    best->waves_per_cu = t.waves_per_cu;
    best->ordered = t.ordered;
    best->reserved = 0;
    if (best_ms) *best_ms = ms;
    return PSD_OK;
}

psd_status psd_octree_workspace_size(const psd_particles* p, const psd_octree_params* op,
                                     size_t* bytes)
{
    if (!bytes) return fail(PSD_ERR_ARG, "bytes is null");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!octree_params_ok(op)) return fail(PSD_ERR_ARG, "bad octree parameters");
    const psd::OctreeArgs A = octree_args(nullptr, p, op);
    *bytes = psd::octree_workspace_layout(A).bytes + psd::octree_queue_bytes(A);
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
    {
        // a NaN would turn the subblock boxes, and so the counts, into garbage
        const psd_status s = check_positions(
            pos, particle_count(p), static_cast<char*>(ws) + psd::octree_workspace_layout(A).counts,
            reinterpret_cast<hipStream_t>(stream), "build_octree");
        if (s != PSD_OK) return s;
    }
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
    if (flags & ~(uint32_t)(PSD_OUT_DENSITY | PSD_ACCUMULATE | PSD_CHECK_FINITE | PSD_WORK_COUNTERS))
        return fail(PSD_ERR_UNSUPPORTED, "octree deposit supports PSD_OUT_DENSITY, PSD_ACCUMULATE, "
                                         "PSD_CHECK_FINITE and PSD_WORK_COUNTERS");
    if (!tuning_ok(opt)) return fail(PSD_ERR_ARG, "bad tuning");
    const psd::OctreeArgs A = octree_args(pos, p, op);
    if (!ws || ws_bytes < psd::octree_workspace_layout(A).bytes + psd::octree_queue_bytes(A))
        return fail(PSD_ERR_WORKSPACE, "workspace too small");
    if (flags & PSD_CHECK_FINITE) {
        const psd_status s = check_positions(
            pos, particle_count(p), static_cast<char*>(ws) + psd::octree_workspace_layout(A).counts,
            reinterpret_cast<hipStream_t>(stream), "deposit_octree");
        if (s != PSD_OK) return s;
    }
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
                                              n_nodes, n_leaves * B * B * B, ws, ws_bytes,
                                              (flags & PSD_ACCUMULATE) != 0, tuning_from(opt),
                                              reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "deposit_octree launch");
    return PSD_OK;
}

psd_status psd_octree_coarsen(const psd_octree_node* nodes, int64_t n_nodes, int64_t n_leaves,
                              int32_t block, int32_t max_level, const float* leaves, float* out,
                              uint32_t flags, void* stream)
{
    if (!nodes || !leaves || !out) return fail(PSD_ERR_ARG, "null pointer");
    if (block < 1 || block > 1024 || max_level < 0 || max_level > 7)
        return fail(PSD_ERR_ARG, "bad block or max_level");
    if (n_nodes < 1 || n_leaves < 1 || n_leaves > n_nodes || n_nodes > psd::octree_max_nodes(max_level))
        return fail(PSD_ERR_ARG, "bad node or leaf count");
    if (flags & ~(uint32_t)PSD_OUT_DENSITY) return fail(PSD_ERR_UNSUPPORTED, "flags: PSD_OUT_DENSITY only");
    if (n_nodes > 1 && (block & 1))
        return fail(PSD_ERR_UNSUPPORTED, "coarse levels need an even block (2x2x2 cells per coarse cell)");
    const int64_t cells = (int64_t)block * block * block;
    const char* lb = reinterpret_cast<const char*>(leaves);
    const char* ob = reinterpret_cast<const char*>(out);
    if (lb < ob + n_nodes * cells * 4 && ob < lb + n_leaves * cells * 4)
        return fail(PSD_ERR_ARG, "out overlaps leaves");
    hipError_t e = psd::launch_octree_coarsen(reinterpret_cast<const psd::OctNode*>(nodes), n_nodes,
                                              n_leaves, block, max_level, (flags & PSD_OUT_DENSITY) != 0,
                                              leaves, out, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "octree_coarsen");
    return PSD_OK;
}

psd_status psd_reorder_workspace_size(const int32_t np[3], size_t* bytes)
{
    if (!np || !bytes) return fail(PSD_ERR_ARG, "null pointer");
    for (int a = 0; a < 3; ++a)
        if (np[a] < 1) return fail(PSD_ERR_ARG, "bad Lagrangian grid size");
    if ((double)np[0] * np[1] * np[2] > 4.0e12) return fail(PSD_ERR_ARG, "Lagrangian grid too large");
    *bytes = psd::reorder_workspace_bytes((int64_t)np[0] * np[1] * np[2]);
    return PSD_OK;
}

psd_status psd_reorder_by_id(const int64_t* ids, const float* pos_in, int64_t n, int64_t id_base,
                             const int32_t np[3], float* pos_out, int64_t* check, void* ws,
                             size_t ws_bytes, void* stream)
{
    if (!np || !pos_out) return fail(PSD_ERR_ARG, "null pointer");
    if (n < 0 || n > ((int64_t)1 << 42)) return fail(PSD_ERR_ARG, "bad record count");
    if (n > 0 && (!ids || !pos_in)) return fail(PSD_ERR_ARG, "null pointer");
    for (int a = 0; a < 3; ++a)
        if (np[a] < 1) return fail(PSD_ERR_ARG, "bad Lagrangian grid size");
    if ((double)np[0] * np[1] * np[2] > 4.0e12) return fail(PSD_ERR_ARG, "Lagrangian grid too large");
    const int64_t slots = (int64_t)np[0] * np[1] * np[2];
    if (n > 0) {
        const char* ib = reinterpret_cast<const char*>(pos_in);
        const char* ob = reinterpret_cast<const char*>(pos_out);
        if (ib < ob + slots * 12 && ob < ib + n * 12) return fail(PSD_ERR_ARG, "pos_out overlaps pos_in");
    }
    if (check && (!ws || ws_bytes < psd::reorder_workspace_bytes(slots)))
        return fail(PSD_ERR_WORKSPACE, "workspace too small for the check");
    hipError_t e = psd::launch_reorder_by_id(ids, pos_in, n, id_base, slots, pos_out, check, ws,
                                             reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "reorder_by_id");
    return PSD_OK;
}

}  // extern "C"

extern "C" {

psd_status psd_surrogate_examples_workspace_size(int64_t n_cubes, size_t* bytes)
{
    if (!bytes) return fail(PSD_ERR_ARG, "bytes is null");
    if (n_cubes < 0 || n_cubes > (int64_t)1 << 40) return fail(PSD_ERR_ARG, "bad cube count");
    *bytes = psd::example_workspace_bytes(6 * n_cubes);
    return PSD_OK;
}

psd_status psd_surrogate_examples(const float* pos, const psd_particles* p, const int32_t nc[3],
                                  int64_t first_cube, int64_t n_cubes, int32_t min_cells,
                                  float* feat, double* frac, uint8_t* mask, int64_t* tet_id,
                                  int64_t capacity, int64_t* n_out, void* ws, size_t ws_bytes,
                                  void* stream)
{
    if (!pos || !n_out) return fail(PSD_ERR_ARG, "pos or n_out is null");
    if (!particles_ok(p)) return fail(PSD_ERR_ARG, "bad particle description");
    if (!grid_ok(nc)) return fail(PSD_ERR_ARG, "bad grid size");
    const int64_t ncube = (int64_t)p->np[0] * p->np[1] * p->np[2];
    if (first_cube < 0 || n_cubes < 0 || first_cube + n_cubes > ncube)
        return fail(PSD_ERR_ARG, "cube range outside the Lagrangian grid");
    if (min_cells < 1 || min_cells > 8) return fail(PSD_ERR_ARG, "min_cells must be 1..8");
    if (capacity < 0 || (capacity > 0 && (!feat || !frac || !mask)))
        return fail(PSD_ERR_ARG, "bad capacity or null output");
    if (!ws || ws_bytes < psd::example_workspace_bytes(6 * n_cubes))
        return fail(PSD_ERR_WORKSPACE, "workspace too small");
    psd::UniformArgs A;
    memset(&A, 0, sizeof(A));
    A.pos = pos;
    for (int a = 0; a < 3; ++a) {
        A.np[a] = p->np[a];
        A.nc[a] = nc[a];
        A.scale[a] = (double)nc[a] / p->box;
    }
    hipError_t e = psd::launch_examples(A, first_cube, n_cubes, min_cells, feat, frac, mask, tet_id,
                                        capacity, ws, n_out, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "surrogate_examples");
    return PSD_OK;
}

psd_status psd_exact_fractions(const float* tets, double* frac, int64_t n, void* stream)
{
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(PSD_ERR_ARG, "bad tetrahedron count");
    if (n > 0 && (!tets || !frac)) return fail(PSD_ERR_ARG, "null pointer");
    hipError_t e = psd::launch_exact_fractions(tets, frac, n, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "exact_fractions");
    return PSD_OK;
}

psd_status psd_surrogate_forward(const float* params, const float* feat, const uint8_t* mask,
                                 int64_t n, float* probs, void* stream)
{
    if (n < 0) return fail(PSD_ERR_ARG, "negative sample count");
    if (!params || (n > 0 && (!feat || !mask || !probs))) return fail(PSD_ERR_ARG, "null pointer");
    hipError_t e = psd::launch_surrogate_forward(params, feat, mask, n, probs,
                                                 reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "surrogate_forward");
    return PSD_OK;
}

psd_status psd_surrogate_backward(const float* params, const float* feat, const double* frac,
                                  const uint8_t* mask, const int64_t* idx, int64_t n, float* grad,
                                  double* loss, void* stream)
{
    if (n < 0) return fail(PSD_ERR_ARG, "negative sample count");
    if (!params || !grad || (n > 0 && (!feat || !frac || !mask)))
        return fail(PSD_ERR_ARG, "null pointer");
    hipError_t e = psd::launch_surrogate_backward(params, feat, frac, mask, idx, n, grad, loss,
                                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "surrogate_backward");
    return PSD_OK;
}

psd_status psd_surrogate_adam(float* params, const float* grad, float* m, float* v, int64_t step,
                              float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!params || !grad || !m || !v) return fail(PSD_ERR_ARG, "null pointer");
    if (step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(PSD_ERR_ARG, "bad Adam hyper-parameters");
    hipError_t e = psd::launch_surrogate_adam(params, grad, m, v, step, lr, beta1, beta2, eps,
                                              reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "surrogate_adam");
    return PSD_OK;
}

psd_status psd_surrogate_train_steps(float* params, const float* feat, const double* frac,
                                     const uint8_t* mask, const int64_t* order, int64_t n,
                                     int64_t batch, int64_t steps, int64_t step0, const float* lr,
                                     float beta1, float beta2, float eps, float* m, float* v,
                                     float* grad, double* losses, void* stream)
{
    if (batch < 1 || steps < 0 || n < 0 || step0 < 0) return fail(PSD_ERR_ARG, "bad batch, step or sample count");
    if (steps > 0 && (steps - 1) >= (n + batch - 1) / batch)
        return fail(PSD_ERR_ARG, "more steps than batches in the sample order");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(PSD_ERR_ARG, "bad Adam hyper-parameters");
    if (steps == 0) return PSD_OK;
    if (!params || !feat || !frac || !mask || !order || !lr || !m || !v || !grad)
        return fail(PSD_ERR_ARG, "null pointer");
    hipError_t e = psd::launch_surrogate_train(params, feat, frac, mask, order, n, batch, steps, step0, lr,
                                               beta1, beta2, eps, m, v, grad, losses,
                                               reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "surrogate_train_steps");
    return PSD_OK;
}

}  // extern "C"
