/*
 * psd.h -- phase-space-element density deposition on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpsd.so.  Plain C types only; a HIP stream is passed as void*
 * (a hipStream_t, NULL = the default stream).
 *
 * The method (Kaehler, "Massively Parallel Computation of Accurate Densities
 * for N-body Dark Matter Simulations using the Phase-Space-Element Method"):
 * tracers sit on a Lagrangian grid of fixed connectivity and equal mass
 * (Section 2); each hexahedral cell of that grid is split into 6 tetrahedra
 * (Section 2; here the Freudenthal split along the 000-111 diagonal); the
 * density is Eq. (1), rho(x) = m sum_i 1/V_i(x), and its average over a
 * cubical cell C is M_C / h^3 with M_C = sum_T m |T cap C| / |T|, where
 * |T cap C| is the exact intersection volume (Section 6.3).
 *
 * Conventions shared by every call:
 *   - Positions: float32 [np0][np1][np2][3], C order (x index slowest), in a
 *     periodic cube of side `box`; any finite value is accepted and wrapped.
 *     Each cube's corners are unwrapped to the minimum image of corner 000.
 *   - Mass per tetrahedron m = total_mass / (6 np0 np1 np2).
 *   - Grids: [nc0][nc1][nc2], C order, cell (a,b,c) covers
 *     [a,a+1) x [b,b+1) x [c,c+1) in units of h_k = box / nc_k.
 *   - All data pointers are DEVICE pointers unless marked (host).  The
 *     caller allocates every buffer, including the workspace; calls never
 *     allocate device memory, keep no state between calls and never free
 *     caller memory.
 *   - Calls enqueue work on `stream` and return without synchronising,
 *     except where stated.  On error nothing is enqueued and outputs are
 *     unspecified.  No C++ exception crosses this boundary.
 */
#ifndef PSD_H
#define PSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSD_OK = 0,
    PSD_ERR_ARG = -1,         /* null pointer, non-positive size, bad value   */
    PSD_ERR_WORKSPACE = -2,   /* workspace smaller than psd_*_workspace_size  */
    PSD_ERR_CAPACITY = -3,    /* octree node array too small (see below)      */
    PSD_ERR_NONFINITE = -4,   /* reserved                                      */
    PSD_ERR_UNSUPPORTED = -5, /* flag combination not supported               */
    PSD_ERR_HIP = -6          /* a HIP runtime call failed (see detail string) */
} psd_status;

enum {
    PSD_OUT_DENSITY = 1u << 0, /* write mass / h^3 instead of cell mass        */
    PSD_ACCUMULATE = 1u << 1,  /* add into `out` instead of overwriting it     */
    PSD_PREC_FP64 = 1u << 2,   /* FP64 output grid (`out` is double); with
                                  PSD_METHOD_CELL also FP64 clipping          */
    PSD_METHOD_CELL = 1u << 3  /* per-cell exact clip in cell-local FP32
                                  coordinates (Section 6.1 loop cell by cell);
                                  default: cumulative FP64 volumes            */
};

typedef struct {
    int32_t np[3];     /* Lagrangian grid size (particles per axis), each >= 1 */
    double box;        /* periodic box side, > 0                              */
    double total_mass; /* mass of all particles                               */
} psd_particles;

/* Launch shape of the cumulative deposit (all zero = defaults). */
typedef struct {
    int32_t lds_cap;      /* FP64 entries of the per-wavefront LDS buffer:
                             512, 1024 or 2048 (0 = 1024)                     */
    int32_t waves_per_cu; /* persistent wavefronts per compute unit (0 = 8)   */
    int32_t ordered;      /* 1: process 64-tet chunks in decreasing estimated
                             cost (bbox cells); 0: in index order             */
    int32_t reserved;     /* must be 0                                        */
} psd_tuning;

typedef struct {
    uint32_t flags;    /* PSD_* flags above                                   */
    int64_t* stats;    /* optional DEVICE int64[8] counters, added into:
                          [0] tets, [1] (tet, bbox cell) pairs, [2] exact
                          clips (per-cell method) or bbox columns (cumulative),
                          [3] non-zero deposits, [4] inverted tets,
                          [5] zero-volume tets, [6..7] reserved; may be NULL */
    const psd_tuning* tuning; /* host, may be NULL                           */
} psd_options;

/* Workspace bytes (host out) needed by psd_deposit_uniform for this problem. */
psd_status psd_uniform_workspace_size(const psd_particles* p, const int32_t nc[3],
                                      const psd_options* opt, size_t* bytes);

/*
 * Cell masses (or densities) of the whole tessellation on a periodic uniform
 * grid (Section 6.1 deposit loop; Section 6.3 exact intersection).
 * Default method: for each column (a,b) of a tetrahedron's bounding box, the
 * volumes of T cap {x<=a+1, y<=b+1} per z-cell (two-plane splitting plus the
 * exact distribution along z), cell volumes by 2-D differences, all FP64.
 * PSD_METHOD_CELL: classify each bbox cell and clip the non-trivial ones
 * exactly, cell-local FP32 (FP64 for distances to the tetrahedron's planes).
 *   pos       DEVICE float [np0][np1][np2][3]
 *   p, nc     host; nc[k] >= 1
 *   out       DEVICE float [nc0][nc1][nc2] (double with PSD_PREC_FP64);
 *             zeroed first unless PSD_ACCUMULATE
 *   mass_sum  DEVICE double[1] or NULL: set (or, with PSD_ACCUMULATE, added)
 *             to the FP64 sum of every mass deposited by this call
 *   opt       host, may be NULL (flags 0)
 *   ws        DEVICE workspace of ws_bytes >= psd_uniform_workspace_size
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_HIP.  Asynchronous.
 */
psd_status psd_deposit_uniform(const float* pos, const psd_particles* p, const int32_t nc[3],
                               void* out, double* mass_sum, const psd_options* opt, void* ws,
                               size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Many independent boxes in one launch                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float* pos;  /* DEVICE float [np0][np1][np2][3] of this box          */
    psd_particles p;   /* its Lagrangian grid, box side and total mass         */
    int32_t nc[3];     /* its periodic deposit grid                           */
    float* out;        /* DEVICE float [nc0][nc1][nc2]                        */
} psd_box;

/* Workspace bytes (host out) for psd_deposit_batched with these options. */
psd_status psd_batched_workspace_size(const psd_box* boxes, int32_t n_boxes,
                                      const psd_options* opt, size_t* bytes);

/*
 * Deposits every box of a batch (each box exactly as psd_deposit_uniform
 * with the default method would) in one persistent launch.  Workgroups pop
 * 64-tetrahedron chunks of all boxes from one device counter; with
 * tuning->ordered the chunks are first binned by their bbox cell count and
 * processed from the most to the least expensive, which balances boxes of
 * very different size (the kernel-level load balancing of Section 5).
 *   boxes      host array of n_boxes descriptors (n_boxes >= 1)
 *   mass_sums  DEVICE double[n_boxes] or NULL: per-box FP64 mass sums
 *   flags      PSD_OUT_DENSITY, PSD_ACCUMULATE
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_UNSUPPORTED, PSD_ERR_HIP.
 * Asynchronous.
 */
psd_status psd_deposit_batched(const psd_box* boxes, int32_t n_boxes, double* mass_sums,
                               const psd_options* opt, void* ws, size_t ws_bytes, void* stream);

/*
 * Chooses the launch shape (psd_tuning) of psd_deposit_batched for this batch
 * by timing candidates with HIP events on `stream`: LDS buffer of 1024 or
 * 2048 FP64 entries, 4 or 8 wavefronts per compute unit, chunks in index or
 * cost order.  The boxes' outputs are overwritten with a valid deposit.  If
 * cache_path (host string, may be NULL) names a JSON file, a result for the
 * same device and batch signature is read from it instead of measuring, and
 * new results are added to it.  The workspace must be sized for ordered
 * chunks (psd_batched_workspace_size with tuning->ordered = 1).
 * Synchronizes `stream`.
 */
psd_status psd_autotune_batched(const psd_box* boxes, int32_t n_boxes, const psd_options* opt,
                                void* ws, size_t ws_bytes, void* stream, const char* cache_path,
                                psd_tuning* best, double* best_ms);

/* ------------------------------------------------------------------------ */
/* Adaptive octree (Section 4)                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t block_cells; /* B: cells per leaf side (the paper's tests use 128
                            and 64; 16 here), >= 1                            */
    int32_t max_level;   /* refinements below the root, 0..7                 */
    int32_t subblock;    /* Lagrangian cubes per subblock side (paper: 8)    */
    int32_t reserved;    /* must be 0                                        */
    int64_t threshold;   /* a node is refined iff its count > threshold      */
} psd_octree_params;

typedef struct {
    int32_t level;       /* 0 = root (the whole periodic box)                */
    int32_t ix, iy, iz;  /* position among the 2^level nodes per axis        */
    int32_t first_child; /* index of the first of 8 contiguous children, or -1 */
    int32_t leaf_id;     /* leaf number (node order) or -1                   */
    int64_t count;       /* overlap estimate of tetrahedra in the node       */
} psd_octree_node;

/* Workspace bytes (host out) for psd_build_octree and psd_deposit_octree. */
psd_status psd_octree_workspace_size(const psd_particles* p, const psd_octree_params* op,
                                     size_t* bytes);

/*
 * Octree refined where many tetrahedra overlap (Section 4): starting from
 * the root box, a node is split into 8 children while its count exceeds
 * `threshold` and its level is below `max_level`.  The count is the paper's
 * memory-efficient estimate from Lagrangian subblocks of subblock^3 cubes,
 * made integer-exact: sum over subblocks of floor(ntets * |bbox cap node| /
 * |bbox|), bounding boxes (min/max of the subblock's unwrapped cube corners)
 * snapped outward to the finest lattice G = B * 2^max_level, overlaps over
 * periodic images.  The result is bit-reproducible.
 *   nodes     DEVICE psd_octree_node[capacity]: canonical order -- by level,
 *             Morton order (x most significant) within a level, the 8
 *             children of a node contiguous -- leaves numbered in node order
 *   n_nodes, n_leaves  host out
 * Returns PSD_ERR_CAPACITY (with *n_nodes, *n_leaves set) when capacity is
 * too small.  Synchronizes `stream`.
 */
psd_status psd_build_octree(const float* pos, const psd_particles* p, const psd_octree_params* op,
                            psd_octree_node* nodes, int64_t capacity, int64_t* n_nodes,
                            int64_t* n_leaves, void* ws, size_t ws_bytes, void* stream);

/*
 * Cell masses (densities with PSD_OUT_DENSITY) of the octree's leaves: a leaf
 * at level l covers box/2^l per axis with B^3 cells of side box/(B 2^l);
 * tetrahedra crossing leaves deposit into each (Section 4 leaf patches,
 * Section 6 deposit).  Same exact volumes as psd_deposit_uniform at the
 * leaf's resolution.
 *   nodes     DEVICE array from psd_build_octree (n_nodes entries)
 *   out       DEVICE float [n_leaves][B][B][B], zeroed first unless
 *             PSD_ACCUMULATE
 *   mass_sum  DEVICE double[1] or NULL (FP64 sum of deposited mass)
 *   flags     PSD_OUT_DENSITY, PSD_ACCUMULATE
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_UNSUPPORTED, PSD_ERR_HIP.
 * Asynchronous.
 */
psd_status psd_deposit_octree(const float* pos, const psd_particles* p, const psd_octree_params* op,
                              const psd_octree_node* nodes, int64_t n_nodes, int64_t n_leaves,
                              float* out, double* mass_sum, const psd_options* opt, void* ws,
                              size_t ws_bytes, void* stream);

/* Human-readable name of a status code (static string). */
const char* psd_status_string(psd_status s);

/* Detail of the last error raised on the calling host thread (thread-local). */
const char* psd_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif
