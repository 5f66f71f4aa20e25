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
 *     A tetrahedron with a NaN or infinite vertex coordinate cannot be
 *     placed: the deposits drop it (stats[7] counts it, mass_sum misses its
 *     mass) unless PSD_CHECK_FINITE asks for the positions to be checked
 *     first, in which case the call fails with PSD_ERR_NONFINITE.
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
    PSD_ERR_NONFINITE = -4,   /* a position is NaN or infinite (only reported
                                 when checked: PSD_CHECK_FINITE, and always
                                 by psd_build_octree)                         */
    PSD_ERR_UNSUPPORTED = -5, /* flag combination not supported               */
    PSD_ERR_HIP = -6          /* a HIP runtime call failed (see detail string) */
} psd_status;

enum {
    PSD_OUT_DENSITY = 1u << 0, /* write mass / h^3 instead of cell mass        */
    PSD_ACCUMULATE = 1u << 1,  /* add into `out` instead of overwriting it     */
    PSD_PREC_FP64 = 1u << 2,   /* FP64 output grid (`out` is double); with
                                  PSD_METHOD_CELL also FP64 clipping          */
    PSD_METHOD_CELL = 1u << 3, /* per-cell exact clip in cell-local FP32
                                  coordinates (Section 6.1 loop cell by cell);
                                  default: cumulative FP64 volumes            */
    PSD_SURROGATE = 1u << 4,   /* tetrahedra whose bbox holds 2..8 cells
                                  inside a 2x2x2 block are deposited with the
                                  learned overlap network (psd_options.
                                  surrogate, see the end of this header)
                                  instead of the exact clip; default method
                                  only                                         */
    PSD_CHECK_FINITE = 1u << 5, /* before any work, scan every position on the
                                  device and return PSD_ERR_NONFINITE (with
                                  nothing else enqueued and the outputs
                                  untouched) if one is NaN or infinite.  The
                                  call then synchronizes `stream`.            */
    PSD_WORK_COUNTERS = 1u << 6, /* with stats: stats holds 16 entries and the
                                  default (cumulative) method runs an
                                  instrumented kernel that also adds its work
                                  events into [8] pieces of the first split,
                                  [9] pieces of the second split (z
                                  distributions set up), [10] z levels walked
                                  by those pieces, [11] (column, level) slots
                                  of the walked tiles; [12..15] reserved.  For
                                  measurement: the plain kernel is faster.    */
    PSD_METHOD_SLAB = 1u << 7   /* cached slab clipping in FP32 (Section 6.3's
                                  splitting, each split computed once where
                                  its pieces serve many cells): per bbox row
                                  x in [a, a+1) the pieces of T cut by
                                  x >= a and x <= a+1 (FP64 planes, kept in
                                  FP32 relative to the tile), per column the
                                  row's pieces cut by y >= b and y <= b+1 in
                                  FP32, and the leaves' exact z distribution
                                  summed into the column's cells.  Cell
                                  volumes are formed directly (no differences
                                  of cumulative values), so FP32 keeps its
                                  relative precision in every cell.  FP32
                                  grids only; not with PSD_PREC_FP64,
                                  PSD_METHOD_CELL, PSD_SURROGATE or
                                  PSD_WORK_COUNTERS.                          */
};

typedef struct {
    int32_t np[3];     /* Lagrangian grid size (particles per axis), each >= 1 */
    double box;        /* periodic box side, > 0                              */
    double total_mass; /* mass of all particles                               */
} psd_particles;

/* Launch shape of the cumulative deposit (all zero = defaults). */
typedef struct {
    int32_t lds_cap;      /* FP64 entries of the per-wavefront LDS buffer:
                             512 (16-tet groups), 960 (32 tets set up at
                             once, 16 tiles a batch), 1024 (8-tet groups, the
                             pieces of all columns walked 64 at a time from a
                             ring), 1408 (8-tet groups, each column's pieces
                             on its own lane) or 2048 (32-tet groups); 0 =
                             1024 when every box has >= 1.5 grid cells per
                             Lagrangian spacing (large tets), else 960;
                             octree leaves always 960                         */
    int32_t waves_per_cu; /* persistent wavefronts per compute unit (0 = as
                             many as fit: 12 at 960, 1024 or 1408 entries on
                             gfx950)                                          */
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
                          [5] zero-volume tets, [6] tets deposited by the
                          surrogate (their bbox pairs are not in [1]),
                          [7] tets dropped because a vertex coordinate is
                          NaN or infinite (their mass is deposited nowhere
                          and is missing from mass_sum); may be NULL.
                          An octree deposit walks the tetrahedra once per
                          level that has leaves and counts [0], [4], [7]
                          on each such walk.                               */
    const psd_tuning* tuning; /* host, may be NULL                           */
    const float* surrogate;   /* DEVICE float[PSD_SURROGATE_PARAMS], the
                                 network for PSD_SURROGATE; else ignored     */
} psd_options;

/* Workspace bytes (host out) needed by psd_deposit_uniform for this problem
 * and these options (PSD_SURROGATE adds 8 bytes per 64 tetrahedra; the
 * cost-ordered tuning adds its chunk order). */
psd_status psd_uniform_workspace_size(const psd_particles* p, const int32_t nc[3],
                                      const psd_options* opt, size_t* bytes);

/*
 * Cell masses (or densities) of the whole tessellation on a periodic uniform
 * grid (Section 6.1 deposit loop; Section 6.3 exact intersection).
 * Default method: for each column (a,b) of a tetrahedron's bounding box, the
 * volumes of T cap {x<=a+1, y<=b+1} per z-cell (two-plane splitting plus the
 * exact distribution along z), cell volumes by 2-D differences, all FP64.
 * PSD_METHOD_CELL: classify each bbox cell and clip the non-trivial ones
 * exactly, cell-local FP32 (FP64 for distances to the tetrahedron's planes);
 * it numbers a bbox's cells with 32-bit indices, so it returns
 * PSD_ERR_UNSUPPORTED when (nc0+1)(nc1+1)(nc2+1) >= 2^31.
 *   pos       DEVICE float [np0][np1][np2][3]
 *   p, nc     host; nc[k] >= 1
 *   out       DEVICE float [nc0][nc1][nc2] (double with PSD_PREC_FP64);
 *             zeroed first unless PSD_ACCUMULATE
 *   mass_sum  DEVICE double[1] or NULL: set (or, with PSD_ACCUMULATE, added)
 *             to the FP64 sum of every mass deposited by this call
 *   opt       host, may be NULL (flags 0)
 *   ws        DEVICE workspace of ws_bytes >= psd_uniform_workspace_size
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_HIP, PSD_ERR_NONFINITE
 * (PSD_CHECK_FINITE only).  Asynchronous unless PSD_CHECK_FINITE is set.
 */
psd_status psd_deposit_uniform(const float* pos, const psd_particles* p, const int32_t nc[3],
                               void* out, double* mass_sum, const psd_options* opt, void* ws,
                               size_t ws_bytes, void* stream);

/*
 * psd_deposit_uniform without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, flags, results and
 * errors as psd_deposit_uniform; the workspace is a fixed device array of
 * PSD_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends.  The call allocates nothing.
 *   Limit: problems whose psd_uniform_workspace_size exceeds
 *   PSD_NOALLOC_SCRATCH_BYTES fail with PSD_ERR_WORKSPACE (index order needs
 *   256 bytes at any size; PSD_SURROGATE adds 8 bytes per 64 tetrahedra, so
 *   up to about 134M tetrahedra; cost ordering adds 12 bytes per 64).
 *   Every call on one GPU shares that GPU's array: calls that overlap in
 *   time on one GPU (several streams or host threads) race and give wrong
 *   results; serialise them.  The array keeps the last call's contents; the
 *   call clears what must start at zero.
 * Runs on the current device; `stream` must belong to it.
 */
enum { PSD_NOALLOC_SCRATCH_BYTES = 16 << 20 };
psd_status psd_deposit_uniform_noalloc(const float* pos, const psd_particles* p,
                                       const int32_t nc[3], void* out, double* mass_sum,
                                       const psd_options* opt, void* stream);

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
 *   flags      PSD_OUT_DENSITY, PSD_ACCUMULATE, PSD_CHECK_FINITE (every box)
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_UNSUPPORTED, PSD_ERR_HIP,
 * PSD_ERR_NONFINITE.  Asynchronous unless PSD_CHECK_FINITE is set.
 */
psd_status psd_deposit_batched(const psd_box* boxes, int32_t n_boxes, double* mass_sums,
                               const psd_options* opt, void* ws, size_t ws_bytes, void* stream);

/*
 * Chooses the launch shape (psd_tuning) of psd_deposit_batched for this batch
 * by timing candidates with HIP events on `stream`: LDS buffer of 960, 1024
 * or 2048 FP64 entries, all the wavefronts that fit a compute unit or half
 * of them, chunks in index or cost order.  The boxes' outputs are overwritten with a valid deposit.  If
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
                            and 64; 16 here), 1..1024 (cells within a leaf
                            are indexed in 32 bits)                           */
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
 * too small, PSD_ERR_NONFINITE (nodes untouched) when a position is NaN or
 * infinite (the positions are always checked).  Synchronizes `stream`.
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
 *   flags     PSD_OUT_DENSITY, PSD_ACCUMULATE, PSD_CHECK_FINITE
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_UNSUPPORTED, PSD_ERR_HIP,
 * PSD_ERR_NONFINITE.  Asynchronous unless PSD_CHECK_FINITE is set.
 */
psd_status psd_deposit_octree(const float* pos, const psd_particles* p, const psd_octree_params* op,
                              const psd_octree_node* nodes, int64_t n_nodes, int64_t n_leaves,
                              float* out, double* mass_sum, const psd_options* opt, void* ws,
                              size_t ws_bytes, void* stream);

/*
 * Coarse representations of the internal nodes (Section 8, future work: the
 * leaves' deposit plus coarser levels for multi-resolution rendering).  For
 * every node, the B^3 cells of its region at its own resolution, box / (B
 * 2^level): a leaf's block is copied from `leaves`; an internal node's cell
 * is the sum (PSD_OUT_DENSITY: the average) of the 2x2x2 cells of its
 * children that it covers -- exact, since |T cap C| is additive over a
 * partition of C -- accumulated in FP64 in the fixed order dx, dy, dz (x
 * outermost) and rounded once to FP32 per level.  Levels are filled
 * bottom-up, so node values do not depend on the launch.
 *   nodes     DEVICE node array from psd_build_octree (n_nodes entries)
 *   leaves    DEVICE float [n_leaves][B][B][B] from psd_deposit_octree
 *             (masses, or densities with PSD_OUT_DENSITY)
 *   out       DEVICE float [n_nodes][B][B][B], node order; must not overlap
 *             `leaves`
 *   block     B, the tree's cells per leaf side; even unless the tree is a
 *             single leaf
 *   max_level the tree's max_level
 *   flags     0 (masses) or PSD_OUT_DENSITY
 * Nodes that are malformed (a child range outside the array, two children in
 * one octant, a leaf id >= n_leaves) are skipped and their blocks left as
 * they were.  Errors: PSD_ERR_ARG, PSD_ERR_UNSUPPORTED (odd block with
 * internal nodes), PSD_ERR_HIP.  Asynchronous.
 */
psd_status psd_octree_coarsen(const psd_octree_node* nodes, int64_t n_nodes, int64_t n_leaves,
                              int32_t block, int32_t max_level, const float* leaves, float* out,
                              uint32_t flags, void* stream);

/* ------------------------------------------------------------------------ */
/* Snapshot ingest (Section 3)                                                */
/* ------------------------------------------------------------------------ */

/* Workspace bytes (host out) of psd_reorder_by_id with a check: one bit per
 * Lagrangian slot, rounded up to 32-bit words. */
psd_status psd_reorder_workspace_size(const int32_t np[3], size_t* bytes);

/*
 * Places snapshot records on the Lagrangian grid.  A snapshot holds tracers
 * in an arbitrary order, each with a unique ID that gives its Lagrangian
 * position (Section 3; once sorted by ID the IDs are dropped).  Record r goes
 * to slot ids[r] - id_base, slot (i * np1 + j) * np2 + k holding particle
 * (i, j, k): pos_out[slot][0..2] = pos_in[r][0..2], bit for bit.
 *   ids       DEVICE int64 [n]
 *   pos_in    DEVICE float [n][3]
 *   n         records, >= 0 (need not equal the slot count)
 *   np        host, the Lagrangian grid size (each >= 1)
 *   pos_out   DEVICE float [np0][np1][np2][3]; must not overlap pos_in; slots
 *             that no record names keep their contents; when several records
 *             name one slot and `check` is given, one of them (unspecified)
 *             is stored whole; without `check` the slot then holds an
 *             unspecified mix of their coordinates (three separate stores)
 *   check     DEVICE int64[3] or NULL: set to [0] records whose id is outside
 *             [id_base, id_base + np0 np1 np2) (skipped), [1] records naming a
 *             slot another record already named, [2] slots no record names.
 *             A valid snapshot (a permutation) gives 0, 0, 0.
 *   ws        DEVICE workspace of psd_reorder_workspace_size bytes when check
 *             is not NULL (may be NULL otherwise)
 * Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_HIP.  Asynchronous.
 */
psd_status psd_reorder_by_id(const int64_t* ids, const float* pos_in, int64_t n, int64_t id_base,
                             const int32_t np[3], float* pos_out, int64_t* check, void* ws,
                             size_t ws_bytes, void* stream);

/* Human-readable name of a status code (static string). */
const char* psd_status_string(psd_status s);

/* Detail of the last error raised on the calling host thread (thread-local). */
const char* psd_last_error_detail(void);

/* ------------------------------------------------------------------------ */
/* Learned overlap surrogate (an addition to the paper)                       */
/* ------------------------------------------------------------------------ */
/*
 * For a tetrahedron whose bounding box spans at most 2 cells per axis (lo =
 * floor of the vertex minima, hi = floor of the maxima, hi - lo <= 1 on every
 * axis) a network predicts the fractions |T cap C| / |T| of the cell average
 * of Eq. (1) for the cells C = lo + (dx,dy,dz), indexed c = 4dx + 2dy + dz:
 *   x[12] = float(v_q,a - lo_a), q = 0..3 in split order, a = 0..2
 *   h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), h3 = silu(W3 h2 + b3)
 *   z = W4 h3 + b4, p = softmax of z over the cells inside [lo, hi], else 0
 * Parameters: one float32 vector of PSD_SURROGATE_PARAMS values, in order
 * W1[64][12], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[8][64],
 * b4[8] (matrices row-major [out][in]).  The matrices are used rounded to
 * bfloat16 (nearest even) on the matrix cores with float32 accumulation;
 * each feature enters as two bfloat16 parts (high, residual); biases,
 * activations' SiLU and the softmax are float32, activations are rounded to
 * bfloat16 between layers.  In a deposit the probabilities are renormalised
 * in FP64 and the last cell takes the residual, so each tetrahedron deposits
 * exactly m.  Tetrahedra inside one cell and zero-volume ones stay exact.
 */
enum { PSD_SURROGATE_PARAMS = 9672 };

/* Workspace bytes (host out) of psd_surrogate_examples over n_cubes cubes. */
psd_status psd_surrogate_examples_workspace_size(int64_t n_cubes, size_t* bytes);

/*
 * Training or test examples: the eligible tetrahedra of Lagrangian cubes
 * first_cube .. first_cube + n_cubes - 1 (cube id (i*np1 + j)*np2 + k,
 * tetrahedron id 6*cube + p) with a non-zero volume and at least min_cells
 * (1..8) cells in their bbox, in tetrahedron order, labelled with exact FP64
 * overlap fractions (splitting of Section 6.3).
 *   feat    DEVICE float  [capacity][12]  features as above
 *   frac    DEVICE double [capacity][8]   |T cap C| / |T|; 0 outside [lo, hi]
 *   mask    DEVICE uint8  [capacity]      bit c set iff cell c is inside [lo, hi]
 *   tet_id  DEVICE int64  [capacity] or NULL
 *   n_out   host: number of eligible tetrahedra; may exceed capacity, in which
 *           case only the first `capacity` are written
 * Synchronizes the stream.  Errors: PSD_ERR_ARG, PSD_ERR_WORKSPACE, PSD_ERR_HIP.
 */
psd_status psd_surrogate_examples(const float* pos, const psd_particles* p, const int32_t nc[3],
                                  int64_t first_cube, int64_t n_cubes, int32_t min_cells,
                                  float* feat, double* frac, uint8_t* mask, int64_t* tet_id,
                                  int64_t capacity, int64_t* n_out, void* ws, size_t ws_bytes,
                                  void* stream);

/*
 * Exact labels for given tetrahedra (Section 6.3 splitting, FP64): for each
 * tetrahedron i, tets[i][4][3] (DEVICE float) are its vertices relative to
 * the low corner of a 2x2x2 block of cells, in cell units, every coordinate
 * in [0, 2); frac[i][c] (DEVICE double [n][8], overwritten) = |T cap C_c|/|T|
 * for cell c = 4 dx + 2 dy + dz of the block.  A zero-volume tetrahedron
 * (|det| <= 1e-12 (longest edge)^3, the rule of the deposits) gives 1 in its
 * centroid's cell.  A tetrahedron with a vertex outside [0, 2)^3 or not
 * finite gives NaN in all 8 entries (no error is returned: the data stay on
 * the device).  Asynchronous.  Errors: PSD_ERR_ARG (n < 0, null pointers),
 * PSD_ERR_HIP.
 */
psd_status psd_exact_fractions(const float* tets, double* frac, int64_t n, void* stream);

/* probs[n][8] (DEVICE float) = p of the network `params` for feat[n][12] and
 * mask[n].  Asynchronous. */
psd_status psd_surrogate_forward(const float* params, const float* feat, const uint8_t* mask,
                                 int64_t n, float* probs, void* stream);

/*
 * grad (DEVICE float[PSD_SURROGATE_PARAMS], overwritten) = gradient of the
 * mean over the batch of -sum_c y_c log p_c, y = frac of the sample, with
 * respect to the parameters (taken at the bfloat16-rounded matrices);
 * loss (DEVICE double[1] or NULL, overwritten) = that mean.  The batch is
 * samples idx[0..n-1] (DEVICE int64) of the example arrays, or 0..n-1 when
 * idx is NULL.  Asynchronous.
 */
psd_status psd_surrogate_backward(const float* params, const float* feat, const double* frac,
                                  const uint8_t* mask, const int64_t* idx, int64_t n, float* grad,
                                  double* loss, void* stream);

/* One Adam update (bias-corrected moments, Kingma & Ba) of params with the
 * moment vectors m and v (DEVICE float[PSD_SURROGATE_PARAMS]); step >= 1 is
 * the update's 1-based count.  Asynchronous. */
psd_status psd_surrogate_adam(float* params, const float* grad, float* m, float* v, int64_t step,
                              float lr, float beta1, float beta2, float eps, void* stream);

/*
 * `steps` training steps in one launch (cooperative: its workgroups, one per
 * 64-sample tile of a batch up to 256, are resident together and meet at
 * grid-wide barriers).  Step s (0-based) takes the samples
 * order[s*batch .. min((s+1)*batch, n) - 1] (DEVICE int64, n entries), forms
 * their mean-loss gradient at the current params as psd_surrogate_backward
 * does, then applies one Adam update as psd_surrogate_adam does, with step
 * count step0 + s + 1 and learning rate lr[s] (DEVICE float[steps]).
 * losses (DEVICE double[steps], or NULL) receives each step's mean loss;
 * grad (DEVICE float[PSD_SURROGATE_PARAMS]) is scratch and ends zeroed.
 * The result equals the per-step calls up to the order of the FP32 gradient
 * sums across workgroups.  PSD_ERR_ARG: batch < 1, steps or n or step0
 * negative, a step past the end of order, bad Adam hyper-parameters, a null
 * pointer; PSD_ERR_HIP: the launch failed (e.g. the grid cannot be
 * resident at once).  Asynchronous.
 */
psd_status psd_surrogate_train_steps(float* params, const float* feat, const double* frac,
                                     const uint8_t* mask, const int64_t* order, int64_t n,
                                     int64_t batch, int64_t steps, int64_t step0, const float* lr,
                                     float beta1, float beta2, float eps, float* m, float* v,
                                     float* grad, double* losses, void* stream);

#ifdef __cplusplus
}
#endif
#endif
