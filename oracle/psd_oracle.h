/*
 * psd_oracle.h -- FP64 CPU oracle for phase-space-element density deposition.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; the two meet only in the
 * seeded input generator.
 *
 * What it computes (Kaehler, "Massively Parallel Computation of Accurate
 * Densities for N-body Dark Matter Simulations using the Phase-Space-Element
 * Method"):
 *   - Section 2, Eq. (1): the density of the tessellation is m * sum_i 1/V_i
 *     over the tetrahedra covering a point.  Averaged over a cubical cell C
 *     this is  M_C = sum_T m |T cap C| / |T|  (cell mass), rho_C = M_C / h^3.
 *   - Section 2: each hexahedral Lagrangian cell is split into 6 tetrahedra
 *     of equal mass; the split used here is the Freudenthal/Kuhn one along the
 *     000-111 diagonal (the paper does not say which 6).
 *   - Section 6.3: |T cap C| is an exact intersection volume.  The oracle gets
 *     it from a general convex-polytope clipper (face polygons, divergence
 *     theorem), unrelated to the tetrahedron-splitting the paper describes.
 *   - Section 6.1: trivial cells (no overlap, C inside T, T inside C) may be
 *     short-cut; ORC_TRIVIAL turns the short-cuts on.
 *   - Section 4: octree refinement from subblock bounding-box overlap
 *     estimates, made integer-exact (see orc_build_octree).
 * Counting mode ORC_PAPER re-computes non-trivial volumes with the paper's own
 * iterative splitting (Section 6.3: x and y planes recursively with a 16-case
 * inside-mask table, the last axis by subtracting the outside parts) and
 * counts its work; it is used for the algorithmic operation counts.
 *
 * All coordinates are in cell units unless stated; positions are float32 in
 * [0, box) and are converted exactly to double.
 */
#ifndef PSD_ORACLE_H
#define PSD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n_tet;         /* tetrahedra processed                                */
    int64_t n_pair;        /* (tet, bbox cell) pairs                              */
    int64_t n_nontrivial;  /* pairs that needed an exact clip                     */
    int64_t n_nonzero;     /* pairs with a positive deposit                       */
    int64_t n_inverted;    /* tets whose orientation differs from the lattice's   */
    int64_t n_degenerate;  /* tets handled by the zero-volume rule                */
    int64_t n_ambiguous;   /* cubes with an unwrapped offset beyond a quarter box */
    int64_t n_pv;          /* ORC_PAPER: (sub-tet, plane) visits                  */
    int64_t n_cut;         /* ORC_PAPER: edge-plane intersections                 */
    int64_t n_sub;         /* ORC_PAPER: sub-tetrahedra generated                 */
} orc_counters;

enum {
    ORC_TRIVIAL = 1,  /* classify cells first; clip only the non-trivial ones      */
    ORC_PAPER = 2     /* non-trivial volumes by the paper's splitting, with counts */
};

/* Volume of T cap [lo,hi] for a tetrahedron v[4][3] (any orientation). */
double orc_clip_tet_box(const double* v, const double* lo, const double* hi);

/* Same volume by the paper's splitting scheme; counts[3] += (visits, cuts, subtets). */
double orc_clip_tet_box_paper(const double* v, const double* lo, const double* hi,
                              int64_t* counts);

/* The 6 tetrahedra of Lagrangian cube (i,j,k), unwrapped, in cell units of an
 * nc[3] grid over a periodic box: tets[6][4][3].  Returns the signed
 * determinants D[6] (|T| = |D|/6) through det (may be NULL). */
void orc_cube_tets(const float* pos, const int* np, double box, const int* nc,
                   int64_t i, int64_t j, int64_t k, double* tets, double* det);

/* Cell masses on a periodic uniform grid nc[3].
 *   region_lo/region_n: the cell block to fill (no wrap inside the block);
 *     NULL means the whole grid.  out is [region_n0][region_n1][region_n2].
 *   cubes/n_cubes: Lagrangian cube indices (i*np1+j)*np2+k to deposit; NULL
 *     means all cubes.
 *   mode: ORC_TRIVIAL | ORC_PAPER.  nthreads <= 0: OpenMP default.
 * out is overwritten.  Returns 0, or -1 on bad arguments. */
int orc_deposit_uniform(const float* pos, const int* np, double box, double total_mass,
                        const int* nc, const int* region_lo, const int* region_n,
                        const int64_t* cubes, int64_t n_cubes, int mode, int nthreads,
                        double* out, orc_counters* cnt);

typedef struct {
    int32_t level, ix, iy, iz;
    int32_t first_child;   /* -1 for a leaf      */
    int32_t leaf_id;       /* -1 for an interior */
    int64_t count;
} orc_node;

/* Octree over the periodic box (Section 4).  Root = the whole box (level 0).
 * A node at level l spans box/2^l per axis; its count is
 *   sum_sb floor( ntets(sb) * Vol(bbox(sb) cap node) / Vol(bbox(sb)) )
 * over subblocks sb of subblock^3 Lagrangian cubes, with bounding boxes
 * snapped outward to the finest integer lattice G = block * 2^max_level and
 * overlaps taken over periodic images.  A node is refined iff
 * count > threshold and level < max_level.  Node order: by level, Morton
 * order (x most significant) within a level; leaves numbered in node order.
 * Returns 0, -1 on bad arguments, -3 if capacity is too small (*n_nodes then
 * holds the required count). */
int orc_build_octree(const float* pos, const int* np, double box, int block, int max_level,
                     int subblock, int64_t threshold, orc_node* nodes, int64_t capacity,
                     int64_t* n_nodes, int64_t* n_leaves);

/* Cell masses of selected leaves: out[n_sel][block][block][block]. */
int orc_deposit_octree(const float* pos, const int* np, double box, double total_mass, int block,
                       const orc_node* nodes, int64_t n_nodes, const int64_t* leaf_sel,
                       int64_t n_sel, int mode, int nthreads, double* out, orc_counters* cnt);

/* Training and test examples for the learned overlap surrogate (an addition
 * to the paper: a network that predicts the overlap fractions |T cap C|/|T|
 * of the cell average of Eq. (1) for small tetrahedra).  For the 6*count
 * tetrahedra of Lagrangian cubes first .. first+count-1 (cube index
 * (i*np1+j)*np2+k, then split permutation 0..5), written at slot
 * 6*(cube-first)+p:
 *   flag[t]        1 if |D| > 1e-12 l^3 and hi-lo <= 1 on every axis, with
 *                  lo = floor(min v), hi = floor(max v) in cell units;
 *   feat[t][4][3]  float(v - lo), vertex order of the split;
 *   mask[t]        bit 4dx+2dy+dz set iff cell lo+(dx,dy,dz) lies in [lo,hi];
 *   frac[t][8]     |T cap C| / |T| for the masked-in cells, 0 elsewhere;
 *   lo[t][3]       the bbox origin wrapped into [0, nc) (may be NULL).
 * Unflagged slots are zero.  Returns 0, or -1 on bad arguments. */
int orc_surrogate_examples(const float* pos, const int* np, double box, const int* nc,
                           int64_t first, int64_t count, int nthreads, uint8_t* flag,
                           float* feat, uint8_t* mask, double* frac, int32_t* lo);

#ifdef __cplusplus
}
#endif
#endif
