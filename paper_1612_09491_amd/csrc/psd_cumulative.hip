// psd_cumulative.hip -- exact deposit by cumulative (inclusion-exclusion) volumes.
//
// Same result as the per-cell clip (Section 6.3 intersection volumes summed
// as in Section 6.1), organised for a SIMD machine:
//
//   D(a,b,l) = |T cap {x <= a+1} cap {y <= b+1} cap {l <= z <= l+1}| / |T|
//
// for every vertex column (a,b) of the bounding box (coordinates relative to
// its origin).  Each column needs T split by only two half-spaces -- with the
// inside-mask table of Section 6.3, at most 3 x 3 pieces -- and each piece's
// share of every z-cell follows from the exact distribution of z over a
// tetrahedron, which plays the role of the paper's subtraction along the
// last axis.  A cell's volume is then the 2-D difference
// D(i,j) - D(i-1,j) - D(i,j-1) + D(i-1,j-1).  Differences cancel, so
// everything is FP64 (full VALU rate on gfx950).
//
// Work: persistent single-wavefront workgroups pop 64-tetrahedron chunks
// from a device counter (optionally in decreasing order of estimated cost)
// over a table of independent boxes -- one periodic grid, the levels of an
// octree, or a batch of uneven boxes.  Per chunk, lanes build the
// tetrahedra into LDS a group at a time; small ones are batched so that
// their D arrays share an LDS buffer, larger ones are tiled.  (tet, column) pairs go over the lanes 64
// at a time: phase 1 fills a window's D columns, phase 2 then walks the
// cells of the same columns, takes the differences and scatters the
// non-zero cell masses with global atomics.
#include <string.h>

#include <atomic>
#include <type_traits>
#include <vector>

#include "psd_internal.h"

namespace psd {

namespace {

// A tetrahedron in its walk frame: axes 0 and 1 are split by the column
// planes, axis 2 gets the exact distribution.  Axis 2 is the longest side of
// the bbox, which makes the fewest columns for the same cells.
struct CTet {
    double vr[4][3];  // vertices relative to the bbox origin, walk-frame axes (cell units), exact,
                      // in increasing walk-frame x
    int lo[3];        // bbox origin wrapped into [0, nc), grid axes
    int ext[3];       // bbox extent in cells, walk-frame axes
    int ncell;        // ext0 * ext1 * ext2 (0: nothing to do)
    int axes;         // grid axis of walk axis k in bits 2k..2k+1
};

__device__ __forceinline__ int walk_axis(const CTet& S, int k) { return (S.axes >> (2 * k)) & 3; }

// A tile of one tetrahedron's cells: x in [a0, a0+ta), y in [b0, b0+tb),
// z in [l0, l0+tl).  Its D buffer covers columns a in [a0-ha, a0+ta),
// b in [b0-hb, b0+tb) (ha, hb = 1 when a lower neighbour column exists).
// Extents and the D offset are below the buffer size (<= 4096 entries), so
// they take 16 bits: a 28-byte record.
struct Tile {
    int a0, b0, l0;
    int16_t ta, tb, tl;
    int16_t doff;    // offset in the D buffer
    uint8_t ha, hb;
    float inv_wb;    // 1 / (tb + hb), the hardware reciprocal (fdivi's bound holds for it)
};

// q = n / d for 0 <= n < 2^21 via a float reciprocal of relative error up to
// 2^-23 (the hardware's): (n + 1/2) * inv_d is off from (n + 1/2) / d by less
// than (n + 1/2) * 1.8e-7 / d < 1/(2d), so it stays inside (q, q + 1).
__device__ __forceinline__ int fdivi(int n, float inv_d)
{
    return (int)(((float)n + 0.5f) * inv_d);
}

// Tile shape for a tetrahedron whose D array exceeds the buffer:
// (ta+1)*(tb+1)*tl <= CAP with ta, tb >= 1.
template <int CAP>
__device__ __forceinline__ void tile_shape(const CTet& S, int& ta, int& tb, int& tl, int& ntiles)
{
    tl = min(S.ext[2], CAP / 4);
    tb = min(S.ext[1], CAP / (2 * tl) - 1);
    ta = min(S.ext[0], CAP / (tl * (tb + 1)) - 1);
    ntiles = ((S.ext[0] + ta - 1) / ta) * ((S.ext[1] + tb - 1) / tb) * ((S.ext[2] + tl - 1) / tl);
}

// The slab form's tiles (no halo columns, at most `rows` tile rows):
// ta*tb*tl <= CAP.
template <int CAP>
__device__ __forceinline__ void tile_shape_slab(const CTet& S, int rows, int& ta, int& tb, int& tl,
                                                int& ntiles)
{
    tl = min(S.ext[2], CAP / 4);
    tb = min(S.ext[1], CAP / (2 * tl));
    ta = min(min(S.ext[0], rows), CAP / (tl * tb));
    ntiles = ((S.ext[0] + ta - 1) / ta) * ((S.ext[1] + tb - 1) / tb) * ((S.ext[2] + tl - 1) / tl);
}

__device__ __forceinline__ int tile_cols(const Tile& t) { return (t.ta + t.ha) * (t.tb + t.hb); }
__device__ __forceinline__ int tile_dsize(const Tile& t) { return tile_cols(t) * t.tl; }
__device__ __forceinline__ int tile_cells(const Tile& t) { return t.ta * t.tb * t.tl; }

__device__ __forceinline__ int wrap_add(int base, int off, int n)
{
    int x = base + off;
    return x >= n ? x - n : x;
}

// Output index of grid cell (x,y,z) (wrapped into [0,nc)), or -1 when the
// cell belongs to no leaf of this octree level.
__device__ __forceinline__ int64_t out_index(const BoxDesc& P, int x, int y, int z)
{
    if (!P.leaf_map) return ((int64_t)x * P.nc[1] + y) * P.nc[2] + z;
    const int B = P.leaf_block, side = P.leaf_side;
    // cells below 2^20 (the largest grid): node quotients by fdivi
    const float invB = __builtin_amdgcn_rcpf((float)B);
    const int nx = fdivi(x, invB), ny = fdivi(y, invB), nz = fdivi(z, invB);
    const int leaf = global_view(P.leaf_map)[(nx * side + ny) * side + nz];
    if (leaf < 0) return -1;
    return (int64_t)leaf * B * B * B + ((x - nx * B) * B + (y - ny * B)) * B + (z - nz * B);
}

// Does the wrapped box [lo, lo+ext) meet a leaf of this level?  Boxes wider
// than a few nodes are not tested (they are simply processed).
__device__ __forceinline__ bool touches_leaf(const BoxDesc& P, const int lo[3], const int ext[3])
{
    const int B = P.leaf_block, side = P.leaf_side;
    int n0[3], nn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        n0[c] = lo[c] / B;
        nn[c] = (lo[c] + ext[c] - 1) / B - n0[c] + 1;
        if (nn[c] > 4) return true;
    }
    for (int a = 0; a < nn[0]; ++a)
        for (int b = 0; b < nn[1]; ++b)
            for (int c = 0; c < nn[2]; ++c) {
                const int x = (n0[0] + a) % side, y = (n0[1] + b) % side, z = (n0[2] + c) % side;
                if (global_view(P.leaf_map)[(x * side + y) * side + z] >= 0) return true;
            }
    return false;
}

// Distribution of height z over one tetrahedral piece.  With the vertex
// heights sorted, s0 <= s1 <= s2 <= s3, the fraction of the piece below a
// plane z = k is a piecewise cubic:
//   s0 < k <= s1 : u^3 / ((s1-s0)(s2-s0)(s3-s0)),      u = k - s0
//   s2 <= k < s3 : 1 - w^3 / ((s3-s0)(s3-s1)(s3-s2)),  w = s3 - k
//   s1 < k < s2  : t02 t03 (1 - t13) + t02 (1 - t12) t13 + t12 t13,
//                  t0j = (k - s0)/(sj - s0), t1j = (k - s1)/(sj - s1)
// (the inside-part fractions of a plane split, Section 6.3's table, for a
// plane parallel to the cell faces; every term is a product of factors in
// [0, 1], so nothing cancels).
// R is the arithmetic type: double in the cumulative walk (its differences
// cancel), float in the slab form (cell volumes summed directly).
template <typename R>
struct ZDist {
    R s0, s1, s2, s3;
    R iA, iC;            // reciprocal products of the two end regions
    R r20, r30, r21, r31;
};

// 1/d for d > 0, else 0: the FP64 estimate refined by one Newton step, or the
// FP32 hardware reciprocal (1 ulp).
__device__ __forceinline__ double rcp_or0(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return d > 0.0 ? r : 0.0;
}
__device__ __forceinline__ float rcp_or0(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    return d > 0.0f ? r : 0.0f;
}

template <typename R>
__device__ __forceinline__ void zdist_init(const R z[4], ZDist<R>& Z)
{
    R a = fmin(z[0], z[1]), b = fmax(z[0], z[1]);
    R c = fmin(z[2], z[3]), d = fmax(z[2], z[3]);
    const R s0 = fmin(a, c), t1 = fmax(a, c);
    const R s3 = fmax(b, d), t2 = fmin(b, d);
    Z.s0 = s0;
    Z.s1 = fmin(t1, t2);
    Z.s2 = fmax(t1, t2);
    Z.s3 = s3;
    const R d10 = Z.s1 - s0, d20 = Z.s2 - s0, d30 = s3 - s0;
    const R d21 = Z.s2 - Z.s1, d31 = s3 - Z.s1, d32 = s3 - Z.s2;
    // the middle region's four reciprocals from one: all four differences
    // are positive whenever that region is not empty (else they are unused)
    const R P1 = d20 * d30, P2 = d21 * d31;
    const R Rp = rcp_or0(P1 * P2);
    Z.r20 = d30 * P2 * Rp;
    Z.r30 = d20 * P2 * Rp;
    Z.r21 = P1 * d31 * Rp;
    Z.r31 = P1 * d21 * Rp;
    Z.iA = rcp_or0(d10 * d20 * d30);
    Z.iC = rcp_or0(d30 * d31 * d32);
}

template <typename R>
__device__ __forceinline__ R zdist_below(const ZDist<R>& Z, R k)
{
    const R one = R(1);
    const R u = k - Z.s0, w = Z.s3 - k, t = k - Z.s1;
    const R lowr = u * u * u * Z.iA;
    const R highr = one - w * w * w * Z.iC;
    const R t02 = u * Z.r20, t03 = u * Z.r30;
    const R t12 = t * Z.r21, t13 = t * Z.r31;
    const R mid = t02 * t03 * (one - t13) + t02 * (one - t12) * t13 + t12 * t13;
    R F = k <= Z.s1 ? lowr : (k >= Z.s2 ? highr : mid);
    F = k >= Z.s3 ? one : F;
    return k <= Z.s0 ? R(0) : F;
}

// Work events of the cumulative walk, counted only by the instrumented
// kernel instances (psd_options flag PSD_WORK_COUNTERS).
struct WorkCount {
    unsigned long long xpiece;  // pieces of the first (u) split
    unsigned long long piece;   // pieces of the second (v) split: z distributions set up
    unsigned long long level;   // z levels walked by those pieces
};

// LDS add with no returned value (one ds_add_f64): the lane does not wait for
// the old value, as a read-modify-write of its own column would.
template <typename R>
__device__ __forceinline__ void lds_add(R* p, R v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds frac * (share of each z-cell of the tile) for one piece.  The levels
// are walked region by region of the piecewise cubic; every cubic is scaled
// by frac up front.  On (s1, s2) the cubic is expanded in t = k - s1: each
// expanded term is bounded by 1 there (t <= s2 - s1 <= s3 - s1 and
// s1 - s0 <= s2 - s0, s3 - s0), so Horner's rule loses only a few ulps.
// Inside a region a level's share is the cubic's difference over a unit
// step, a quadratic evaluated directly (nothing is carried from level to
// level, so no error accumulates); the end regions' quadratics have only
// positive terms.
template <bool WORK, typename R>
__device__ __forceinline__ void spread_z(const R z[4], R frac, const Tile& t, R* Dcol,
                                         WorkCount& wc)
{
    ZDist<R> Z;
    zdist_init(z, Z);
    const int lfirst = (int)floor(Z.s0);
    const int lA = max(lfirst, t.l0);
    const int lB = min((int)floor(Z.s3), t.l0 + t.tl - 1);
    if (lA > lB) return;
    if constexpr (WORK) wc.level += (unsigned long long)(lB - lA + 1);
    R Fprev = (lA <= lfirst) ? R(0) : frac * zdist_below(Z, (R)lA);
    R* p = Dcol + (lA - t.l0);
    R k = (R)(lA + 1);       // upper plane of the level
    const R kB = (R)(lB + 1);
    // Each region: its first level from F at both planes (the lower plane
    // may lie in the region before), the others from the difference of the
    // region's cubic over a unit step, a quadratic in the upper plane.
    // k <= s1: F = fA u^3, u = k - s0; step fA (3u^2 - 3u + 1), u >= 1
    const R fA = frac * Z.iA;
    const R kLow = fmin(Z.s1, kB);
    if (k <= kLow) {
        R u = k - Z.s0;
        lds_add(p, fA * (u * u * u) - Fprev);
        k += R(1);
        ++p;
        const R g = R(3) * fA;
        for (; k <= kLow; k += R(1), ++p) {
            u = k - Z.s0;
            lds_add(p, fma(u, fma(g, u, -g), fA));
        }
        u = (k - R(1)) - Z.s0;
        Fprev = fA * (u * u * u);
    }
    // s1 < k < s2: F = c0 + c1 t + c2 t^2 + c3 t^3, t = k - s1;
    // step q0 + q1 t + q2 t^2
    if (k < Z.s2 && k <= kB) {
        const R a = Z.s1 - Z.s0;
        const R A = Z.r20 * Z.r30, B = Z.r20 * Z.r31;
        const R c0 = frac * (A * a * a);
        const R c1 = frac * (a * (A * (R(2) - Z.r31 * a) + B));
        const R c2 = frac * (A * (R(1) - R(2) * a * Z.r31) + B * (R(1) - a * Z.r21) + Z.r21 * Z.r31);
        const R c3 = -frac * (A * Z.r31 + B * Z.r21);
        R tt = k - Z.s1;
        lds_add(p, fma(fma(fma(c3, tt, c2), tt, c1), tt, c0) - Fprev);
        k += R(1);
        ++p;
        const R q0 = c1 - c2 + c3, q1 = R(2) * c2 - R(3) * c3, q2 = R(3) * c3;
        for (; k < Z.s2 && k <= kB; k += R(1), ++p) {
            tt = k - Z.s1;
            lds_add(p, fma(fma(q2, tt, q1), tt, q0));
        }
        tt = (k - R(1)) - Z.s1;
        Fprev = fma(fma(fma(c3, tt, c2), tt, c1), tt, c0);
    }
    // s2 <= k: F = frac - fC w^3, w = s3 - k (frac once k >= s3);
    // step fC (3w^2 + 3w + 1) while k < s3
    if (k <= kB) {
        const R fC = frac * Z.iC;
        R w = Z.s3 - k;
        lds_add(p, (w > R(0) ? frac - fC * (w * w * w) : frac) - Fprev);
        k += R(1);
        ++p;
        const R g = R(3) * fC;
        for (; k < Z.s3 && k <= kB; k += R(1), ++p) {
            w = Z.s3 - k;
            lds_add(p, fma(w, fma(g, w, g), fC));
        }
        // the level whose upper plane passes s3
        if (k <= kB) {
            w = Z.s3 - (k - R(1));
            lds_add(p, fC * (w * w * w));
        }
    }
}

// Whether column row a of tile t takes the complement of the x split: T has
// three vertices with x <= a+1 (the vertices are in increasing x), so the
// inside part is a prism of three pieces while the outside part x > a+1 is
// one tetrahedron, and the tile holds the bbox's last row, whose D columns
// are all of T below y = b+1 (no x plane cuts there).  Such a column is
// walked as minus the outside tetrahedron; the 2-D differences add the last
// row's column back where the complement starts or ends.
__device__ __forceinline__ bool x_complement(const CTet& S, const Tile& t, int a)
{
    const double X = (double)(a + 1);
    return a + 1 < S.ext[0] && X - S.vr[2][0] >= 0.0 && X - S.vr[3][0] < 0.0 &&
           t.a0 + t.ta == S.ext[0];
}

// D column (a,b) of one tile: T cut by x <= a+1 and y <= b+1, the
// complement walked where a split leaves three vertices inside (for y, the
// x-piece whole minus its one outside tetrahedron: two z walks instead of
// three; for x, see x_complement).
template <bool WORK>
__device__ __forceinline__ void column(const CTet& S, int a, int b, const Tile& t, double* Dcol,
                                       WorkCount& wc)
{
    for (int l = 0; l < t.tl; ++l) Dcol[l] = 0.0;
    const bool cx = a + 1 < S.ext[0];
    const bool cy = b + 1 < S.ext[1];
    const double X = (double)(a + 1), Y = (double)(b + 1);
    double v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[q][c] = S.vr[q][c];

    // level 1: x <= X (inside when X - x >= 0); the vertices are in
    // increasing x, so the inside ones come first
    double dx[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) dx[q] = cx ? X - v[q][0] : 1.0;
    const int nin = (dx[0] >= 0.0 ? 1 : 0) + (dx[1] >= 0.0 ? 1 : 0) + (dx[2] >= 0.0 ? 1 : 0) +
                    (dx[3] >= 0.0 ? 1 : 0);
    const bool cmp = x_complement(S, t, a);
    double d[4], P1[4][2];
    d[0] = cmp ? -dx[3] : dx[0];
    d[1] = cmp ? -dx[0] : dx[1];
    d[2] = cmp ? -dx[1] : dx[2];
    d[3] = cmp ? -dx[2] : dx[3];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        P1[0][c] = cmp ? v[3][c + 1] : v[0][c + 1];
        P1[1][c] = cmp ? v[0][c + 1] : v[1][c + 1];
        P1[2][c] = cmp ? v[1][c + 1] : v[2][c + 1];
        P1[3][c] = cmp ? v[2][c + 1] : v[3][c + 1];
    }
    const double xsign = cmp ? -1.0 : 1.0;
    Split<double> s1;
    s1.nin = cmp ? 1 : nin;
    s1.ia = 0;
    s1.ib = 1;
    s1.ic = 2;
    s1.id = 3;
    split_ordered(d[0], d[1], d[2], d[3], s1.nin, s1);
    if (s1.nin == 0) return;
    const bool a1 = s1.nin == 1, a2 = s1.nin == 2, a3 = s1.nin == 3, a4 = s1.nin == 4;
    double U0[2], U1[2], U2[2], W0[2], W1[2], W2[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double va = P1[0][c], vb = P1[1][c], vc = P1[2][c], vd = P1[3][c];
        const double in1 = a3 ? vb : va, in2 = a1 ? va : (a2 ? vb : vc);
        const double out0 = a1 ? vb : (a2 ? vc : vd), out1 = a1 ? vc : vd, out2 = a2 ? vc : vd;
        const double c0 = va + s1.t0 * (out0 - va);
        const double c1 = in1 + s1.t1 * (out1 - in1);
        const double c2 = in2 + s1.t2 * (out2 - in2);
        const double c3 = vb + s1.t3 * (vd - vb);
        U0[c] = va;
        U1[c] = (a3 || a4) ? vb : c0;
        U2[c] = (a3 || a4) ? vc : c1;
        W0[c] = a2 ? vb : c0;
        W1[c] = a2 ? c2 : c1;
        W2[c] = a4 ? vd : (a2 ? c3 : c2);
    }
    const int n1 = (a2 || a3) ? 3 : 1;
    if constexpr (WORK) wc.xpiece += (unsigned long long)n1;
    for (int j = 0; j < n1; ++j) {
        double cv[4][2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            cv[0][c] = U0[c];
            cv[1][c] = j == 2 ? W0[c] : U1[c];
            cv[2][c] = j == 0 ? U2[c] : W1[c];
            cv[3][c] = W2[c];
        }
        const double f1 = xsign * (j == 0 ? s1.f0 : (j == 1 ? s1.f1 : s1.f2));
        // level 2: y <= Y
        double dy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dy[q] = cy ? Y - cv[q][0] : 1.0;
        Split<double> s2;
        split_plane(dy, s2);
        if (s2.nin == 0) continue;
        double za = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ia);
        double zb = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ib);
        double zc = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ic);
        double zd = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.id);
        const bool b1 = s2.nin == 1, b2 = s2.nin == 2, b3 = s2.nin == 3, b4 = s2.nin == 4;
        const double in1 = b3 ? zb : za, in2 = b1 ? za : (b2 ? zb : zc);
        const double out0 = b1 ? zb : (b2 ? zc : zd), out1 = b1 ? zc : zd, out2 = b2 ? zc : zd;
        const double c0 = za + s2.t0 * (out0 - za);
        const double c1 = in1 + s2.t1 * (out1 - in1);
        const double c2 = in2 + s2.t2 * (out2 - in2);
        const double c3 = zb + s2.t3 * (zd - zb);
        const double u0 = za, u1 = (b3 || b4) ? zb : c0, u2 = (b3 || b4) ? zc : c1;
        const double w0 = b2 ? zb : c0, w1 = b2 ? c2 : c1, w2 = b4 ? zd : (b2 ? c3 : c2);
        // three inside: the x-piece whole, then minus its one outside
        // tetrahedron (zd, c0, c1, c2), whose edges from zd keep 1 - t
        if (b3) {
            s2.f0 = 1.0;
            s2.f1 = -((1.0 - s2.t0) * (1.0 - s2.t1) * (1.0 - s2.t2));
        }
        const int n2 = b2 ? 3 : (b3 ? 2 : 1);
        if constexpr (WORK) wc.piece += (unsigned long long)n2;
        for (int k = 0; k < n2; ++k) {
            const bool c1k = b3 && k == 1;
            const double z[4] = {c1k ? zd : u0, (k == 2 || c1k) ? w0 : u1, k == 0 ? u2 : w1,
                                 (b3 && k == 0) ? zd : w2};
            const double f2 = k == 0 ? s2.f0 : (k == 1 ? s2.f1 : s2.f2);
            spread_z<WORK, double>(z, f1 * f2, t, Dcol, wc);
        }
    }
}


// Orders a wavefront's LDS accesses before the ones that follow: they
// complete in issue order, so a wavefront fence (no wait on the global atomics
// in flight) is enough for values other lanes wrote.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pieces of the two-plane splits waiting for their z walk: a ring of QCAP
// records in LDS (QCAP a power of two), one per piece: its four vertex
// heights, its volume fraction of the tetrahedron, and where its levels go
// (D-buffer offset of its column and tile index, packed).  Every lane of the
// wavefront produces the pieces of its own column, 0 to 9 of them; the z
// walks then go over the lanes 64 pieces at a time, so a column cut into nine
// pieces no longer holds the other 63 lanes back.
template <int QCAP, typename R>
struct PieceRing {
    R z[4][QCAP];
    R frac[QCAP];
    uint16_t where[QCAP];  // D offset << 4 | tile
};

// The z walks of the next min(count, 64) queued pieces, one per lane.
// Wave-uniform: every lane calls it with the same head and count.
template <bool WORK, int QCAP, typename R>
__device__ __forceinline__ void drain_round(PieceRing<QCAP, R>& Q, int& head, int& count,
                                            const Tile* tiles, R* Dbuf, WorkCount& wc,
                                            bool local_z = false)
{
    wave_lds_sync();  // the ring's records were written by other lanes
    const int lane = threadIdx.x;
    const int ntake = count < kWave ? count : kWave;
    if (lane < ntake) {
        const int q = (head + lane) & (QCAP - 1);
        const R z[4] = {Q.z[0][q], Q.z[1][q], Q.z[2][q], Q.z[3][q]};
        const int w = Q.where[q];
        Tile t = tiles[w & 15];
        if (local_z) t.l0 = 0;  // heights relative to the tile's first level
        spread_z<WORK, R>(z, Q.frac[q], t, Dbuf + (w >> 4), wc);
    }
    head = (head + ntake) & (QCAP - 1);
    count -= ntake;
}

// Column (a,b) of one tile (valid lanes only; every lane of the wavefront
// calls it; the D column is zeroed with the batch's): splits T by x <= a+1
// and y <= b+1 as column() does, and queues the pieces; full rounds of 64 are
// walked as they fill.  Where a split leaves three vertices inside, the
// complement is walked instead (Section 6.3's inside-mask split, read from
// the outside): for y, the whole x-piece plus minus its one outside
// tetrahedron (two pieces, not three); for x, see x_complement.  Loops run to
// the wavefront's largest piece count, so that the rounds are taken with
// every lane present.
template <bool WORK, int QCAP>
__device__ __forceinline__ void column_queue(bool valid, const CTet& S, int a, int b, const Tile& t,
                                             int tile_idx, int doff, double* Dbuf,
                                             PieceRing<QCAP, double>& Q, int& head, int& count,
                                             const Tile* tiles, WorkCount& wc)
{
    const int lane = threadIdx.x;
    int n1 = 0;
    Split<double> s1;
    double U0[2], U1[2], U2[2], W0[2], W1[2], W2[2];
    double xsign = 1.0;
    if (valid) {  // the batch's D columns were zeroed before its first window
        const bool cx = a + 1 < S.ext[0];
        const double X = (double)(a + 1);
        double v[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[q][c] = S.vr[q][c];
        double dx[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dx[q] = cx ? X - v[q][0] : 1.0;
        const int nin = (dx[0] >= 0.0 ? 1 : 0) + (dx[1] >= 0.0 ? 1 : 0) + (dx[2] >= 0.0 ? 1 : 0) +
                        (dx[3] >= 0.0 ? 1 : 0);
        // the complement: vertex 3 alone inside x >= X (its value x - X > 0;
        // the others' are <= 0, a vertex on the plane cut at itself)
        const bool cmp = x_complement(S, t, a);
        double d[4], P1[4][2];
        d[0] = cmp ? -dx[3] : dx[0];
        d[1] = cmp ? -dx[0] : dx[1];
        d[2] = cmp ? -dx[1] : dx[2];
        d[3] = cmp ? -dx[2] : dx[3];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            P1[0][c] = cmp ? v[3][c + 1] : v[0][c + 1];
            P1[1][c] = cmp ? v[0][c + 1] : v[1][c + 1];
            P1[2][c] = cmp ? v[1][c + 1] : v[2][c + 1];
            P1[3][c] = cmp ? v[2][c + 1] : v[3][c + 1];
        }
        xsign = cmp ? -1.0 : 1.0;
        s1.nin = cmp ? 1 : nin;
        s1.ia = 0;
        s1.ib = 1;
        s1.ic = 2;
        s1.id = 3;
        split_ordered(d[0], d[1], d[2], d[3], s1.nin, s1);
        if (s1.nin > 0) {
            const bool a1 = s1.nin == 1, a2 = s1.nin == 2, a3 = s1.nin == 3, a4 = s1.nin == 4;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double va = P1[0][c], vb = P1[1][c], vc = P1[2][c], vd = P1[3][c];
                const double in1 = a3 ? vb : va, in2 = a1 ? va : (a2 ? vb : vc);
                const double out0 = a1 ? vb : (a2 ? vc : vd), out1 = a1 ? vc : vd, out2 = a2 ? vc : vd;
                const double c0 = va + s1.t0 * (out0 - va);
                const double c1 = in1 + s1.t1 * (out1 - in1);
                const double c2 = in2 + s1.t2 * (out2 - in2);
                const double c3 = vb + s1.t3 * (vd - vb);
                U0[c] = va;
                U1[c] = (a3 || a4) ? vb : c0;
                U2[c] = (a3 || a4) ? vc : c1;
                W0[c] = a2 ? vb : c0;
                W1[c] = a2 ? c2 : c1;
                W2[c] = a4 ? vd : (a2 ? c3 : c2);
            }
            n1 = (a2 || a3) ? 3 : 1;
            if constexpr (WORK) wc.xpiece += (unsigned long long)n1;
        }
    }
    const int nj = __ballot(n1 == 3) ? 3 : (__ballot(n1 == 1) ? 1 : 0);
    const bool cy = b + 1 < S.ext[1];
    const double Y = (double)(b + 1);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int j = 0; j < nj; ++j) {
        int n2 = 0;
        Split<double> s2;
        double u0 = 0.0, u1 = 0.0, u2 = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0, e = 0.0, f1 = 0.0;
        bool ycmp = false;
        if (j < n1) {
            double cv[4][2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                cv[0][c] = U0[c];
                cv[1][c] = j == 2 ? W0[c] : U1[c];
                cv[2][c] = j == 0 ? U2[c] : W1[c];
                cv[3][c] = W2[c];
            }
            f1 = xsign * (j == 0 ? s1.f0 : (j == 1 ? s1.f1 : s1.f2));
            double dy[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) dy[q] = cy ? Y - cv[q][0] : 1.0;
            split_plane(dy, s2);
            if (s2.nin > 0) {
                const double za = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ia);
                const double zb = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ib);
                const double zc = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ic);
                const double zd = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.id);
                const bool b1 = s2.nin == 1, b2 = s2.nin == 2, b3 = s2.nin == 3, b4 = s2.nin == 4;
                const double in1 = b3 ? zb : za, in2 = b1 ? za : (b2 ? zb : zc);
                const double out0 = b1 ? zb : (b2 ? zc : zd), out1 = b1 ? zc : zd, out2 = b2 ? zc : zd;
                const double c0 = za + s2.t0 * (out0 - za);
                const double c1 = in1 + s2.t1 * (out1 - in1);
                const double c2 = in2 + s2.t2 * (out2 - in2);
                const double c3 = zb + s2.t3 * (zd - zb);
                u0 = za;
                u1 = (b3 || b4) ? zb : c0;
                u2 = (b3 || b4) ? zc : c1;
                w0 = b2 ? zb : c0;
                w1 = b2 ? c2 : c1;
                w2 = b4 ? zd : (b2 ? c3 : c2);
                e = zd;
                // three inside: the x-piece (za, zb, zc, zd) whole, then minus
                // the outside tetrahedron (zd, c0, c1, c2), whose edges from zd
                // keep 1 - t of the parent's
                ycmp = b3;
                if (b3) {
                    s2.f0 = 1.0;
                    s2.f1 = -((1.0 - s2.t0) * (1.0 - s2.t1) * (1.0 - s2.t2));
                }
                n2 = b2 ? 3 : (b3 ? 2 : 1);
                if constexpr (WORK) wc.piece += (unsigned long long)n2;
            }
        }
        const int nk = __ballot(n2 == 3) ? 3 : (__ballot(n2 == 2) ? 2 : (__ballot(n2 == 1) ? 1 : 0));
        for (int k = 0; k < nk; ++k) {
            const bool has = k < n2;
            const uint64_t bal = __ballot(has);
            if (has) {
                const int q = (head + count + __popcll(bal & below)) & (QCAP - 1);
                const bool c1k = ycmp && k == 1;
                Q.z[0][q] = c1k ? e : u0;
                Q.z[1][q] = (k == 2 || c1k) ? w0 : u1;
                Q.z[2][q] = k == 0 ? u2 : w1;
                Q.z[3][q] = (ycmp && k == 0) ? e : w2;
                Q.frac[q] = f1 * (k == 0 ? s2.f0 : (k == 1 ? s2.f1 : s2.f2));
                Q.where[q] = (uint16_t)((doff << 4) | tile_idx);
            }
            count += __popcll(bal);
            if (count >= kWave) drain_round<WORK, QCAP, double>(Q, head, count, tiles, Dbuf, wc);
        }
    }
}

// ---------------------------------------------------------------------------
// Slab form: the cells' volumes directly, each split computed once where
// the pieces can be reused.  A tile row a (the slab a <= x < a+1 of the walk
// frame) is cut from T once by x >= a and x <= a+1 (FP64 planes on the exact
// bbox-local vertices); its <= 9 pieces are kept in LDS in FP32, relative to
// the tile's first column and level.  Every column (a, b) of the row takes
// them, splits each by y >= b and y <= b+1 in FP32 and sends the leaves to
// the piece ring, whose z walks add each leaf's exact z distribution into the
// column's cells: no cumulative values, so nothing cancels and FP32 keeps its
// relative precision in every cell.
// ---------------------------------------------------------------------------

constexpr int kSlabPieces = 9;

template <int ROWS>
struct SlabCache {
    float v[ROWS][kSlabPieces][4][2];  // (y - b0, z - l0) of the 4 vertices
    float frac[ROWS][kSlabPieces];
    int n[ROWS];
};

// Pieces of T cut by x >= a and x <= a+1 (walk frame, bbox-local vertices):
// each inside part of the first cut is cut again.  The planes that do not
// meet the bbox (a = 0, a + 1 = ext0) keep every vertex inside.
template <int ROWS>
__device__ __forceinline__ void slab_row(const CTet& S, int a, const Tile& t, int row,
                                         SlabCache<ROWS>& C)
{
    const bool cut0 = a > 0, cut1 = a + 1 < S.ext[0];
    double v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[q][c] = S.vr[q][c];
    double d0[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) d0[q] = cut0 ? v[q][0] - (double)a : 1.0;
    Split<double> s0;
    split_plane(d0, s0);
    int n = 0;
    if (s0.nin > 0) {
        double U0[3], U1[3], U2[3], W0[3], W1[3], W2[3];
        const bool a1 = s0.nin == 1, a2 = s0.nin == 2, a3 = s0.nin == 3, a4 = s0.nin == 4;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double va = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s0.ia);
            const double vb = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s0.ib);
            const double vc = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s0.ic);
            const double vd = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s0.id);
            const double in1 = a3 ? vb : va, in2 = a1 ? va : (a2 ? vb : vc);
            const double out0 = a1 ? vb : (a2 ? vc : vd), out1 = a1 ? vc : vd, out2 = a2 ? vc : vd;
            const double c0 = va + s0.t0 * (out0 - va);
            const double c1 = in1 + s0.t1 * (out1 - in1);
            const double c2 = in2 + s0.t2 * (out2 - in2);
            const double c3 = vb + s0.t3 * (vd - vb);
            U0[c] = va;
            U1[c] = (a3 || a4) ? vb : c0;
            U2[c] = (a3 || a4) ? vc : c1;
            W0[c] = a2 ? vb : c0;
            W1[c] = a2 ? c2 : c1;
            W2[c] = a4 ? vd : (a2 ? c3 : c2);
        }
        const int n0 = (a2 || a3) ? 3 : 1;
        for (int j = 0; j < n0; ++j) {
            double cv[4][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cv[0][c] = U0[c];
                cv[1][c] = j == 2 ? W0[c] : U1[c];
                cv[2][c] = j == 0 ? U2[c] : W1[c];
                cv[3][c] = W2[c];
            }
            const double f0 = j == 0 ? s0.f0 : (j == 1 ? s0.f1 : s0.f2);
            double d1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) d1[q] = cut1 ? (double)(a + 1) - cv[q][0] : 1.0;
            Split<double> s1;
            split_plane(d1, s1);
            if (s1.nin == 0) continue;
            const bool b1 = s1.nin == 1, b2 = s1.nin == 2, b3 = s1.nin == 3, b4 = s1.nin == 4;
            float u0[2], u1[2], u2[2], w0[2], w1[2], w2[2];
            const double org[2] = {(double)t.b0, (double)t.l0};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double va = sel4(cv[0][c + 1], cv[1][c + 1], cv[2][c + 1], cv[3][c + 1], s1.ia);
                const double vb = sel4(cv[0][c + 1], cv[1][c + 1], cv[2][c + 1], cv[3][c + 1], s1.ib);
                const double vc = sel4(cv[0][c + 1], cv[1][c + 1], cv[2][c + 1], cv[3][c + 1], s1.ic);
                const double vd = sel4(cv[0][c + 1], cv[1][c + 1], cv[2][c + 1], cv[3][c + 1], s1.id);
                const double in1 = b3 ? vb : va, in2 = b1 ? va : (b2 ? vb : vc);
                const double out0 = b1 ? vb : (b2 ? vc : vd), out1 = b1 ? vc : vd, out2 = b2 ? vc : vd;
                const double c0 = va + s1.t0 * (out0 - va);
                const double c1 = in1 + s1.t1 * (out1 - in1);
                const double c2 = in2 + s1.t2 * (out2 - in2);
                const double c3 = vb + s1.t3 * (vd - vb);
                u0[c] = (float)(va - org[c]);
                u1[c] = (float)(((b3 || b4) ? vb : c0) - org[c]);
                u2[c] = (float)(((b3 || b4) ? vc : c1) - org[c]);
                w0[c] = (float)((b2 ? vb : c0) - org[c]);
                w1[c] = (float)((b2 ? c2 : c1) - org[c]);
                w2[c] = (float)((b4 ? vd : (b2 ? c3 : c2)) - org[c]);
            }
            const int n1 = (b2 || b3) ? 3 : 1;
            for (int k = 0; k < n1; ++k, ++n) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    C.v[row][n][0][c] = u0[c];
                    C.v[row][n][1][c] = k == 2 ? w0[c] : u1[c];
                    C.v[row][n][2][c] = k == 0 ? u2[c] : w1[c];
                    C.v[row][n][3][c] = w2[c];
                }
                C.frac[row][n] = (float)(f0 * (k == 0 ? s1.f0 : (k == 1 ? s1.f1 : s1.f2)));
            }
        }
    }
    C.n[row] = n;
}

// Column (a, b) of the slab form (valid lanes only; every lane calls it):
// zeroes the column's cells, splits the row's slab pieces by y >= b and
// y <= b+1 and queues the leaves; full rounds of 64 are walked as they fill.
template <bool WORK, int QCAP, int ROWS>
__device__ __forceinline__ void column_slab(bool valid, const CTet& S, int b, const Tile& t,
                                            int tile_idx, int row, int doff, float* Dbuf,
                                            const SlabCache<ROWS>& C, PieceRing<QCAP, float>& Q,
                                            int& head, int& count, const Tile* tiles, WorkCount& wc)
{
    const int lane = threadIdx.x;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    int ns = 0;
    if (valid) {
        float* Dcol = Dbuf + doff;
        for (int l = 0; l < t.tl; ++l) Dcol[l] = 0.0f;
        ns = C.n[row];
    }
    // the wavefront's largest slab piece count (at most 9)
    int nsmax = ns;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) nsmax = max(nsmax, __shfl_xor(nsmax, off, kWave));
    const bool cut0 = b > 0, cut1 = b + 1 < S.ext[1];
    const float yb = (float)(b - t.b0);  // the column's lower y plane, tile-relative
    for (int p = 0; p < nsmax; ++p) {
        int n1 = 0;
        Split<float> s1;
        float U0[2], U1[2], U2[2], W0[2], W1[2], W2[2];
        float fp = 0.0f;
        if (p < ns) {
            float v[4][2];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q][0] = C.v[row][p][q][0] - yb;  // column-local y
                v[q][1] = C.v[row][p][q][1];
            }
            fp = C.frac[row][p];
            float d[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) d[q] = cut0 ? v[q][0] : 1.0f;
            split_plane(d, s1);
            if (s1.nin > 0) {
                const bool a1 = s1.nin == 1, a2 = s1.nin == 2, a3 = s1.nin == 3, a4 = s1.nin == 4;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float va = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s1.ia);
                    const float vb = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s1.ib);
                    const float vc = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s1.ic);
                    const float vd = sel4(v[0][c], v[1][c], v[2][c], v[3][c], s1.id);
                    const float in1 = a3 ? vb : va, in2 = a1 ? va : (a2 ? vb : vc);
                    const float out0 = a1 ? vb : (a2 ? vc : vd), out1 = a1 ? vc : vd, out2 = a2 ? vc : vd;
                    const float c0 = va + s1.t0 * (out0 - va);
                    const float c1 = in1 + s1.t1 * (out1 - in1);
                    const float c2 = in2 + s1.t2 * (out2 - in2);
                    const float c3 = vb + s1.t3 * (vd - vb);
                    U0[c] = va;
                    U1[c] = (a3 || a4) ? vb : c0;
                    U2[c] = (a3 || a4) ? vc : c1;
                    W0[c] = a2 ? vb : c0;
                    W1[c] = a2 ? c2 : c1;
                    W2[c] = a4 ? vd : (a2 ? c3 : c2);
                }
                n1 = (a2 || a3) ? 3 : 1;
                if constexpr (WORK) wc.xpiece += (unsigned long long)n1;
            }
        }
        const int nj = __ballot(n1 == 3) ? 3 : (__ballot(n1 == 1) ? 1 : 0);
        for (int j = 0; j < nj; ++j) {
            int n2 = 0;
            Split<float> s2;
            float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f, w0 = 0.0f, w1 = 0.0f, w2 = 0.0f, f1 = 0.0f;
            if (j < n1) {
                float cv[4][2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    cv[0][c] = U0[c];
                    cv[1][c] = j == 2 ? W0[c] : U1[c];
                    cv[2][c] = j == 0 ? U2[c] : W1[c];
                    cv[3][c] = W2[c];
                }
                f1 = fp * (j == 0 ? s1.f0 : (j == 1 ? s1.f1 : s1.f2));
                float d[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) d[q] = cut1 ? 1.0f - cv[q][0] : 1.0f;
                split_plane(d, s2);
                if (s2.nin > 0) {
                    const float za = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ia);
                    const float zb = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ib);
                    const float zc = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.ic);
                    const float zd = sel4(cv[0][1], cv[1][1], cv[2][1], cv[3][1], s2.id);
                    const bool b1 = s2.nin == 1, b2 = s2.nin == 2, b3 = s2.nin == 3, b4 = s2.nin == 4;
                    const float in1 = b3 ? zb : za, in2 = b1 ? za : (b2 ? zb : zc);
                    const float out0 = b1 ? zb : (b2 ? zc : zd), out1 = b1 ? zc : zd, out2 = b2 ? zc : zd;
                    const float c0 = za + s2.t0 * (out0 - za);
                    const float c1 = in1 + s2.t1 * (out1 - in1);
                    const float c2 = in2 + s2.t2 * (out2 - in2);
                    const float c3 = zb + s2.t3 * (zd - zb);
                    u0 = za;
                    u1 = (b3 || b4) ? zb : c0;
                    u2 = (b3 || b4) ? zc : c1;
                    w0 = b2 ? zb : c0;
                    w1 = b2 ? c2 : c1;
                    w2 = b4 ? zd : (b2 ? c3 : c2);
                    n2 = (b2 || b3) ? 3 : 1;
                    if constexpr (WORK) wc.piece += (unsigned long long)n2;
                }
            }
            const int nk = __ballot(n2 == 3) ? 3 : (__ballot(n2 == 1) ? 1 : 0);
            for (int k = 0; k < nk; ++k) {
                const bool has = k < n2;
                const uint64_t bal = __ballot(has);
                if (has) {
                    const int q = (head + count + __popcll(bal & below)) & (QCAP - 1);
                    Q.z[0][q] = u0;
                    Q.z[1][q] = k == 2 ? w0 : u1;
                    Q.z[2][q] = k == 0 ? u2 : w1;
                    Q.z[3][q] = w2;
                    Q.frac[q] = f1 * (k == 0 ? s2.f0 : (k == 1 ? s2.f1 : s2.f2));
                    Q.where[q] = (uint16_t)((doff << 4) | tile_idx);
                }
                count += __popcll(bal);
                if (count >= kWave) drain_round<WORK, QCAP, float>(Q, head, count, tiles, Dbuf, wc, true);
            }
        }
    }
}

// Index of the box holding global chunk g (boxes sorted by chunk_begin).
__device__ __forceinline__ int box_of(const QueueArgs& Q, int64_t g)
{
    if (!Q.boxes) return 0;
    int lo = 0, hi = Q.n_boxes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (Q.boxes[mid].chunk_begin <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Position of the k-th set bit (k from 0, k < popcount(m)) of m.
__device__ __forceinline__ int nth_bit(uint64_t m, int k)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = (1ull << w) - 1ull;
        const int c = __popcll(m & low);
        const bool up = k >= c;
        k = up ? k - c : k;
        m = up ? m >> w : m & low;
        pos += up ? w : 0;
    }
    return pos;
}

// Builds tetrahedron `tid` of box P into slot S; returns its bbox cell count
// (0 when nothing is left to do) and deposits the cases that need no walk.
template <typename OutT>
// With `pend` (the group-tile instances), a tetrahedron whose whole mass goes
// to one cell (inside one cell, or zero volume) is not added here: its cell
// (wrapped grid coordinates) is returned in pend[0..2] and pend[3] = 1, and
// the caller adds it to the group's tile.
__device__ __forceinline__ int setup_tet(const BoxDesc& P, int64_t tid, CTet& S, double& macc,
                                         unsigned long long& n_pair, unsigned long long& n_nz,
                                         unsigned long long& n_inv, unsigned long long& n_deg,
                                         unsigned long long* stats, int* pend = nullptr)
{
    const int64_t cube = tid / 6;
    const int p = (int)(tid - cube * 6);
    const int64_t kk = cube % P.np[2];
    const int64_t jj = (cube / P.np[2]) % P.np[1];
    const int64_t ii = cube / ((int64_t)P.np[1] * P.np[2]);
    Tet64 T;
    make_tet(P.pos, P.np[0], P.np[1], P.np[2], P.scale, P.nc, ii, jj, kk, p, T);
    OutT* out = reinterpret_cast<OutT*>(P.out);
    if ((double)kuhn_sign(p) * T.D < 0.0) ++n_inv;
    if (!(isfinite(T.D) && isfinite(T.l3))) {
        // a NaN or infinite vertex cannot be placed: dropped, and counted
        // (rare, so straight to the counter rather than a register)
        if (stats) atomicAdd(stats + 7, 1ull);
        return 0;
    }
    if (fabs(T.D) <= 1e-12 * T.l3) {
        // zero-volume tetrahedron: all mass to the centroid's cell
        ++n_deg;
        int g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x = 0.25 * (T.v[0][c] + T.v[1][c] + T.v[2][c] + T.v[3][c]);
            g[c] = wrap_index(floor(x), P.nc[c]);
        }
        const int64_t idx = out_index(P, g[0], g[1], g[2]);
        if (idx >= 0) {
            ++n_nz;
            if (pend) {
                pend[0] = g[0];
                pend[1] = g[1];
                pend[2] = g[2];
                pend[3] = 1;
            } else {
                global_add(out + idx, (OutT)(P.m * P.out_scale));
            }
            macc += P.m;
        }
        return 0;
    }
    bool ok = true;
    double lof[3];
    int e[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double mn = fmin(fmin(T.v[0][c], T.v[1][c]), fmin(T.v[2][c], T.v[3][c]));
        const double mx = fmax(fmax(T.v[0][c], T.v[1][c]), fmax(T.v[2][c], T.v[3][c]));
        lof[c] = floor(mn);
        e[c] = (int)(floor(mx) - lof[c]) + 1;
        // minimum-image offsets bound the extent by nc + 1 cells
        ok = ok && e[c] >= 1 && e[c] <= P.nc[c] + 1;
        S.lo[c] = wrap_index(lof[c], P.nc[c]);
    }
    // a bbox can exceed 2^31 cells on grids above ~1290 cells per axis: the
    // count only picks the tiled walk, which handles any size
    const int64_t ncell64 = ok ? (int64_t)e[0] * e[1] * e[2] : 0;
    int ncell = ncell64 > 0x7FFFFFFF ? 0x7FFFFFFF : (int)ncell64;
    if (ncell && P.leaf_map && !touches_leaf(P, S.lo, e)) ncell = 0;
    // deposited by the learned surrogate instead
    if (P.skip_small && ncell >= 2 && e[0] <= 2 && e[1] <= 2 && e[2] <= 2) return 0;
    // walk frame: the longest axis last (ties keep the later grid axis)
    const int w2 = (e[0] > e[1] && e[0] > e[2]) ? 0 : (e[1] > e[2] ? 1 : 2);
    int w0 = w2 == 0 ? 1 : 0, w1 = w2 == 2 ? 1 : 2;
    {
        // Of the two others, the first split goes along the one with fewer
        // three-piece columns: rows whose plane has two vertices on each side
        // (floor of the 3rd smallest coordinate minus floor of the 2nd, in
        // bbox-local units) times the row's length, the other axis' extent.
        double rows[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int c = k == 0 ? w0 : w1;
            const double lo = c == 0 ? lof[0] : (c == 1 ? lof[1] : lof[2]);
            double x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = (c == 0 ? T.v[q][0] : (c == 1 ? T.v[q][1] : T.v[q][2])) - lo;
            const double a = fmin(x[0], x[1]), b = fmax(x[0], x[1]);
            const double cc = fmin(x[2], x[3]), d = fmax(x[2], x[3]);
            const double m1 = fmin(fmax(a, cc), fmin(b, d)), m2 = fmax(fmax(a, cc), fmin(b, d));
            rows[k] = floor(m2) - floor(m1);
        }
        const int e0 = w0 == 0 ? e[0] : (w0 == 1 ? e[1] : e[2]);
        const int e1 = w1 == 0 ? e[0] : (w1 == 1 ? e[1] : e[2]);
        if (rows[1] * (double)e0 < rows[0] * (double)e1) {
            const int t = w0;
            w0 = w1;
            w1 = t;
        }
    }
    S.axes = w0 | (w1 << 2) | (w2 << 4);
    const int wa[3] = {w0, w1, w2};
    double w[4][3];
    int id[4] = {0, 1, 2, 3};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int c = wa[k];
        const double lo = c == 0 ? lof[0] : (c == 1 ? lof[1] : lof[2]);
        S.ext[k] = c == 0 ? e[0] : (c == 1 ? e[1] : e[2]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q][k] = (c == 0 ? T.v[q][0] : (c == 1 ? T.v[q][1] : T.v[q][2])) - lo;
    }
    // vertices in increasing walk-frame x (ties by vertex index): every
    // plane x <= a+1 then has its inside vertices first (split_prefix)
    auto order = [&](int i, int j) {
        const bool sw = w[i][0] > w[j][0] || (w[i][0] == w[j][0] && id[i] > id[j]);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double t = w[i][k];
            w[i][k] = sw ? w[j][k] : t;
            w[j][k] = sw ? t : w[j][k];
        }
        const int ti = id[i];
        id[i] = sw ? id[j] : ti;
        id[j] = sw ? ti : id[j];
    };
    order(0, 1);
    order(2, 3);
    order(0, 2);
    order(1, 3);
    order(1, 2);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) S.vr[q][k] = w[q][k];
    if (ncell == 1) {
        // the tetrahedron lies inside one cell
        ++n_pair;
        const int64_t idx = out_index(P, S.lo[0], S.lo[1], S.lo[2]);
        if (idx >= 0) {
            ++n_nz;
            if (pend) {
                pend[0] = S.lo[0];
                pend[1] = S.lo[1];
                pend[2] = S.lo[2];
                pend[3] = 1;
            } else {
                global_add(out + idx, (OutT)(P.m * P.out_scale));
            }
            macc += P.m;
        }
        ncell = 0;
    }
    return ncell;
}

__device__ __forceinline__ void flush_mass(const BoxDesc& P, double& macc)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) macc += __shfl_xor(macc, off, kWave);
    if (threadIdx.x == 0 && P.mass_sum && macc != 0.0) global_add(P.mass_sum, macc);
    macc = 0.0;
}

// A 64-tet chunk is built in groups of GROUP tetrahedra (one per lane) and
// each group is walked in batches of at most TILES tiles: the tet slots of a
// group and the D buffer of CAP FP64 entries share the LDS of a wavefront.
// Three wavefronts per SIMD (12 per compute unit) need at most 13.6 KB of
// LDS each and at most 168 registers (the launch bounds); the instances
// trade slots for buffer: 32 tets set up at once with 960 entries and 16
// tiles a batch suit small tetrahedra (many per batch), 8 tets with 1024
// entries and a 128-piece ring (QCAP) large ones, whose columns are cut into
// 1 to 9 pieces walking up to tens of levels each; 8 tets with 1408 entries
// and no ring is the same walk with each column's pieces on its own lane.
// The 2048-entry instance runs at two per SIMD.
// SLAB selects the slab form (FP32 cell volumes, CAP FP32 entries, at most
// SLAB_ROWS tile rows a batch); otherwise the cumulative walk in FP64.
template <typename OutT, int CAP, int GROUP, int TILES, bool WORK, int QCAP, bool SLAB = false>
__global__ __launch_bounds__(kWave, ((SLAB ? CAP / 2 : CAP) <= 1408 ? 3 : 2)) void queue_kernel(QueueArgs Q)
{
    static_assert(kWave % GROUP == 0 && GROUP <= kWave && TILES <= GROUP, "chunk of whole groups");
    static_assert(QCAP == 0 || (QCAP >= 2 * kWave && (QCAP & (QCAP - 1)) == 0 && TILES <= 16 &&
                                CAP <= 4096), "piece ring: a power of two of at least 128; its "
                                              "records hold D offset and tile in 16 bits");
    static_assert(CAP <= 32767 && TILES <= 256 && GROUP <= 256, "16-bit tile fields, 8-bit slots");
    static_assert(!SLAB || (QCAP > 0 && GROUP < 16), "the slab form queues its leaves");
    using DT = typename std::conditional<SLAB, float, double>::type;
    constexpr int SLAB_ROWS = SLAB ? 16 : 1;
    // the cumulative walk takes the x complement (column, column_queue)
    constexpr bool XCMP = !SLAB;
    __shared__ CTet slots[GROUP];
    __shared__ __attribute__((aligned(16))) DT Dbuf[CAP];
    __shared__ Tile tiles[TILES];
    __shared__ uint8_t t_slot[TILES];
    __shared__ uint16_t s_incl[TILES];  // columns of the batch's tiles, inclusive prefix (<= CAP)
    __shared__ int64_t s_item;
    __shared__ PieceRing<(QCAP > 0 ? QCAP : 1), DT> ring;
    __shared__ SlabCache<SLAB_ROWS> slab;
    __shared__ int s_row0[SLAB ? TILES : 1];
    // Small tetrahedra (the <= 960-entry instances): a group's tets come from
    // neighbouring Lagrangian cubes and share most of their cells, so their
    // masses are summed in an LDS tile over the group's union bbox and each
    // non-zero cell is flushed with one global atomic (a group whose union is
    // larger than the tile adds straight to the grid).
    constexpr bool AGG = CAP <= 960 && QCAP == 0 && !SLAB;
    constexpr int ACC = AGG ? 192 : 1;
    __shared__ OutT acc[ACC];

    const int lane = threadIdx.x;
    double macc = 0.0;
    unsigned long long n_tet = 0, n_pair = 0, n_col = 0, n_nz = 0, n_inv = 0, n_deg = 0;
    WorkCount wc = {0ull, 0ull, 0ull};
    unsigned long long n_colcell = 0;
    int cur_box = -1;
    BoxDesc P = Q.box0;

    for (;;) {
        if (lane == 0) s_item = (int64_t)atomicAdd(Q.next, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= Q.n_chunks) break;
        const int64_t g = Q.order ? global_view(Q.order)[item] : item;
        const int bi = box_of(Q, g);
        if (bi != cur_box) {
            if (cur_box >= 0) flush_mass(P, macc);
            cur_box = bi;
            if (Q.boxes) P = Q.boxes[bi];
        }
        if (P.level_has_leaf && *global_view(P.level_has_leaf) == 0) {
            // a level without leaves: in index order its remaining chunks
            // are skipped in one step (the counter only moves forward)
            if (!Q.order && lane == 0) {
                const unsigned long long end =
                    (Q.boxes && bi + 1 < Q.n_boxes) ? (unsigned long long)Q.boxes[bi + 1].chunk_begin
                                                    : (unsigned long long)Q.n_chunks;
                atomicMax(Q.next, end);
            }
            continue;
        }
        OutT* out = reinterpret_cast<OutT*>(P.out);

        // The chunk's tets to deposit: all of them, or those the surrogate
        // left (its mask), taken in order GROUP at a time.
        const int64_t first = (g - P.chunk_begin) * kWave;
        const int64_t left = P.ntet - first;
        const int nvalid = left < kWave ? (int)left : kWave;
        if (lane == 0) n_tet += nvalid;
        const uint64_t todo = P.exact_mask ? P.exact_mask[g - P.chunk_begin] : 0ull;
        const int ntodo = P.exact_mask ? __popcll(todo) : nvalid;
        for (int grp = 0; grp * GROUP < ntodo; ++grp) {
        const int k = grp * GROUP + lane;  // rank among the chunk's tets to do
        int ncell = 0;
        int pend[4] = {0, 0, 0, 0};
        if (lane < GROUP && k < ntodo) {
            const int64_t tid = first + (P.exact_mask ? nth_bit(todo, k) : k);
            ncell = setup_tet<OutT>(P, tid, slots[lane], macc, n_pair, n_nz, n_inv, n_deg,
                                    Q.stats, AGG ? pend : nullptr);
        }
        if (lane < GROUP) slots[lane].ncell = ncell;
        __syncthreads();
        // The group tile: origin gref (wrapped grid cell of the first tet with
        // anything to add), box [gmn, gmn + gE) relative to it (minimum image).
        int gref[3] = {0, 0, 0}, gmn[3] = {0, 0, 0}, gE[3] = {1, 1, 1};
        bool tiled = false;
        if constexpr (AGG) {
            int lo_l[3] = {0, 0, 0}, hi_l[3] = {0, 0, 0};
            bool has = false;
            if (lane < GROUP && ncell > 0) {
                const CTet& S = slots[lane];
                has = true;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int c = walk_axis(S, q);
                    lo_l[c] = S.lo[c];
                    hi_l[c] = S.ext[q] - 1;
                }
            } else if (pend[3]) {
                has = true;
#pragma unroll
                for (int c = 0; c < 3; ++c) lo_l[c] = pend[c];
            }
            const uint64_t hb = __ballot(has);
            if (hb) {
                const int src = __ffsll((long long)hb) - 1;
                int mn[3], mx[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gref[c] = __shfl(lo_l[c], src, kWave);
                    const int nca = P.nc[c];
                    int d = lo_l[c] - gref[c];
                    if (2 * d > nca) d -= nca;
                    else if (2 * d < -nca) d += nca;
                    mn[c] = has ? d : 0x3FFFFFFF;
                    mx[c] = has ? d + hi_l[c] : -0x3FFFFFFF;
                }
#pragma unroll
                for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        mn[c] = min(mn[c], __shfl_xor(mn[c], off, kWave));
                        mx[c] = max(mx[c], __shfl_xor(mx[c], off, kWave));
                    }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gmn[c] = mn[c];
                    gE[c] = mx[c] - mn[c] + 1;
                }
                tiled = (int64_t)gE[0] * gE[1] * gE[2] <= ACC;
            }
            if (tiled) {
                for (int i = lane; i < gE[0] * gE[1] * gE[2]; i += kWave) acc[i] = OutT(0);
                __syncthreads();
            }
            if (pend[3]) {
                const double mass = P.m * P.out_scale;
                if (tiled) {
                    int li[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int nca = P.nc[c];
                        int d = pend[c] - gref[c];
                        if (2 * d > nca) d -= nca;
                        else if (2 * d < -nca) d += nca;
                        li[c] = d - gmn[c];
                    }
                    lds_add(acc + (li[0] * gE[1] + li[1]) * gE[2] + li[2], (OutT)mass);
                } else {
                    global_add(out + out_index(P, pend[0], pend[1], pend[2]), (OutT)mass);
                }
            }
        }

        // Walk the group's tetrahedra in tile batches that fit the D buffer.
        int cur = 0;       // next slot to start
        int cur_tile = 0;  // for a tiled tetrahedron, linear index of its next tile
        // a tiled tetrahedron's tile shape (set at its first tile) and the
        // position (ix, iy, iz) of tile cur_tile in its nx * ny * nz grid
        int sh_ta = 1, sh_tb = 1, sh_tl = 1, sh_nx = 1, sh_ny = 1, sh_n = 1;
        int ix = 0, iy = 0, iz = 0;
        while (cur < GROUP) {
            // Wave-uniform planning (every lane computes the same list).
            // With 16-tet groups (small tets, many per batch) runs of
            // untiled tetrahedra are laid out by all lanes at once: one slot
            // per lane and a scan of their D sizes.
            int nt = 0, used = 0, rows = 0;
            while (cur < GROUP && nt < TILES) {
                if constexpr (GROUP >= 16) {
                    if (cur_tile == 0 && slots[cur].ncell <= CAP) {
                        const int s = cur + lane;
                        const int nc = s < GROUP ? slots[s].ncell : 0;
                        const uint64_t tiled = __ballot(s < GROUP && nc > CAP);
                        const int lim = tiled ? __ffsll((long long)tiled) - 1 : GROUP - cur;
                        const int ds = lane < lim ? nc : 0;  // an untiled tile's D size is its cells
                        int incl = ds;
#pragma unroll
                        for (int off = 1; off < kWave; off <<= 1) {
                            const int y = __shfl_up(incl, off, kWave);
                            if (lane >= off) incl += y;
                        }
                        const uint64_t busy = __ballot(ds > 0);
                        const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
                        const int rank = __popcll(busy & upto);  // tiles up to this slot
                        // a prefix of the lanes: each condition is monotone in the lane
                        const bool take = lane < lim && used + incl <= CAP && nt + rank <= TILES;
                        const int ntake = __popcll(__ballot(take));
                        if (take && ds > 0) {
                            const CTet& S = slots[s];
                            Tile t;
                            t.a0 = 0; t.ta = S.ext[0]; t.b0 = 0; t.tb = S.ext[1];
                            t.l0 = 0; t.tl = S.ext[2]; t.ha = 0; t.hb = 0;
                            t.doff = used + incl - ds;
                            t.inv_wb = __builtin_amdgcn_rcpf((float)t.tb);
                            tiles[nt + rank - 1] = t;
                            t_slot[nt + rank - 1] = s;
                        }
                        if (ntake > 0) {
                            nt += __shfl(rank, ntake - 1, kWave);
                            used += __shfl(incl, ntake - 1, kWave);
                            cur += ntake;
                        }
                        if (ntake < lim) break;  // buffer or tile list full
                        continue;
                    }
                }
                const CTet& S = slots[cur];
                if (S.ncell == 0) {
                    ++cur;
                    cur_tile = 0;
                    continue;
                }
                Tile t;
                int ntiles = 1;
                if (S.ncell <= CAP && (!SLAB || S.ext[0] <= SLAB_ROWS)) {
                    t.a0 = 0; t.ta = S.ext[0]; t.b0 = 0; t.tb = S.ext[1];
                    t.l0 = 0; t.tl = S.ext[2]; t.ha = 0; t.hb = 0;
                } else {
                    if (cur_tile == 0) {
                        if constexpr (SLAB) tile_shape_slab<CAP>(S, SLAB_ROWS, sh_ta, sh_tb, sh_tl, sh_n);
                        else tile_shape<CAP>(S, sh_ta, sh_tb, sh_tl, sh_n);
                        sh_nx = (S.ext[0] + sh_ta - 1) / sh_ta;
                        sh_ny = (S.ext[1] + sh_tb - 1) / sh_tb;
                        ix = iy = iz = 0;
                    }
                    ntiles = sh_n;
                    t.a0 = ix * sh_ta; t.ta = min(sh_ta, S.ext[0] - t.a0);
                    t.b0 = iy * sh_tb; t.tb = min(sh_tb, S.ext[1] - t.b0);
                    t.l0 = iz * sh_tl; t.tl = min(sh_tl, S.ext[2] - t.l0);
                    // the cumulative walk differences against the neighbour
                    // column below; the slab form needs none
                    t.ha = (!SLAB && t.a0 > 0) ? 1 : 0;
                    t.hb = (!SLAB && t.b0 > 0) ? 1 : 0;
                }
                const int ds = tile_dsize(t);
                if (used + ds > CAP) break;  // buffer full: run this batch first
                if (SLAB && rows + t.ta > SLAB_ROWS) break;  // row cache full
                if constexpr (SLAB) {
                    if (lane == 0) s_row0[nt] = rows;
                    rows += t.ta;
                }
                t.doff = used;
                t.inv_wb = __builtin_amdgcn_rcpf((float)(t.tb + t.hb));
                used += ds;
                if (lane == 0) {
                    tiles[nt] = t;
                    t_slot[nt] = cur;
                }
                ++nt;
                if (++cur_tile >= ntiles) {
                    ++cur;
                    cur_tile = 0;
                } else if (++ix == sh_nx) {  // the next tile: x fastest, then y, then z
                    ix = 0;
                    if (++iy == sh_ny) {
                        iy = 0;
                        ++iz;
                    }
                }
            }
            __syncthreads();
            if (nt == 0) continue;

            // (tile, column) pairs over lanes, 64 at a time, columns numbered
            // row by row.  Phase 1 fills the D columns of every window of the
            // batch (one column per lane, or through the piece ring); after a
            // barrier phase 2 walks the cells of each window's columns, whose
            // lower neighbours (a-1, b), (a, b-1), (a-1, b-1) and, for the x
            // complement, the tile's last row are then final.
            {
                // columns of a tile are at most its D entries, so the sums stay below CAP
                const int c = lane < nt ? tile_cols(tiles[lane]) : 0;
                int incl = c;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const int y = __shfl_up(incl, off, kWave);
                    if (lane >= off) incl += y;
                }
                if (lane < TILES) s_incl[lane] = (uint16_t)incl;  // nt <= TILES
                __syncthreads();
                const int total = __shfl(incl, kWave - 1, kWave);
                // the tile of pair idx and its column's rank r within the tile
                auto locate = [&](int64_t idx, int& lo, int& r) {
                    lo = 0;
                    int hi = nt - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_incl[mid] > idx) hi = mid;
                        else lo = mid + 1;
                    }
                    r = (int)(idx - (s_incl[lo] - tile_cols(tiles[lo])));
                };
                if constexpr (SLAB) {
                    // The slab pieces of every tile row of the batch, one row
                    // per lane (rows <= SLAB_ROWS <= 64).
                    int nrows = 0;
                    for (int k = 0; k < nt; ++k) nrows += tiles[k].ta;
                    if (lane < nrows) {
                        int k = 0;
                        while (k + 1 < nt && s_row0[k + 1] <= lane) ++k;
                        const Tile t = tiles[k];
                        slab_row<SLAB_ROWS>(slots[t_slot[k]], t.a0 + (lane - s_row0[k]), t, lane, slab);
                    }
                    __syncthreads();
                }
                if constexpr (QCAP > 0 && !SLAB) {
                    // the batch's D columns (used entries) zeroed by all lanes
                    // at once, two entries a lane per store
                    double2* Z = reinterpret_cast<double2*>(Dbuf);
                    for (int i = lane; 2 * i < used; i += kWave) Z[i] = make_double2(0.0, 0.0);
                    wave_lds_sync();
                }
                if constexpr (QCAP > 0) {
                    // Phase 1 for every window of the batch, the pieces of all
                    // columns walked 64 at a time; phase 2 follows once the
                    // ring is empty.
                    int head = 0, count = 0;
                    for (int64_t base = 0; base < total; base += kWave) {
                        const int64_t idx = base + lane;
                        const bool valid = idx < total;
                        int lo = 0, r = 0;
                        if (valid) locate(idx, lo, r);
                        const Tile t = tiles[lo];
                        const CTet& S = slots[t_slot[lo]];
                        const int wb = t.tb + t.hb;
                        const int qa = fdivi(r, t.inv_wb);
                        const int a = t.a0 - t.ha + qa;
                        const int b = t.b0 - t.hb + (r - qa * wb);
                        if constexpr (SLAB)
                            column_slab<WORK, QCAP, SLAB_ROWS>(valid, S, b, t, lo, s_row0[lo] + qa,
                                                               t.doff + r * t.tl, Dbuf, slab, ring,
                                                               head, count, tiles, wc);
                        else
                            column_queue<WORK, QCAP>(valid, S, a, b, t, lo, t.doff + r * t.tl, Dbuf,
                                                     ring, head, count, tiles, wc);
                        if (valid) {
                            ++n_col;
                            if constexpr (WORK) n_colcell += (unsigned long long)t.tl;
                        }
                    }
                    while (count > 0)
                        drain_round<WORK, QCAP, DT>(ring, head, count, tiles, Dbuf, wc, SLAB);
                    __syncthreads();
                }
                if constexpr (QCAP == 0) {
                    // phase 1 for every window of the batch first: the columns
                    // that take the x complement need the last row's
                    for (int64_t base = 0; base < total; base += kWave) {
                        const int64_t idx = base + lane;
                        if (idx < total) {
                            int lo = 0, r = 0;
                            locate(idx, lo, r);
                            const Tile t = tiles[lo];
                            const CTet& S = slots[t_slot[lo]];
                            const int wb = t.tb + t.hb;
                            const int qa = fdivi(r, t.inv_wb);
                            const int a = t.a0 - t.ha + qa;
                            const int b = t.b0 - t.hb + (r - qa * wb);
                            if constexpr (!SLAB) column<WORK>(S, a, b, t, Dbuf + t.doff + r * t.tl, wc);
                            ++n_col;
                            if constexpr (WORK) n_colcell += (unsigned long long)t.tl;
                        }
                    }
                    __syncthreads();
                }
                for (int64_t base = 0; base < total; base += kWave) {
                    const int64_t idx = base + lane;
                    int lo = 0, r = 0;
                    if (idx < total) locate(idx, lo, r);
                    // Phase 2: the cells (i, j, l) of this lane's column, l
                    // walking the tile's levels; halo columns have no cells.
                    if (idx < total) {
                        const Tile t = tiles[lo];
                        const CTet& S = slots[t_slot[lo]];
                        const int wb = t.tb + t.hb;
                        const int ca = fdivi(r, t.inv_wb), cb = r - ca * wb;
                        const int i = ca - t.ha, j = cb - t.hb;
                        if (i >= 0 && j >= 0) {
                            // the slab form holds the cells' own volumes: no differences
                            const bool has_a = !SLAB && (t.a0 + i) > 0, has_b = !SLAB && (t.b0 + j) > 0;
                            // the lower neighbours' columns; an absent one is read
                            // from this column and weighted by 0, which gives
                            // (d11 - d01) - (d10 - d00) with that term 0, bit for bit
                            const DT* D11 = Dbuf + t.doff + r * t.tl;
                            const DT* D01 = has_a ? D11 - wb * t.tl : D11;
                            const DT* D10 = has_b ? D11 - t.tl : D11;
                            const DT* D00 = (has_a && has_b) ? D11 - (wb + 1) * t.tl : D11;
                            const double ma = has_a ? 1.0 : 0.0, mb = has_b ? 1.0 : 0.0;
                            const double mab = ma * mb;
                            // Rows that took the x complement hold D minus the last
                            // row's column: across a row where that starts (ce = 1)
                            // or ends (ce = -1, the last row) the difference also
                            // carries the last row's own y difference E(b) - E(b-1).
                            double ce = 0.0;
                            const DT* E1 = D11;
                            const DT* E0 = D11;
                            if constexpr (XCMP) {
                                const int a = t.a0 + i;
                                const bool c1 = x_complement(S, t, a);
                                const bool c0 = a > 0 && x_complement(S, t, a - 1);
                                ce = (c1 ? 1.0 : 0.0) - (c0 ? 1.0 : 0.0);
                                E1 = Dbuf + t.doff + ((t.ta + t.ha - 1) * wb + cb) * t.tl;
                                E0 = has_b ? E1 - t.tl : E1;
                            }
                            auto volume = [&](int l) {
                                double V = fma(-ma, (double)D01[l], (double)D11[l]) -
                                           fma(-mab, (double)D00[l], mb * (double)D10[l]);
                                if constexpr (XCMP) V = fma(ce, fma(-mb, (double)E0[l], (double)E1[l]), V);
                                return V;
                            };
                            // grid cell of level 0, and the grid axis the levels walk
                            const int o0 = t.a0 + i, o1 = t.b0 + j, o2 = t.l0;
                            const int k0 = walk_axis(S, 0), k1 = walk_axis(S, 1), k2 = walk_axis(S, 2);
                            const int gx = wrap_add(S.lo[0], k0 == 0 ? o0 : (k1 == 0 ? o1 : o2), P.nc[0]);
                            const int gy = wrap_add(S.lo[1], k0 == 1 ? o0 : (k1 == 1 ? o1 : o2), P.nc[1]);
                            const int gz = wrap_add(S.lo[2], k0 == 2 ? o0 : (k1 == 2 ? o1 : o2), P.nc[2]);
                            const int gw = k2 == 0 ? gx : (k2 == 1 ? gy : gz);
                            const int nw = k2 == 0 ? P.nc[0] : (k2 == 1 ? P.nc[1] : P.nc[2]);
                            n_pair += t.tl;
                            // in the group tile: level 0's cell and the walk axis' stride
                            int li = 0, lstep = 0;
                            if (AGG && tiled) {
                                int lc[3];
#pragma unroll
                                for (int c = 0; c < 3; ++c) {
                                    const int nca = P.nc[c];
                                    int d = S.lo[c] - gref[c];
                                    if (2 * d > nca) d -= nca;
                                    else if (2 * d < -nca) d += nca;
                                    lc[c] = d - gmn[c] + (k0 == c ? o0 : (k1 == c ? o1 : o2));
                                }
                                li = (lc[0] * gE[1] + lc[1]) * gE[2] + lc[2];
                                lstep = k2 == 0 ? gE[1] * gE[2] : (k2 == 1 ? gE[2] : 1);
                            }
                            // the cell's mass: (d11 - d01) - (d10 - d00); differences of
                            // values up to 1 carry ~1e-16 noise, which is dropped
                            if (!P.leaf_map) {
                                // plain grid: the element of level 0, then one stride of
                                // the walk axis per level; the levels from lw on lie
                                // past the periodic wrap, nw strides back (a second
                                // loop, empty for nearly every column)
                                const int64_t step = k2 == 0 ? (int64_t)P.nc[1] * P.nc[2]
                                                             : (k2 == 1 ? (int64_t)P.nc[2] : 1);
                                OutT* po = out + ((int64_t)gx * P.nc[1] + gy) * P.nc[2] + gz;
                                auto cell = [&](int l) {
                                    const double V = volume(l);
                                    if (V > 4e-15) {
                                        ++n_nz;
                                        const double mass = P.m * V;
                                        if (AGG && tiled) lds_add(acc + li, (OutT)(mass * P.out_scale));
                                        else global_add(po, (OutT)(mass * P.out_scale));
                                        macc += mass;
                                    }
                                    li += lstep;
                                    po += step;
                                };
                                const int lw = min(t.tl, nw - gw);
                                int l = 0;
                                for (; l + 1 < lw; l += 2) {  // pairs: one ds_read2 per D column
                                    cell(l);
                                    cell(l + 1);
                                }
                                if (l < lw) cell(l);
                                po -= step * nw;
                                for (int l = lw; l < t.tl; ++l) cell(l);
                            } else if constexpr (CAP <= 960) {
                                // octree level (the instances for small tets): the node
                                // and in-leaf offset of level 0, then one cell of the
                                // walk axis per level; the leaf map is read again where
                                // the walk enters the next node
                                const int B = P.leaf_block, side = P.leaf_side;
                                const int cx = gx / B, cy = gy / B, cz = gz / B;
                                const int rx = gx - cx * B, ry = gy - cy * B, rz = gz - cz * B;
                                int off = (rx * B + ry) * B + rz;  // < B^3 <= 2^30
                                int node = (cx * side + cy) * side + cz;
                                const int ostep = k2 == 0 ? B * B : (k2 == 1 ? B : 1);
                                const int nstep = k2 == 0 ? side * side : (k2 == 1 ? side : 1);
                                int rw = k2 == 0 ? rx : (k2 == 1 ? ry : rz);
                                int qw = k2 == 0 ? cx : (k2 == 1 ? cy : cz);
                                int leaf = global_view(P.leaf_map)[node];
                                for (int l = 0; l < t.tl; ++l) {
                                    const double V = volume(l);
                                    if (V > 4e-15 && leaf >= 0) {
                                        ++n_nz;
                                        const double mass = P.m * V;
                                        if (AGG && tiled) lds_add(acc + li, (OutT)(mass * P.out_scale));
                                        else global_add(out + ((int64_t)leaf * B * B * B + off),
                                                        (OutT)(mass * P.out_scale));
                                        macc += mass;
                                    }
                                    li += lstep;
                                    off += ostep;
                                    if (++rw == B) {
                                        rw = 0;
                                        off -= B * ostep;
                                        node += nstep;
                                        if (++qw == side) {
                                            qw = 0;
                                            node -= side * nstep;
                                        }
                                        leaf = global_view(P.leaf_map)[node];
                                    }
                                }
                            } else {
                                // octree level (large-tet instances, which have no
                                // registers to spare): each non-zero cell mapped alone
                                for (int l = 0; l < t.tl; ++l) {
                                    const double V = volume(l);
                                    if (V > 4e-15) {
                                        const int w = wrap_add(gw, l, nw);
                                        const int64_t gi = out_index(P, k2 == 0 ? w : gx,
                                                                     k2 == 1 ? w : gy, k2 == 2 ? w : gz);
                                        if (gi >= 0) {
                                            ++n_nz;
                                            const double mass = P.m * V;
                                            global_add(out + gi, (OutT)(mass * P.out_scale));
                                            macc += mass;
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();
        if constexpr (AGG) {
            if (tiled) {
                // the group tile to the grid: one atomic per non-zero cell.
                // Cell i of the tile is (i / (E1 E2), i / E2 mod E1, i mod E2)
                // and its grid cell (base + that) mod nc, base the tile's
                // origin wrapped once; every quotient has a numerator below
                // 2^21 (i < 192, base + offset < nc + 192 with nc <= 2^20), so it
                // comes from a float reciprocal (fdivi), not an integer division.
                const int ncells = gE[0] * gE[1] * gE[2];
                const int e12 = gE[1] * gE[2];
                const float inv12 = __builtin_amdgcn_rcpf((float)e12);
                const float inv2 = __builtin_amdgcn_rcpf((float)gE[2]);
                int base[3];
                float invn[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int nca = P.nc[c];
                    const int x = (gref[c] + gmn[c]) % nca;
                    base[c] = x < 0 ? x + nca : x;
                    invn[c] = __builtin_amdgcn_rcpf((float)nca);
                }
                for (int i = lane; i < ncells; i += kWave) {
                    const OutT v = acc[i];
                    if (v == OutT(0)) continue;
                    const int q0 = fdivi(i, inv12), r0 = i - q0 * e12;
                    const int q1 = fdivi(r0, inv2);
                    const int li[3] = {q0, q1, r0 - q1 * gE[2]};
                    int g3[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int x = base[c] + li[c];
                        g3[c] = x - fdivi(x, invn[c]) * P.nc[c];
                    }
                    const int64_t idx = out_index(P, g3[0], g3[1], g3[2]);
                    if (idx >= 0) global_add(out + idx, v);
                }
                __syncthreads();
            }
        }
        }
    }
    if (cur_box >= 0) flush_mass(P, macc);

#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        n_tet += __shfl_xor(n_tet, off, kWave);
        n_pair += __shfl_xor(n_pair, off, kWave);
        n_col += __shfl_xor(n_col, off, kWave);
        if constexpr (WORK) {
            wc.xpiece += __shfl_xor(wc.xpiece, off, kWave);
            wc.piece += __shfl_xor(wc.piece, off, kWave);
            wc.level += __shfl_xor(wc.level, off, kWave);
            n_colcell += __shfl_xor(n_colcell, off, kWave);
        }
        n_nz += __shfl_xor(n_nz, off, kWave);
        n_inv += __shfl_xor(n_inv, off, kWave);
        n_deg += __shfl_xor(n_deg, off, kWave);
    }
    if (lane == 0 && Q.stats) {
        atomicAdd(Q.stats + 0, n_tet);
        atomicAdd(Q.stats + 1, n_pair);
        atomicAdd(Q.stats + 2, n_col);
        if constexpr (WORK) {
            atomicAdd(Q.stats + 8, wc.xpiece);
            atomicAdd(Q.stats + 9, wc.piece);
            atomicAdd(Q.stats + 10, wc.level);
            atomicAdd(Q.stats + 11, n_colcell);
        }
        atomicAdd(Q.stats + 3, n_nz);
        atomicAdd(Q.stats + 4, n_inv);
        atomicAdd(Q.stats + 5, n_deg);
    }
}

// ---------------------------------------------------------------------------
// Ordering by estimated cost: the number of bbox cells of a chunk's
// tetrahedra, bucketed by its base-2 logarithm; buckets run from the most to
// the least expensive so that the longest chunks start first.
// ---------------------------------------------------------------------------

constexpr int kBuckets = 64;

__global__ __launch_bounds__(kWave) void chunk_cost_kernel(QueueArgs Q, int* bucket,
                                                           unsigned long long* hist)
{
    const int64_t g = blockIdx.x;
    if (g >= Q.n_chunks) return;
    const BoxDesc P = Q.boxes ? Q.boxes[box_of(Q, g)] : Q.box0;
    const int64_t tid = (g - P.chunk_begin) * kWave + threadIdx.x;
    unsigned long long cells = 0;
    if (tid < P.ntet) {
        const int64_t cube = tid / 6;
        const int p = (int)(tid - cube * 6);
        const int64_t kk = cube % P.np[2];
        const int64_t jj = (cube / P.np[2]) % P.np[1];
        const int64_t ii = cube / ((int64_t)P.np[1] * P.np[2]);
        Tet64 T;
        make_tet(P.pos, P.np[0], P.np[1], P.np[2], P.scale, P.nc, ii, jj, kk, p, T);
        if (isfinite(T.D) && isfinite(T.l3)) {
            unsigned long long n = 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double mn = fmin(fmin(T.v[0][c], T.v[1][c]), fmin(T.v[2][c], T.v[3][c]));
                const double mx = fmax(fmax(T.v[0][c], T.v[1][c]), fmax(T.v[2][c], T.v[3][c]));
                n *= (unsigned long long)(floor(mx) - floor(mn) + 1.0);
            }
            cells = n;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) cells += __shfl_xor(cells, off, kWave);
    if (threadIdx.x == 0) {
        const int b = cells ? min(kBuckets - 1, 63 - __builtin_clzll(cells)) : 0;
        bucket[g] = b;
        atomicAdd(hist + b, 1ull);
    }
}

// Exclusive offsets of the buckets, most expensive first (one wavefront).
__global__ __launch_bounds__(kWave) void bucket_offsets_kernel(unsigned long long* hist,
                                                               unsigned long long* cursor)
{
    const int lane = threadIdx.x;
    const int b = kBuckets - 1 - lane;  // descending cost
    unsigned long long v = hist[b];
    unsigned long long incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned long long y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += y;
    }
    cursor[b] = incl - v;
}

__global__ void scatter_order_kernel(QueueArgs Q, const int* bucket, unsigned long long* cursor,
                                     int64_t* order)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= Q.n_chunks) return;
    const unsigned long long at = atomicAdd(cursor + bucket[g], 1ull);
    order[at] = g;
}

template <typename T>
__global__ void zero_kernel(T* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

struct QueueLayout {
    size_t next, boxes, bucket, hist, cursor, order, bytes;
};

QueueLayout queue_layout(int64_t n_chunks, int n_boxes, bool ordered)
{
    QueueLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    L.next = take(sizeof(unsigned long long));
    L.boxes = take(n_boxes > 1 ? sizeof(BoxDesc) * (size_t)n_boxes : 0);
    L.bucket = take(ordered ? sizeof(int) * (size_t)n_chunks : 0);
    L.hist = take(ordered ? sizeof(unsigned long long) * kBuckets : 0);
    L.cursor = take(ordered ? sizeof(unsigned long long) * kBuckets : 0);
    L.order = take(ordered ? sizeof(int64_t) * (size_t)n_chunks : 0);
    L.bytes = off;
    return L;
}

// Kernel instances by buffer size: (entries, tets per group, tiles per
// batch), plain or counting the walk's work events.
template <typename OutT, bool WORK>
const void* queue_kernel_for(int cap)
{
    if (cap <= 512) return reinterpret_cast<const void*>(&queue_kernel<OutT, 512, 16, 16, WORK, 0>);
    if (cap <= 960) return reinterpret_cast<const void*>(&queue_kernel<OutT, 960, 32, 16, WORK, 0>);
    if (cap <= 1024) return reinterpret_cast<const void*>(&queue_kernel<OutT, 1024, 8, 8, WORK, 128>);
    if (cap <= 1408) return reinterpret_cast<const void*>(&queue_kernel<OutT, 1408, 8, 8, WORK, 0>);
    return reinterpret_cast<const void*>(&queue_kernel<OutT, 2048, 32, 32, WORK, 0>);
}

// The slab form (PSD_METHOD_SLAB): 2048 FP32 entries, 16 tile rows a batch,
// 8-tet groups, 128-leaf ring; FP32 grids only, no work counters.
const void* slab_kernel() { return reinterpret_cast<const void*>(&queue_kernel<float, 2048, 8, 8, false, 128, true>); }

template <typename OutT, bool WORK>
hipError_t launch_queue_kernel(const QueueArgs& Q, int cap, bool slab, int grid, hipStream_t stream)
{
    const void* k = slab ? slab_kernel() : queue_kernel_for<OutT, WORK>(cap);
    hipLaunchKernelGGL(reinterpret_cast<void (*)(QueueArgs)>(const_cast<void*>(k)), dim3(grid), dim3(kWave),
                       0, stream, Q);
    return hipGetLastError();
}

}  // namespace

Tuning default_tuning()
{
    Tuning t;
    t.cap = 0;           // chosen from the boxes (auto_cap)
    t.waves_per_cu = 0;  // as many as fit a compute unit
    t.ordered = 0;
    t.work_counters = 0;
    t.slab = 0;
    return t;
}

int auto_cap(const BoxDesc* boxes, int n_boxes)
{
    // Grid cells per Lagrangian spacing: from about 1.5 on, tetrahedra span
    // hundreds of cells and a few of them fill the buffer; octree levels
    // always hold small ones.
    double ratio = 1e30;
    for (int b = 0; b < n_boxes; ++b) {
        if (boxes[b].leaf_map) return 960;
        for (int a = 0; a < 3; ++a)
            ratio = fmin(ratio, (double)boxes[b].nc[a] / (double)boxes[b].np[a]);
    }
    return ratio >= 1.5 ? 1024 : 960;
}

hipError_t queue_resident_waves(int cap, bool out_fp64, int& waves, bool work, bool slab)
{
    if (slab) {
        static std::atomic<int> known_slab{0};
        int n = known_slab.load(std::memory_order_relaxed);
        if (n == 0) {
            const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, slab_kernel(), kWave, 0);
            if (e != hipSuccess) return e;
            if (n < 1) n = 1;
            known_slab.store(n, std::memory_order_relaxed);
        }
        waves = n;
        return hipSuccess;
    }
    // one kernel instance per (buffer size, output type, counters); the
    // answer only depends on the instance, so it is asked once
    static std::atomic<int> known[5][2][2];
    const int ci = cap <= 512 ? 0 : (cap <= 960 ? 1 : (cap <= 1024 ? 2 : (cap <= 1408 ? 3 : 4)));
    const int ti = out_fp64 ? 1 : 0;
    const int wi = work ? 1 : 0;
    int n = known[ci][ti][wi].load(std::memory_order_relaxed);
    if (n == 0) {
        const void* k = out_fp64 ? (work ? queue_kernel_for<double, true>(cap)
                                         : queue_kernel_for<double, false>(cap))
                                 : (work ? queue_kernel_for<float, true>(cap)
                                         : queue_kernel_for<float, false>(cap));
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kWave, 0);
        if (e != hipSuccess) return e;
        if (n < 1) n = 1;
        known[ci][ti][wi].store(n, std::memory_order_relaxed);
    }
    waves = n;
    return hipSuccess;
}

size_t queue_workspace_bytes(int64_t n_chunks, int n_boxes, bool ordered)
{
    return queue_layout(n_chunks, n_boxes, ordered).bytes;
}

int64_t queue_chunks(const BoxDesc* boxes, int n_boxes)
{
    int64_t n = 0;
    for (int b = 0; b < n_boxes; ++b) n += (boxes[b].ntet + kWave - 1) / kWave;
    return n;
}

hipError_t launch_queue(const BoxDesc* boxes_in, int n_boxes, bool out_fp64, const Tuning& tune,
                        void* ws, size_t ws_bytes, unsigned long long* stats, hipStream_t stream)
{
    if (n_boxes < 1) return hipErrorInvalidValue;
    // a plain grid or an octree's levels fit the local table: no host
    // allocation on those paths
    BoxDesc local[8];
    std::vector<BoxDesc> many;
    BoxDesc* boxes = local;
    if (n_boxes > 8) {
        many.assign(boxes_in, boxes_in + n_boxes);
        boxes = many.data();
    } else {
        for (int b = 0; b < n_boxes; ++b) local[b] = boxes_in[b];
    }
    int64_t n_chunks = 0;
    for (int b = 0; b < n_boxes; ++b) {
        boxes[b].chunk_begin = n_chunks;
        n_chunks += (boxes[b].ntet + kWave - 1) / kWave;
    }
    const bool ordered = tune.ordered != 0;
    const QueueLayout L = queue_layout(n_chunks, n_boxes, ordered);
    if (ws_bytes < L.bytes) return hipErrorInvalidValue;
    char* base = reinterpret_cast<char*>(ws);
    QueueArgs Q;
    memset(&Q, 0, sizeof(Q));
    Q.box0 = boxes[0];
    Q.n_boxes = n_boxes;
    Q.n_chunks = n_chunks;
    Q.next = reinterpret_cast<unsigned long long*>(base + L.next);
    Q.stats = stats;
    hipError_t e;
    if (n_boxes > 1) {
        e = hipMemcpyAsync(base + L.boxes, boxes, sizeof(BoxDesc) * (size_t)n_boxes,
                           hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
        Q.boxes = reinterpret_cast<const BoxDesc*>(base + L.boxes);
    }
    hipLaunchKernelGGL(zero_kernel<unsigned long long>, dim3(1), dim3(64), 0, stream, Q.next,
                       (int64_t)1);
    if (n_chunks == 0) return hipGetLastError();
    if (ordered) {
        int* bucket = reinterpret_cast<int*>(base + L.bucket);
        unsigned long long* hist = reinterpret_cast<unsigned long long*>(base + L.hist);
        unsigned long long* cursor = reinterpret_cast<unsigned long long*>(base + L.cursor);
        int64_t* order = reinterpret_cast<int64_t*>(base + L.order);
        hipLaunchKernelGGL(zero_kernel<unsigned long long>, dim3(1), dim3(64), 0, stream, hist,
                           (int64_t)kBuckets);
        hipLaunchKernelGGL(chunk_cost_kernel, dim3((unsigned)n_chunks), dim3(kWave), 0, stream, Q,
                           bucket, hist);
        hipLaunchKernelGGL(bucket_offsets_kernel, dim3(1), dim3(kWave), 0, stream, hist, cursor);
        hipLaunchKernelGGL(scatter_order_kernel, dim3((unsigned)((n_chunks + 255) / 256)), dim3(256),
                           0, stream, Q, (const int*)bucket, cursor, order);
        Q.order = order;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    const int cap = tune.cap > 0 ? tune.cap : auto_cap(boxes, n_boxes);
    const bool slab = tune.slab != 0;
    if (slab && out_fp64) return hipErrorInvalidValue;  // the slab form writes FP32 grids
    const bool work = tune.work_counters != 0 && stats != nullptr && !slab;
    int waves = tune.waves_per_cu;
    if (waves <= 0) {
        const hipError_t e = queue_resident_waves(cap, out_fp64, waves, work, slab);
        if (e != hipSuccess) return e;
    }
    int64_t grid = (int64_t)cus * waves;
    if (grid > n_chunks) grid = n_chunks;
    if (grid < 1) grid = 1;
    if (work)
        return out_fp64 ? launch_queue_kernel<double, true>(Q, cap, slab, (int)grid, stream)
                        : launch_queue_kernel<float, true>(Q, cap, slab, (int)grid, stream);
    return out_fp64 ? launch_queue_kernel<double, false>(Q, cap, slab, (int)grid, stream)
                    : launch_queue_kernel<float, false>(Q, cap, slab, (int)grid, stream);
}

}  // namespace psd
