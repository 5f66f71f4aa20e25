// psd_device.h -- device building blocks of the deposition kernels (gfx950).
//
// Tetrahedron generation (Section 2: six tetrahedra per Lagrangian cube) and
// the exact tetrahedron/cell intersection (Section 6.3: iterative splitting
// against planes with a table indexed by the inside-vertex mask).
//
// The splitting here tracks, for every sub-tetrahedron, only what later
// planes need: its four vertices' attributes (cell-local coordinates, or
// signed distances to the remaining planes) and its volume as a fraction of
// the root.  When a plane cuts a tetrahedron at parameters t along its edges,
// each piece's volume fraction is a product of t and (1 - t) factors, so no
// determinant is ever formed and nothing cancels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psd {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R sel4(R a0, R a1, R a2, R a3, int i)
{
    R lo = (i & 1) ? a1 : a0;
    R hi = (i & 1) ? a3 : a2;
    return (i & 2) ? hi : lo;
}

// Global-memory views of generic pointers: loads and atomics through them
// compile to global instructions rather than flat ones, which the hardware
// also counts as LDS accesses (every wait on the wavefront's LDS reads then
// waits for them too).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_view(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void global_add(T* p, T v)
{
    __hip_atomic_fetch_add((__attribute__((address_space(1))) T*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// A cell index of an unwrapped tetrahedron (an integer-valued double in
// [-n, 2n): its vertices lie within half a box of corner 0, which is in
// [0, n)) wrapped into [0, n) without a division.
__device__ __forceinline__ int wrap_index(double x, int n)
{
    const int i = (int)x;
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Quotient a / b for b > 0 with a few ulps of error (the FP64 reciprocal
// estimate refined by one Newton step, which doubles its correct bits).
__device__ __forceinline__ float fdiv_pos(float a, float b)
{
    return a * __builtin_amdgcn_rcpf(b);
}
__device__ __forceinline__ double fdiv_pos(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    return a * r;
}

// Edge parameter of a cut from an inside end (value i >= 0) toward an outside
// end (value o < 0); 0 for pairs that are not a valid cut.
template <typename R>
__device__ __forceinline__ R cut_t(R i, R o)
{
    R den = i - o;
    return den > R(0) ? fdiv_pos(i, den) : R(0);
}

// For an inside-vertex mask (bit v set when vertex v is inside), the vertex
// order with the inside vertices first, then the outside ones, ascending
// within each group; 2 bits per index, 8 bits per mask.
constexpr uint64_t perm_word(int first)
{
    uint64_t w = 0;
    for (int m = first; m < first + 8; ++m) {
        int order[4] = {0, 0, 0, 0}, n = 0;
        for (int v = 0; v < 4; ++v)
            if ((m >> v) & 1) order[n++] = v;
        for (int v = 0; v < 4; ++v)
            if (!((m >> v) & 1)) order[n++] = v;
        uint64_t code = (uint64_t)(order[0] | (order[1] << 2) | (order[2] << 4) | (order[3] << 6));
        w |= code << (8 * (m - first));
    }
    return w;
}

__device__ __forceinline__ uint32_t perm_code(int mask)
{
    constexpr uint64_t lo = perm_word(0);
    constexpr uint64_t hi = perm_word(8);
    uint64_t w = (mask & 8) ? hi : lo;
    return (uint32_t)(w >> ((mask & 7) * 8)) & 0xFFu;
}

// ---------------------------------------------------------------------------
// One split of a tetrahedron by a plane.
//
// With the vertices ordered (a, b, c, d), inside ones first, the inside part is
//   1 inside : the tet (a, p_ab, p_ac, p_ad)
//   2 inside : the prism (a, p_ac, p_ad) / (b, p_bc, p_bd)
//   3 inside : the prism (a, b, c) / (p_ad, p_bd, p_cd)
//   4 inside : the tet itself
// where p_xy is the cut point on edge xy at parameter t_xy from x.  A prism
// (u0,u1,u2)/(w0,w1,w2) with lateral edges u_i w_i is cut into the three
// tetrahedra (u0,u1,u2,w2), (u0,u1,w1,w2), (u0,w0,w1,w2), whose volume
// fractions of the parent are (barycentric determinants):
//   2 inside : t_ac t_ad (1 - t_bd),  t_ac (1 - t_bc) t_bd,  t_bc t_bd
//   3 inside : t_cd,  t_bd (1 - t_cd),  t_ad (1 - t_bd)(1 - t_cd)
//   1 inside : t_ab t_ac t_ad        4 inside : 1
// Cut slots: 1 inside (ab, ac, ad); 2 inside (ac, ad, bc, bd);
// 3 inside (ad, bd, cd).
// ---------------------------------------------------------------------------

template <typename R>
struct Split {
    int nin;
    int ia, ib, ic, id;
    R t0, t1, t2, t3;
    R f0, f1, f2;
};

// Cut parameters and piece fractions from the plane values of the ordered
// vertices (inside ones first).
template <typename R>
__device__ __forceinline__ void split_ordered(R da, R db, R dc, R dd, int nin, Split<R>& s)
{
    bool n1 = nin == 1, n2 = nin == 2, n3 = nin == 3;
    R i0 = da, o0 = n1 ? db : (n2 ? dc : dd);
    R i1 = n3 ? db : da, o1 = n1 ? dc : dd;
    R i2 = n1 ? da : (n2 ? db : dc), o2 = n2 ? dc : dd;
    s.t0 = cut_t(i0, o0);
    s.t1 = cut_t(i1, o1);
    s.t2 = cut_t(i2, o2);
    s.t3 = cut_t(db, dd);
    const R one = R(1);
    R f0, f1 = R(0), f2 = R(0);
    if (n1) {
        f0 = s.t0 * s.t1 * s.t2;
    } else if (n2) {
        f0 = s.t0 * s.t1 * (one - s.t3);
        f1 = s.t0 * (one - s.t2) * s.t3;
        f2 = s.t2 * s.t3;
    } else if (n3) {
        f0 = s.t2;
        f1 = s.t1 * (one - s.t2);
        f2 = s.t0 * (one - s.t1) * (one - s.t2);
    } else {
        f0 = nin == 4 ? one : R(0);
    }
    s.f0 = f0;
    s.f1 = f1;
    s.f2 = f2;
}

template <typename R>
__device__ __forceinline__ void split_plane(const R d[4], Split<R>& s)
{
    int mask = (d[0] >= R(0) ? 1 : 0) | (d[1] >= R(0) ? 2 : 0) | (d[2] >= R(0) ? 4 : 0) |
               (d[3] >= R(0) ? 8 : 0);
    int nin = __builtin_popcount(mask);
    uint32_t pc = perm_code(mask);
    s.nin = nin;
    s.ia = pc & 3;
    s.ib = (pc >> 2) & 3;
    s.ic = (pc >> 4) & 3;
    s.id = (pc >> 6) & 3;
    split_ordered(sel4(d[0], d[1], d[2], d[3], s.ia), sel4(d[0], d[1], d[2], d[3], s.ib),
                  sel4(d[0], d[1], d[2], d[3], s.ic), sel4(d[0], d[1], d[2], d[3], s.id), nin, s);
}

// The same split when the plane values do not increase with the vertex
// index (d[0] >= d[1] >= d[2] >= d[3]): the inside vertices are a prefix,
// already in the order above, so the permutation is the identity.
template <typename R>
__device__ __forceinline__ void split_prefix(const R d[4], Split<R>& s)
{
    const int nin = (d[0] >= R(0) ? 1 : 0) + (d[1] >= R(0) ? 1 : 0) + (d[2] >= R(0) ? 1 : 0) +
                    (d[3] >= R(0) ? 1 : 0);
    s.nin = nin;
    s.ia = 0;
    s.ib = 1;
    s.ic = 2;
    s.id = 3;
    split_ordered(d[0], d[1], d[2], d[3], nin, s);
}

// Plane evaluators.  Planes are compacted per lane so that the k planes that
// actually cut the root come first; level L of the search splits by plane L
// and the last active plane only contributes the inside fraction.
//
// Cell frame: attributes are the vertices' signed distances to the (compacted)
// face planes of the tetrahedron; plane L is attribute L.
template <typename R>
struct CellEval {
    static constexpr int A = 4;
    template <int L>
    __device__ __forceinline__ R dist(const R (&v)[4]) const { return v[L]; }
};

// Tet frame: attributes are cell-local coordinates; plane slot L is
// off[L] + sgn[L] * coordinate[axis[L]] (x>=0: 0 + x, x<=1: 1 - x, ...).
template <typename R>
struct TetEval {
    static constexpr int A = 3;
    int axis[6];
    R sgn[6], off[6];
    template <int L>
    __device__ __forceinline__ R dist(const R (&v)[3]) const
    {
        R c = axis[L] == 0 ? v[0] : (axis[L] == 1 ? v[1] : v[2]);
        return off[L] + sgn[L] * c;
    }
};

// Volume fraction of the tetrahedron with vertex attributes v that lies
// inside the first k planes (k >= 1), starting at level L.  Depth-first over
// the table's pieces; each level is instantiated once, so code size is linear
// in the number of planes.
template <typename R, int L, int KMAX, typename Ev>
__device__ __forceinline__ R inside_fraction(const R (&v)[4][Ev::A], int k, const Ev& ev)
{
    constexpr int A = Ev::A;
    R d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = ev.template dist<L>(v[q]);
    Split<R> s;
    split_plane(d, s);
    if (s.nin == 0) return R(0);
    if constexpr (L == KMAX - 1) {
        return s.f0 + s.f1 + s.f2;
    } else {
        if (L >= k - 1) return s.f0 + s.f1 + s.f2;
        const bool n1 = s.nin == 1, n2 = s.nin == 2, n3 = s.nin == 3, n4 = s.nin == 4;
        R u0[A], u1[A], u2[A], w0[A], w1[A], w2[A];
#pragma unroll
        for (int a = 0; a < A; ++a) {
            R va = sel4(v[0][a], v[1][a], v[2][a], v[3][a], s.ia);
            R vb = sel4(v[0][a], v[1][a], v[2][a], v[3][a], s.ib);
            R vc = sel4(v[0][a], v[1][a], v[2][a], v[3][a], s.ic);
            R vd = sel4(v[0][a], v[1][a], v[2][a], v[3][a], s.id);
            // cut points (same endpoint pattern as split_plane)
            R in1 = n3 ? vb : va, in2 = n1 ? va : (n2 ? vb : vc);
            R out0 = n1 ? vb : (n2 ? vc : vd), out1 = n1 ? vc : vd, out2 = n2 ? vc : vd;
            R c0 = va + s.t0 * (out0 - va);
            R c1 = in1 + s.t1 * (out1 - in1);
            R c2 = in2 + s.t2 * (out2 - in2);
            R c3 = vb + s.t3 * (vd - vb);
            u0[a] = va;
            u1[a] = (n3 || n4) ? vb : c0;
            u2[a] = (n3 || n4) ? vc : c1;
            w0[a] = n2 ? vb : c0;
            w1[a] = n2 ? c2 : c1;
            w2[a] = n4 ? vd : (n2 ? c3 : c2);
        }
        const int nchild = (n2 || n3) ? 3 : 1;
        R acc = R(0);
        for (int j = 0; j < nchild; ++j) {
            R cv[4][A];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                cv[0][a] = u0[a];
                cv[1][a] = j == 2 ? w0[a] : u1[a];
                cv[2][a] = j == 0 ? u2[a] : w1[a];
                cv[3][a] = w2[a];
            }
            R f = j == 0 ? s.f0 : (j == 1 ? s.f1 : s.f2);
            acc += f * inside_fraction<R, L + 1, KMAX, Ev>(cv, k, ev);
        }
        return acc;
    }
}

// ---------------------------------------------------------------------------
// Lagrangian tetrahedra (Section 2).  Corner index q = 4a + 2b + c of cube
// corner (a,b,c); tetrahedron p of the Freudenthal split (axis permutations
// 012, 021, 102, 120, 201, 210) has corners (0, q1, q2, 7).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int kuhn_q1(int p) { return (0x112244 >> (4 * p)) & 0xF; }
__device__ __forceinline__ int kuhn_q2(int p) { return (0x353656 >> (4 * p)) & 0xF; }
__device__ __forceinline__ int kuhn_sign(int p) { return ((0x19 >> p) & 1) ? 1 : -1; }  // + - - + + -

struct Tet64 {
    double v[4][3];  // unwrapped vertex coordinates, cell units (corner 0 wrapped into [0,nc))
    double D;        // signed determinant det(v1-v0, v2-v0, v3-v0)
    double l3;       // (longest edge)^3
};

// Builds tetrahedron p of cube (i,j,k).  Unwrap: each corner is moved to the
// minimum image of its offset from corner 0 (offsets of exactly half a box
// keep their sign).  Contraction is off so the determinant matches a plain
// evaluation bit for bit.
__device__ __forceinline__ void make_tet(const float* __restrict__ pos, int np0, int np1, int np2,
                                         const double sc[3], const int nc[3], int64_t i,
                                         int64_t j, int64_t k, int p, Tet64& T)
{
#pragma clang fp contract(off)
    int qs[4] = {0, kuhn_q1(p), kuhn_q2(p), 7};
    double c[4][3];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        int q = qs[m];
        int64_t ii = i + ((q >> 2) & 1), jj = j + ((q >> 1) & 1), kk = k + (q & 1);
        if (ii == np0) ii = 0;
        if (jj == np1) jj = 0;
        if (kk == np2) kk = 0;
        const __attribute__((address_space(1))) float* pp =
            global_view(pos) + 3 * ((ii * np1 + jj) * np2 + kk);
        c[m][0] = (double)pp[0] * sc[0];
        c[m][1] = (double)pp[1] * sc[1];
        c[m][2] = (double)pp[2] * sc[2];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double n = (double)nc[a];
        // 1/n to about an ulp (the hardware estimate and two Newton steps)
        // instead of a division per quotient: the quotients only pick integer
        // shifts, a floor that lands corner 0 outside [0, n) (c/n within an ulp
        // of an integer) is corrected to the same value, and the minimum image
        // can differ only for a displacement within an ulp of half the box
        double r = __builtin_amdgcn_rcp(n);
        r = fma(fma(-n, r, 1.0), r, r);
        r = fma(fma(-n, r, 1.0), r, r);
        double c0w = c[0][a] - n * floor(c[0][a] * r);
        c0w = c0w >= n ? c0w - n : (c0w < 0.0 ? c0w + n : c0w);
        T.v[0][a] = c0w;
#pragma unroll
        for (int m = 1; m < 4; ++m) {
            double d = c[m][a] - c[0][a];
            d -= n * rint(d * r);
            T.v[m][a] = c0w + d;
        }
    }
    double e[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int a = 0; a < 3; ++a) e[m][a] = T.v[m + 1][a] - T.v[0][a];
    T.D = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
          e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
          e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    double l2 = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n2 = m + 1; n2 < 4; ++n2) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) s += (T.v[m][a] - T.v[n2][a]) * (T.v[m][a] - T.v[n2][a]);
            l2 = s > l2 ? s : l2;
        }
    T.l3 = l2 * sqrt(l2);
}

}  // namespace psd
