/*
 * psd_oracle.c -- FP64 CPU oracle for phase-space-element density deposition.
 *
 * TEST INFRASTRUCTURE ONLY (see psd_oracle.h for what it computes and who
 * may use it).  Plain loops, double precision, no fast-math.
 */
#include "psd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Convex polytope as a list of outward-oriented face polygons.              */
/* ------------------------------------------------------------------------ */

#define ORC_MAXV 32
#define ORC_MAXF 12

typedef struct {
    int n;
    double p[ORC_MAXV][3];
} orc_face;

typedef struct {
    int nf;
    orc_face f[ORC_MAXF];
} orc_poly;

static double det3(const double a[3], const double b[3], const double c[3])
{
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
}

static double tet_det(const double v[4][3])
{
    double e1[3], e2[3], e3[3];
    for (int a = 0; a < 3; ++a) {
        e1[a] = v[1][a] - v[0][a];
        e2[a] = v[2][a] - v[0][a];
        e3[a] = v[3][a] - v[0][a];
    }
    return det3(e1, e2, e3);
}

/* Faces of a tetrahedron, wound counter-clockwise seen from outside. */
static void poly_from_tet(orc_poly* P, const double v[4][3])
{
    /* For a positively oriented tet these index triples face outward. */
    static const int F[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    int pos = tet_det(v) > 0.0;
    P->nf = 4;
    for (int f = 0; f < 4; ++f) {
        int ids[3] = {F[f][0], pos ? F[f][1] : F[f][2], pos ? F[f][2] : F[f][1]};
        P->f[f].n = 3;
        for (int i = 0; i < 3; ++i)
            for (int a = 0; a < 3; ++a) P->f[f].p[i][a] = v[ids[i]][a];
    }
}

/* Divergence theorem: fan every face from its first vertex, apex r. */
static double poly_volume(const orc_poly* P, const double r[3])
{
    double V = 0.0;
    for (int f = 0; f < P->nf; ++f) {
        const orc_face* F = &P->f[f];
        if (F->n < 3) continue;
        double a[3], b[3], c[3];
        for (int k = 0; k < 3; ++k) a[k] = F->p[0][k] - r[k];
        for (int i = 1; i + 1 < F->n; ++i) {
            for (int k = 0; k < 3; ++k) {
                b[k] = F->p[i][k] - r[k];
                c[k] = F->p[i + 1][k] - r[k];
            }
            V += det3(a, b, c);
        }
    }
    return V / 6.0;
}

static double plane_eval(const double a[3], double b, const double p[3])
{
    return a[0] * p[0] + a[1] * p[1] + a[2] * p[2] + b;
}

static int same_point(const double p[3], const double q[3])
{
    return p[0] == q[0] && p[1] == q[1] && p[2] == q[2];
}

/* Keep the part of `in` where a.x + b >= 0 (A4 reading: on-plane counts as
 * inside; cut points only where the sign changes strictly). */
static void poly_clip(const orc_poly* in, orc_poly* out, const double a[3], double b)
{
    int has_pos = 0, has_neg = 0;
    for (int f = 0; f < in->nf; ++f)
        for (int i = 0; i < in->f[f].n; ++i) {
            double d = plane_eval(a, b, in->f[f].p[i]);
            if (d > 0.0) has_pos = 1;
            if (d < 0.0) has_neg = 1;
        }
    if (!has_neg) {
        if (out != in) *out = *in;
        return;
    }
    if (!has_pos) {
        out->nf = 0;
        return;
    }

    static const int CAPMAX = 4 * ORC_MAXF * ORC_MAXV;
    double cap[4 * ORC_MAXF * ORC_MAXV][3];
    int ncap = 0;
    orc_poly tmp;
    tmp.nf = 0;

    for (int f = 0; f < in->nf; ++f) {
        const orc_face* F = &in->f[f];
        orc_face G;
        G.n = 0;
        for (int i = 0; i < F->n; ++i) {
            const double* P = F->p[i];
            const double* Q = F->p[(i + 1) % F->n];
            double dP = plane_eval(a, b, P);
            double dQ = plane_eval(a, b, Q);
            if (dP >= 0.0) {
                for (int k = 0; k < 3; ++k) G.p[G.n][k] = P[k];
                G.n++;
                if (dP == 0.0 && ncap < CAPMAX) {
                    for (int k = 0; k < 3; ++k) cap[ncap][k] = P[k];
                    ncap++;
                }
            }
            if ((dP > 0.0 && dQ < 0.0) || (dP < 0.0 && dQ > 0.0)) {
                /* Always interpolate from the inside end so that the two faces
                 * sharing this edge produce the identical point. */
                const double* I = dP > 0.0 ? P : Q;
                const double* O = dP > 0.0 ? Q : P;
                double dI = dP > 0.0 ? dP : dQ;
                double dO = dP > 0.0 ? dQ : dP;
                double t = dI / (dI - dO);
                for (int k = 0; k < 3; ++k) G.p[G.n][k] = I[k] + t * (O[k] - I[k]);
                if (ncap < CAPMAX) {
                    for (int k = 0; k < 3; ++k) cap[ncap][k] = G.p[G.n][k];
                    ncap++;
                }
                G.n++;
            }
        }
        if (G.n >= 3) tmp.f[tmp.nf++] = G;
    }

    /* Cap polygon on the plane: unique points sorted by angle, wound so its
     * normal is -a (outward for the kept side). */
    double uq[4 * ORC_MAXF * ORC_MAXV][3];
    int nu = 0;
    for (int i = 0; i < ncap; ++i) {
        int dup = 0;
        for (int j = 0; j < nu && !dup; ++j) dup = same_point(cap[i], uq[j]);
        if (!dup) {
            for (int k = 0; k < 3; ++k) uq[nu][k] = cap[i][k];
            nu++;
        }
    }
    if (nu >= 3 && nu <= ORC_MAXV && tmp.nf < ORC_MAXF) {
        double c[3] = {0, 0, 0};
        for (int i = 0; i < nu; ++i)
            for (int k = 0; k < 3; ++k) c[k] += uq[i][k];
        for (int k = 0; k < 3; ++k) c[k] /= nu;
        double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double n[3] = {-a[0] / na, -a[1] / na, -a[2] / na};
        /* u: unit vector orthogonal to n; w = n x u. */
        int m = 0;
        if (fabs(n[1]) < fabs(n[m])) m = 1;
        if (fabs(n[2]) < fabs(n[m])) m = 2;
        double e[3] = {0, 0, 0};
        e[m] = 1.0;
        double u[3] = {n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2],
                       n[0] * e[1] - n[1] * e[0]};
        double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int k = 0; k < 3; ++k) u[k] /= un;
        double w[3] = {n[1] * u[2] - n[2] * u[1], n[2] * u[0] - n[0] * u[2],
                       n[0] * u[1] - n[1] * u[0]};
        double ang[4 * ORC_MAXF * ORC_MAXV];
        for (int i = 0; i < nu; ++i) {
            double r[3] = {uq[i][0] - c[0], uq[i][1] - c[1], uq[i][2] - c[2]};
            ang[i] = atan2(w[0] * r[0] + w[1] * r[1] + w[2] * r[2],
                           u[0] * r[0] + u[1] * r[1] + u[2] * r[2]);
        }
        for (int i = 1; i < nu; ++i) { /* insertion sort by angle */
            double ak = ang[i], pk[3] = {uq[i][0], uq[i][1], uq[i][2]};
            int j = i - 1;
            while (j >= 0 && ang[j] > ak) {
                ang[j + 1] = ang[j];
                for (int k = 0; k < 3; ++k) uq[j + 1][k] = uq[j][k];
                --j;
            }
            ang[j + 1] = ak;
            for (int k = 0; k < 3; ++k) uq[j + 1][k] = pk[k];
        }
        orc_face* G = &tmp.f[tmp.nf++];
        G->n = nu;
        for (int i = 0; i < nu; ++i)
            for (int k = 0; k < 3; ++k) G->p[i][k] = uq[i][k];
    }
    *out = tmp;
}

double orc_clip_tet_box(const double* v, const double* lo, const double* hi)
{
    /* Work relative to lo: the box becomes [0,w]. */
    double t[4][3], w[3];
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) t[i][k] = v[3 * i + k] - lo[k];
    for (int k = 0; k < 3; ++k) w[k] = hi[k] - lo[k];
    if (tet_det(t) == 0.0) return 0.0;
    orc_poly P, Q;
    poly_from_tet(&P, t);
    for (int k = 0; k < 3; ++k) {
        double a[3] = {0, 0, 0};
        a[k] = 1.0; /* x_k >= 0 */
        poly_clip(&P, &Q, a, 0.0);
        if (Q.nf == 0) return 0.0;
        a[k] = -1.0; /* x_k <= w_k */
        poly_clip(&Q, &P, a, w[k]);
        if (P.nf == 0) return 0.0;
    }
    double r[3] = {0.5 * w[0], 0.5 * w[1], 0.5 * w[2]};
    double V = poly_volume(&P, r);
    return V > 0.0 ? V : 0.0;
}

/* ------------------------------------------------------------------------ */
/* The paper's splitting scheme (Section 6.3), for work counts.              */
/* A tetrahedron is split against one plane at a time; the inside part is    */
/* re-triangulated by the number of inside vertices (0:none, 1:one tet,      */
/* 2:a prism in three tets, 3:a truncated tet in three tets, 4:unchanged).   */
/* x and y planes recurse; the z pair subtracts the outside parts.           */
/* ------------------------------------------------------------------------ */

typedef struct {
    double v[4][3];
} orc_tet;

static double tet_abs_vol(const orc_tet* t)
{
    return fabs(tet_det(t->v)) / 6.0;
}

/* Point on edge (p inside, q outside) where the plane value vanishes. */
static void cut_point(const double p[3], double dp, const double q[3], double dq, double out[3])
{
    double s = dp / (dp - dq);
    for (int k = 0; k < 3; ++k) out[k] = p[k] + s * (q[k] - p[k]);
}

/* Inside part of t for the plane value d_i = sgn * v_i[axis] + off >= 0. */
static int split_inside(const orc_tet* t, int axis, double sgn, double off, orc_tet out[3],
                        int64_t* ncut)
{
    double d[4];
    int in[4], out_[4], ni = 0, no = 0;
    for (int i = 0; i < 4; ++i) {
        d[i] = sgn * t->v[i][axis] + off;
        if (d[i] >= 0.0) in[ni++] = i;
        else out_[no++] = i;
    }
    if (ni == 0) return 0;
    if (ni == 4) {
        out[0] = *t;
        return 1;
    }
    if (ni == 1) {
        int a = in[0];
        double c[3][3];
        for (int j = 0; j < 3; ++j) cut_point(t->v[a], d[a], t->v[out_[j]], d[out_[j]], c[j]);
        *ncut += 3;
        memcpy(out[0].v[0], t->v[a], sizeof(double) * 3);
        for (int j = 0; j < 3; ++j) memcpy(out[0].v[j + 1], c[j], sizeof(double) * 3);
        return 1;
    }
    if (ni == 2) {
        int a = in[0], b = in[1], c = out_[0], e = out_[1];
        double ac[3], ae[3], bc[3], be[3];
        cut_point(t->v[a], d[a], t->v[c], d[c], ac);
        cut_point(t->v[a], d[a], t->v[e], d[e], ae);
        cut_point(t->v[b], d[b], t->v[c], d[c], bc);
        cut_point(t->v[b], d[b], t->v[e], d[e], be);
        *ncut += 4;
        /* prism with ends (a, ac, ae) and (b, bc, be) */
        const double* pr[6] = {t->v[a], ac, ae, t->v[b], bc, be};
        static const int S[3][4] = {{0, 1, 2, 5}, {0, 1, 4, 5}, {0, 3, 4, 5}};
        for (int m = 0; m < 3; ++m)
            for (int j = 0; j < 4; ++j) memcpy(out[m].v[j], pr[S[m][j]], sizeof(double) * 3);
        return 3;
    }
    /* ni == 3: remove the corner at the single outside vertex */
    {
        int a = in[0], b = in[1], c = in[2], e = out_[0];
        double ae[3], be[3], ce[3];
        cut_point(t->v[a], d[a], t->v[e], d[e], ae);
        cut_point(t->v[b], d[b], t->v[e], d[e], be);
        cut_point(t->v[c], d[c], t->v[e], d[e], ce);
        *ncut += 3;
        const double* pr[6] = {t->v[a], t->v[b], t->v[c], ae, be, ce};
        static const int S[3][4] = {{0, 1, 2, 5}, {0, 1, 4, 5}, {0, 3, 4, 5}};
        for (int m = 0; m < 3; ++m)
            for (int j = 0; j < 4; ++j) memcpy(out[m].v[j], pr[S[m][j]], sizeof(double) * 3);
        return 3;
    }
}

/* counts: [0] plane visits, [1] edge cuts, [2] sub-tets */
static double paper_z_part(const orc_tet* t, double wz, int64_t* counts)
{
    double V = tet_abs_vol(t);
    orc_tet part[3];
    /* z <= 0 part */
    counts[0]++;
    int n = split_inside(t, 2, -1.0, 0.0, part, &counts[1]);
    counts[2] += n;
    for (int i = 0; i < n; ++i) V -= tet_abs_vol(&part[i]);
    /* z >= wz part */
    counts[0]++;
    n = split_inside(t, 2, 1.0, -wz, part, &counts[1]);
    counts[2] += n;
    for (int i = 0; i < n; ++i) V -= tet_abs_vol(&part[i]);
    return V;
}

static double paper_dfs(const orc_tet* t, int plane, const double w[3], int64_t* counts)
{
    if (plane == 4) return paper_z_part(t, w[2], counts);
    int axis = plane / 2;
    double sgn = (plane & 1) ? -1.0 : 1.0;
    double off = (plane & 1) ? w[axis] : 0.0;
    counts[0]++;
    orc_tet kids[3];
    int64_t nc = 0;
    int n = split_inside(t, axis, sgn, off, kids, &nc);
    if (n == 1 && nc == 0) return paper_dfs(t, plane + 1, w, counts); /* untouched */
    counts[1] += nc;
    counts[2] += n;
    double V = 0.0;
    for (int i = 0; i < n; ++i) V += paper_dfs(&kids[i], plane + 1, w, counts);
    return V;
}

double orc_clip_tet_box_paper(const double* v, const double* lo, const double* hi,
                              int64_t* counts)
{
    orc_tet t;
    double w[3];
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) t.v[i][k] = v[3 * i + k] - lo[k];
    for (int k = 0; k < 3; ++k) w[k] = hi[k] - lo[k];
    int64_t local[3] = {0, 0, 0};
    double V = paper_dfs(&t, 0, w, counts ? counts : local);
    return V > 0.0 ? V : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Tetrahedra of the Lagrangian grid (Section 2).                            */
/* ------------------------------------------------------------------------ */

/* Axis permutations in lexicographic order, and their parities. */
static const int KUHN[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int KUHN_SIGN[6] = {+1, -1, -1, +1, +1, -1};

static int64_t wrap64(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* Corners of cube (i,j,k) in cell units, unwrapped to the minimum image of
 * each corner relative to corner 000.  corner index = 4a + 2b + c. */
static void cube_corners(const float* pos, const int* np, double box, const int* nc, int64_t i,
                         int64_t j, int64_t k, double c[8][3], int* ambiguous)
{
    double scale[3] = {nc[0] / box, nc[1] / box, nc[2] / box};
    *ambiguous = 0;
    for (int q = 0; q < 8; ++q) {
        int64_t ii = wrap64(i + ((q >> 2) & 1), np[0]);
        int64_t jj = wrap64(j + ((q >> 1) & 1), np[1]);
        int64_t kk = wrap64(k + (q & 1), np[2]);
        const float* p = pos + 3 * ((ii * np[1] + jj) * np[2] + kk);
        for (int a = 0; a < 3; ++a) c[q][a] = (double)p[a] * scale[a];
    }
    for (int q = 1; q < 8; ++q)
        for (int a = 0; a < 3; ++a) {
            double d = c[q][a] - c[0][a];
            d -= nc[a] * rint(d / nc[a]);
            if (fabs(d) > 0.25 * nc[a]) *ambiguous = 1;
            c[q][a] = c[0][a] + d;
        }
}

static void kuhn_tet(const double c[8][3], int p, double v[4][3])
{
    int q0 = 0;
    int q1 = q0 | (4 >> KUHN[p][0]);
    int q2 = q1 | (4 >> KUHN[p][1]);
    int q3 = 7;
    int qs[4] = {q0, q1, q2, q3};
    for (int i = 0; i < 4; ++i)
        for (int a = 0; a < 3; ++a) v[i][a] = c[qs[i]][a];
}

void orc_cube_tets(const float* pos, const int* np, double box, const int* nc, int64_t i,
                   int64_t j, int64_t k, double* tets, double* det)
{
    double c[8][3];
    int amb;
    cube_corners(pos, np, box, nc, i, j, k, c, &amb);
    for (int p = 0; p < 6; ++p) {
        double v[4][3];
        kuhn_tet(c, p, v);
        memcpy(tets + 12 * p, v, sizeof(v));
        if (det) det[p] = tet_det(v);
    }
}

/* ------------------------------------------------------------------------ */
/* Deposit onto a periodic uniform grid.                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const int* nc;
    int rlo[3], rn[3];
    double* out;
    int atomic;
} orc_sink;

static void sink_add(const orc_sink* s, int64_t a, int64_t b, int64_t c, double m)
{
    int64_t ia = wrap64(a, s->nc[0]) - s->rlo[0];
    int64_t ib = wrap64(b, s->nc[1]) - s->rlo[1];
    int64_t ic = wrap64(c, s->nc[2]) - s->rlo[2];
    if (ia < 0 || ia >= s->rn[0] || ib < 0 || ib >= s->rn[1] || ic < 0 || ic >= s->rn[2]) return;
    double* dst = s->out + (ia * s->rn[1] + ib) * s->rn[2] + ic;
    if (s->atomic) {
#pragma omp atomic
        *dst += m;
    } else {
        *dst += m;
    }
}

/* Does the (periodic) integer cell range [lo,hi] along an axis meet the region? */
static int range_hits(int64_t lo, int64_t hi, int n, int rlo, int rn)
{
    if (hi - lo + 1 >= n) return 1;
    for (int64_t a = lo; a <= hi; ++a) {
        int64_t w = wrap64(a, n);
        if (w >= rlo && w < rlo + rn) return 1;
    }
    return 0;
}

/* Inside half-spaces a_f.x + b_f >= 0 of the four faces. */
static void tet_planes(const double v[4][3], double A[4][3], double B[4])
{
    static const int F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int f = 0; f < 4; ++f) {
        const double* p0 = v[F[f][0]];
        const double* p1 = v[F[f][1]];
        const double* p2 = v[F[f][2]];
        double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
        double b = -(n[0] * p0[0] + n[1] * p0[1] + n[2] * p0[2]);
        /* the opposite vertex (index f) must be inside */
        if (n[0] * v[f][0] + n[1] * v[f][1] + n[2] * v[f][2] + b < 0.0) {
            n[0] = -n[0];
            n[1] = -n[1];
            n[2] = -n[2];
            b = -b;
        }
        for (int k = 0; k < 3; ++k) A[f][k] = n[k];
        B[f] = b;
    }
}

/* Deposit one tetrahedron.  Returns nothing; updates sink and counters. */
static void deposit_tet(const double v[4][3], int sign_ref, double m, int mode,
                        const orc_sink* s, orc_counters* cnt)
{
    double D = tet_det(v);
    cnt->n_tet++;
    if (sign_ref * D < 0.0) cnt->n_inverted++;
    double l3 = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j) {
            double e2 = 0.0;
            for (int a = 0; a < 3; ++a) e2 += (v[i][a] - v[j][a]) * (v[i][a] - v[j][a]);
            if (e2 > l3) l3 = e2;
        }
    l3 = l3 * sqrt(l3); /* (max edge length)^3 */
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        double mn = v[0][a], mx = v[0][a];
        for (int i = 1; i < 4; ++i) {
            if (v[i][a] < mn) mn = v[i][a];
            if (v[i][a] > mx) mx = v[i][a];
        }
        lo[a] = (int64_t)floor(mn);
        hi[a] = (int64_t)floor(mx);
    }
    /* Reject early when the bbox misses the output region. */
    for (int a = 0; a < 3; ++a)
        if (!range_hits(lo[a], hi[a], s->nc[a], s->rlo[a], s->rn[a])) {
            /* still count pairs for the whole bbox only if the region is the grid */
            return;
        }
    if (fabs(D) <= 1e-12 * l3) {
        /* zero-volume tetrahedron: all its mass at the centroid's cell */
        cnt->n_degenerate++;
        double g[3];
        for (int a = 0; a < 3; ++a) g[a] = 0.25 * (v[0][a] + v[1][a] + v[2][a] + v[3][a]);
        sink_add(s, (int64_t)floor(g[0]), (int64_t)floor(g[1]), (int64_t)floor(g[2]), m);
        cnt->n_nonzero++;
        return;
    }
    double VT = fabs(D) / 6.0;
    double A[4][3], B[4];
    tet_planes(v, A, B);
    int single = lo[0] == hi[0] && lo[1] == hi[1] && lo[2] == hi[2];
    for (int64_t a = lo[0]; a <= hi[0]; ++a)
        for (int64_t b = lo[1]; b <= hi[1]; ++b)
            for (int64_t c = lo[2]; c <= hi[2]; ++c) {
                cnt->n_pair++;
                double V;
                double clo[3] = {(double)a, (double)b, (double)c};
                double chi[3] = {(double)a + 1, (double)b + 1, (double)c + 1};
                if (mode & ORC_TRIVIAL) {
                    if (single) {
                        V = VT; /* T inside C */
                    } else {
                        int inside_all = 1, separated = 0;
                        for (int f = 0; f < 4 && !separated; ++f) {
                            double mn = 1e300, mx = -1e300;
                            for (int q = 0; q < 8; ++q) {
                                double p[3] = {clo[0] + ((q >> 2) & 1), clo[1] + ((q >> 1) & 1),
                                               clo[2] + (q & 1)};
                                double d = A[f][0] * p[0] + A[f][1] * p[1] + A[f][2] * p[2] + B[f];
                                if (d < mn) mn = d;
                                if (d > mx) mx = d;
                            }
                            if (mx <= 0.0) separated = 1;
                            if (mn < 0.0) inside_all = 0;
                        }
                        if (separated) {
                            V = 0.0;
                        } else if (inside_all) {
                            V = 1.0; /* C inside T */
                        } else {
                            cnt->n_nontrivial++;
                            if (mode & ORC_PAPER) {
                                int64_t k3[3] = {0, 0, 0};
                                V = orc_clip_tet_box_paper(&v[0][0], clo, chi, k3);
                                cnt->n_pv += k3[0];
                                cnt->n_cut += k3[1];
                                cnt->n_sub += k3[2];
                            } else {
                                V = orc_clip_tet_box(&v[0][0], clo, chi);
                            }
                        }
                    }
                } else {
                    cnt->n_nontrivial++;
                    V = orc_clip_tet_box(&v[0][0], clo, chi);
                }
                if (V > 0.0) {
                    cnt->n_nonzero++;
                    sink_add(s, a, b, c, m * (V / VT));
                }
            }
}

static void counters_add(orc_counters* dst, const orc_counters* src)
{
    dst->n_tet += src->n_tet;
    dst->n_pair += src->n_pair;
    dst->n_nontrivial += src->n_nontrivial;
    dst->n_nonzero += src->n_nonzero;
    dst->n_inverted += src->n_inverted;
    dst->n_degenerate += src->n_degenerate;
    dst->n_ambiguous += src->n_ambiguous;
    dst->n_pv += src->n_pv;
    dst->n_cut += src->n_cut;
    dst->n_sub += src->n_sub;
}

int orc_deposit_uniform(const float* pos, const int* np, double box, double total_mass,
                        const int* nc, const int* region_lo, const int* region_n,
                        const int64_t* cubes, int64_t n_cubes, int mode, int nthreads,
                        double* out, orc_counters* cnt)
{
    if (!pos || !np || !nc || !out || box <= 0.0) return -1;
    for (int a = 0; a < 3; ++a)
        if (np[a] < 1 || nc[a] < 1) return -1;
    int rlo[3] = {0, 0, 0}, rn[3] = {nc[0], nc[1], nc[2]};
    if (region_lo && region_n)
        for (int a = 0; a < 3; ++a) {
            rlo[a] = region_lo[a];
            rn[a] = region_n[a];
            if (rlo[a] < 0 || rn[a] < 1 || rlo[a] + rn[a] > nc[a]) return -1;
        }
    int64_t n_out = (int64_t)rn[0] * rn[1] * rn[2];
    memset(out, 0, sizeof(double) * n_out);
    int64_t ncube_all = (int64_t)np[0] * np[1] * np[2];
    int64_t ncw = cubes ? n_cubes : ncube_all;
    double m = total_mass / (6.0 * (double)ncube_all);
    if (nthreads <= 0) {
#ifdef _OPENMP
        nthreads = omp_get_max_threads();
#else
        nthreads = 1;
#endif
    }
    /* Private buffers when small, shared atomics otherwise. */
    int use_private = n_out * (int64_t)nthreads * 8 <= ((int64_t)256 << 20) && nthreads > 1;
    orc_counters total;
    memset(&total, 0, sizeof(total));

#pragma omp parallel num_threads(nthreads)
    {
        orc_counters lc;
        memset(&lc, 0, sizeof(lc));
        double* buf = out;
        if (use_private) buf = (double*)calloc((size_t)n_out, sizeof(double));
        orc_sink s = {nc, {rlo[0], rlo[1], rlo[2]}, {rn[0], rn[1], rn[2]}, buf,
                      (!use_private && nthreads > 1)};
#pragma omp for schedule(dynamic, 64)
        for (int64_t w = 0; w < ncw; ++w) {
            int64_t id = cubes ? cubes[w] : w;
            int64_t k = id % np[2];
            int64_t j = (id / np[2]) % np[1];
            int64_t i = id / ((int64_t)np[1] * np[2]);
            double c[8][3];
            int amb;
            cube_corners(pos, np, box, nc, i, j, k, c, &amb);
            lc.n_ambiguous += amb;
            for (int p = 0; p < 6; ++p) {
                double v[4][3];
                kuhn_tet(c, p, v);
                deposit_tet(v, KUHN_SIGN[p], m, mode, &s, &lc);
            }
        }
        if (use_private) {
#pragma omp critical
            {
                for (int64_t q = 0; q < n_out; ++q) out[q] += buf[q];
            }
            free(buf);
        }
#pragma omp critical
        counters_add(&total, &lc);
    }
    if (cnt) *cnt = total;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Octree (Section 4).                                                       */
/* ------------------------------------------------------------------------ */

static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

/* Length of the periodic images of [lo,hi) inside [nlo,nhi), period G. */
static int64_t periodic_overlap(int64_t lo, int64_t hi, int64_t nlo, int64_t nhi, int64_t G)
{
    int64_t total = 0;
    int64_t k0 = floor_div(nlo - hi, G);
    int64_t k1 = floor_div(nhi - lo, G) + 1;
    for (int64_t k = k0; k <= k1; ++k) {
        int64_t a = lo + k * G, b = hi + k * G;
        if (a < nlo) a = nlo;
        if (b > nhi) b = nhi;
        if (b > a) total += b - a;
    }
    return total;
}

typedef struct {
    int64_t lo[3], hi[3]; /* finest-lattice integer box [lo,hi) */
    int64_t ntets;
} orc_subblock;

static orc_subblock* subblock_boxes(const float* pos, const int* np, double box, int64_t G,
                                    int S, int64_t* nsb_out)
{
    int64_t ns[3];
    for (int a = 0; a < 3; ++a) ns[a] = (np[a] + S - 1) / S;
    int64_t nsb = ns[0] * ns[1] * ns[2];
    orc_subblock* sb = (orc_subblock*)calloc((size_t)nsb, sizeof(orc_subblock));
    int gnc[3] = {(int)G, (int)G, (int)G};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < nsb; ++s) {
        int64_t si = s / (ns[1] * ns[2]), sj = (s / ns[2]) % ns[1], sk = s % ns[2];
        int64_t i0 = si * S, j0 = sj * S, k0 = sk * S;
        int64_t i1 = i0 + S < np[0] ? i0 + S : np[0];
        int64_t j1 = j0 + S < np[1] ? j0 + S : np[1];
        int64_t k1 = k0 + S < np[2] ? k0 + S : np[2];
        /* reference: the subblock's first particle, in finest units */
        const float* pr = pos + 3 * ((i0 * np[1] + j0) * np[2] + k0);
        double ref[3];
        for (int a = 0; a < 3; ++a) ref[a] = (double)pr[a] * (G / box);
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t j = j0; j < j1; ++j)
                for (int64_t k = k0; k < k1; ++k) {
                    double c[8][3];
                    int amb;
                    cube_corners(pos, np, box, gnc, i, j, k, c, &amb);
                    /* shift the cube to the image nearest the reference */
                    double sh[3];
                    for (int a = 0; a < 3; ++a) {
                        double d = c[0][a] - ref[a];
                        sh[a] = -(double)G * rint(d / (double)G);
                    }
                    for (int q = 0; q < 8; ++q)
                        for (int a = 0; a < 3; ++a) {
                            double x = c[q][a] + sh[a];
                            if (x < mn[a]) mn[a] = x;
                            if (x > mx[a]) mx[a] = x;
                        }
                }
        for (int a = 0; a < 3; ++a) {
            sb[s].lo[a] = (int64_t)floor(mn[a]);
            sb[s].hi[a] = (int64_t)ceil(mx[a]);
            if (sb[s].hi[a] <= sb[s].lo[a]) sb[s].hi[a] = sb[s].lo[a] + 1;
        }
        sb[s].ntets = 6 * (i1 - i0) * (j1 - j0) * (k1 - k0);
    }
    *nsb_out = nsb;
    return sb;
}

static uint64_t morton3(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint64_t m = 0;
    for (int b = bits - 1; b >= 0; --b) {
        m = (m << 3) | ((uint64_t)((x >> b) & 1) << 2) | ((uint64_t)((y >> b) & 1) << 1) |
            (uint64_t)((z >> b) & 1);
    }
    return m;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int orc_build_octree(const float* pos, const int* np, double box, int block, int max_level,
                     int subblock, int64_t threshold, orc_node* nodes, int64_t capacity,
                     int64_t* n_nodes, int64_t* n_leaves)
{
    if (!pos || !np || !n_nodes || !n_leaves || block < 1 || max_level < 0 || max_level > 10 ||
        subblock < 1 || box <= 0.0)
        return -1;
    int64_t G = (int64_t)block << max_level;
    int64_t nsb;
    orc_subblock* sb = subblock_boxes(pos, np, box, G, subblock, &nsb);

    /* Level by level: the current level's node coordinates in Morton order. */
    int64_t cap_total = 1;
    for (int l = 1; l <= max_level; ++l) cap_total += (int64_t)1 << (3 * l);
    orc_node* all = (orc_node*)malloc(sizeof(orc_node) * (size_t)cap_total);
    int64_t n_all = 0;
    int64_t level_begin = 0, level_end = 1;
    all[0].level = 0;
    all[0].ix = all[0].iy = all[0].iz = 0;
    all[0].first_child = -1;
    all[0].leaf_id = -1;
    all[0].count = 0;
    n_all = 1;
    for (int l = 0; l <= max_level; ++l) {
        int64_t side = (int64_t)1 << l;
        int64_t w = G / side;
        int64_t* dense = (int64_t*)calloc((size_t)(side * side * side), sizeof(int64_t));
        /* count estimate for every node position of this level */
        for (int64_t s = 0; s < nsb; ++s) {
            int64_t vol = (sb[s].hi[0] - sb[s].lo[0]) * (sb[s].hi[1] - sb[s].lo[1]) *
                          (sb[s].hi[2] - sb[s].lo[2]);
            int64_t* ov[3];
            for (int a = 0; a < 3; ++a) {
                ov[a] = (int64_t*)calloc((size_t)side, sizeof(int64_t));
                for (int64_t n = 0; n < side; ++n)
                    ov[a][n] = periodic_overlap(sb[s].lo[a], sb[s].hi[a], n * w, (n + 1) * w, G);
            }
            for (int64_t x = 0; x < side; ++x) {
                if (!ov[0][x]) continue;
                for (int64_t y = 0; y < side; ++y) {
                    if (!ov[1][y]) continue;
                    for (int64_t z = 0; z < side; ++z) {
                        if (!ov[2][z]) continue;
                        int64_t num = sb[s].ntets * ov[0][x] * ov[1][y] * ov[2][z];
                        dense[(x * side + y) * side + z] += num / vol;
                    }
                }
            }
            for (int a = 0; a < 3; ++a) free(ov[a]);
        }
        /* children of refined nodes, in Morton order of the next level */
        int64_t nkids = 0;
        for (int64_t q = level_begin; q < level_end; ++q) {
            orc_node* nd = &all[q];
            nd->count = dense[((int64_t)nd->ix * side + nd->iy) * side + nd->iz];
            if (nd->count > threshold && l < max_level) {
                nd->first_child = (int32_t)(level_end + nkids);
                nkids += 8;
            }
        }
        free(dense);
        if (nkids == 0) break;
        for (int64_t q = level_begin; q < level_end; ++q) {
            orc_node* nd = &all[q];
            if (nd->first_child < 0) continue;
            for (int c = 0; c < 8; ++c) {
                orc_node* ch = &all[nd->first_child + c];
                ch->level = l + 1;
                ch->ix = 2 * nd->ix + ((c >> 2) & 1);
                ch->iy = 2 * nd->iy + ((c >> 1) & 1);
                ch->iz = 2 * nd->iz + (c & 1);
                ch->first_child = -1;
                ch->leaf_id = -1;
                ch->count = 0;
            }
        }
        n_all = level_end + nkids;
        level_begin = level_end;
        level_end = n_all;
    }
    /* Parents are visited in Morton order, so the children are too; check. */
    {
        int64_t lb = 0;
        while (lb < n_all) {
            int64_t le = lb;
            while (le < n_all && all[le].level == all[lb].level) ++le;
            uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(le - lb));
            for (int64_t q = lb; q < le; ++q)
                keys[q - lb] = morton3(all[q].ix, all[q].iy, all[q].iz, all[q].level);
            uint64_t* sorted = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(le - lb));
            memcpy(sorted, keys, sizeof(uint64_t) * (size_t)(le - lb));
            qsort(sorted, (size_t)(le - lb), sizeof(uint64_t), cmp_u64);
            int ok = memcmp(sorted, keys, sizeof(uint64_t) * (size_t)(le - lb)) == 0;
            free(keys);
            free(sorted);
            if (!ok) {
                free(all);
                free(sb);
                return -1;
            }
            lb = le;
        }
    }
    int64_t nl = 0;
    for (int64_t q = 0; q < n_all; ++q)
        if (all[q].first_child < 0) all[q].leaf_id = (int32_t)nl++;
    *n_nodes = n_all;
    *n_leaves = nl;
    free(sb);
    if (!nodes || capacity < n_all) {
        free(all);
        return -3;
    }
    memcpy(nodes, all, sizeof(orc_node) * (size_t)n_all);
    free(all);
    return 0;
}

int orc_deposit_octree(const float* pos, const int* np, double box, double total_mass, int block,
                       const orc_node* nodes, int64_t n_nodes, const int64_t* leaf_sel,
                       int64_t n_sel, int mode, int nthreads, double* out, orc_counters* cnt)
{
    if (!pos || !np || !nodes || !out || !leaf_sel || block < 1) return -1;
    if (cnt) memset(cnt, 0, sizeof(*cnt));
    int64_t B3 = (int64_t)block * block * block;
    for (int64_t s = 0; s < n_sel; ++s) {
        const orc_node* leaf = NULL;
        for (int64_t q = 0; q < n_nodes; ++q)
            if (nodes[q].leaf_id == leaf_sel[s]) {
                leaf = &nodes[q];
                break;
            }
        if (!leaf) return -1;
        /* The leaf's cells are the cells of a uniform grid at its level. */
        int n = block << leaf->level;
        int nc[3] = {n, n, n};
        int rlo[3] = {leaf->ix * block, leaf->iy * block, leaf->iz * block};
        int rn[3] = {block, block, block};
        orc_counters c1;
        int rc = orc_deposit_uniform(pos, np, box, total_mass, nc, rlo, rn, NULL, 0, mode,
                                     nthreads, out + s * B3, &c1);
        if (rc) return rc;
        if (cnt) counters_add(cnt, &c1);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Examples for the learned overlap surrogate.                              */
/* ------------------------------------------------------------------------ */

int orc_surrogate_examples(const float* pos, const int* np, double box, const int* nc,
                           int64_t first, int64_t count, int nthreads, uint8_t* flag,
                           float* feat, uint8_t* mask, double* frac, int32_t* lo_out)
{
    if (!pos || !np || !nc || !flag || !feat || !mask || !frac || count < 0 || first < 0)
        return -1;
    int64_t ncube = (int64_t)np[0] * np[1] * np[2];
    if (first + count > ncube) return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t w = 0; w < count; ++w) {
        int64_t cube = first + w;
        int64_t i = cube / ((int64_t)np[1] * np[2]);
        int64_t j = (cube / np[2]) % np[1];
        int64_t k = cube % np[2];
        double c[8][3];
        int amb;
        cube_corners(pos, np, box, nc, i, j, k, c, &amb);
        for (int p = 0; p < 6; ++p) {
            int64_t t = 6 * w + p;
            double v[4][3];
            kuhn_tet(c, p, v);
            flag[t] = 0;
            mask[t] = 0;
            if (lo_out) lo_out[3 * t] = lo_out[3 * t + 1] = lo_out[3 * t + 2] = 0;
            for (int q = 0; q < 12; ++q) feat[12 * t + q] = 0.0f;
            for (int q = 0; q < 8; ++q) frac[8 * t + q] = 0.0;
            double D = tet_det(v);
            double l3 = 0.0;
            for (int a = 0; a < 4; ++a)
                for (int b = a + 1; b < 4; ++b) {
                    double e2 = 0.0;
                    for (int x = 0; x < 3; ++x) e2 += (v[a][x] - v[b][x]) * (v[a][x] - v[b][x]);
                    if (e2 > l3) l3 = e2;
                }
            l3 = l3 * sqrt(l3);
            if (fabs(D) <= 1e-12 * l3) continue;
            double lo[3];
            int span[3], ok = 1;
            for (int x = 0; x < 3; ++x) {
                double mn = v[0][x], mx = v[0][x];
                for (int a = 1; a < 4; ++a) {
                    if (v[a][x] < mn) mn = v[a][x];
                    if (v[a][x] > mx) mx = v[a][x];
                }
                lo[x] = floor(mn);
                span[x] = (int)(floor(mx) - lo[x]);
                if (span[x] > 1) ok = 0;
            }
            if (!ok) continue;
            flag[t] = 1;
            if (lo_out)
                for (int x = 0; x < 3; ++x)
                    lo_out[3 * t + x] = (int32_t)wrap64((int64_t)lo[x], nc[x]);
            for (int a = 0; a < 4; ++a)
                for (int x = 0; x < 3; ++x) feat[12 * t + 3 * a + x] = (float)(v[a][x] - lo[x]);
            double VT = fabs(D) / 6.0;
            for (int q = 0; q < 8; ++q) {
                int d[3] = {(q >> 2) & 1, (q >> 1) & 1, q & 1};
                if (d[0] > span[0] || d[1] > span[1] || d[2] > span[2]) continue;
                mask[t] |= (uint8_t)(1u << q);
                double clo[3], chi[3];
                for (int x = 0; x < 3; ++x) {
                    clo[x] = lo[x] + d[x];
                    chi[x] = clo[x] + 1.0;
                }
                frac[8 * t + q] = orc_clip_tet_box(&v[0][0], clo, chi) / VT;
            }
        }
    }
    return 0;
}
