// psd_uniform.hip -- deposit onto a periodic uniform grid.
//
// Section 6.1 loop (per tetrahedron, per cell of its bounding box: trivial
// classification, exact clip otherwise) with the GPU structure of its
// Section 6.2 re-shaped for a 64-lane wavefront: lanes classify 64 cells in
// lock-step, trivial cells scatter at once, and the non-trivial ones are
// compacted (ballot + popcount prefix) into LDS queues that are clipped 64
// at a time.  Queues are split by the expected size of the clip so that the
// lanes of one flush follow similar paths.
#include <string.h>

#include "psd_internal.h"

namespace psd {

namespace {

// Per-tetrahedron record kept in LDS while its cells are walked.
struct TetSlot {
    double vr[4][3];  // vertices relative to the bbox origin (cell units), exact
    float N[4][3];    // face normals (inside positive), for classification
    float c[4];       // plane offsets: N.x + c with x relative to the bbox origin
    float neg[4];     // sum of the negative components of N
    float pos[4];     // sum of the positive components of N
    float tol[4];     // bound on the float rounding of N.x + c over the bbox
    double m_over_v;  // m / |T|, |T| in cell units
    int lo[3];        // bbox origin, wrapped into [0, nc)
    int ext[3];       // bbox extent in cells
    int frac;         // bit a: the vertices' largest coordinate on axis a is not an integer
};

constexpr int kQueues = 4;
constexpr int kQCap = 2 * kWave;
constexpr uint32_t kTetFrameBit = 1u << 15;

__device__ __forceinline__ int wrap_add(int base, int off, int n)
{
    int x = base + off;
    return x >= n ? x - n : x;
}

template <typename OutT>
__device__ __forceinline__ void scatter(OutT* out, const UniformArgs& P, int a, int b, int c,
                                        double mass, double& acc)
{
    int64_t idx = ((int64_t)a * P.nc[1] + b) * P.nc[2] + c;
    OutT val = (OutT)(mass * P.out_scale);
    global_add(out + idx, val);
    acc += mass;
}

__device__ __forceinline__ void decode_cell(const TetSlot& S, uint32_t r, int& ci, int& cj, int& ck)
{
    const uint32_t ez = (uint32_t)S.ext[2], eyz = (uint32_t)S.ext[1] * ez;
    ci = (int)(r / eyz);
    const uint32_t rem = r - (uint32_t)ci * eyz;
    cj = (int)(rem / ez);
    ck = (int)(rem - (uint32_t)cj * ez);
}

// Cell frame: the cell's six Freudenthal tetrahedra against the tetrahedron's
// active face planes (tmask), distances in FP64.  Returns |T cap C| in cells^3.
__device__ __forceinline__ double cell_frame_volume(const TetSlot& S, int ci, int cj, int ck, uint32_t tmask)
{
    // FP64 face planes in the cell's local frame (origin at its low corner).
    double Nn[4][3], cc[4];
    const double o[3] = {(double)ci, (double)cj, (double)ck};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int i0 = f == 0 ? 1 : 0, i1 = f <= 1 ? 2 : 1, i2 = f <= 2 ? 3 : 2;
        double p0[3], e1[3], e2[3], w[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p0[a] = S.vr[i0][a] - o[a];
            e1[a] = S.vr[i1][a] - S.vr[i0][a];
            e2[a] = S.vr[i2][a] - S.vr[i0][a];
            w[a] = S.vr[f][a] - S.vr[i0][a];
        }
        double n0 = e1[1] * e2[2] - e1[2] * e2[1];
        double n1 = e1[2] * e2[0] - e1[0] * e2[2];
        double n2 = e1[0] * e2[1] - e1[1] * e2[0];
        double sg = (n0 * w[0] + n1 * w[1] + n2 * w[2]) < 0.0 ? -1.0 : 1.0;
        Nn[f][0] = sg * n0;
        Nn[f][1] = sg * n1;
        Nn[f][2] = sg * n2;
        cc[f] = -(Nn[f][0] * p0[0] + Nn[f][1] * p0[1] + Nn[f][2] * p0[2]);
    }
    // Compact the active planes and tabulate their values at the 8 corners.
    const int k = __builtin_popcount(tmask);
    double dq[8][4];
    uint32_t m = tmask;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int f = m ? __builtin_ctz(m) : 0;
        m &= m - 1;
        const double nx = sel4(Nn[0][0], Nn[1][0], Nn[2][0], Nn[3][0], f);
        const double ny = sel4(Nn[0][1], Nn[1][1], Nn[2][1], Nn[3][1], f);
        const double nz = sel4(Nn[0][2], Nn[1][2], Nn[2][2], Nn[3][2], f);
        const double d0 = sel4(cc[0], cc[1], cc[2], cc[3], f);
        dq[0][s] = d0;
        dq[4][s] = d0 + nx;
        dq[2][s] = d0 + ny;
        dq[6][s] = dq[4][s] + ny;
        dq[1][s] = d0 + nz;
        dq[5][s] = dq[4][s] + nz;
        dq[3][s] = dq[2][s] + nz;
        dq[7][s] = dq[6][s] + nz;
    }
    CellEval<double> ev;
    double vol = 0.0;
    for (int p = 0; p < 6; ++p) {
        const int q1 = kuhn_q1(p), q2 = kuhn_q2(p);
        double t[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            t[0][s] = dq[0][s];
            t[1][s] = q1 == 4 ? dq[4][s] : (q1 == 2 ? dq[2][s] : dq[1][s]);
            t[2][s] = q2 == 6 ? dq[6][s] : (q2 == 5 ? dq[5][s] : dq[3][s]);
            t[3][s] = dq[7][s];
        }
        vol += inside_fraction<double, 0, 4>(t, k, ev);
    }
    return vol / 6.0;
}

// Tet frame: the tetrahedron against the cell's active planes (cmask bits:
// x>=0, x<=1, y>=0, y<=1, z>=0, z<=1), cell-local coordinates rounded once
// to R.  Returns the fraction of T inside the cell.
template <typename R>
__device__ __forceinline__ R tet_frame_fraction(const TetSlot& S, int ci, int cj, int ck, uint32_t cmask)
{
    const int k = __builtin_popcount(cmask);
    if (k == 0) return R(1);
    const double o[3] = {(double)ci, (double)cj, (double)ck};
    R x[4][3];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int a = 0; a < 3; ++a) x[v][a] = (R)(S.vr[v][a] - o[a]);
    TetEval<R> ev;
    uint32_t m = cmask;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int id = m ? __builtin_ctz(m) : 0;
        m &= m - 1;
        ev.axis[s] = id >> 1;
        ev.sgn[s] = (id & 1) ? R(-1) : R(1);
        ev.off[s] = (id & 1) ? R(1) : R(0);
    }
    return inside_fraction<R, 0, 6>(x, k, ev);
}

template <typename R>
__device__ __forceinline__ double clip_mass(const TetSlot& S, uint32_t r, uint32_t masks, double m)
{
    int ci, cj, ck;
    decode_cell(S, r, ci, cj, ck);
    if (masks & kTetFrameBit) return m * (double)tet_frame_fraction<R>(S, ci, cj, ck, (masks >> 4) & 0x3F);
    return S.m_over_v * cell_frame_volume(S, ci, cj, ck, masks & 0xF);
}

template <typename R, typename OutT>
__global__ __launch_bounds__(kWave) void deposit_uniform_kernel(UniformArgs P)
{
    __shared__ TetSlot slots[kWave];
    __shared__ int64_t s_incl[kWave];
    __shared__ int64_t s_excl[kWave];
    __shared__ uint32_t q_cell[kQueues][kQCap];
    __shared__ uint16_t q_mask[kQueues][kQCap];
    __shared__ uint8_t q_slot[kQueues][kQCap];

    OutT* out = reinterpret_cast<OutT*>(P.out);
    const int lane = threadIdx.x;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const double sc[3] = {P.scale[0], P.scale[1], P.scale[2]};
    double macc = 0.0;
    unsigned long long n_tet = 0, n_pair = 0, n_clip = 0, n_nz = 0, n_inv = 0, n_deg = 0;
    int qn[kQueues] = {0, 0, 0, 0};

    auto flush = [&](int qi, int base, int count) {
        if (lane < count) {
            const int e = base + lane;
            const TetSlot& S = slots[q_slot[qi][e]];
            const uint32_t rr = q_cell[qi][e];
            const double mass = clip_mass<R>(S, rr, q_mask[qi][e], P.m);
            ++n_clip;
            if (mass > 0.0) {
                int ci, cj, ck;
                decode_cell(S, rr, ci, cj, ck);
                ++n_nz;
                scatter(out, P, wrap_add(S.lo[0], ci, P.nc[0]), wrap_add(S.lo[1], cj, P.nc[1]),
                        wrap_add(S.lo[2], ck, P.nc[2]), mass, macc);
            }
        }
    };

    for (int64_t chunk = blockIdx.x; chunk * kWave < P.ntet; chunk += gridDim.x) {
        const int64_t tid = chunk * kWave + lane;
        int nb = 0;
        if (tid < P.ntet) {
            const int64_t cube = tid / 6;
            const int p = (int)(tid - cube * 6);
            const int64_t kk = cube % P.np[2];
            const int64_t jj = (cube / P.np[2]) % P.np[1];
            const int64_t ii = cube / ((int64_t)P.np[1] * P.np[2]);
            Tet64 T;
            make_tet(P.pos, P.np[0], P.np[1], P.np[2], sc, P.nc, ii, jj, kk, p, T);
            ++n_tet;
            if ((double)kuhn_sign(p) * T.D < 0.0) ++n_inv;
            // Non-finite input cannot be placed; such a tetrahedron is dropped.
            const bool finite_tet = isfinite(T.D) && isfinite(T.l3);
            if (!finite_tet) {
                // nothing deposited; counted
                if (P.stats) atomicAdd(P.stats + 7, 1ull);
            } else if (fabs(T.D) <= 1e-12 * T.l3) {
                // zero-volume tetrahedron: all mass to the centroid's cell
                ++n_deg;
                ++n_nz;
                int g[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double x = 0.25 * (T.v[0][a] + T.v[1][a] + T.v[2][a] + T.v[3][a]);
                    g[a] = wrap_index(floor(x), P.nc[a]);
                }
                scatter(out, P, g[0], g[1], g[2], P.m, macc);
            } else {
                TetSlot& S = slots[lane];
                int ext[3], frac = 0;
                bool ext_ok = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double mn = fmin(fmin(T.v[0][a], T.v[1][a]), fmin(T.v[2][a], T.v[3][a]));
                    const double mx = fmax(fmax(T.v[0][a], T.v[1][a]), fmax(T.v[2][a], T.v[3][a]));
                    const double lo = floor(mn);
                    const double hi = floor(mx);
                    ext[a] = (int)(hi - lo) + 1;
                    // minimum-image offsets bound the extent by nc + 1 cells
                    ext_ok = ext_ok && ext[a] >= 1 && ext[a] <= P.nc[a] + 1;
                    frac |= (mx > hi) ? (1 << a) : 0;
                    S.lo[a] = wrap_index(lo, P.nc[a]);
                    S.ext[a] = ext[a];
#pragma unroll
                    for (int v = 0; v < 4; ++v) S.vr[v][a] = T.v[v][a] - lo;
                }
                S.frac = frac;
                S.m_over_v = P.m / (fabs(T.D) / 6.0);
                const double emax = (double)max(ext[0], max(ext[1], ext[2]));
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const int i0 = f == 0 ? 1 : 0, i1 = f <= 1 ? 2 : 1, i2 = f <= 2 ? 3 : 2;
                    double e1[3], e2[3], n[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        e1[a] = S.vr[i1][a] - S.vr[i0][a];
                        e2[a] = S.vr[i2][a] - S.vr[i0][a];
                    }
                    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
                    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
                    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
                    double cc = -(n[0] * S.vr[i0][0] + n[1] * S.vr[i0][1] + n[2] * S.vr[i0][2]);
                    const double sv = n[0] * S.vr[f][0] + n[1] * S.vr[f][1] + n[2] * S.vr[f][2] + cc;
                    const double sg = sv < 0.0 ? -1.0 : 1.0;
                    double ng = 0.0, ps = 0.0, an = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        n[a] *= sg;
                        S.N[f][a] = (float)n[a];
                        ng += n[a] < 0.0 ? n[a] : 0.0;
                        ps += n[a] > 0.0 ? n[a] : 0.0;
                        an += fabs(n[a]);
                    }
                    cc *= sg;
                    S.c[f] = (float)cc;
                    S.neg[f] = (float)ng;
                    S.pos[f] = (float)ps;
                    // float evaluation of N.o + c and the corner offsets
                    S.tol[f] = (float)(1e-6 * (an * (emax + 1.0) + fabs(cc)));
                }
                nb = ext_ok ? ext[0] * ext[1] * ext[2] : 0;
                if (nb == 1) {
                    // the tetrahedron lies inside one cell
                    ++n_pair;
                    ++n_nz;
                    scatter(out, P, S.lo[0], S.lo[1], S.lo[2], P.m, macc);
                    nb = 0;
                }
            }
        }
        // inclusive scan of the bbox cell counts across the wave
        int64_t incl = nb;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int64_t y = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += y;
        }
        s_incl[lane] = incl;
        s_excl[lane] = incl - nb;
        __syncthreads();
        const int64_t total = __shfl(incl, kWave - 1, kWave);

        for (int64_t base = 0; base < total; base += kWave) {
            const int64_t idx = base + lane;
            int cls = -1, slot = 0;
            uint32_t r = 0, masks = 0;
            if (idx < total) {
                int lo = 0, hi = kWave - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_incl[mid] > idx) hi = mid;
                    else lo = mid + 1;
                }
                slot = lo;
                r = (uint32_t)(idx - s_excl[slot]);
                const TetSlot& S = slots[slot];
                int ci, cj, ck;
                decode_cell(S, r, ci, cj, ck);
                ++n_pair;
                const float fi = (float)ci, fj = (float)cj, fk = (float)ck;
                bool full = true, sep = false;
                uint32_t tmask = 0;
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const float d0 = fmaf(S.N[f][0], fi, fmaf(S.N[f][1], fj, fmaf(S.N[f][2], fk, S.c[f])));
                    const float mn = d0 + S.neg[f], mx = d0 + S.pos[f];
                    sep = sep || (mx < -S.tol[f]);
                    const bool inside = mn > S.tol[f];
                    full = full && inside;
                    tmask |= inside ? 0u : (1u << f);
                }
                // Cell planes that cut T: x>=0 needs ci >= 1; x<=1 needs some
                // vertex beyond ci+1.  A cell whose low face only touches the
                // bbox's top (integer maximum) has zero volume.
                uint32_t cmask = 0;
                bool touch = false;
                const int cidx[3] = {ci, cj, ck};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int e = S.ext[a], i = cidx[a];
                    const bool fr = (S.frac >> a) & 1;
                    cmask |= (i >= 1) ? (1u << (2 * a)) : 0u;
                    cmask |= (i <= e - 3 || (i == e - 2 && fr)) ? (2u << (2 * a)) : 0u;
                    touch = touch || (i == e - 1 && !fr && e > 1);
                }
                if (!sep && !touch) {
                    if (full) {
                        ++n_nz;
                        scatter(out, P, wrap_add(S.lo[0], ci, P.nc[0]), wrap_add(S.lo[1], cj, P.nc[1]),
                                wrap_add(S.lo[2], ck, P.nc[2]), S.m_over_v, macc);
                    } else {
                        const int kT = __builtin_popcount(tmask);
                        const int kC = __builtin_popcount(cmask);
                        const bool tet_frame = kC <= kT + 1;
                        masks = tmask | (cmask << 4) | (tet_frame ? kTetFrameBit : 0u);
                        cls = tet_frame ? (kC <= 2 ? 2 : 3) : (kT == 1 ? 0 : (kT == 2 ? 1 : 3));
                    }
                }
            }
#pragma unroll
            for (int qi = 0; qi < kQueues; ++qi) {
                const uint64_t bal = __ballot(cls == qi);
                if (cls == qi) {
                    const int at = qn[qi] + __popcll(bal & lt_mask);
                    q_cell[qi][at] = r;
                    q_slot[qi][at] = (uint8_t)slot;
                    q_mask[qi][at] = (uint16_t)masks;
                }
                qn[qi] += __popcll(bal);
            }
            __syncthreads();
            // clip every full queue (one call site keeps the clip code single)
            uint32_t due = 0;
#pragma unroll
            for (int qi = 0; qi < kQueues; ++qi) due |= (qn[qi] >= kWave) ? (1u << qi) : 0u;
            while (due) {
                const int qi = __builtin_ctz(due);
                due &= due - 1;
                const int n = qi == 0 ? qn[0] : (qi == 1 ? qn[1] : (qi == 2 ? qn[2] : qn[3]));
                flush(qi, n - kWave, kWave);
#pragma unroll
                for (int q = 0; q < kQueues; ++q) qn[q] -= (q == qi) ? kWave : 0;
            }
            __syncthreads();
        }
        // drain this chunk's queues before its slots are overwritten
        for (int qi = 0; qi < kQueues; ++qi) {
            const int n = qi == 0 ? qn[0] : (qi == 1 ? qn[1] : (qi == 2 ? qn[2] : qn[3]));
            if (n > 0) flush(qi, 0, n);
        }
#pragma unroll
        for (int q = 0; q < kQueues; ++q) qn[q] = 0;
        __syncthreads();
    }

    // wave reductions: FP64 mass partial and counters
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        macc += __shfl_xor(macc, off, kWave);
        n_tet += __shfl_xor(n_tet, off, kWave);
        n_pair += __shfl_xor(n_pair, off, kWave);
        n_clip += __shfl_xor(n_clip, off, kWave);
        n_nz += __shfl_xor(n_nz, off, kWave);
        n_inv += __shfl_xor(n_inv, off, kWave);
        n_deg += __shfl_xor(n_deg, off, kWave);
    }
    if (lane == 0) {
        if (P.mass_sum) global_add(P.mass_sum, macc);
        if (P.stats) {
            atomicAdd(P.stats + 0, n_tet);
            atomicAdd(P.stats + 1, n_pair);
            atomicAdd(P.stats + 2, n_clip);
            atomicAdd(P.stats + 3, n_nz);
            atomicAdd(P.stats + 4, n_inv);
            atomicAdd(P.stats + 5, n_deg);
        }
    }
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

BoxDesc box_from_uniform(const UniformArgs& P)
{
    BoxDesc b;
    memset(&b, 0, sizeof(b));
    b.pos = P.pos;
    for (int a = 0; a < 3; ++a) {
        b.np[a] = P.np[a];
        b.nc[a] = P.nc[a];
        b.scale[a] = P.scale[a];
    }
    b.m = P.m;
    b.out_scale = P.out_scale;
    b.out = P.out;
    b.mass_sum = P.mass_sum;
    b.ntet = P.ntet;
    b.leaf_map = P.leaf_map;
    b.level_has_leaf = P.level_has_leaf;
    b.leaf_block = P.leaf_block;
    b.leaf_side = P.leaf_side;
    b.skip_small = P.surrogate != nullptr;
    return b;
}

hipError_t launch_deposit_uniform(const UniformArgs& P, bool fp64, bool accumulate,
                                  bool cell_method, const Tuning& tune, void* ws, size_t ws_bytes,
                                  hipStream_t stream)
{
    const int64_t ncell = (int64_t)P.nc[0] * P.nc[1] * P.nc[2];
    if (!accumulate) {
        const int64_t want = (ncell + 255) / 256;
        const int blocks = (int)(want < 65536 ? want : 65536);
        if (fp64)
            hipLaunchKernelGGL(fill_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                               (double*)P.out, ncell, 0.0);
        else
            hipLaunchKernelGGL(fill_kernel<float>, dim3(blocks), dim3(256), 0, stream,
                               (float*)P.out, ncell, 0.0f);
        if (P.mass_sum)
            hipLaunchKernelGGL(fill_kernel<double>, dim3(1), dim3(64), 0, stream, P.mass_sum,
                               (int64_t)1, 0.0);
    }
    if (!cell_method) {
        BoxDesc b = box_from_uniform(P);
        size_t qbytes = ws_bytes;
        if (P.surrogate) {
            // the network's pass first: it marks the tets left to the exact pass
            const int64_t n_chunks = (P.ntet + kWave - 1) / kWave;
            qbytes = queue_workspace_bytes(n_chunks, 1, tune.ordered != 0);
            const size_t off = surrogate_mask_offset(qbytes);
            if (off + surrogate_mask_bytes(P.ntet) > ws_bytes) return hipErrorInvalidValue;
            unsigned long long* mask =
                reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) + off);
            hipError_t e = launch_surrogate_deposit(P, fp64, mask, stream);
            if (e != hipSuccess) return e;
            b.exact_mask = mask;
        }
        return launch_queue(&b, 1, fp64, tune, ws, qbytes, P.stats, stream);
    }
    if (P.surrogate) return hipErrorInvalidValue;
    const int64_t nchunk = (P.ntet + kWave - 1) / kWave;
    int grid = (int)(nchunk < (int64_t)P.grid_limit ? nchunk : (int64_t)P.grid_limit);
    if (grid < 1) grid = 1;
    if (fp64)
        hipLaunchKernelGGL((deposit_uniform_kernel<double, double>), dim3(grid), dim3(kWave), 0,
                           stream, P);
    else
        hipLaunchKernelGGL((deposit_uniform_kernel<float, float>), dim3(grid), dim3(kWave), 0,
                           stream, P);
    return hipGetLastError();
}

}  // namespace psd
