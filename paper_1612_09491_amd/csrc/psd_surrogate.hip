// psd_surrogate.hip -- the learned overlap surrogate for small tetrahedra.
//
// For a tetrahedron whose bounding box spans at most 2 cells per axis, a small
// network predicts the overlap fractions |T cap C| / |T| (the cell average of
// Eq. (1)) for the 2x2x2 cells at the bbox origin lo = floor(min v):
//   x (12) = vertices minus lo in cell units  ->  64 -> 64 -> 64 (SiLU)  ->  8
// followed by a softmax over the cells that lie inside [lo, hi].  The three
// 64-wide products and the output layer run on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulate); the input layer takes the
// float32 features split into two BF16 halves (hi + lo) in one 32-deep
// product, so the inputs keep 16 significant bits.  Everything here is an
// addition to the paper; the training labels come from the exact splitting
// of Section 6.3.
//
// Wavefront tiling (64 tetrahedra per wave): activations live in LDS as
// [tet][unit] BF16 rows; a layer computes D[unit][tet] = W[unit][:] . H[tet][:]
// as 4 x 4 tiles of 16 x 16, the weight fragments (A operand) stay in
// registers for the life of the wave, and each lane of the epilogue writes 4
// consecutive units of one tetrahedron.

#include <hip/hip_cooperative_groups.h>

#include "psd_internal.h"

namespace psd {
namespace {

constexpr int kH = 64;   // hidden width
constexpr int kIn = 12;  // 4 vertices x 3 coordinates
constexpr int kOut = 8;  // 2 x 2 x 2 cells, c = 4 dx + 2 dy + dz
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kOut * kH, kNParams = oB4 + kOut;
static_assert(kNParams == 9672, "packed parameter layout");

constexpr int kHS = 72;  // row stride (BF16) of a 64-wide activation tile
constexpr int kXS = 40;  // row stride of the 32-wide input tile (hi 12, lo 12, zero 8)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// float -> bfloat16, round to nearest even (finite inputs).
// Round to nearest even (the hardware conversion, v_cvt_pk_bf16_f32).
__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }

__device__ __forceinline__ float from_bf16(__bf16 h)
{
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, h) << 16);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ bf16x8 ld8s(const __bf16* p, int stride)
{
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = p[e * stride];
    return r;
}

__device__ __forceinline__ int wrap_cell(int x, int n) { return x >= n ? x - n : x; }

// 1 / (1 + e^-z) with the hardware reciprocal (1 ulp; 0 when e^-z overflows).
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// The deposit kernel runs the network on pre-activations scaled by -log2(e):
// with y = -log2(e) z, 2^y = e^-z, so the sigmoid needs no multiply, and the
// stored activation y * sigmoid(z) = -log2(e) silu(z) feeds the next layer
// unscaled (its bias scaled by -log2(e) gives that layer's y).  The output
// layer with negated weights and its bias times log2(e) then yields log2(e)
// times the logits, so the softmax takes powers of 2.
constexpr float kNegLog2e = -1.4426950408889634f;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float sigmoid_pow2(float y) { return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y)); }

// q = n / d for 0 <= n < 2^21 from the hardware reciprocal (relative error
// up to 2^-23): (n + 1/2) * inv_d stays within (q, q + 1) because its error,
// under (n + 1/2) * 1.8e-7 / d, is below 1/(2d).
__device__ __forceinline__ int quot_small(int n, float inv_d) { return (int)(((float)n + 0.5f) * inv_d); }

// Weight fragments of the A operand and bias columns, held per wave.
// Lane l holds row (l & 15) of a 16-row tile, k = 8 (l >> 4) + 0..7.
struct Net {
    bf16x8 w1[4][1];   // [unit tile][k step] (k: hi 0..11, lo 12..23, zero)
    bf16x8 w2[4][2];   // [unit tile][k step]
    bf16x8 w3[4][2];
    bf16x8 w4[2];      // rows 0..7 = cells, 8..15 zero
    const float* w;    // the packed parameters (biases are read from here, cached)
};

__device__ __forceinline__ void load_net(const float* __restrict__ w, Net& N, bool neg_out = false)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int u = mt * 16 + r;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
            const float v = k < kIn ? w[oW1 + u * kIn + k] : (k < 2 * kIn ? w[oW1 + u * kIn + k - kIn] : 0.0f);
            N.w1[mt][0][e] = to_bf16(v);
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = ks * 32 + 8 * g + e;
                N.w2[mt][ks][e] = to_bf16(w[oW2 + u * kH + k]);
                N.w3[mt][ks][e] = to_bf16(w[oW3 + u * kH + k]);
            }
    }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = ks * 32 + 8 * g + e;
            const float v = r < kOut ? w[oW4 + r * kH + k] : 0.0f;
            N.w4[ks][e] = to_bf16(neg_out ? -v : v);
        }
    N.w = w;
}

// Writes the features of one tetrahedron (12 floats) as row t of an input
// tile: BF16 high parts, BF16 residuals, zeros.
__device__ __forceinline__ void put_features(__bf16* row, const float (&x)[kIn])
{
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        const __bf16 hi = to_bf16(x[k]);
        row[k] = hi;
        row[kIn + k] = to_bf16(x[k] - from_bf16(hi));
    }
#pragma unroll
    for (int k = 2 * kIn; k < 32; ++k) row[k] = to_bf16(0.0f);
}

// Canonical pose: the overlap fractions do not depend on the order of the
// vertices, and reflecting an axis whose bbox spans 2 cells (x -> 2 - x) only
// swaps that axis's cells.  Every straddling axis whose vertex sum exceeds 4
// (centroid beyond the middle plane) is reflected, then the vertices are
// sorted lexicographically.  Returns the reflected axes' cell bits r: the
// network's canonical cell c' is the tetrahedron's cell c' ^ r.
__device__ __forceinline__ bool vless(const float (&x)[kIn], int i, int j)
{
    const float* a = x + 3 * i;
    const float* b = x + 3 * j;
    return a[0] < b[0] || (a[0] == b[0] && (a[1] < b[1] || (a[1] == b[1] && a[2] < b[2])));
}

__device__ __forceinline__ void vswap_if(float (&x)[kIn], int i, int j)
{
    const bool sw = vless(x, j, i);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = x[3 * i + a], w = x[3 * j + a];
        x[3 * i + a] = sw ? w : u;
        x[3 * j + a] = sw ? u : w;
    }
}

__device__ __forceinline__ int canonical_pose(float (&x)[kIn], int mask)
{
    int r = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int bit = 4 >> a;
        const double s = (((double)x[a] + (double)x[3 + a]) + (double)x[6 + a]) + (double)x[9 + a];
        const bool refl = ((mask >> bit) & 1) && s > 4.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) x[3 * q + a] = refl ? 2.0f - x[3 * q + a] : x[3 * q + a];
        r |= refl ? bit : 0;
    }
    // 4-element sorting network
    vswap_if(x, 0, 1);
    vswap_if(x, 2, 3);
    vswap_if(x, 0, 2);
    vswap_if(x, 1, 3);
    vswap_if(x, 1, 2);
    return r;
}

// p[c] <- p[c ^ r] for a 3-bit r, with selects (no indexed registers).
__device__ __forceinline__ void xor_cells(float (&p)[kOut], int r)
{
#pragma unroll
    for (int bit = 4; bit >= 1; bit >>= 1) {
        const bool sw = (r & bit) != 0;
#pragma unroll
        for (int c = 0; c < kOut; ++c) {
            if (c & bit) continue;
            const float a = p[c], b = p[c | bit];
            p[c] = sw ? b : a;
            p[c | bit] = sw ? a : b;
        }
    }
}

// One hidden layer over the wave's 64 tetrahedra: out[t][u] = silu(W in[t] + b),
// optionally sp[t][u] = silu'(z).  `in` and `out` may be the same buffer (each
// 16-tet tile is read completely before it is written).
// With POW2 the layer works on y = -log2(e) z (bias scaled here, the input
// already scaled) and writes y * sigmoid(z); sp must then be null.
template <int KS, int IN_STRIDE, bool POW2 = false>
__device__ __forceinline__ void hidden_layer(const __bf16* in, __bf16* out, __bf16* sp,
                                             const bf16x8 (&w)[4][KS], const float* __restrict__ bias)
{
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    f32x4 b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) b[mt][i] = POW2 ? kNegLog2e * bias[mt * 16 + 4 * g + i] : bias[mt * 16 + 4 * g + i];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int t = nt * 16 + col;
        bf16x8 bx[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bx[ks] = ld8(in + t * IN_STRIDE + ks * 32 + 8 * g);
        f32x4 acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            acc[mt] = b[mt];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) acc[mt] = mfma(w[mt][ks], bx[ks], acc[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[mt][i];
                const float s = POW2 ? sigmoid_pow2(z) : sigmoid(z);
                const int u = mt * 16 + 4 * g + i;
                out[t * kHS + u] = to_bf16(z * s);
                if (!POW2 && sp) sp[t * kHS + u] = to_bf16(s * (1.0f + z * (1.0f - s)));
            }
    }
}

// Output layer: logits lg[t][c] (float, row stride 8) for the wave's 64 tets.
// With POW2 (negated output weights, base-2 activations) the logits come out
// multiplied by log2(e).
template <bool POW2 = false>
__device__ __forceinline__ void output_layer(const __bf16* h3, float* lg, const Net& N)
{
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int t = nt * 16 + col;
        f32x4 acc;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = 4 * g + i < kOut ? (POW2 ? kLog2e : 1.0f) * N.w[oB4 + 4 * g + i] : 0.0f;
        acc = mfma(N.w4[0], ld8(h3 + t * kHS + 8 * g), acc);
        acc = mfma(N.w4[1], ld8(h3 + t * kHS + 32 + 8 * g), acc);
        if (g < 2) *reinterpret_cast<f32x4*>(lg + t * kOut + 4 * g) = acc;
    }
}

// Softmax of the logits over the cells in `mask`; p is 0 outside it.
__device__ __forceinline__ void masked_softmax(const float* lg, int mask, float (&p)[kOut])
{
    float mx = -INFINITY;
#pragma unroll
    for (int c = 0; c < kOut; ++c)
        if ((mask >> c) & 1) mx = fmaxf(mx, lg[c]);
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        p[c] = ((mask >> c) & 1) ? __expf(lg[c] - mx) : 0.0f;
        s += p[c];
    }
    const float inv = 1.0f / s;
#pragma unroll
    for (int c = 0; c < kOut; ++c) p[c] *= inv;
}

// ---------------------------------------------------------------------------
// Eligibility and exact labels
// ---------------------------------------------------------------------------

// Decides whether tetrahedron T goes to the network: finite, non-zero volume
// (|D| > 1e-12 l^3, the zero-volume rule of the exact path) and a bbox of at
// most 2 cells per axis holding at least min_cells cells.  Fills the
// vertices relative to the unwrapped bbox origin and the per-axis spans.
__device__ __forceinline__ bool small_tet(const Tet64& T, int min_cells, double (&vr)[4][3],
                                          double (&lo)[3], int (&span)[3])
{
    if (!(isfinite(T.D) && isfinite(T.l3))) return false;
    if (fabs(T.D) <= 1e-12 * T.l3) return false;
    int cells = 1;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double mn = fmin(fmin(T.v[0][a], T.v[1][a]), fmin(T.v[2][a], T.v[3][a]));
        const double mx = fmax(fmax(T.v[0][a], T.v[1][a]), fmax(T.v[2][a], T.v[3][a]));
        lo[a] = floor(mn);
        const double sp = floor(mx) - lo[a];
        ok = ok && sp <= 1.0;
        span[a] = sp <= 1.0 ? (int)sp : 2;
        cells *= span[a] + 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) vr[q][a] = T.v[q][a] - lo[a];
    }
    return ok && cells >= min_cells;
}

__device__ __forceinline__ int cell_mask(const int (&span)[3])
{
    int m = 0;
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
        if (dx <= span[0] && dy <= span[1] && dz <= span[2]) m |= 1 << c;
    }
    return m;
}

// Exact fraction of T (vertices vr relative to lo) in cell lo + d: the middle
// plane of every axis with span 1 bounds the cell (x <= 1 for d = 0, x >= 1
// for d = 1), coordinates taken relative to the cell's low corner.
__device__ __forceinline__ double exact_fraction(const double (&vr)[4][3], const int (&span)[3], int c)
{
    const int d[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
    double x[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) x[q][a] = vr[q][a] - (double)d[a];
    TetEval<double> ev;
    int k = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (span[a] != 1) continue;
        ev.axis[k] = a;
        ev.sgn[k] = d[a] ? 1.0 : -1.0;  // x >= 0 or 1 - x >= 0
        ev.off[k] = d[a] ? 0.0 : 1.0;
        ++k;
    }
    for (int s = k; s < 6; ++s) {
        ev.axis[s] = 0;
        ev.sgn[s] = 1.0;
        ev.off[s] = 0.0;
    }
    if (k == 0) return 1.0;
    return inside_fraction<double, 0, 3>(x, k, ev);
}

// Exact fractions of given tetrahedra (vertices relative to the low corner
// of a 2x2x2 block of cells, every coordinate in [0, 2)) in the block's 8
// cells, cell c = 4 dx + 2 dy + dz.  A zero-volume tetrahedron (the rule of
// the deposit, |D| <= 1e-12 l^3) puts everything in its centroid's cell;
// vertices outside the block or non-finite give NaN in all 8 entries.
__global__ __launch_bounds__(256) void exact_fractions_kernel(const float* tets, double* frac,
                                                               int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[4][3];
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[q][a] = (double)tets[(i * 4 + q) * 3 + a];
            ok = ok && v[q][a] >= 0.0 && v[q][a] < 2.0;  // false for NaN
        }
    double* f = frac + i * kOut;
    if (!ok) {
#pragma unroll
        for (int c = 0; c < kOut; ++c) f[c] = __builtin_nan("");
        return;
    }
    double e[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int a = 0; a < 3; ++a) e[m][a] = v[m + 1][a] - v[0][a];
    const double D = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                     e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                     e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    double l2 = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int k = m + 1; k < 4; ++k) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) s += (v[m][a] - v[k][a]) * (v[m][a] - v[k][a]);
            l2 = fmax(l2, s);
        }
    if (fabs(D) <= 1e-12 * l2 * sqrt(l2)) {
        int cc = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double x = 0.25 * (v[0][a] + v[1][a] + v[2][a] + v[3][a]);
            cc |= (x >= 1.0 ? 1 : 0) << (2 - a);
        }
#pragma unroll
        for (int c = 0; c < kOut; ++c) f[c] = c == cc ? 1.0 : 0.0;
        return;
    }
    // bbox origin lo (0 or 1 per axis) and span, then the cells inside it
    double vr[4][3];
    int lo[3], span[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double mn = fmin(fmin(v[0][a], v[1][a]), fmin(v[2][a], v[3][a]));
        const double mx = fmax(fmax(v[0][a], v[1][a]), fmax(v[2][a], v[3][a]));
        lo[a] = mn >= 1.0 ? 1 : 0;
        span[a] = (mx >= 1.0 ? 1 : 0) - lo[a];
#pragma unroll
        for (int q = 0; q < 4; ++q) vr[q][a] = v[q][a] - (double)lo[a];
    }
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        const int d[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
        bool in = true;
        int cl = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int r = d[a] - lo[a];
            in = in && r >= 0 && r <= span[a];
            cl |= (r & 1) << (2 - a);
        }
        f[c] = in ? exact_fraction(vr, span, cl) : 0.0;
    }
}

struct ExampleArgs {
    const float* pos;
    int np[3];
    int nc[3];
    double scale[3];
    int64_t tet0;       // first tetrahedron (6 * first cube)
    int64_t ntet;       // tetrahedra to scan
    int min_cells;
    float* feat;        // [capacity][12]
    double* frac;       // [capacity][8]
    uint8_t* mask;      // [capacity]
    int64_t* tet_id;    // [capacity] or null
    int64_t capacity;
    unsigned int* block_count;         // [nblocks]
    unsigned long long* block_offset;  // [nblocks + 1]
};

constexpr int kExBlock = 256;

__device__ __forceinline__ bool example_of(const ExampleArgs& A, int64_t tid, Tet64& T,
                                           double (&vr)[4][3], double (&lo)[3], int (&span)[3])
{
    if (tid >= A.tet0 + A.ntet) return false;
    const int64_t cube = tid / 6;
    const int p = (int)(tid - cube * 6);
    const int64_t kk = cube % A.np[2];
    const int64_t jj = (cube / A.np[2]) % A.np[1];
    const int64_t ii = cube / ((int64_t)A.np[1] * A.np[2]);
    make_tet(A.pos, A.np[0], A.np[1], A.np[2], A.scale, A.nc, ii, jj, kk, p, T);
    return small_tet(T, A.min_cells, vr, lo, span);
}

__global__ __launch_bounds__(kExBlock) void example_count_kernel(ExampleArgs A)
{
    const int64_t tid = A.tet0 + (int64_t)blockIdx.x * kExBlock + threadIdx.x;
    Tet64 T;
    double vr[4][3], lo[3];
    int span[3];
    const bool e = example_of(A, tid, T, vr, lo, span);
    const int n = __syncthreads_count(e);
    if (threadIdx.x == 0) A.block_count[blockIdx.x] = (unsigned)n;
}

// Exclusive scan of the block counts (one workgroup).
__global__ __launch_bounds__(1024) void example_scan_kernel(const unsigned int* count,
                                                            unsigned long long* offset, int64_t n)
{
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = t * per, e = b + per < n ? b + per : n;
    unsigned long long s = 0;
    for (int64_t i = b; i < e; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        unsigned long long run = 0;
        for (int i = 0; i < 1024; ++i) {
            const unsigned long long v = part[i];
            part[i] = run;
            run += v;
        }
        offset[n] = run;
    }
    __syncthreads();
    unsigned long long run = part[t];
    for (int64_t i = b; i < e; ++i) {
        offset[i] = run;
        run += count[i];
    }
}

__global__ __launch_bounds__(kExBlock) void example_write_kernel(ExampleArgs A)
{
    __shared__ unsigned int wave_base[kExBlock / 64];
    const int64_t tid = A.tet0 + (int64_t)blockIdx.x * kExBlock + threadIdx.x;
    Tet64 T;
    double vr[4][3], lo[3];
    int span[3];
    const bool e = example_of(A, tid, T, vr, lo, span);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t bal = __ballot(e);
    if (lane == 0) wave_base[w] = (unsigned)__popcll(bal);
    __syncthreads();
    unsigned int base = 0;
    for (int i = 0; i < w; ++i) base += wave_base[i];
    if (!e) return;
    const unsigned int rank = base + (unsigned)__popcll(bal & ((1ull << lane) - 1ull));
    const int64_t dst = (int64_t)A.block_offset[blockIdx.x] + rank;
    if (dst >= A.capacity) return;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) A.feat[dst * kIn + 3 * q + a] = (float)vr[q][a];
    const int m = cell_mask(span);
    A.mask[dst] = (uint8_t)m;
    for (int c = 0; c < kOut; ++c)
        A.frac[dst * kOut + c] = ((m >> c) & 1) ? exact_fraction(vr, span, c) : 0.0;
    if (A.tet_id) A.tet_id[dst] = tid;
}

// ---------------------------------------------------------------------------
// Forward (probabilities) for a feature list
// ---------------------------------------------------------------------------

struct NetIO {
    const float* w;       // packed parameters, float32
    const float* feat;    // [n][12]
    const uint8_t* mask;  // [n]
    const double* frac;   // [n][8] labels (backward)
    const int64_t* idx;   // sample indices of the batch, or null (identity)
    int64_t n;
    float* probs;         // [n][8] (forward)
    float* grad;          // [kNParams] (backward, accumulated)
    double* loss;         // mean loss (backward, accumulated), may be null
};

__device__ __forceinline__ void load_row(const float* feat, int64_t s, float (&x)[kIn])
{
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = feat[s * kIn + k];
}

__global__ __launch_bounds__(64) void forward_kernel(NetIO io)
{
    __shared__ __attribute__((aligned(16))) __bf16 hb[64 * kHS];
    __shared__ __attribute__((aligned(16))) float lg[64 * kOut];
    Net N;
    load_net(io.w, N);
    const int lane = threadIdx.x;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < io.n; base += (int64_t)gridDim.x * 64) {
        const int64_t s = base + lane;
        float x[kIn];
        int m = 0, r = 0;
        if (s < io.n) {
            load_row(io.feat, s, x);
            m = io.mask[s];
            r = canonical_pose(x, m);
        } else {
#pragma unroll
            for (int k = 0; k < kIn; ++k) x[k] = 0.0f;
        }
        put_features(hb + lane * kHS, x);
        __syncthreads();
        hidden_layer<1, kHS>(hb, hb, nullptr, N.w1, N.w + oB1);
        hidden_layer<2, kHS>(hb, hb, nullptr, N.w2, N.w + oB2);
        hidden_layer<2, kHS>(hb, hb, nullptr, N.w3, N.w + oB3);
        output_layer(hb, lg, N);
        __syncthreads();
        if (s < io.n) {
            float p[kOut];
            masked_softmax(lg + lane * kOut, m, p);
#pragma unroll
            for (int c = 0; c < kOut; ++c) io.probs[s * kOut + (c ^ r)] = p[c];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Backward: gradient of the mean soft-label cross entropy over the n samples
// ---------------------------------------------------------------------------

// Transposed weight fragment: A[row = v][k = u] = W[u][v] for a 64 x 64 matrix.
__device__ __forceinline__ bf16x8 wt_frag(const float* __restrict__ W, int mt, int ks)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    bf16x8 f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = to_bf16(W[(ks * 32 + 8 * g + e) * kH + mt * 16 + r]);
    return f;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// dW[u][v] += sum_t G[t][u] H[t][v] over the wave's 64 samples (16-row tiles
// of u: NU, of v: NV; H row stride HS) and db[u] += sum_t G[t][u].
template <int NU, int NV, int HS>
__device__ __forceinline__ void weight_grad(const __bf16* G, const __bf16* H, float* dW, int ldw,
                                            int v_fold, float* db)
{
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    for (int mt = 0; mt < NU; ++mt) {
        bf16x8 a[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) a[ks] = ld8s(G + (ks * 32 + 8 * g) * kHS + mt * 16 + col, kHS);
        for (int nt = 0; nt < NV; ++nt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                acc = mfma(a[ks], ld8s(H + (ks * 32 + 8 * g) * HS + nt * 16 + col, HS), acc);
            const int v = nt * 16 + col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = mt * 16 + 4 * g + i;
                if (v_fold > 0) {
                    // input layer: columns hi (k) and lo (k + 12) both belong to x_k
                    if (v < v_fold) atomicAdd(dW + u * ldw + v, acc[i]);
                    else if (v < 2 * v_fold) atomicAdd(dW + u * ldw + v - v_fold, acc[i]);
                } else {
                    atomicAdd(dW + u * ldw + v, acc[i]);
                }
            }
        }
    }
    if (db) {
        float s = 0.0f;
        for (int t = 0; t < 64; ++t) s += from_bf16(G[t * kHS + lane]);
        atomicAdd(db + lane, s);
    }
}

// G_out[t][v] = sp[t][v] * sum_u Wt-fragment[v][u] G_in[t][u]  (64 x 64 weights)
__device__ __forceinline__ void input_grad(const __bf16* Gin, __bf16* Gout, const __bf16* sp,
                                           const float* __restrict__ W)
{
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 a0 = wt_frag(W, mt, 0), a1 = wt_frag(W, mt, 1);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int t = nt * 16 + col;
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma(a0, ld8(Gin + t * kHS + 8 * g), acc);
            acc = mfma(a1, ld8(Gin + t * kHS + 32 + 8 * g), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = mt * 16 + 4 * g + i;
                Gout[t * kHS + v] = to_bf16(acc[i] * from_bf16(sp[t * kHS + v]));
            }
        }
    }
}

struct BackLds {
    __bf16 x[64 * kXS];
    __bf16 h1[64 * kHS], h2[64 * kHS], h3[64 * kHS];
    __bf16 s1[64 * kHS], s2[64 * kHS], s3[64 * kHS];
    __bf16 ga[64 * kHS], gb[64 * kHS];
};

// One wave per workgroup; the workgroups share the batch's 64-sample tiles
// (blockIdx.x, stepping by gridDim.x) and add into io.grad and io.loss.
__device__ __forceinline__ void backward_pass(const NetIO& io, BackLds& L)
{
    Net N;
    load_net(io.w, N);
    const int lane = threadIdx.x;
    const float inv_n = 1.0f / (float)io.n;
    const float* W = io.w;
    float* dW = io.grad;
    float db4[kOut];
#pragma unroll
    for (int c = 0; c < kOut; ++c) db4[c] = 0.0f;
    double lsum = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < io.n; base += (int64_t)gridDim.x * 64) {
        const int64_t pos = base + lane;
        const bool valid = pos < io.n;
        const int64_t s = valid ? (io.idx ? io.idx[pos] : pos) : 0;
        float x[kIn];
        const int m = valid ? io.mask[s] : 0;
        int r = 0;
        if (valid) {
            load_row(io.feat, s, x);
            r = canonical_pose(x, m);
        } else {
#pragma unroll
            for (int k = 0; k < kIn; ++k) x[k] = 0.0f;
        }
        // input tile: the first 32 columns of a kXS-wide row
        {
            __bf16* row = L.x + lane * kXS;
            put_features(row, x);
        }
        __syncthreads();
        hidden_layer<1, kXS>(L.x, L.h1, L.s1, N.w1, N.w + oB1);
        hidden_layer<2, kHS>(L.h1, L.h2, L.s2, N.w2, N.w + oB2);
        hidden_layer<2, kHS>(L.h2, L.h3, L.s3, N.w3, N.w + oB3);
        float* lg = reinterpret_cast<float*>(L.gb);
        output_layer(L.h3, lg, N);
        __syncthreads();
        // dz4 = (p sum(y) - y) / n on the masked-in cells; row t of ga holds
        // dz4 in columns 0..7 and zeros up to 31 (the K depth of dH3).
        float dz[kOut];
        {
            float p[kOut];
            if (valid) masked_softmax(lg + lane * kOut, m, p);
            // labels in the canonical cell order (the mask is the same in both poses)
            float ysum = 0.0f, y[kOut];
#pragma unroll
            for (int c = 0; c < kOut; ++c) {
                y[c] = valid && ((m >> c) & 1) ? (float)io.frac[s * kOut + (c ^ r)] : 0.0f;
                ysum += y[c];
            }
            // loss from the log-softmax, log p_c = z_c - max - log(sum exp(z - max))
            double l = 0.0;
            if (valid) {
                const float* z = lg + lane * kOut;
                double mx = -INFINITY, se = 0.0;
#pragma unroll
                for (int c = 0; c < kOut; ++c)
                    if ((m >> c) & 1) mx = fmax(mx, (double)z[c]);
#pragma unroll
                for (int c = 0; c < kOut; ++c)
                    if ((m >> c) & 1) se += exp((double)z[c] - mx);
                const double lse = mx + log(se);
#pragma unroll
                for (int c = 0; c < kOut; ++c)
                    if (((m >> c) & 1) && y[c] != 0.0f) l -= (double)y[c] * ((double)z[c] - lse);
            }
#pragma unroll
            for (int c = 0; c < kOut; ++c) {
                const bool in = valid && ((m >> c) & 1);
                dz[c] = in ? (p[c] * ysum - y[c]) * inv_n : 0.0f;
                db4[c] += dz[c];
            }
            lsum += l;
        }
        __syncthreads();
        {
            __bf16* row = L.ga + lane * kHS;
#pragma unroll
            for (int c = 0; c < kOut; ++c) row[c] = to_bf16(dz[c]);
#pragma unroll
            for (int c = kOut; c < 32; ++c) row[c] = to_bf16(0.0f);
        }
        __syncthreads();
        // output layer: dW4[c][u] = sum_t dz4[t][c] h3[t][u] (rows c >= 8 dropped)
        {
            const int col = lane & 15, g = lane >> 4;
            bf16x8 a[2];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) a[ks] = ld8s(L.ga + (ks * 32 + 8 * g) * kHS + col, kHS);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks)
                    acc = mfma(a[ks], ld8s(L.h3 + (ks * 32 + 8 * g) * kHS + nt * 16 + col, kHS), acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = 4 * g + i;
                    if (c < kOut) atomicAdd(dW + oW4 + c * kH + nt * 16 + col, acc[i]);
                }
            }
            // dz3[t][u] = silu'(z3) * sum_c W4[c][u] dz4[t][c]  -> gb
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                bf16x8 w4t;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int c = 8 * g + e;
                    w4t[e] = to_bf16(c < kOut ? W[oW4 + c * kH + mt * 16 + col] : 0.0f);
                }
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int t = nt * 16 + col;
                    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                    acc = mfma(w4t, ld8(L.ga + t * kHS + 8 * g), acc);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int u = mt * 16 + 4 * g + i;
                        L.gb[t * kHS + u] = to_bf16(acc[i] * from_bf16(L.s3[t * kHS + u]));
                    }
                }
            }
        }
        __syncthreads();
        weight_grad<4, 4, kHS>(L.gb, L.h2, dW + oW3, kH, 0, dW + oB3);
        input_grad(L.gb, L.ga, L.s2, W + oW3);
        __syncthreads();
        weight_grad<4, 4, kHS>(L.ga, L.h1, dW + oW2, kH, 0, dW + oB2);
        input_grad(L.ga, L.gb, L.s1, W + oW2);
        __syncthreads();
        weight_grad<4, 2, kXS>(L.gb, L.x, dW + oW1, kIn, kIn, dW + oB1);
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        const float v = wave_sum(db4[c]);
        if (lane == 0) atomicAdd(dW + oB4 + c, v);
    }
    lsum = wave_sum(lsum);
    if (lane == 0 && io.loss) atomicAdd(io.loss, lsum / (double)io.n);
}

__global__ __launch_bounds__(64) void backward_kernel(NetIO io)
{
    __shared__ __attribute__((aligned(16))) BackLds L;
    backward_pass(io, L);
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Adam (Kingma & Ba) for parameter i: moments from gradient g[i], update
// with the bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__device__ __forceinline__ void adam_update(float* w, float gi, float* m, float* v, int64_t i, float lr,
                                            float b1, float b2, float eps, float c1, float c2)
{
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    adam_update(w, g[i], m, v, i, lr, b1, b2, eps, c1, c2);
}

// Several training steps in one cooperative launch: per step, the batch's
// gradient (every workgroup adds its tiles), a grid barrier, Adam over the
// parameters with the gradient cleared behind it, a grid barrier.  Every
// workgroup runs the same steps, so every barrier is reached by all.
struct TrainArgs {
    float* w;
    const float* feat;
    const double* frac;
    const uint8_t* mask;
    const int64_t* order;  // sample order; step s takes order[s * batch ..]
    int64_t n;             // entries of order
    int64_t batch;
    int64_t steps;
    int64_t step0;         // Adam updates done before this launch
    const float* lr;       // [steps]
    float b1, b2, eps;
    float* m;
    float* v;
    float* grad;           // [kNParams], scratch: cleared here, cleared again at the end
    double* losses;        // [steps] or null
};

__global__ __launch_bounds__(64) void train_kernel(TrainArgs A)
{
    __shared__ __attribute__((aligned(16))) BackLds L;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int64_t gt = (int64_t)blockIdx.x * 64 + threadIdx.x, gs = (int64_t)gridDim.x * 64;
    for (int64_t i = gt; i < kNParams; i += gs) A.grad[i] = 0.0f;
    if (A.losses)
        for (int64_t i = gt; i < A.steps; i += gs) A.losses[i] = 0.0;
    grid.sync();
    for (int64_t s = 0; s < A.steps; ++s) {
        NetIO io = {};
        io.w = A.w;
        io.feat = A.feat;
        io.frac = A.frac;
        io.mask = A.mask;
        io.idx = A.order + s * A.batch;
        io.n = min(A.batch, A.n - s * A.batch);
        io.grad = A.grad;
        io.loss = A.losses ? A.losses + s : nullptr;
        backward_pass(io, L);
        grid.sync();
        const double t = (double)(A.step0 + s + 1);
        const float c1 = (float)(1.0 - pow((double)A.b1, t)), c2 = (float)(1.0 - pow((double)A.b2, t));
        const float lr = A.lr[s];
        for (int64_t i = gt; i < kNParams; i += gs) {
            adam_update(A.w, A.grad[i], A.m, A.v, i, lr, A.b1, A.b2, A.eps, c1, c2);
            A.grad[i] = 0.0f;
        }
        grid.sync();
    }
}

// ---------------------------------------------------------------------------
// Deposit of the small tetrahedra through the network
// ---------------------------------------------------------------------------

constexpr int kRing = 128;  // per-wave queue of eligible tetrahedra

template <typename OutT>
__global__ __launch_bounds__(64, 2) void surrogate_deposit_kernel(UniformArgs P, int64_t n_chunks,
                                                                   unsigned long long* exact_mask)
{
    __shared__ __attribute__((aligned(16))) float qx[kRing * kIn];
    __shared__ int qm[kRing * 4];  // mask, lo wrapped into [0, nc) per axis
    __shared__ __attribute__((aligned(16))) __bf16 hb[64 * kHS];
    __shared__ __attribute__((aligned(16))) float lg[64 * kOut];
    Net N;
    load_net(P.surrogate, N, true);
    OutT* out = reinterpret_cast<OutT*>(P.out);
    const int lane = threadIdx.x;
    int head = 0, qn = 0;
    double macc = 0.0;
    unsigned long long n_sur = 0, n_nz = 0, n_inv = 0;

    // After the network, the activation buffer holds the batch's cell masses:
    // a tile over the union of the n tets' 2x2x2 blocks, flushed with one
    // global atomic per non-zero cell (the batch's tets come from neighbouring
    // Lagrangian cubes and share most of their cells).  A batch whose union
    // is larger than the buffer adds straight to the grid.
    constexpr int kAcc = (int)(sizeof(hb) / (sizeof(OutT)));  // OutT entries in the bytes of hb
    static_assert(kAcc < (1 << 21), "flush quotients");
    OutT* acc = reinterpret_cast<OutT*>(hb);
    auto run = [&](int n) {
        if (lane < n) {
            const int slot = (head + lane) & (kRing - 1);
            float x[kIn];
#pragma unroll
            for (int k = 0; k < kIn; ++k) x[k] = kNegLog2e * qx[slot * kIn + k];
            put_features(hb + lane * kHS, x);
        } else {
            float x[kIn];
#pragma unroll
            for (int k = 0; k < kIn; ++k) x[k] = 0.0f;
            put_features(hb + lane * kHS, x);
        }
        __syncthreads();
        hidden_layer<1, kHS, true>(hb, hb, nullptr, N.w1, N.w + oB1);
        hidden_layer<2, kHS, true>(hb, hb, nullptr, N.w2, N.w + oB2);
        hidden_layer<2, kHS, true>(hb, hb, nullptr, N.w3, N.w + oB3);
        output_layer<true>(hb, lg, N);
        __syncthreads();
        // the union box, in cells relative to lane 0's block (minimum image)
        const int slot0 = head & (kRing - 1);
        int lo[3], mn[3], mx[3], E[3];
        {
            const int slot = (head + (lane < n ? lane : 0)) & (kRing - 1);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int ref = qm[slot0 * 4 + 1 + a], nca = P.nc[a];
                int d = qm[slot * 4 + 1 + a] - ref;
                if (2 * d > nca) d -= nca;
                else if (2 * d < -nca) d += nca;
                lo[a] = d;
                mn[a] = d;
                mx[a] = d;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(mn[a], __shfl_xor(mn[a], off, 64));
                    mx[a] = max(mx[a], __shfl_xor(mx[a], off, 64));
                }
#pragma unroll
            for (int a = 0; a < 3; ++a) E[a] = mx[a] - mn[a] + 2;
        }
        const bool tiled = (int64_t)E[0] * E[1] * E[2] <= kAcc;
        const int ncell = E[0] * E[1] * E[2];
        if (tiled) {
            for (int i = lane; i < ncell; i += 64) acc[i] = OutT(0);
            __syncthreads();
        }
        if (lane < n) {
            const int slot = (head + lane) & (kRing - 1);
            const int m = qm[slot * 4] & 0xFF, r = qm[slot * 4] >> 8;
            // softmax of the base-2 logits over the cells in m (the largest
            // term is 1, so the sum is at least 1), in the tet's own cell order
            float p[kOut], mx = -INFINITY, s = 0.0f;
#pragma unroll
            for (int c = 0; c < kOut; ++c)
                if ((m >> c) & 1) mx = fmaxf(mx, lg[lane * kOut + c]);
#pragma unroll
            for (int c = 0; c < kOut; ++c) {
                p[c] = ((m >> c) & 1) ? __builtin_amdgcn_exp2f(lg[lane * kOut + c] - mx) : 0.0f;
                s += p[c];
            }
            xor_cells(p, r);
            const float inv = __builtin_amdgcn_rcpf(s);
            // FP64 shares; the last cell takes the residual so the deposits
            // sum to m
            int last = 0;
#pragma unroll
            for (int c = 0; c < kOut; ++c)
                if ((m >> c) & 1) last = c;
            const int ib = ((lo[0] - mn[0]) * E[1] + (lo[1] - mn[1])) * E[2] + (lo[2] - mn[2]);
            double given = 0.0;
#pragma unroll
            for (int c = 0; c < kOut; ++c) {
                if (!((m >> c) & 1)) continue;
                const double d = c == last ? P.m - given : (double)(p[c] * inv) * P.m;
                given += d;
                if (d == 0.0) continue;
                if (tiled) {
                    const int i = ib + ((c >> 2) & 1) * E[1] * E[2] + ((c >> 1) & 1) * E[2] + (c & 1);
                    __hip_atomic_fetch_add(acc + i, (OutT)(d * P.out_scale), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    const int a = wrap_cell(qm[slot * 4 + 1] + ((c >> 2) & 1), P.nc[0]);
                    const int b = wrap_cell(qm[slot * 4 + 2] + ((c >> 1) & 1), P.nc[1]);
                    const int z = wrap_cell(qm[slot * 4 + 3] + (c & 1), P.nc[2]);
                    global_add(out + ((int64_t)a * P.nc[1] + b) * P.nc[2] + z, (OutT)(d * P.out_scale));
                }
                ++n_nz;
            }
            macc += given;
        }
        __syncthreads();
        if (tiled) {
            // one global atomic per non-zero cell of the tile; ncell <= kAcc
            // keeps the quotients exact, and the cell coordinates lie in
            // [-nc/2, 2 nc) (lane 0's wrapped block plus offsets of at most
            // nc/2 + E - 1), so one correction wraps them
            const int E12 = E[1] * E[2];
            const float rE2 = __builtin_amdgcn_rcpf((float)E[2]), rE12 = __builtin_amdgcn_rcpf((float)E12);
            for (int i = lane; i < ncell; i += 64) {
                const OutT v = acc[i];
                if (v == OutT(0)) continue;
                const int i0 = quot_small(i, rE12), rem = i - i0 * E12;
                const int i1 = quot_small(rem, rE2), i2 = rem - i1 * E[2];
                int g[3];
                const int li[3] = {i0, i1, i2};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int x = qm[slot0 * 4 + 1 + a] + mn[a] + li[a], nca = P.nc[a];
                    g[a] = x < 0 ? x + nca : (x >= nca ? x - nca : x);
                }
                global_add(out + ((int64_t)g[0] * P.nc[1] + g[1]) * P.nc[2] + g[2], v);
            }
            __syncthreads();
        }
        head = (head + n) & (kRing - 1);
        qn -= n;
    };

    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        const int64_t tid = chunk * 64 + lane;
        bool e = false;
        double vr[4][3], lo[3];
        int span[3];
        if (tid < P.ntet) {
            const int64_t cube = tid / 6;
            const int p = (int)(tid - cube * 6);
            const int64_t kk = cube % P.np[2];
            const int64_t jj = (cube / P.np[2]) % P.np[1];
            const int64_t ii = cube / ((int64_t)P.np[1] * P.np[2]);
            Tet64 T;
            make_tet(P.pos, P.np[0], P.np[1], P.np[2], P.scale, P.nc, ii, jj, kk, p, T);
            e = small_tet(T, 2, vr, lo, span);
            // the exact pass skips these tets, so their orientation is counted here
            if (e && (double)kuhn_sign(p) * T.D < 0.0) ++n_inv;
        }
        const uint64_t bal = __ballot(e);
        if (exact_mask) {
            const uint64_t rest = __ballot(tid < P.ntet && !e);
            if (lane == 0) exact_mask[chunk] = rest;
        }
        if (e) {
            const int rank = (int)__popcll(bal & ((1ull << lane) - 1ull));
            const int slot = (head + qn + rank) & (kRing - 1);
            float x[kIn];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int a = 0; a < 3; ++a) x[3 * q + a] = (float)vr[q][a];
            const int m = cell_mask(span);
            const int r = canonical_pose(x, m);
#pragma unroll
            for (int k = 0; k < kIn; ++k) qx[slot * kIn + k] = x[k];
            qm[slot * 4] = m | (r << 8);
#pragma unroll
            for (int a = 0; a < 3; ++a) qm[slot * 4 + 1 + a] = wrap_index(lo[a], P.nc[a]);
            ++n_sur;
        }
        qn += (int)__popcll(bal);
        __syncthreads();
        if (qn >= 64) run(64);
    }
    if (qn > 0) run(qn);

    macc = wave_sum(macc);
    if (lane == 0 && P.mass_sum && macc != 0.0) global_add(P.mass_sum, macc);
    if (P.stats) {
        unsigned long long a = n_sur, b = n_nz, c = n_inv;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
            c += __shfl_xor(c, off, 64);
        }
        if (lane == 0) {
            if (a) atomicAdd(P.stats + 6, a);
            if (b) atomicAdd(P.stats + 3, b);
            if (c) atomicAdd(P.stats + 4, c);
        }
    }
}

}  // namespace

int surrogate_param_count() { return kNParams; }

size_t example_workspace_bytes(int64_t ntet)
{
    const int64_t nb = (ntet + kExBlock - 1) / kExBlock;
    return (size_t)nb * sizeof(unsigned int) + 256 + (size_t)(nb + 1) * sizeof(unsigned long long);
}

hipError_t launch_examples(const UniformArgs& P, int64_t first_cube, int64_t n_cubes, int min_cells,
                           float* feat, double* frac, uint8_t* mask, int64_t* tet_id,
                           int64_t capacity, void* ws, int64_t* n_out, hipStream_t stream)
{
    ExampleArgs A;
    A.pos = P.pos;
    for (int a = 0; a < 3; ++a) {
        A.np[a] = P.np[a];
        A.nc[a] = P.nc[a];
        A.scale[a] = P.scale[a];
    }
    A.tet0 = 6 * first_cube;
    A.ntet = 6 * n_cubes;
    A.min_cells = min_cells;
    A.feat = feat;
    A.frac = frac;
    A.mask = mask;
    A.tet_id = tet_id;
    A.capacity = capacity;
    const int64_t nb = (A.ntet + kExBlock - 1) / kExBlock;
    char* base = static_cast<char*>(ws);
    A.block_count = reinterpret_cast<unsigned int*>(base);
    size_t off = ((size_t)nb * sizeof(unsigned int) + 255) & ~(size_t)255;
    A.block_offset = reinterpret_cast<unsigned long long*>(base + off);
    *n_out = 0;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(example_count_kernel, dim3((unsigned)nb), dim3(kExBlock), 0, stream, A);
    hipLaunchKernelGGL(example_scan_kernel, dim3(1), dim3(1024), 0, stream,
                       (const unsigned int*)A.block_count, A.block_offset, nb);
    hipLaunchKernelGGL(example_write_kernel, dim3((unsigned)nb), dim3(kExBlock), 0, stream, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long total = 0;
    e = hipMemcpyAsync(&total, A.block_offset + nb, sizeof(total), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    *n_out = (int64_t)total;
    return hipSuccess;
}

static int net_grid(int64_t n)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    const int64_t tiles = (n + 63) / 64;
    const int64_t cap = (int64_t)cus * 8;
    return (int)(tiles < cap ? (tiles > 0 ? tiles : 1) : cap);
}

// Workgroups of a training launch: one per 64-sample tile of a batch, at most
// 256 (the batch's tiles are shared out when there are more).
static int train_grid(int64_t batch) { return (int)((batch + 63) / 64 < 256 ? (batch + 63) / 64 : 256); }

hipError_t launch_exact_fractions(const float* tets, double* frac, int64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(exact_fractions_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       tets, frac, n);
    return hipGetLastError();
}

hipError_t launch_surrogate_forward(const float* w, const float* feat, const uint8_t* mask, int64_t n,
                                    float* probs, hipStream_t stream)
{
    NetIO io = {};
    io.w = w;
    io.feat = feat;
    io.mask = mask;
    io.n = n;
    io.probs = probs;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(forward_kernel, dim3(net_grid(n)), dim3(64), 0, stream, io);
    return hipGetLastError();
}

hipError_t launch_surrogate_backward(const float* w, const float* feat, const double* frac,
                                     const uint8_t* mask, const int64_t* idx, int64_t n, float* grad,
                                     double* loss, hipStream_t stream)
{
    hipLaunchKernelGGL(fill_kernel<float>, dim3((kNParams + 255) / 256), dim3(256), 0, stream, grad,
                       (int64_t)kNParams, 0.0f);
    if (loss) hipLaunchKernelGGL(fill_kernel<double>, dim3(1), dim3(64), 0, stream, loss, (int64_t)1, 0.0);
    if (n > 0) {
        NetIO io = {};
        io.w = w;
        io.feat = feat;
        io.frac = frac;
        io.mask = mask;
        io.idx = idx;
        io.n = n;
        io.grad = grad;
        io.loss = loss;
        hipLaunchKernelGGL(backward_kernel, dim3(net_grid(n)), dim3(64), 0, stream, io);
    }
    return hipGetLastError();
}

hipError_t launch_surrogate_adam(float* w, const float* grad, float* m, float* v, int64_t step,
                                 float lr, float beta1, float beta2, float eps, hipStream_t stream)
{
    const double c1 = 1.0 - pow((double)beta1, (double)step);
    const double c2 = 1.0 - pow((double)beta2, (double)step);
    hipLaunchKernelGGL(adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, stream, w, grad, m, v,
                       (int64_t)kNParams, lr, beta1, beta2, eps, (float)c1, (float)c2);
    return hipGetLastError();
}

hipError_t launch_surrogate_train(float* w, const float* feat, const double* frac, const uint8_t* mask,
                                  const int64_t* order, int64_t n, int64_t batch, int64_t steps,
                                  int64_t step0, const float* lr, float beta1, float beta2, float eps,
                                  float* m, float* v, float* grad, double* losses, hipStream_t stream)
{
    if (steps == 0) return hipSuccess;
    TrainArgs A;
    A.w = w;
    A.feat = feat;
    A.frac = frac;
    A.mask = mask;
    A.order = order;
    A.n = n;
    A.batch = batch;
    A.steps = steps;
    A.step0 = step0;
    A.lr = lr;
    A.b1 = beta1;
    A.b2 = beta2;
    A.eps = eps;
    A.m = m;
    A.v = v;
    A.grad = grad;
    A.losses = losses;
    void* args[] = {&A};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(train_kernel), dim3(train_grid(batch)),
                                      dim3(64), args, 0, stream);
}

hipError_t launch_surrogate_deposit(const UniformArgs& P, bool fp64, unsigned long long* exact_mask,
                                    hipStream_t stream)
{
    const int64_t n_chunks = (P.ntet + 63) / 64;
    if (n_chunks == 0) return hipSuccess;
    int grid = net_grid(P.ntet);
    if (fp64)
        hipLaunchKernelGGL(surrogate_deposit_kernel<double>, dim3(grid), dim3(64), 0, stream, P, n_chunks,
                           exact_mask);
    else
        hipLaunchKernelGGL(surrogate_deposit_kernel<float>, dim3(grid), dim3(64), 0, stream, P, n_chunks,
                           exact_mask);
    return hipGetLastError();
}

}  // namespace psd
