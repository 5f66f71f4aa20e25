// psd_octree.hip -- adaptive octree over the periodic box (Section 4).
//
// The paper refines a node while the number of tetrahedra overlapping it
// exceeds a threshold, estimating that number from the bounding boxes of
// Lagrangian subblocks (8^3 cells in its tests) weighted by the overlapping
// volume.  Here the estimate is made integer-exact so that the tree is
// bit-reproducible whatever the summation order:
//
//   count(node) = sum_sb floor( ntets(sb) * |bbox(sb) cap node| / |bbox(sb)| )
//
// with bounding boxes snapped outward to the finest lattice G = B * 2^lmax
// and overlaps taken over periodic images.  Kernels:
//   1. subblock_bbox   one wavefront per subblock, FP64 corners, integer box
//   2. level_counts    one thread per subblock, integer atomics into a dense
//                      count array for every level
//   3. assemble        one workgroup: level by level, refine flags, block scans
//                      give the canonical order (by level, Morton within a
//                      level, children of a node contiguous), leaves numbered
//                      in node order.
#include "psd_internal.h"

namespace psd {

namespace {

constexpr int kAsm = 256;  // threads of the assembly workgroup

__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

// Length of the periodic images of [lo,hi) inside [nlo,nhi), period G.
__device__ __forceinline__ int64_t periodic_overlap(int64_t lo, int64_t hi, int64_t nlo,
                                                    int64_t nhi, int64_t G)
{
    int64_t total = 0;
    const int64_t k0 = floor_div64(nlo - hi, G);
    const int64_t k1 = floor_div64(nhi - lo, G) + 1;
    for (int64_t k = k0; k <= k1; ++k) {
        int64_t a = lo + k * G, b = hi + k * G;
        if (a < nlo) a = nlo;
        if (b > nhi) b = nhi;
        if (b > a) total += b - a;
    }
    return total;
}

__global__ __launch_bounds__(kWave) void subblock_bbox_kernel(OctreeArgs A, SubblockBox* out)
{
#pragma clang fp contract(off)
    const int64_t s = blockIdx.x;
    const int64_t nsb = (int64_t)A.ns[0] * A.ns[1] * A.ns[2];
    if (s >= nsb) return;
    const int lane = threadIdx.x;
    const int64_t si = s / ((int64_t)A.ns[1] * A.ns[2]);
    const int64_t sj = (s / A.ns[2]) % A.ns[1];
    const int64_t sk = s % A.ns[2];
    const int S = A.subblock;
    const int64_t i0 = si * S, j0 = sj * S, k0 = sk * S;
    const int64_t i1 = min(i0 + S, (int64_t)A.np[0]);
    const int64_t j1 = min(j0 + S, (int64_t)A.np[1]);
    const int64_t k1 = min(k0 + S, (int64_t)A.np[2]);
    const int64_t ni = i1 - i0, nj = j1 - j0, nk = k1 - k0;
    const double G = (double)A.G;
    const float* pr = A.pos + 3 * ((i0 * A.np[1] + j0) * A.np[2] + k0);
    double ref[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ref[c] = (double)pr[c] * A.gscale;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t q = lane; q < ni * nj * nk; q += kWave) {
        const int64_t ci = i0 + q / (nj * nk), cj = j0 + (q / nk) % nj, ck = k0 + q % nk;
        double c[8][3];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int64_t ii = ci + ((m >> 2) & 1), jj = cj + ((m >> 1) & 1), kk = ck + (m & 1);
            if (ii == A.np[0]) ii = 0;
            if (jj == A.np[1]) jj = 0;
            if (kk == A.np[2]) kk = 0;
            const float* pp = A.pos + 3 * ((ii * A.np[1] + jj) * A.np[2] + kk);
#pragma unroll
            for (int a = 0; a < 3; ++a) c[m][a] = (double)pp[a] * A.gscale;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                double d = c[m][a] - c[0][a];
                const double t = G * rint(d / G);
                d -= t;
                c[m][a] = c[0][a] + d;
            }
            const double d0 = c[0][a] - ref[a];
            const double sh = -G * rint(d0 / G);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const double x = c[m][a] + sh;
                mn[a] = x < mn[a] ? x : mn[a];
                mx[a] = x > mx[a] ? x : mx[a];
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], __shfl_xor(mn[a], off, kWave));
            mx[a] = fmax(mx[a], __shfl_xor(mx[a], off, kWave));
        }
    if (lane == 0) {
        SubblockBox b;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = (int64_t)floor(mn[a]);
            b.hi[a] = (int64_t)ceil(mx[a]);
            if (b.hi[a] <= b.lo[a]) b.hi[a] = b.lo[a] + 1;
        }
        b.ntets = 6 * ni * nj * nk;
        out[s] = b;
    }
}

// Offset of level l in the dense count array (levels 0..l-1 before it).
__device__ __host__ __forceinline__ int64_t level_offset(int l)
{
    int64_t off = 0;
    for (int k = 0; k < l; ++k) off += (int64_t)1 << (3 * k);
    return off;
}

__global__ void level_counts_kernel(OctreeArgs A, const SubblockBox* sb, unsigned long long* dense)
{
    const int64_t nsb = (int64_t)A.ns[0] * A.ns[1] * A.ns[2];
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= nsb) return;
    const SubblockBox b = sb[s];
    const int64_t vol = (b.hi[0] - b.lo[0]) * (b.hi[1] - b.lo[1]) * (b.hi[2] - b.lo[2]);
    for (int l = 0; l <= A.max_level; ++l) {
        const int64_t side = (int64_t)1 << l;
        const int64_t w = A.G / side;
        unsigned long long* dl = dense + level_offset(l);
        for (int64_t x = 0; x < side; ++x) {
            const int64_t ox = periodic_overlap(b.lo[0], b.hi[0], x * w, (x + 1) * w, A.G);
            if (!ox) continue;
            for (int64_t y = 0; y < side; ++y) {
                const int64_t oy = periodic_overlap(b.lo[1], b.hi[1], y * w, (y + 1) * w, A.G);
                if (!oy) continue;
                for (int64_t z = 0; z < side; ++z) {
                    const int64_t oz = periodic_overlap(b.lo[2], b.hi[2], z * w, (z + 1) * w, A.G);
                    if (!oz) continue;
                    const int64_t num = b.ntets * ox * oy * oz;
                    const unsigned long long add = (unsigned long long)(num / vol);
                    if (add) atomicAdd(dl + (x * side + y) * side + z, add);
                }
            }
        }
    }
}

// Block-wide exclusive scan of small non-negative ints (kAsm threads).
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int& total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kAsm; off <<= 1) {
        const int y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    total = sh[kAsm - 1];
    const int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kAsm) void assemble_kernel(OctreeArgs A,
                                                         const unsigned long long* dense,
                                                         OctNode* work, OctNode* nodes,
                                                         int64_t capacity, int64_t* counts_out)
{
    __shared__ int sh[kAsm];
    const int t = threadIdx.x;
    if (t == 0) {
        OctNode r;
        r.level = 0;
        r.ix = r.iy = r.iz = 0;
        r.first_child = -1;
        r.leaf_id = -1;
        r.count = 0;
        work[0] = r;
    }
    __threadfence();
    __syncthreads();
    int64_t beg = 0, end = 1;
    for (int l = 0; l <= A.max_level; ++l) {
        const int64_t side = (int64_t)1 << l;
        const unsigned long long* dl = dense + level_offset(l);
        int64_t refined = 0;
        for (int64_t c = beg; c < end; c += kAsm) {
            const int64_t i = c + t;
            int ref = 0;
            OctNode nd;
            if (i < end) {
                nd = work[i];
                nd.count = (int64_t)dl[((int64_t)nd.ix * side + nd.iy) * side + nd.iz];
                ref = (nd.count > A.threshold && l < A.max_level) ? 1 : 0;
            }
            int tot;
            const int ex = block_excl_scan(ref, sh, tot);
            if (i < end) {
                nd.first_child = ref ? (int32_t)(end + 8 * (refined + ex)) : -1;
                work[i] = nd;
                if (ref) {
                    for (int q = 0; q < 8; ++q) {
                        OctNode ch;
                        ch.level = l + 1;
                        ch.ix = 2 * nd.ix + ((q >> 2) & 1);
                        ch.iy = 2 * nd.iy + ((q >> 1) & 1);
                        ch.iz = 2 * nd.iz + (q & 1);
                        ch.first_child = -1;
                        ch.leaf_id = -1;
                        ch.count = 0;
                        work[nd.first_child + q] = ch;
                    }
                }
            }
            refined += tot;
        }
        __threadfence();
        __syncthreads();
        beg = end;
        end += 8 * refined;
        if (refined == 0) break;
    }
    // leaf ids in node order, and the copy to the caller's array
    int64_t nleaf = 0;
    for (int64_t c = 0; c < end; c += kAsm) {
        const int64_t i = c + t;
        int leaf = 0;
        OctNode nd;
        if (i < end) {
            nd = work[i];
            leaf = nd.first_child < 0 ? 1 : 0;
        }
        int tot;
        const int ex = block_excl_scan(leaf, sh, tot);
        if (i < end) {
            nd.leaf_id = leaf ? (int32_t)(nleaf + ex) : -1;
            if (i < capacity) nodes[i] = nd;
            work[i] = nd;
        }
        nleaf += tot;
    }
    if (t == 0) {
        counts_out[0] = end;
        counts_out[1] = nleaf;
    }
}

template <typename T>
__global__ void zero_kernel(T* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

__global__ void fill_int_kernel(int* p, int64_t n, int v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Dense per-level map (level offsets as for the counts) node -> leaf id, and
// a flag per level telling whether it holds any leaf.  Nodes outside the
// valid range are ignored.
__global__ void leaf_map_kernel(const OctNode* nodes, int64_t n_nodes, int64_t n_leaves,
                                int max_level, int* map, int* level_flag)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const OctNode nd = nodes[i];
    if (nd.leaf_id < 0 || nd.leaf_id >= n_leaves || nd.level < 0 || nd.level > max_level) return;
    const int64_t side = (int64_t)1 << nd.level;
    if (nd.ix < 0 || nd.iy < 0 || nd.iz < 0 || nd.ix >= side || nd.iy >= side || nd.iz >= side) return;
    map[level_offset(nd.level) + ((int64_t)nd.ix * side + nd.iy) * side + nd.iz] = nd.leaf_id;
    level_flag[nd.level] = 1;
}

}  // namespace

int64_t octree_max_nodes(int max_level)
{
    int64_t n = 0;
    for (int l = 0; l <= max_level; ++l) n += (int64_t)1 << (3 * l);
    return n;
}

OctreeWorkspace octree_workspace_layout(const OctreeArgs& A)
{
    OctreeWorkspace w;
    const int64_t nsb = (int64_t)A.ns[0] * A.ns[1] * A.ns[2];
    const int64_t maxn = octree_max_nodes(A.max_level);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    w.boxes = take(sizeof(SubblockBox) * nsb);
    w.dense = take(sizeof(unsigned long long) * maxn);
    w.work = take(sizeof(OctNode) * maxn);
    w.counts = take(sizeof(int64_t) * 2);
    w.leafmap = take(sizeof(int) * maxn);
    w.levelflag = take(sizeof(int) * (A.max_level + 1));
    w.bytes = off;
    return w;
}

hipError_t launch_build_octree(const OctreeArgs& A, void* ws, OctNode* nodes, int64_t capacity,
                               int64_t* counts_host, hipStream_t stream)
{
    const OctreeWorkspace w = octree_workspace_layout(A);
    char* base = reinterpret_cast<char*>(ws);
    SubblockBox* boxes = reinterpret_cast<SubblockBox*>(base + w.boxes);
    unsigned long long* dense = reinterpret_cast<unsigned long long*>(base + w.dense);
    OctNode* work = reinterpret_cast<OctNode*>(base + w.work);
    int64_t* counts = reinterpret_cast<int64_t*>(base + w.counts);
    const int64_t nsb = (int64_t)A.ns[0] * A.ns[1] * A.ns[2];
    const int64_t maxn = octree_max_nodes(A.max_level);

    hipLaunchKernelGGL(zero_kernel<unsigned long long>, dim3((unsigned)((maxn + 255) / 256 < 4096 ? (maxn + 255) / 256 : 4096)),
                       dim3(256), 0, stream, dense, maxn);
    hipLaunchKernelGGL(subblock_bbox_kernel, dim3((unsigned)nsb), dim3(kWave), 0, stream, A, boxes);
    hipLaunchKernelGGL(level_counts_kernel, dim3((unsigned)((nsb + 127) / 128)), dim3(128), 0, stream,
                       A, (const SubblockBox*)boxes, dense);
    hipLaunchKernelGGL(assemble_kernel, dim3(1), dim3(kAsm), 0, stream, A,
                       (const unsigned long long*)dense, work, nodes, capacity, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(counts_host, counts, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

size_t octree_queue_bytes(const OctreeArgs& A)
{
    int64_t chunks = 0;
    const int64_t ntet = 6 * (int64_t)A.np[0] * A.np[1] * A.np[2];
    for (int l = 0; l <= A.max_level; ++l) chunks += (ntet + kWave - 1) / kWave;
    return queue_workspace_bytes(chunks, A.max_level + 1, true);
}

hipError_t launch_deposit_octree(const OctreeArgs& A, const UniformArgs& base, const OctNode* nodes,
                                 int64_t n_nodes, int64_t n_leaf_cells, void* ws, size_t ws_bytes,
                                 bool accumulate, const Tuning& tune, hipStream_t stream)
{
    const OctreeWorkspace w = octree_workspace_layout(A);
    char* wsb = reinterpret_cast<char*>(ws);
    int* map = reinterpret_cast<int*>(wsb + w.leafmap);
    int* flags = reinterpret_cast<int*>(wsb + w.levelflag);
    const int64_t maxn = octree_max_nodes(A.max_level);
    const unsigned gmap = (unsigned)((maxn + 255) / 256 < 4096 ? (maxn + 255) / 256 : 4096);
    hipLaunchKernelGGL(fill_int_kernel, dim3(gmap), dim3(256), 0, stream, map, maxn, -1);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, stream, flags,
                       (int64_t)(A.max_level + 1), 0);
    if (n_nodes > 0)
        hipLaunchKernelGGL(leaf_map_kernel, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0,
                           stream, nodes, n_nodes, n_leaf_cells / ((int64_t)A.block * A.block * A.block),
                           A.max_level, map, flags);
    if (!accumulate) {
        const unsigned g = (unsigned)((n_leaf_cells + 255) / 256 < 65536 ? (n_leaf_cells + 255) / 256 : 65536);
        if (n_leaf_cells > 0)
            hipLaunchKernelGGL(zero_kernel<float>, dim3(g), dim3(256), 0, stream,
                               reinterpret_cast<float*>(base.out), n_leaf_cells);
        if (base.mass_sum)
            hipLaunchKernelGGL(zero_kernel<double>, dim3(1), dim3(64), 0, stream, base.mass_sum,
                               (int64_t)1);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BoxDesc boxes[8];
    const int nl = A.max_level + 1;
    for (int l = 0; l < nl; ++l) {
        UniformArgs P = base;
        const int n = A.block << l;
        for (int c = 0; c < 3; ++c) {
            P.nc[c] = n;
            P.scale[c] = (double)n / A.box;
        }
        if (base.out_scale != 1.0) P.out_scale = (double)n * n * n / (A.box * A.box * A.box);
        P.leaf_map = map + level_offset(l);
        P.level_has_leaf = flags + l;
        P.leaf_block = A.block;
        P.leaf_side = 1 << l;
        boxes[l] = box_from_uniform(P);
    }
    const size_t used = w.bytes;
    return launch_queue(boxes, nl, false, tune, wsb + used, ws_bytes - used, base.stats, stream);
}

}  // namespace psd
