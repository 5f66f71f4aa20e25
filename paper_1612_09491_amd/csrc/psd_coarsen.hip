// psd_coarsen.hip -- coarse representations of an octree's internal nodes.
//
// The deposit fills the leaves; multi-resolution volume rendering also wants
// every internal node as a block of the same B^3 cells at the node's own,
// coarser resolution (Section 8, future work).  The exact intersection volume
// is additive over a partition of a cell, |T cap C| = sum over the 8 octants
// of |T cap C_q|, so a coarse cell's mass is the sum of the 2x2x2 finer cells
// it covers, and its density their average.  Levels are filled bottom-up,
// one launch per level: a node at level l reads its children's blocks, which
// the launch for level l + 1 wrote.
//
// HBM-bound: per internal-node cell 8 reads and one write of 4 bytes, per
// leaf cell one read and one write.
#include "psd_internal.h"

namespace psd {

namespace {

constexpr int kCoarsenBlock = 256;

// One workgroup per node; nodes not at `level` return at once.
__global__ __launch_bounds__(kCoarsenBlock) void coarsen_level_kernel(
    const OctNode* __restrict__ nodes, int64_t n_nodes, int64_t n_leaves, int B, int level,
    float scale, const float* __restrict__ leaves, float* __restrict__ out)
{
    const int64_t n = blockIdx.x;
    const OctNode nd = nodes[n];
    if (nd.level != level) return;
    const int64_t cells = (int64_t)B * B * B;
    float* dst = out + n * cells;
    if (nd.first_child < 0) {
        if (nd.leaf_id < 0 || nd.leaf_id >= n_leaves) return;  // not a valid leaf
        const float* src = leaves + (int64_t)nd.leaf_id * cells;
        for (int64_t c = threadIdx.x; c < cells; c += blockDim.x) dst[c] = src[c];
        return;
    }
    if (nd.first_child <= n || (int64_t)nd.first_child + 8 > n_nodes) return;  // malformed
    // node index of the child in each octant q = 4 dx + 2 dy + dz, from the
    // children's own positions (2 ix + dx, ...)
    __shared__ int64_t child[8];
    __shared__ int complete;
    if (threadIdx.x == 0) {
        for (int q = 0; q < 8; ++q) child[q] = -1;
        for (int k = 0; k < 8; ++k) {
            const OctNode ch = nodes[nd.first_child + k];
            child[((ch.ix & 1) << 2) | ((ch.iy & 1) << 1) | (ch.iz & 1)] = nd.first_child + k;
        }
        int ok = 1;
        for (int q = 0; q < 8; ++q) ok &= child[q] >= 0 ? 1 : 0;
        complete = ok;
    }
    __syncthreads();
    if (!complete) return;  // malformed: two children in one octant
    const int h = B / 2;
    for (int64_t c = threadIdx.x; c < cells; c += blockDim.x) {
        const int x = (int)(c / ((int64_t)B * B)), y = (int)((c / B) % B), z = (int)(c % B);
        const int q = ((x >= h) << 2) | ((y >= h) << 1) | (z >= h);
        const float* src = out + child[q] * cells;
        const int x0 = 2 * (x % h), y0 = 2 * (y % h), z0 = 2 * (z % h);
        // fixed order: x outermost, then y, then z
        double s = 0.0;
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dz = 0; dz < 2; ++dz)
                    s += (double)src[((int64_t)(x0 + dx) * B + (y0 + dy)) * B + (z0 + dz)];
        dst[c] = (float)(s * (double)scale);
    }
}

}  // namespace

hipError_t launch_octree_coarsen(const OctNode* nodes, int64_t n_nodes, int64_t n_leaves, int B,
                                 int max_level, bool density, const float* leaves, float* out,
                                 hipStream_t stream)
{
    // masses add; densities of the 8 equal octants average
    const float scale = density ? 0.125f : 1.0f;
    for (int l = max_level; l >= 0; --l)
        hipLaunchKernelGGL(coarsen_level_kernel, dim3((unsigned)n_nodes), dim3(kCoarsenBlock), 0,
                           stream, nodes, n_nodes, n_leaves, B, l, scale, leaves, out);
    return hipGetLastError();
}

}  // namespace psd
