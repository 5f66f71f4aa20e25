// psd_ingest.hip -- snapshot ingest: particles into their Lagrangian grid slots.
//
// A snapshot stores tracers in an arbitrary order, each with a unique ID that
// names its place in the Lagrangian grid (Section 3: the IDs give the
// Lagrangian positions; once the tracers are sorted by ID the IDs are no
// longer needed).  The IDs are a permutation of the slots, so on one GPU the
// sort is a single scatter: record r goes to slot ids[r] - id_base.
//
// HBM-bound: 8 B of ID and 12 B of position read and 12 B written per record,
// reads coalesced, writes wherever the IDs send them.  With the optional check
// a one-bit-per-slot occupancy map (an atomic OR per record) finds duplicate
// IDs -- only the record that claims a slot first writes it -- and a popcount
// pass finds the slots no record names.
#include "psd_internal.h"

namespace psd {

namespace {

constexpr int kIngestBlock = 256;

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <bool CHECK>
__global__ __launch_bounds__(kIngestBlock) void scatter_by_id_kernel(
    const int64_t* __restrict__ ids, const float* __restrict__ pos_in, int64_t n, int64_t id_base,
    int64_t n_slots, float* __restrict__ pos_out, unsigned* __restrict__ occupied,
    unsigned long long* __restrict__ check)
{
    unsigned long long bad = 0, dup = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += stride) {
        // modular difference: an id below id_base wraps to a huge value
        const uint64_t slot = (uint64_t)ids[r] - (uint64_t)id_base;
        if (slot >= (uint64_t)n_slots) {
            ++bad;
            continue;
        }
        if (CHECK) {
            // the record that sets the slot's bit first is the one stored, whole;
            // later records naming the slot are only counted
            const unsigned bit = 1u << (unsigned)(slot & 31);
            const unsigned old = atomicOr(occupied + (slot >> 5), bit);
            if (old & bit) {
                ++dup;
                continue;
            }
        }
        const float x = pos_in[3 * r + 0], y = pos_in[3 * r + 1], z = pos_in[3 * r + 2];
        float* o = pos_out + 3 * slot;
        o[0] = x;
        o[1] = y;
        o[2] = z;
    }
    if (CHECK) {
        bad = wave_sum(bad);
        dup = wave_sum(dup);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            if (bad) atomicAdd(check + 0, bad);
            if (dup) atomicAdd(check + 1, dup);
        }
    }
}

// check[2] = n_slots - (number of set bits), i.e. the slots no record named;
// the map's bits beyond n_slots are never set.
__global__ __launch_bounds__(kIngestBlock) void missing_slots_kernel(const unsigned* __restrict__ occupied,
                                                                     int64_t n_words, int64_t n_slots,
                                                                     unsigned long long* check)
{
    unsigned long long set = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n_words; w += stride)
        set += (unsigned long long)__popc(occupied[w]);
    set = wave_sum(set);
    // every wave subtracts its share; the first thread adds n_slots once
    if ((threadIdx.x & (kWave - 1)) == 0 && set) atomicAdd(check + 2, (unsigned long long)(-(int64_t)set));
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(check + 2, (unsigned long long)n_slots);
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

unsigned blocks_for(int64_t n, int64_t per_block, int64_t cap)
{
    int64_t b = (n + per_block - 1) / per_block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

size_t reorder_workspace_bytes(int64_t n_slots)
{
    return (size_t)((n_slots + 31) / 32) * sizeof(unsigned);
}

hipError_t launch_reorder_by_id(const int64_t* ids, const float* pos_in, int64_t n, int64_t id_base,
                                int64_t n_slots, float* pos_out, int64_t* check, void* ws,
                                hipStream_t stream)
{
    // enough workgroups to fill the chip several times over; each thread
    // then strides over the records
    const unsigned grid = blocks_for(n, kIngestBlock, 256 * 32);
    if (!check) {
        if (n > 0)
            hipLaunchKernelGGL(scatter_by_id_kernel<false>, dim3(grid), dim3(kIngestBlock), 0, stream,
                               ids, pos_in, n, id_base, n_slots, pos_out, nullptr, nullptr);
        return hipGetLastError();
    }
    unsigned long long* c = reinterpret_cast<unsigned long long*>(check);
    unsigned* occupied = reinterpret_cast<unsigned*>(ws);
    const int64_t n_words = (n_slots + 31) / 32;
    hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(1), dim3(64), 0, stream, c, (int64_t)3,
                       0ull);
    hipLaunchKernelGGL(fill_kernel<unsigned>, dim3(blocks_for(n_words, kIngestBlock, 8192)),
                       dim3(kIngestBlock), 0, stream, occupied, n_words, 0u);
    if (n > 0)
        hipLaunchKernelGGL(scatter_by_id_kernel<true>, dim3(grid), dim3(kIngestBlock), 0, stream, ids,
                           pos_in, n, id_base, n_slots, pos_out, occupied, c);
    hipLaunchKernelGGL(missing_slots_kernel, dim3(blocks_for(n_words, kIngestBlock, 2048)),
                       dim3(kIngestBlock), 0, stream, (const unsigned*)occupied, n_words, n_slots, c);
    return hipGetLastError();
}

}  // namespace psd
