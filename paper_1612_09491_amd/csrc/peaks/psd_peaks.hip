// psd_peaks.hip -- microbenchmarks of the rates a deposit is priced against.
//
// Measurement code, built into its own library (libpsd_peaks.so) beside the
// deposit library.  Each call enqueues one kernel on `stream`; the caller
// times it with events on that stream and divides by the operation count the
// call returns.
//
//   peaks_global_atomic_f32: FP32 global atomic adds whose result is unused
//     (global_atomic_add_f32 without return), the scatter of the deposit's
//     phase 2.  pattern 0: lanes of a wavefront hit consecutive words
//     (coalesced); pattern 1: every add goes to a hashed word of the array
//     (random); pattern 2: every lane walks runs of 8 consecutive cells along
//     one axis of a 512^3 grid from a hashed start, the axis (stride 1, 512
//     or 512^2 words) the same across a wavefront and changing from one
//     wavefront to the next -- the deposit's phase 2, where each lane walks
//     the levels of its own column along the tetrahedron's walk axis;
//     pattern 3: the lanes in groups of 8 (a tile row of 8 neighbouring
//     columns, one cell apart along one axis of the 512^3 grid) from a hashed
//     start per group, each lane walking runs of 8 cells along another axis,
//     the pair of axes the same across a wavefront and one of the six from
//     one wavefront to the next -- phase 2 as the deposit lays its columns
//     out, row by row over the lanes.  n is a power of two and addresses are
//     masked to n - 1, so every access is in bounds.
//   peaks_lds_atomic: LDS atomic adds without return (ds_add_f32 or
//     ds_add_f64, the deposit's level increments) to lane-consecutive words
//     of a 2048-word array per workgroup, bank-conflict free.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    // integer hash (xorshift-multiply), used only to scatter addresses
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(kBlock) void global_atomic_kernel(float* __restrict__ buf, uint32_t mask,
                                                               int iters, int pattern)
{
    const uint32_t tid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t nthreads = gridDim.x * kBlock;
    for (int i = 0; i < iters; ++i) {
        uint32_t a;
        if (pattern == 0) {
            a = ((uint32_t)i * nthreads + tid) & mask;
        } else if (pattern == 1) {
            a = mix32(tid * 0x9e3779b9u + (uint32_t)i * 0x85ebca6bu) & mask;
        } else if (pattern == 2) {
            const uint32_t wave = tid >> 6;
            const uint32_t stride = (wave % 3u) == 0u ? 1u : ((wave % 3u) == 1u ? 512u : 512u * 512u);
            const uint32_t start = mix32(tid * 0x9e3779b9u + (uint32_t)(i >> 3) * 0x85ebca6bu);
            a = (start + (uint32_t)(i & 7) * stride) & mask;
        } else {
            const uint32_t wave = tid >> 6, pair = wave % 6u;
            const uint32_t s[3] = {1u, 512u, 512u * 512u};
            const uint32_t across = s[pair / 2u];                            // along the row
            const uint32_t walk = s[(pair / 2u + 1u + (pair & 1u)) % 3u];    // another axis
            const uint32_t group = tid >> 3;
            const uint32_t start = mix32(group * 0x9e3779b9u + (uint32_t)(i >> 3) * 0x85ebca6bu);
            a = (start + (tid & 7u) * across + (uint32_t)(i & 7) * walk) & mask;
        }
        __hip_atomic_fetch_add(buf + a, 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void lds_atomic_kernel(T* __restrict__ out, int iters)
{
    constexpr int kWords = 2048;
    __shared__ T s[kWords];
    for (int w = threadIdx.x; w < kWords; w += kBlock) s[w] = T(0);
    __syncthreads();
    const int lane0 = threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        const int a = (lane0 + i * kBlock) & (kWords - 1);
        __hip_atomic_fetch_add(s + a, T(1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    // keep the adds live: one word per thread of the block's sums
    T acc = T(0);
    for (int w = threadIdx.x; w < kWords; w += kBlock) acc += s[w];
    out[blockIdx.x * kBlock + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

// n words of buf (a power of two, 1 <= n <= 2^31), `blocks` workgroups of 256
// threads, each thread `iters` adds.  Returns the number of atomic adds
// enqueued, or -1.
int64_t peaks_global_atomic_f32(float* buf, int64_t n, int blocks, int iters, int pattern,
                                void* stream)
{
    if (!buf || n < 1 || n > (1ll << 31) || (n & (n - 1)) != 0 || blocks < 1 || iters < 1 ||
        pattern < 0 || pattern > 3)
        return -1;
    hipLaunchKernelGGL(global_atomic_kernel, dim3(blocks), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), buf, (uint32_t)(n - 1), iters, pattern);
    if (hipGetLastError() != hipSuccess) return -1;
    return (int64_t)blocks * kBlock * iters;
}

// out holds blocks * 256 elements (float when fp64 == 0, else double).
// Returns the number of LDS atomic adds enqueued, or -1.
int64_t peaks_lds_atomic(void* out, int blocks, int iters, int fp64, void* stream)
{
    if (!out || blocks < 1 || iters < 1) return -1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (fp64)
        hipLaunchKernelGGL(lds_atomic_kernel<double>, dim3(blocks), dim3(kBlock), 0, s,
                           static_cast<double*>(out), iters);
    else
        hipLaunchKernelGGL(lds_atomic_kernel<float>, dim3(blocks), dim3(kBlock), 0, s,
                           static_cast<float*>(out), iters);
    if (hipGetLastError() != hipSuccess) return -1;
    return (int64_t)blocks * kBlock * iters;
}

}  // extern "C"
