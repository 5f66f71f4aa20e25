// psd_finite.hip -- check that every position is a finite number.
//
// The deposits accept any finite coordinate (Section 2: tracer positions in a
// periodic box); a NaN or infinity cannot be placed.  This scan backs the
// PSD_CHECK_FINITE flag and the check psd_build_octree always makes.
#include "psd_internal.h"

namespace psd {

namespace {

// Non-finite floats among p[0..n): grid-stride over 16-byte vectors (the
// array is 4-byte aligned; the head up to a 16-byte boundary and the tail are
// read as scalars by the first wavefront), one atomic per wavefront that
// found any.
__global__ __launch_bounds__(256) void count_nonfinite_kernel(const float* __restrict__ p,
                                                              int64_t n,
                                                              unsigned long long* count)
{
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    int64_t head = (int64_t)(((16 - (addr & 15)) & 15) >> 2);
    if (head > n) head = n;
    const int64_t nvec = (n - head) >> 2;
    const float4* v = reinterpret_cast<const float4*>(p + head);
    unsigned bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvec; i += stride) {
        const float4 q = v[i];
        bad += !isfinite(q.x) + !isfinite(q.y) + !isfinite(q.z) + !isfinite(q.w);
    }
    if (blockIdx.x == 0 && threadIdx.x < 8) {
        // at most 3 head floats and 3 tail floats
        const int t = threadIdx.x;
        int64_t i = -1;
        if (t < 4 && t < head) i = t;
        if (t >= 4 && head + 4 * nvec + (t - 4) < n) i = head + 4 * nvec + (t - 4);
        if (i >= 0) bad += !isfinite(p[i]);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) bad += __shfl_xor(bad, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(count, (unsigned long long)bad);
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

}  // namespace

hipError_t count_nonfinite(const float* p, int64_t n, unsigned long long* dcount,
                           hipStream_t stream, unsigned long long& host_count)
{
    host_count = 0;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, stream, dcount);
    if (n > 0) {
        int64_t blocks = (n / 4 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(count_nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p,
                           n, dcount);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long c = 0;
    e = hipMemcpyAsync(&c, dcount, sizeof(c), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    host_count = c;
    return hipSuccess;
}

}  // namespace psd
