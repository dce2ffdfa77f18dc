// lsort_stream.hip -- two reference streams over plain memory, the practical
// ceilings against which the sort's passes are measured: a copy (one read and
// one write per word, like the scatter and the base case) and a read-only
// reduction (one read per word, like the histogram).
#include <algorithm>

#include "lsort_kernels.hpp"

namespace ls {

#define LAUNCH(kernel, grid, block, stream, ...)                                     \
    do {                                                                             \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

// Copy: one 8-byte word per thread and step, grid-strided; read: each
// workgroup takes runs of 32768 contiguous words (256 KB) and keeps eight
// loads in flight per thread.  These shapes measured fastest on this GPU
// among grid-strided and run-per-workgroup variants with 4-16 loads in
// flight and 8- or 16-byte accesses.
constexpr int ST_COPY_THREADS = 256;
constexpr int ST_READ_THREADS = 512;
constexpr int ST_U = 8;                  // loads in flight per thread (read)
constexpr uint64_t ST_RUN = 32768;       // words per workgroup run (read)

__global__ __launch_bounds__(ST_COPY_THREADS) void k_stream_copy(const uint64_t* __restrict__ src,
                                                                 uint64_t* __restrict__ dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * ST_COPY_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * ST_COPY_THREADS + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_stream_zero(unsigned long long* out) {
    if (threadIdx.x == 0) *out = 0;
}

__global__ __launch_bounds__(ST_READ_THREADS) void k_stream_read(const uint64_t* __restrict__ src, uint64_t n,
                                                                 unsigned long long* out) {
    __shared__ uint64_t red[ST_READ_THREADS / 64];
    uint64_t s = 0;
    const uint64_t nrun = (n + ST_RUN - 1) / ST_RUN;
    for (uint64_t r = blockIdx.x; r < nrun; r += gridDim.x) {
        const uint64_t base = r * ST_RUN;
        for (uint64_t i0 = 0; i0 < ST_RUN; i0 += (uint64_t)ST_READ_THREADS * ST_U) {
            uint64_t v[ST_U];
#pragma unroll
            for (int u = 0; u < ST_U; u++) {
                const uint64_t i = base + i0 + u * ST_READ_THREADS + threadIdx.x;
                v[u] = i < n ? src[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < ST_U; u++) s += v[u];
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < ST_READ_THREADS / 64; w++) t += red[w];
        atomicAdd(out, (unsigned long long)t);
    }
}

hipError_t launch_stream_copy(const uint64_t* src, uint64_t* dst, uint64_t n, uint32_t cus, hipStream_t st) {
    const uint64_t want = (n + ST_COPY_THREADS - 1) / ST_COPY_THREADS;
    LAUNCH(k_stream_copy, (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * 16)),
           ST_COPY_THREADS, st, src, dst, n);
}

hipError_t launch_stream_read(const uint64_t* src, uint64_t n, uint64_t* sum, uint32_t cus, hipStream_t st) {
    hipLaunchKernelGGL(k_stream_zero, dim3(1), dim3(64), 0, st, (unsigned long long*)sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    const uint64_t nrun = (n + ST_RUN - 1) / ST_RUN;
    LAUNCH(k_stream_read, (uint32_t)std::min<uint64_t>(nrun, (uint64_t)cus * 16), ST_READ_THREADS, st, src, n,
           (unsigned long long*)sum);
}

}  // namespace ls
