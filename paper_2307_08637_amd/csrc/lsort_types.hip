// lsort_types.hip -- the key types and payload width that the partition
// engine does not handle natively, mapped onto the ones it does:
//   * int64 keys: adding 2^63 (flipping the sign bit) is an order-preserving
//     bijection onto uint64; the engine sorts the flipped words and the
//     flip is undone afterwards, in place.
//   * float32 keys: each key is widened, by integer arithmetic on its bits,
//     to the binary64 number of the same value (exact: every binary32 value
//     is a binary64 value); a NaN becomes the binary64 NaN of the same sign
//     carrying the 23-bit payload in the top of its mantissa.  The map keeps
//     IEEE totalOrder, so the engine sorts the widened words and they are
//     narrowed back bit for bit.
//   * 64-bit payloads: the engine sorts (key, original index) pairs stably;
//     the payload is then gathered through the sorted indices.
// Every pass here is a plain streaming kernel (grid-strided, one element per
// thread and step); the gather reads at random.
#include <algorithm>

#include "lsort_kernels.hpp"

namespace ls {

constexpr int TY_THREADS = 256;

__device__ __forceinline__ uint64_t widen_f32(uint32_t b) {
    const uint64_t s = (uint64_t)(b >> 31) << 63;
    const uint32_t e = (b >> 23) & 0xFF, m = b & 0x7FFFFF;
    if (e == 0xFF) return s | 0x7FF0000000000000ull | ((uint64_t)m << 29);  // inf (m = 0) or NaN
    if (e == 0) {
        if (m == 0) return s;  // signed zero
        // subnormal m * 2^-149: normalise on its leading bit p (0..22)
        const int p = 31 - __builtin_clz(m);
        const uint64_t e64 = (uint64_t)(p - 149 + 1023);
        return s | (e64 << 52) | (((uint64_t)m << (52 - p)) & 0xFFFFFFFFFFFFFull);
    }
    return s | ((uint64_t)(e + 896) << 52) | ((uint64_t)m << 29);
}

// Inverse of widen_f32 on its image.
__device__ __forceinline__ uint32_t narrow_f64(uint64_t b) {
    const uint32_t s = (uint32_t)(b >> 63) << 31;
    const uint32_t e = (uint32_t)(b >> 52) & 0x7FF;
    const uint64_t m = b & 0xFFFFFFFFFFFFFull;
    if (e == 0x7FF) return s | 0x7F800000u | (uint32_t)(m >> 29);
    if (e == 0) return s;
    const int E = (int)e - 896;
    if (E >= 1) return s | ((uint32_t)E << 23) | (uint32_t)(m >> 29);
    const int sh = 29 + 1 - E;  // binary32 subnormal: (1.m) * 2^(E - 127) with E <= 0
    return s | (uint32_t)(((1ull << 52) | m) >> sh);
}

__global__ __launch_bounds__(TY_THREADS) void k_flip_sign(uint64_t* k, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * TY_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * TY_THREADS + threadIdx.x; i < n; i += stride)
        k[i] ^= 0x8000000000000000ull;
}

__global__ __launch_bounds__(TY_THREADS) void k_widen(const uint32_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                      uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * TY_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * TY_THREADS + threadIdx.x; i < n; i += stride) dst[i] = widen_f32(src[i]);
}

__global__ __launch_bounds__(TY_THREADS) void k_narrow(const uint64_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                       uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * TY_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * TY_THREADS + threadIdx.x; i < n; i += stride) dst[i] = narrow_f64(src[i]);
}

// idx[i] = i within each array (segment-relative offsets are not needed: the
// gather reads save[] at absolute positions, so the index is absolute); the
// payload is saved for the gather.
__global__ __launch_bounds__(TY_THREADS) void k_index_save(const uint64_t* __restrict__ pay,
                                                           uint64_t* __restrict__ save, uint32_t* __restrict__ idx,
                                                           uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * TY_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * TY_THREADS + threadIdx.x; i < n; i += stride) {
        save[i] = pay[i];
        idx[i] = (uint32_t)i;
    }
}

__global__ __launch_bounds__(TY_THREADS) void k_gather64(const uint64_t* __restrict__ save,
                                                         const uint32_t* __restrict__ idx, uint64_t* __restrict__ pay,
                                                         uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * TY_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * TY_THREADS + threadIdx.x; i < n; i += stride) pay[i] = save[idx[i]];
}

static uint32_t ty_grid(uint64_t n, uint32_t cus) {
    const uint64_t want = (n + TY_THREADS - 1) / TY_THREADS;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * 16));
}

#define TY_LAUNCH(kernel, n, cus, st, ...)                                                        \
    do {                                                                                          \
        if ((n) == 0) return hipSuccess;                                                          \
        hipLaunchKernelGGL(kernel, dim3(ty_grid((n), (cus))), dim3(TY_THREADS), 0, st, __VA_ARGS__); \
        return hipGetLastError();                                                                 \
    } while (0)

hipError_t launch_flip_sign(uint64_t* k, uint64_t n, uint32_t cus, hipStream_t st) {
    TY_LAUNCH(k_flip_sign, n, cus, st, k, n);
}
hipError_t launch_widen(const uint32_t* src, uint64_t* dst, uint64_t n, uint32_t cus, hipStream_t st) {
    TY_LAUNCH(k_widen, n, cus, st, src, dst, n);
}
hipError_t launch_narrow(const uint64_t* src, uint32_t* dst, uint64_t n, uint32_t cus, hipStream_t st) {
    TY_LAUNCH(k_narrow, n, cus, st, src, dst, n);
}
hipError_t launch_index_save(const uint64_t* pay, uint64_t* save, uint32_t* idx, uint64_t n, uint32_t cus,
                             hipStream_t st) {
    TY_LAUNCH(k_index_save, n, cus, st, pay, save, idx, n);
}
hipError_t launch_gather64(const uint64_t* save, const uint32_t* idx, uint64_t* pay, uint64_t n, uint32_t cus,
                           hipStream_t st) {
    TY_LAUNCH(k_gather64, n, cus, st, save, idx, pay, n);
}

}  // namespace ls
