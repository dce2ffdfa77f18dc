// lsort_base.hip -- base case of the learned sample sort for gfx950: the
// sub-arrays left after the last partition level, sorted directly.
//
// Built on its own with -fno-honor-nans: its only floating-point operations
// are the comparators of the binary64 group sort, whose inputs are checked
// NaN-free first (everything else here is integer code), so v_min_f64 /
// v_max_f64 need no quieting of their operands.
#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {

// ===========================================================================
// Base case (Sec. 4: sub-arrays below the cutoff are sorted directly).
// k_base_small: sub-arrays of at most 512 keys sorted in registers -- up to
// 256 keys by a group of 8 or 16 lanes (group_bitonic, 8 or 4 sub-arrays per
// wavefront), larger ones (and all of them with a payload) by a whole
// wavefront (wave_bitonic); k_base_big: one workgroup per larger sub-array
// (up to 4096) sorted in LDS, and the copies of finished runs.
// ===========================================================================

constexpr int BASE_THREADS = 256;

template <int E, bool PAY>
__device__ __forceinline__ void base_small_item(const Params& P, uint64_t off, uint32_t size, uint32_t srcb, int lane) {
    const uint64_t* in = P.keys[srcb];
    uint64_t* out = P.keys[0];
    const int u64 = P.u64;
    uint64_t k[E];
    uint32_t ix[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = lane * E + e;
        k[e] = i < size ? key_ord(in[off + i], u64) : ~0ull;
        ix[e] = i;
    }
    if (PAY) {
        wave_bitonic<E, true>(k, ix, lane);
        const uint32_t* pin = P.pay[srcb];
        uint32_t* pout = P.pay[0];
        uint32_t pv[E];
#pragma unroll
        for (int e = 0; e < E; e++) pv[e] = (lane * E + e < (int)size) ? pin[off + ix[e]] : 0u;
#pragma unroll
        for (int e = 0; e < E; e++)
            if (lane * E + e < (int)size) pout[off + lane * E + e] = pv[e];
    } else {
        wave_bitonic<E, false>(k, ix, lane);
    }
#pragma unroll
    for (int e = 0; e < E; e++)
        if (lane * E + e < (int)size) out[off + lane * E + e] = key_unord(k[e], u64);
}

// Group items: GPW = 64 / G sub-arrays per wavefront, G lanes and E keys per
// lane each (group_bitonic): items of up to 128 keys on 8 lanes, of 129..256
// keys on 16 lanes, 16 keys per lane.  Loads read key j of a sub-array into
// lane j % G, register j / G (consecutive lanes, consecutive keys: any
// placement of unsorted input is valid); the sorted keys go out through LDS,
// each wave in its own region, so that stores are contiguous too.  binary64
// keys are sorted as numbers unless the wavefront holds a NaN or a -0.0
// (whose order is the bit pattern's), else as ordered integers.
constexpr int GLE = 4, GE = 1 << GLE;
constexpr int G_SLOTS = WAVE * GE + WAVE * GE / 16;  // LDS slots per wave: one pad slot after every 16
static_assert(GE * 8 == GROUP_SMALL_MAX && GE * 16 == GROUP_MAX, "lane groups of 8 and 16 lanes");

__device__ __forceinline__ uint32_t gslot(uint32_t i) { return i + (i >> 4); }

// Wave-local LDS hand-off: the wavefront's own LDS accesses run in order; this
// keeps the compiler from moving them across each other.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Items [lo, hi) of a list, each sorted by the whole wavefront.  Not inlined:
// the group tasks call it only for the rare task holding a NaN or a -0.0, and
// its registers then stay out of the group code's.
__attribute__((noinline)) __device__ void base_items_one_by_one(const Params& P, const uint64_t* items, uint64_t lo,
                                                                uint64_t hi, int lane) {
    for (uint64_t it = lo; it < hi; it++) {
        const uint64_t w = items[it];
        const uint32_t sz = (uint32_t)(w & 0xffffu) + 1;
        if (sz <= 64) base_small_item<1, false>(P, w >> 18, sz, (w >> 17) & 1u, lane);
        else if (sz <= 128) base_small_item<2, false>(P, w >> 18, sz, (w >> 17) & 1u, lane);
        else base_small_item<4, false>(P, w >> 18, sz, (w >> 17) & 1u, lane);
    }
}

// One task: GPW items of the group's list.  U64: ordered-integer network.
// binary64: the numeric network, unless the task holds a NaN or a -0.0; then
// its items go one by one through the whole-wavefront sort instead (rare, and
// it keeps the integer network's registers out of this kernel).
template <int LG, bool U64>
__device__ __forceinline__ void base_group_task(const Params& P, const uint64_t* items, uint64_t task, uint64_t nitem,
                                                uint64_t* lds, int lane) {
    constexpr int G = 1 << LG, GPW = WAVE / G, N = GE * G;
    // per-task copy of the lane id: the sixteen lane offsets r * G + gl are
    // cheap to form again each task, and hoisted out of the task loop they
    // would hold sixteen registers for the whole kernel
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int g = ln >> LG, gl = ln & (G - 1);
    const uint64_t idx = task * GPW + g;
    // every load is in bounds without a branch: an idle group (past the last
    // item) reads the last item and keeps size 0; indices clamp to size - 1
    const uint64_t wd = items[min<uint64_t>(idx, nitem - 1)];
    const uint64_t off = wd >> 18;
    const uint32_t size = idx < nitem ? (uint32_t)(wd & 0xffffu) + 1 : 0u;
    const uint64_t* src = (((wd >> 17) & 1u) ? P.keys[1] : P.keys[0]) + off;
    uint64_t* dst = P.keys[0] + off;
    const uint32_t last = size ? size - 1 : 0u;
    uint64_t raw[GE];
#pragma unroll
    for (int r = 0; r < GE; r++) raw[r] = src[min<uint32_t>(r * G + gl, last)];
    uint64_t* mine = lds + g * (N + N / 16);
    if (U64) {
#pragma unroll
        for (int r = 0; r < GE; r++)
            if ((uint32_t)(r * G + gl) >= size) raw[r] = ~0ull;
        group_bitonic<uint64_t, GLE, LG>(raw, lane);
    } else {
        bool special = false;
#pragma unroll
        for (int r = 0; r < GE; r++) {
            if ((uint32_t)(r * G + gl) >= size) raw[r] = 0x7ff0000000000000ull;  // +inf pads
            special |= (raw[r] << 1) > 0xffe0000000000000ull || raw[r] == 0x8000000000000000ull;  // NaN, -0.0
        }
        if (__ballot(special) != 0) {
            base_items_one_by_one(P, items, task * GPW, min<uint64_t>(nitem, task * GPW + GPW), lane);
            return;
        }
        double k[GE];
#pragma unroll
        for (int r = 0; r < GE; r++) k[r] = __builtin_bit_cast(double, raw[r]);
        group_bitonic<double, GLE, LG>(k, lane);
#pragma unroll
        for (int r = 0; r < GE; r++) raw[r] = __builtin_bit_cast(uint64_t, k[r]);
    }
#pragma unroll
    for (int r = 0; r < GE; r++) mine[gslot(gl * GE + r)] = raw[r];
    wave_lds_sync();
    uint64_t o[GE];
#pragma unroll
    for (int r = 0; r < GE; r++) o[r] = mine[gslot(r * G + gl)];
#pragma unroll
    for (int r = 0; r < GE; r++)
        if ((uint32_t)(r * G + gl) < size) dst[r * G + gl] = o[r];
    wave_lds_sync();  // the next task rewrites the region
}

// Three loops, each grid-strided over every wavefront (so each class is spread
// evenly), largest items first: whole-wave items (257..512 keys), tasks of 4
// items of 129..256 keys, tasks of 8 items of up to 128 keys.  Separate loops
// keep each class's loop-invariant registers out of the others'.  With a
// payload every item is one wave task (the stable pair sort, wave_bitonic).
template <bool PAY, bool U64>
__global__ __launch_bounds__(BASE_THREADS) void k_base_small(Params P) {
    constexpr int W = BASE_THREADS / 64;
    __shared__ uint64_t glds[PAY ? 1 : W][PAY ? 1 : G_SLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * W, wid = (uint64_t)blockIdx.x * W + wv;
    const uint64_t n0 = min<unsigned long long>(P.ctl->nitems, P.item_cap);
    const uint64_t n1 = min<unsigned long long>(P.ctl->nitems_b, P.item_b_cap);
    const uint64_t nw = min<unsigned long long>(P.ctl->nitems_w, P.item_cap);
    const uint64_t nall = PAY ? nw + n1 + n0 : nw;
    for (uint64_t t = wid; t < nall; t += waves) {
        const uint64_t wd = t < nw ? P.items[P.item_cap - 1 - t] : t < nw + n1 ? P.items_b[t - nw] : P.items[t - nw - n1];
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        if (size <= 64) base_small_item<1, PAY>(P, off, size, srcb, lane);
        else if (size <= 128) base_small_item<2, PAY>(P, off, size, srcb, lane);
        else if (size <= 256) base_small_item<4, PAY>(P, off, size, srcb, lane);
        else base_small_item<8, PAY>(P, off, size, srcb, lane);
    }
    if (PAY) return;
    for (uint64_t t = wid; t < (n1 + 3) / 4; t += waves) base_group_task<4, U64>(P, P.items_b, t, n1, glds[wv], lane);
    for (uint64_t t = wid; t < (n0 + 7) / 8; t += waves) base_group_task<3, U64>(P, P.items, t, n0, glds[wv], lane);
}

constexpr int BIG_THREADS = 512;

// One sub-array of 513..4096 keys: gather into registers (BIG_THREADS * E
// elements, padded with the largest key), block_bitonic, write back.  The
// payload follows through the sorted local index, read before any write.
template <int E>
__device__ void base_big_item(const Params& P, uint64_t off, uint32_t size, uint32_t srcb, uint64_t* sk, uint32_t* si) {
    const uint64_t* in = P.keys[srcb];
    uint64_t* out = P.keys[0];
    const int t = threadIdx.x, u64 = P.u64;
    uint64_t k[E];
    uint32_t ix[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = t * E + e;
        k[e] = i < size ? key_ord(in[off + i], u64) : ~0ull;
        ix[e] = i;
    }
    if (P.has_pay) {
        block_bitonic<BIG_THREADS, E, true>(k, ix, sk, si);
        const uint32_t* pin = P.pay[srcb];
        uint32_t* pout = P.pay[0];
        uint32_t pv[E];
#pragma unroll
        for (int e = 0; e < E; e++) pv[e] = t * E + e < size ? pin[off + ix[e]] : 0u;
        __syncthreads();  // every payload read of this sub-array happens before any write
#pragma unroll
        for (int e = 0; e < E; e++)
            if (t * E + e < size) pout[off + t * E + e] = pv[e];
    } else {
        block_bitonic<BIG_THREADS, E, false>(k, ix, sk, si);
    }
#pragma unroll
    for (int e = 0; e < E; e++)
        if (t * E + e < size) out[off + t * E + e] = key_unord(k[e], u64);
    __syncthreads();
}

__global__ __launch_bounds__(BIG_THREADS) void k_base_big(Params P) {
    __shared__ uint64_t sk[C_MAX];
    __shared__ uint32_t si[C_MAX];
    const int tid = threadIdx.x;
    const uint64_t nitems = min<unsigned long long>(P.ctl->nbig, P.big_cap);
    const int has_pay = P.has_pay;
    uint64_t* out = P.keys[0];
    uint32_t* pout = P.pay[0];
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint64_t wd = P.bigs[it];
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u, copy = (wd >> 16) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        const uint64_t* in = P.keys[srcb];
        const uint32_t* pin = P.pay[srcb];
        if (copy) {
            if (srcb)
                for (uint32_t i = tid; i < size; i += BIG_THREADS) {
                    out[off + i] = in[off + i];
                    if (has_pay) pout[off + i] = pin[off + i];
                }
            continue;
        }
        if (size <= 1024) base_big_item<2>(P, off, size, srcb, sk, si);
        else if (size <= 2048) base_big_item<4>(P, off, size, srcb, sk, si);
        else base_big_item<8>(P, off, size, srcb, sk, si);
    }
}


#define LAUNCH(kernel, grid, block, stream, ...)                                     \
    do {                                                                             \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_base_small(const Params& P, uint32_t grid, hipStream_t st) {
    if (P.has_pay) LAUNCH((k_base_small<true, false>), grid, BASE_THREADS, st, P);
    if (P.u64) LAUNCH((k_base_small<false, true>), grid, BASE_THREADS, st, P);
    LAUNCH((k_base_small<false, false>), grid, BASE_THREADS, st, P);
}
hipError_t launch_base_big(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_base_big, grid, BIG_THREADS, st, P); }

}  // namespace ls
