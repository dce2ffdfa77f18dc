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
// k_base_small: keys only, sub-arrays of at most 2048 keys sorted in
// registers by groups of 4, 8, 16, 32 or 64 lanes (group_bitonic, 16 .. 1
// sub-arrays per wavefront); k_base_pay_small: with a payload, sub-arrays of
// at most 512 keys, one per wavefront, as (key, index) pairs
// (packed_pair_sort, else pair_bitonic); k_base_pairs: with a payload,
// 513..1024 keys the same way; k_base_merge: chunk-and-merge items;
// k_base_big: one workgroup per larger sub-array (up to 8192) sorted in LDS,
// and the copies of finished runs.
// ===========================================================================

constexpr int BASE_THREADS = 256;

// A value the same in every lane, moved to scalar registers: addresses formed
// from it are a scalar base plus a lane offset.
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Smallest and largest ordered key of a wavefront's item (pads excluded by
// the caller), in every lane: a butterfly over lane ^ 1 .. lane ^ 32.
template <int S>
__device__ __forceinline__ void wave_span(uint64_t& mn, uint64_t& mx, int lane) {
    if constexpr (S < 6) {
        const uint64_t a = dpp_t<S>(mn, (uint32_t)lane), b = dpp_t<S>(mx, (uint32_t)lane);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
        wave_span<S + 1>(mn, mx, lane);
    }
}

// Stable sort of one wavefront's item of (ordered key, index) pairs, 2^LE per
// lane (indices distinct, below 2^(LE + 6); those at or above size mark
// pads), through the binary64 network.  With IB = LE + 6 index bits, an item
// whose keys span less than 2^(62 - IB) maps each pair to
// (key - min) * 2^IB + index: below 2^62, so the bit pattern of a finite
// non-negative binary64 number, and such numbers order as their bit patterns.
// The numeric network (one v_min_f64 / v_max_f64 per compare-exchange inside
// a lane) then orders by key, then index: the stable order, the same result
// as the pair network, whose 64-bit key and index compares and selects cost
// several times more.  Pads sort last as +inf.  A wider item returns false
// with k and ix untouched (the caller runs the pair network).
template <int LE>
__device__ __forceinline__ bool packed_pair_sort(uint64_t (&k)[1 << LE], uint32_t (&ix)[1 << LE], uint32_t size,
                                                 int lane) {
    constexpr int E = 1 << LE, IB = LE + 6;
    uint64_t mn = ~0ull, mx = 0;
#pragma unroll
    for (int e = 0; e < E; e++) {
        const bool in = ix[e] < size;
        mn = in && k[e] < mn ? k[e] : mn;
        mx = in && k[e] > mx ? k[e] : mx;
    }
    wave_span<0>(mn, mx, lane);
    // the same value in every lane: a uniform branch
    if (__builtin_amdgcn_readfirstlane((int)((mx - mn) >> (62 - IB) != 0))) return false;
    double d[E];
#pragma unroll
    for (int e = 0; e < E; e++)
        d[e] = __builtin_bit_cast(double, ix[e] < size ? ((k[e] - mn) << IB) | ix[e] : 0x7ff0000000000000ull);
    group_bitonic<double, LE, 6>(d, lane);
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint64_t u = __builtin_bit_cast(uint64_t, d[e]);
        k[e] = mn + (u >> IB);
        ix[e] = (uint32_t)u & ((1u << IB) - 1);
    }
    return true;
}

// Group items: 64 / G sub-arrays per wavefront, G lanes and E = 32 keys per
// lane each (group_bitonic): items of up to 128 keys on 4 lanes, 129..256 on
// 8 lanes, 257..512 on 16 lanes, 513..1024 on 32, 1025..2048 on 64.  Loads read key j of a sub-array into lane
// j % G, register j / G (consecutive lanes, consecutive keys: any placement
// of unsorted input is valid).  The sorted keys leave through LDS in phases
// of 16 registers, each wave in its own 8.5 KB region, so that stores are
// contiguous too.  binary64 keys are sorted as numbers unless the task holds
// a NaN or a -0.0 (whose order is the bit pattern's), else as ordered
// integers.
constexpr int GLE = 5, GE = 1 << GLE;
constexpr int GPH = 16;                              // registers per LDS phase
constexpr int G_SLOTS = WAVE * GPH + WAVE * GPH / 16; // LDS slots per wave: one pad slot after every 16
static_assert(GE * 4 == GROUP_SMALL_MAX && GE * 8 == GROUP_MAX && GE * 16 == SMALL_MAX && GE * 32 == GROUP_LARGE_MAX &&
                  GE * 64 == GROUP_WAVE_MAX,
              "lane groups of 4, 8, 16, 32, 64");

__device__ __forceinline__ uint32_t gslot(uint32_t i) { return i + (i >> 4); }

// Wave-local LDS hand-off: the wavefront's own LDS accesses run in order; this
// keeps the compiler from moving them across each other.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A value the compiler cannot see through: lane offsets derived from it are
// formed where they are used instead of being kept in registers across the
// sort (or hoisted out of the task loops).
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Loads and stores of the keys through global (not flat) instructions.
__device__ __forceinline__ uint64_t gload(const uint64_t* p) {
    return *(const __attribute__((address_space(1))) uint64_t*)p;
}
__device__ __forceinline__ void gstore(uint64_t* p, uint64_t v) { *(__attribute__((address_space(1))) uint64_t*)p = v; }

// One payload item of up to 64 * 2^LE keys, one wavefront: a stable sort of
// (ordered key, index) pairs in registers, 2^LE per lane (packed_pair_sort
// when the keys are narrow enough, else pair_bitonic).  Keys and payload are
// read coalesced (element i at lane i % 64, register i / 64: any placement of
// unsorted input is valid), the payload kept in the wave's LDS region by
// position; after the sort element j sits at lane j / 2^LE, register
// j % 2^LE, and takes its payload from LDS through its index.  The sorted
// keys, then the payload, leave through the same region (one pad slot after
// every 2^LE, so that a lane's run starts on a different bank than its
// neighbours') and are stored coalesced.  lr: the wave's region,
// pay_slots(LE) 8-byte slots.
__device__ __forceinline__ constexpr int pay_slots(int LE) { return (WAVE << LE) + WAVE; }

template <int LE>
__device__ __forceinline__ void pay_wave_item(const Params& P, uint64_t off, uint32_t size, uint32_t srcb, int lane,
                                              uint64_t* lr) {
    constexpr int E = 1 << LE;
    const uint64_t* in = P.keys[srcb];
    const uint32_t* pin = P.pay[srcb];
    uint64_t* out = P.keys[0];
    uint32_t* pout = P.pay[0];
    uint32_t* lp = reinterpret_cast<uint32_t*>(lr);
    const int u64 = P.u64;
    auto slot = [](uint32_t j) { return j + (j >> LE); };
    uint64_t k[E];
    uint32_t ix[E];
    {
        // indices clamp to size - 1: every load is in bounds without a branch
        // (the pads' payload slots are never read).  Every load is issued
        // before any is used, so that they are all in flight at once.
        const uint32_t last = size - 1;
        uint32_t pr[E];
#pragma unroll
        for (int r = 0; r < E; r++) {
            const uint32_t c = min<uint32_t>(r * WAVE + opaque(lane), last);
            k[r] = gload(in + off + c);
            pr[r] = pin[off + c];
            // each address formed next to its load
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int r = 0; r < E; r++) {
            const uint32_t i = r * WAVE + lane;
            lp[i] = pr[r];
            k[r] = i < size ? key_ord(k[r], u64) : ~0ull;
            ix[r] = i;
        }
    }
    if (!packed_pair_sort<LE>(k, ix, size, lane)) pair_bitonic<LE, 6>(k, ix, lane);
    wave_lds_sync();
    uint32_t pv[E];
#pragma unroll
    for (int e = 0; e < E; e++) pv[e] = (uint32_t)(lane * E + e) < size ? lp[ix[e]] : 0u;
    wave_lds_sync();  // every gather done before the region is rewritten
#pragma unroll
    for (int e = 0; e < E; e++) lr[slot(lane * E + e)] = k[e];
    wave_lds_sync();
    {
        // every LDS read before any store: one wait for all of them
        uint64_t o[E];
#pragma unroll
        for (int r = 0; r < E; r++) o[r] = lr[slot(r * WAVE + lane)];
#pragma unroll
        for (int r = 0; r < E; r++) {
            const uint32_t j = r * WAVE + opaque(lane);
            if (j < size) gstore(out + off + j, key_unord(o[r], u64));
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; e++) lp[slot(lane * E + e)] = pv[e];
    wave_lds_sync();
    {
        uint32_t o[E];
#pragma unroll
        for (int r = 0; r < E; r++) o[r] = lp[slot(r * WAVE + lane)];
#pragma unroll
        for (int r = 0; r < E; r++) {
            const uint32_t j = r * WAVE + opaque(lane);
            if (j < size) pout[off + j] = o[r];
        }
    }
    wave_lds_sync();  // the next item rewrites the region
}

// One task: 64 / G items, entries [task * GPW, ...) of a list (read from the
// back when REV).  binary64: the numeric network, unless the task holds a NaN
// or a -0.0.  U64: the same network over the differences key - min of each
// item, unless an item spans the +inf bit pattern or more.  Such tasks
// (rarely) hand their items to k_base_mid, which runs after this kernel and
// orders by the totalOrder image (a one-key item is only moved).  Keeping
// the integer network out of this kernel keeps its register count down.
// The descriptor of this lane's item in a task.  Every load is in bounds
// without a branch: an idle group (past the last item) reads the last item
// and gets size 0 from base_group_task.
template <int LG, bool REV>
__device__ __forceinline__ uint64_t group_desc(const uint64_t* items, uint64_t cap, uint64_t task, uint64_t nitem,
                                               int lane) {
    const uint64_t e = min<uint64_t>(task * (WAVE >> LG) + (opaque(lane) >> LG), nitem - 1);
    return items[REV ? cap - 1 - e : e];
}

template <int LG, bool U64>
__device__ __forceinline__ void base_group_task(const Params& P, const uint64_t* k0, const uint64_t* k1, uint64_t wd,
                                                uint64_t task, uint64_t nitem, uint64_t* lds, int lane) {
    constexpr int G = 1 << LG, GPW = WAVE / G;
    // per-task copy of the lane id: the lane offsets r * G + gl are cheap to
    // form again each task, and hoisted out of the task loop they would hold
    // registers for the whole kernel
    const int g = opaque(lane) >> LG, gl = opaque(lane) & (G - 1);
    const uint64_t idx = task * GPW + g;
    // indices clamp to size - 1, so every key load is in bounds too
    const uint64_t off = wd >> 18;
    const uint32_t size = idx < nitem ? (uint32_t)(wd & 0xffffu) + 1 : 0u;
    const uint64_t* src = (((wd >> 17) & 1u) ? k1 : k0) + off;
    uint64_t* dst = const_cast<uint64_t*>(k0) + off;
    const uint32_t last = size ? size - 1 : 0u;
    uint64_t raw[GE];
#pragma unroll
    for (int r = 0; r < GE; r++) {
        raw[r] = gload(src + min<uint32_t>(r * G + gl, last));
        // each address formed next to its load: all of them up front would
        // hold a register pair each until the last load is issued
        __builtin_amdgcn_sched_barrier(0);
    }
    const int gp = opaque(lane) & (G - 1);  // fresh copy: the offsets below are formed again, not kept
    bool special = false;
    uint64_t lo = 0;
    if (U64) {
        // uint64 keys: an item whose keys span less than the +inf bit pattern
        // (max - min < 0x7ff0...) sorts as the binary64 values of the
        // differences key - min: non-negative and finite (subnormal or zero
        // included), their numeric order is the integers' order, so the
        // floating-point network sorts them; min is added back afterwards.
        // A wider item is handed on like a NaN item below.
        uint64_t mn = ~0ull, mx = 0;
#pragma unroll
        for (int r = 0; r < GE; r++) {
            const bool in = (uint32_t)(r * G + gp) < size;
            mn = in && raw[r] < mn ? raw[r] : mn;
            mx = in && raw[r] > mx ? raw[r] : mx;
        }
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {  // over the item's lanes (the low LG lane bits)
            const uint64_t a = __shfl_xor(mn, o), b = __shfl_xor(mx, o);
            mn = a < mn ? a : mn;
            mx = b > mx ? b : mx;
        }
        lo = size ? mn : 0;
        special = size && mx - mn >= 0x7ff0000000000000ull;
#pragma unroll
        for (int r = 0; r < GE; r++)
            raw[r] = (uint32_t)(r * G + gp) < size ? raw[r] - lo : 0x7ff0000000000000ull;  // +inf pads
    } else {
#pragma unroll
        for (int r = 0; r < GE; r++) {
            if ((uint32_t)(r * G + gp) >= size) raw[r] = 0x7ff0000000000000ull;  // +inf pads
            // NaN (any payload, either sign) or -0.0, tested on the bits: no
            // floating-point assumption of this file's build can remove it
            special |= (raw[r] & 0x7fffffffffffffffull) > 0x7ff0000000000000ull || raw[r] == 0x8000000000000000ull;
        }
    }
    if (__ballot(special) != 0) {
        if (gp == 0 && size == 1) {
            if (src != dst) gstore(dst, gload(src));
        } else if (gp == 0 && size > 1) {
            const uint64_t b = atomicAdd(&P.ctl->nbig, 1ull);
            atomicAdd(&P.ctl->nmoved, 1ull);
            if (b < P.big_cap) P.bigs[b] = wd;
            else atomicOr(&P.ctl->overflow, OVF_ITEM);
        }
        return;
    }
    {
        double k[GE];
#pragma unroll
        for (int r = 0; r < GE; r++) k[r] = __builtin_bit_cast(double, raw[r]);
        group_bitonic<double, GLE, LG>(k, lane);
#pragma unroll
        for (int r = 0; r < GE; r++) raw[r] = __builtin_bit_cast(uint64_t, k[r]) + (U64 ? lo : 0ull);
    }
    // Element i of the sub-array is lane i / E, register i % E.  Phase h moves
    // registers 16h .. 16h+15 of every lane: lane c's run lands at LDS slots
    // c*16 .. c*16+15 of the group's region, and is read back as
    // u = rr * G + gl, i.e. element (u / 16) * E + 16h + u % 16, so the G
    // lanes of a store write G consecutive keys.
    const int gs = opaque(lane) & (G - 1);
    uint64_t* mine = lds + (opaque(lane) >> LG) * (G * GPH + G * GPH / 16);
#pragma unroll
    for (int h = 0; h < GE / GPH; h++) {
#pragma unroll
        for (int rr = 0; rr < GPH; rr++) mine[gslot(gs * GPH + rr)] = raw[h * GPH + rr];
        wave_lds_sync();
        uint64_t o[GPH];
#pragma unroll
        for (int rr = 0; rr < GPH; rr++) o[rr] = mine[gslot(rr * G + gs)];
#pragma unroll
        for (int rr = 0; rr < GPH; rr++) {
            const uint32_t u = rr * G + gs, pos = (u / GPH) * GE + h * GPH + u % GPH;
            if (pos < size) gstore(dst + pos, o[rr]);
        }
        wave_lds_sync();  // the next phase (or task) rewrites the region
    }
}

// The tasks of one class, grid-strided over every wavefront; the next task's
// descriptors are loaded before the current task is sorted.
template <int LG, bool U64, bool REV>
__device__ __forceinline__ void group_loop(const Params& P, const uint64_t* items, uint64_t cap, uint64_t nitem,
                                           uint64_t wid, uint64_t waves, uint64_t* lds, int lane) {
    const uint64_t ntask = (nitem + (WAVE >> LG) - 1) / (WAVE >> LG);
    if (wid >= ntask) return;
    const uint64_t* k0 = P.keys[0];
    const uint64_t* k1 = P.keys[1];
    uint64_t wd = group_desc<LG, REV>(items, cap, wid, nitem, lane);
    for (uint64_t t = wid; t < ntask; t += waves) {
        const uint64_t wn = group_desc<LG, REV>(items, cap, min(t + waves, ntask - 1), nitem, lane);
        base_group_task<LG, U64>(P, k0, k1, wd, t, nitem, lds, lane);
        wd = wn;
    }
}

// One loop per group class, each grid-strided over every wavefront (so each
// class is spread evenly), largest items first: tasks of 1 item of
// 1025..2048 keys and of 2 items of 513..1024 (keys only), of 4 items of
// 257..512, of 8 of 129..256, of 16 of up to 128.  Separate loops keep each class's loop-invariant registers
// out of the others'.  Keys only (with a payload: k_base_pay_small).
template <bool U64>
__global__ __launch_bounds__(BASE_THREADS) void k_base_small(Params P) {
    constexpr int W = BASE_THREADS / 64;
    __shared__ uint64_t glds[W][G_SLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * W, wid = (uint64_t)blockIdx.x * W + wv;
    const uint64_t n0 = min<unsigned long long>(P.ctl->nitems, P.item_cap);
    const uint64_t n1 = min<unsigned long long>(P.ctl->nitems_b, P.item_b_cap);
    const uint64_t nw = min<unsigned long long>(P.ctl->nitems_w, P.item_cap);
    const uint64_t nk = min<unsigned long long>(P.ctl->nitems_k, P.item_b_cap);
    const uint64_t nc = min<unsigned long long>(P.ctl->nitems_c, P.item_c_cap);
    // the classes' tasks are dealt out as one list: a class starts at the
    // wavefront after the one the previous class ended on, so that with fewer
    // tasks than wavefronts no wavefront sorts two
    uint64_t o = 0;
    auto first = [&](uint64_t ntask) {
        const uint64_t f = (wid + waves - o % waves) % waves;
        o += ntask;
        return f;
    };
    const uint64_t f6 = first(nc), f5 = first((nk + 1) / 2), f4 = first((nw + 3) / 4), f3 = first((n1 + 7) / 8);
    const uint64_t f2 = first((n0 + 15) / 16);
    group_loop<6, U64, false>(P, P.items_c, P.item_c_cap, nc, f6, waves, glds[wv], lane);
    group_loop<5, U64, true>(P, P.items_b, P.item_b_cap, nk, f5, waves, glds[wv], lane);
    group_loop<4, U64, true>(P, P.items, P.item_cap, nw, f4, waves, glds[wv], lane);
    group_loop<3, U64, false>(P, P.items_b, P.item_b_cap, n1, f3, waves, glds[wv], lane);
    group_loop<2, U64, false>(P, P.items, P.item_cap, n0, f2, waves, glds[wv], lane);
}

constexpr int BIG_THREADS = 512;
constexpr int MID_THREADS = 256, MID_MAX = 2048;

// One sub-array of up to BIG_MAX keys: gather into registers (BIG_THREADS * E
// elements, padded with the largest key), block_bitonic, write back.  The
// payload follows through the sorted local index, read before any write.
template <int E, int NT = BIG_THREADS>
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
        block_bitonic<NT, E, true>(k, ix, sk, si);
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
        block_bitonic<NT, E, false>(k, ix, sk, si);
    }
#pragma unroll
    for (int e = 0; e < E; e++)
        if (t * E + e < size) out[off + t * E + e] = key_unord(k[e], u64);
    __syncthreads();
}

// CAP: the largest item this instantiation sorts (its LDS); the 4096-key one
// also does the copies, the 8192-key one (one workgroup per CU) only the
// few items above 4096 keys.
template <int CAP>
__global__ __launch_bounds__(BIG_THREADS) void k_base_big(Params P) {
    __shared__ uint64_t sk[CAP];
    __shared__ uint32_t si[CAP];
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
        if (CAP > C_MAX) {  // only the large sorts
            if (!copy && size > C_MAX) base_big_item<16>(P, off, size, srcb, sk, si);
            continue;
        }
        if (copy) {
            if (srcb)
                for (uint32_t i = tid; i < size; i += BIG_THREADS) {
                    out[off + i] = in[off + i];
                    if (has_pay) pout[off + i] = pin[off + i];
                }
            continue;
        }
        // items of up to MID_MAX keys: k_base_mid
        if (size > MID_MAX && size <= 4096) base_big_item<8>(P, off, size, srcb, sk, si);
    }
}

// Items of up to MID_MAX keys (with a payload, or keys with NaN / -0): a
// quarter-size workgroup per item, so that four items are in flight per CU.
template <int NT>
__global__ __launch_bounds__(NT) void k_base_mid(Params P) {
    __shared__ uint64_t sk[MID_MAX];
    __shared__ uint32_t si[MID_MAX];
    const uint64_t nitems = min<unsigned long long>(P.ctl->nbig, P.big_cap);
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint64_t wd = P.bigs[it];
        const uint32_t copy = (wd >> 16) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        if (copy || size > MID_MAX) continue;
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u;
        if (size <= NT * 4) base_big_item<4, NT>(P, off, size, srcb, sk, si);
        else base_big_item<MID_MAX / NT, NT>(P, off, size, srcb, sk, si);
    }
}

// Chunk-and-merge items (split_chunks).  Keys only: items of 2049..8192
// keys, whose 2048-key chunks k_base_small has sorted into the caller's
// buffer (k_base_mid the chunks holding a NaN or a -0.0).  With a payload:
// items of 1025..8192 keys, whose 1024-key chunks k_base_pairs has sorted
// stably.  One workgroup per item merges the sorted runs pairwise in LDS,
// runs of one chunk into two, four, eight.  Keys are compared as ordered
// 64-bit images (the totalOrder map), which order every chunk the same way
// whichever kernel sorted it; on equal keys the earlier run's key comes first,
// so the merge of stable runs is stable and the payload follows.  Each
// thread produces 16 consecutive outputs of a round: its start in the pair of
// runs comes from a merge-path search (the number of keys the first run
// contributes to the outputs before it), then it merges sequentially.  The
// item sits in LDS with one pad word after every 16 keys, so that the 16-key
// output runs of a wavefront's lanes fall on distinct banks (17 l mod 32 is a
// bijection).
constexpr int MG_OUT = 16;
static_assert(PAIR_CHUNK % MG_OUT == 0 && GROUP_WAVE_MAX % MG_OUT == 0, "a thread's outputs lie inside one pair of runs");

__device__ __forceinline__ uint32_t mslot(uint32_t i) { return i + (i >> 4); }

// CAP: the largest item of the launch (CAP / 16 threads, its LDS).  Many
// items: each size class (up to 2048 keys, 2049..4096, 4097..8192) has a
// launch of its own with as many workgroups per CU as its LDS allows, and
// skips the others' items.  Few items (ALL): one launch takes every size,
// so that the largest items' merges overlap the others' instead of
// following them.
template <bool PAY, int CAP, bool ALL>
__global__ __launch_bounds__(CAP / MG_OUT) void k_base_merge(Params P) {
    constexpr int MG_THREADS = CAP / MG_OUT;
    constexpr uint32_t NMIN = ALL || CAP <= GROUP_WAVE_MAX ? 0u : CAP / 2;  // items of NMIN+1 .. CAP keys
    static_assert(CAP <= BIG_MAX && CAP % MG_OUT == 0, "item size classes");
    __shared__ uint64_t L[CAP + CAP / 16];
    __shared__ uint32_t Lp[PAY ? CAP + CAP / 16 : 1];
    const int tid = threadIdx.x;
    const uint64_t nm = min<unsigned long long>(P.ctl->nmerge, P.merge_cap);
    uint64_t* keys = P.keys[0];
    uint32_t* pay = P.pay[0];
    const int u64 = P.u64;
    const uint32_t w0 = chunk_keys(PAY);
    for (uint64_t it = blockIdx.x; it < nm; it += gridDim.x) {
        const uint64_t wd = P.merges[it];
        const uint64_t off = wd >> 18;
        const uint32_t n = (uint32_t)(wd & 0xffffu) + 1;
        if (n <= NMIN || n > CAP) continue;  // another launch's item
        {
            uint64_t v[MG_OUT];
#pragma unroll
            for (int r = 0; r < MG_OUT; r++) {
                const uint32_t i = r * MG_THREADS + tid;
                v[r] = i < n ? keys[off + i] : 0ull;
            }
#pragma unroll
            for (int r = 0; r < MG_OUT; r++) {
                const uint32_t i = r * MG_THREADS + tid;
                if (i < n) L[mslot(i)] = key_ord(v[r], u64);
            }
            if (PAY) {
                uint32_t pv[MG_OUT];
#pragma unroll
                for (int r = 0; r < MG_OUT; r++) {
                    const uint32_t i = r * MG_THREADS + tid;
                    pv[r] = i < n ? pay[off + i] : 0u;
                }
#pragma unroll
                for (int r = 0; r < MG_OUT; r++) {
                    const uint32_t i = r * MG_THREADS + tid;
                    if (i < n) Lp[mslot(i)] = pv[r];
                }
            }
        }
        __syncthreads();
        const uint32_t p0 = (uint32_t)tid * MG_OUT;
        for (uint32_t w = w0; w < n; w <<= 1) {
            uint64_t o[MG_OUT];
            uint32_t op[MG_OUT];
            if (p0 < n) {
                const uint32_t a0 = p0 / (2 * w) * (2 * w);     // the pair of runs [a0, a0 + la), [b0, b0 + lb)
                const uint32_t la = min(w, n - a0);
                const uint32_t b0 = a0 + la;
                const uint32_t lb = b0 < n ? min(w, n - b0) : 0u;
                const uint32_t d = p0 - a0;
                // smallest i in [d - lb, min(d, la)] whose A[i] does not precede B[d - i - 1]
                uint32_t lo = d > lb ? d - lb : 0u, hi = min(d, la);
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (L[mslot(a0 + mid)] <= L[mslot(b0 + d - mid - 1)]) lo = mid + 1;
                    else hi = mid;
                }
                uint32_t ia = lo, ib = d - lo;
                uint64_t va = ia < la ? L[mslot(a0 + ia)] : 0ull;
                uint64_t vb = ib < lb ? L[mslot(b0 + ib)] : 0ull;
#pragma unroll
                for (int r = 0; r < MG_OUT; r++) {
                    const bool ta = ib >= lb || (ia < la && va <= vb);
                    o[r] = ta ? va : vb;
                    if (PAY) op[r] = Lp[mslot(ta ? a0 + ia : b0 + ib)];
                    if (ta) {
                        ia++;
                        va = ia < la ? L[mslot(a0 + ia)] : 0ull;
                    } else {
                        ib++;
                        vb = ib < lb ? L[mslot(b0 + ib)] : 0ull;
                    }
                }
            }
            __syncthreads();  // every read of this round is done
#pragma unroll
            for (int r = 0; r < MG_OUT; r++)
                if (p0 + r < n) {
                    L[mslot(p0 + r)] = o[r];
                    if (PAY) Lp[mslot(p0 + r)] = op[r];
                }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < MG_OUT; r++) {
            const uint32_t i = r * MG_THREADS + tid;
            if (i < n) {
                keys[off + i] = key_unord(L[mslot(i)], u64);
                if (PAY) pay[off + i] = Lp[mslot(i)];
            }
        }
        __syncthreads();  // the next item rewrites L
    }
}

// With a payload: items of up to SMALL_MAX keys, one wavefront each
// (pay_wave_item, 1..8 pairs per lane), the three lists dealt out as one.
// (Held to 80 registers for six wavefronts per SIMD it spilled and measured
// 12 % slower.)
__global__ __launch_bounds__(BASE_THREADS) void k_base_pay_small(Params P) {
    constexpr int W = BASE_THREADS / 64;
    __shared__ uint64_t plr[W][pay_slots(3)];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * W, wid = (uint64_t)blockIdx.x * W + wv;
    const uint64_t n0 = min<unsigned long long>(P.ctl->nitems, P.item_cap);
    const uint64_t n1 = min<unsigned long long>(P.ctl->nitems_b, P.item_b_cap);
    const uint64_t nw = min<unsigned long long>(P.ctl->nitems_w, P.item_cap);
    for (uint64_t t = wid; t < nw + n1 + n0; t += waves) {
        const uint64_t wd = wave_uniform(t < nw ? P.items[P.item_cap - 1 - t] : t < nw + n1 ? P.items_b[t - nw]
                                                                                         : P.items[t - nw - n1]);
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        if (size <= 64) pay_wave_item<0>(P, off, size, srcb, lane, plr[wv]);
        else if (size <= 128) pay_wave_item<1>(P, off, size, srcb, lane, plr[wv]);
        else if (size <= 256) pay_wave_item<2>(P, off, size, srcb, lane, plr[wv]);
        else pay_wave_item<3>(P, off, size, srcb, lane, plr[wv]);
    }
}

// With a payload: items and chunks of SMALL_MAX+1 .. PAIR_CHUNK keys, one
// wavefront each (pay_wave_item: 16 pairs per lane, 8 for a chunk of at most
// 512 keys).  Held to 128 registers (four wavefronts per SIMD; a few values
// of the rarely taken pair network go to scratch): measured ~9 % faster than
// with the 172 it would take.
__global__ __launch_bounds__(BASE_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_base_pairs(Params P) {
    constexpr int W = BASE_THREADS / 64;
    __shared__ uint64_t plr[W][pay_slots(4)];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * W, wid = (uint64_t)blockIdx.x * W + wv;
    const uint64_t nc = min<unsigned long long>(P.ctl->nitems_c, P.item_c_cap);
    for (uint64_t t = wid; t < nc; t += waves) {
        const uint64_t wd = wave_uniform(P.items_c[t]);
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        static_assert(SMALL_MAX == 8 * WAVE && PAIR_CHUNK == 16 * WAVE, "8 and 16 pairs per lane");
        if (size <= SMALL_MAX) pay_wave_item<3>(P, off, size, srcb, lane, plr[wv]);
        else pay_wave_item<4>(P, off, size, srcb, lane, plr[wv]);
    }
}

#define LAUNCH(kernel, grid, block, stream, ...)                                     \
    do {                                                                             \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_base_small(const Params& P, uint32_t grid, hipStream_t st) {
    if (P.has_pay) {
        hipLaunchKernelGGL(k_base_pay_small, dim3(grid), dim3(BASE_THREADS), 0, st, P);
        LAUNCH(k_base_pairs, grid, BASE_THREADS, st, P);  // items and chunks of 513..1024 keys
    }
    if (P.u64) LAUNCH(k_base_small<true>, grid, BASE_THREADS, st, P);
    LAUNCH(k_base_small<false>, grid, BASE_THREADS, st, P);
}
hipError_t launch_base_big(const Params& P, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_base_mid<MID_THREADS>, dim3(grid / 2 * 5), dim3(MID_THREADS), 0, st, P);  // 5 per CU
    if (!P.has_pay) LAUNCH(k_base_big<C_MAX>, grid, BIG_THREADS, st, P);  // keys only: copies (large items merge)
    hipLaunchKernelGGL(k_base_big<C_MAX>, dim3(grid), dim3(BIG_THREADS), 0, st, P);
    LAUNCH(k_base_big<BIG_MAX>, grid / 2 ? grid / 2 : 1, BIG_THREADS, st, P);
}
hipError_t launch_base_merge(const Params& P, uint32_t cus, uint32_t classes, hipStream_t st) {
    // workgroups per CU by LDS: keys only 35 / 70 KB (4096 / 8192 keys), with
    // a payload 26 / 52 / 104 KB (2048 / 4096 / 8192)
    if (classes & 8) {  // one launch for every size
        if (P.has_pay) LAUNCH((k_base_merge<true, BIG_MAX, true>), cus, BIG_MAX / MG_OUT, st, P);
        LAUNCH((k_base_merge<false, BIG_MAX, true>), cus * 2, BIG_MAX / MG_OUT, st, P);
    }
    if (P.has_pay) {
        if (classes & 1)
            hipLaunchKernelGGL((k_base_merge<true, GROUP_WAVE_MAX, false>), dim3(cus * 6), dim3(GROUP_WAVE_MAX / MG_OUT), 0,
                               st, P);
        if (classes & 2)
            hipLaunchKernelGGL((k_base_merge<true, 2 * GROUP_WAVE_MAX, false>), dim3(cus * 3),
                               dim3(2 * GROUP_WAVE_MAX / MG_OUT), 0, st, P);
        if (classes & 4)
            hipLaunchKernelGGL((k_base_merge<true, BIG_MAX, false>), dim3(cus), dim3(BIG_MAX / MG_OUT), 0, st, P);
        return hipGetLastError();
    }
    // keys only: merged items hold more than GROUP_WAVE_MAX keys
    if (classes & 2)
        hipLaunchKernelGGL((k_base_merge<false, 2 * GROUP_WAVE_MAX, false>), dim3(cus * 4),
                           dim3(2 * GROUP_WAVE_MAX / MG_OUT), 0, st, P);
    if (classes & 4)
        hipLaunchKernelGGL((k_base_merge<false, BIG_MAX, false>), dim3(cus * 2), dim3(BIG_MAX / MG_OUT), 0, st, P);
    return hipGetLastError();
}

}  // namespace ls
