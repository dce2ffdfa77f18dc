// lsort_dev.hpp -- device-side building blocks of the learned sample sort
// for gfx950 (CDNA4, wave64): key order, model inputs, the three bucket
// functions (monotone RMI, splitter tree with equality buckets, range radix),
// the monotone FP32 MLP, wave-level match and scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lsort_internal.hpp"

namespace ls {

// ---------------------------------------------------------------------------
// Keys
// ---------------------------------------------------------------------------

// Order-preserving image of a key's bits (Sec. 5, float-to-integer key
// extractor): IEEE totalOrder for binary64, identity for uint64.
__device__ __forceinline__ uint64_t key_ord(uint64_t raw, int u64) {
    if (u64) return raw;
    return (raw >> 63) ? ~raw : (raw | 0x8000000000000000ull);
}

__device__ __forceinline__ uint64_t key_unord(uint64_t o, int u64) {
    if (u64) return o;
    return (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
}

// Model input of a key. Returns 0 and sets x for a finite key; -1 / +1 for a
// non-finite binary64 key of negative / positive sign (first / last bucket).
__device__ __forceinline__ int key_x(uint64_t raw, int u64, double& x) {
    if (u64) { x = (double)raw; return 0; }
    if (((raw >> 52) & 0x7ffull) == 0x7ffull) return (raw >> 63) ? -1 : 1;
    x = __longlong_as_double((long long)raw);
    return 0;
}

// ---------------------------------------------------------------------------
// Sampling: SplitMix64 (Steele, Lea & Flood 2014) output k from state seed,
// mapped to [0, n) by the high half of a 64x64 product (Lemire).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t sample_index(uint64_t seed, uint64_t k, uint64_t n) {
    return __umul64hi(splitmix64_at(seed, k), n);
}

// ---------------------------------------------------------------------------
// Bucket functions. Every one is non-decreasing in the key's totalOrder, so a
// partition never misorders keys; rounding can only unbalance buckets.
// ---------------------------------------------------------------------------

// Monotone two-level RMI at total resolution R (Sec. 2.1 formula, Sec. 2.2
// bucket = floor(B F(x)), Sec. 4 clamp intervals).  Stored form (model word 4
// on): 2 + 4L pre-scaled doubles alpha_r, beta_r, then alpha_j, beta_j,
// gamma_j, delta_j per leaf; the bucket is
//   j = clamp(floor(fma(alpha_r, x, beta_r)), 0, L-1)
//   g = clamp(floor(clamp(fma(alpha_j, x, beta_j), gamma_j, delta_j)), 0, R-1).
//
// The partition kernels evaluate an LDS image of it (load_model_lds): header
// and root as stored, the leaf lines as (alpha_j, beta_j) pairs (one 16-byte
// read), then per leaf the bucket range [lo_j, hi_j] its clamp interval
// allows, lo_j = G(gamma_j), hi_j = G(delta_j), G(y) = clamp(floor(y), 0, R-1)
// (lo_j = hi_j = G(delta_j) when gamma_j > delta_j).  G is non-decreasing, so
// G(clamp(t, gamma, delta)) = clamp(G(t), lo, hi); and a saturating
// conversion to uint32 (truncation, negative and NaN to 0) agrees with G
// wherever the bounds do not override it.  Hence
//   j = min(cvt_u32(fma(alpha_r, x, beta_r)), L-1)
//   g = med3(cvt_u32(fma(alpha_j, x, beta_j)), lo_j, hi_j)
// gives the same ids bit for bit with two conversions and two integer clamps
// in place of two floors and six double min/max, and with no branch per key.
constexpr int RMI_PAIRS = 6;  // LDS image: word of the first (alpha_j, beta_j) pair

__device__ __forceinline__ uint32_t cvt_sat_u32(double d) {
    uint32_t r;
    asm("v_cvt_u32_f64 %0, %1" : "=v"(r) : "v"(d));  // saturates; NaN -> 0
    return r;
}

__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t lo, uint32_t hi) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(lo), "v"(hi));
    return r;
}

// The bucket range [lo, hi] that leaf clamp interval [c, d] allows:
// G(c), G(d) with G(y) = clamp(floor(y), 0, R-1); a NaN bound clamps nothing;
// c > d leaves only G(d).
__device__ __forceinline__ void rmi_leaf_range(double c, double d, double Rm1, uint32_t& lo, uint32_t& hi) {
    if (c != c) c = -INFINITY;
    if (d != d) d = INFINITY;
    lo = (uint32_t)fmin(fmax(floor(c), 0.0), Rm1);
    hi = (uint32_t)fmin(fmax(floor(d), 0.0), Rm1);
    if (lo > hi) lo = hi;
}

// LDS image of the leaf table of a stored RMI at src (header first) into dst:
// one leaf per thread of [tid, L) step nt.
__device__ __forceinline__ void rmi_to_lds(uint64_t* dst, const uint64_t* src, int tid, int nt) {
    const RmiModel* h = (const RmiModel*)src;
    const uint32_t L = h->L;
    const double Rm1 = h->R - 1.0;
    for (int i = tid; i < RMI_PAIRS; i += nt) dst[i] = src[i];
    const double* q = (const double*)(src + RMI_PAIRS);
    for (uint32_t j = tid; j < L; j += nt) {
        dst[RMI_PAIRS + 2 * j] = __double_as_longlong(q[4 * j]);
        dst[RMI_PAIRS + 2 * j + 1] = __double_as_longlong(q[4 * j + 1]);
        uint32_t lo, hi;
        rmi_leaf_range(q[4 * j + 2], q[4 * j + 3], Rm1, lo, hi);
        dst[RMI_PAIRS + 2 * L + j] = (uint64_t)lo | ((uint64_t)hi << 32);
    }
}

// Bucket of a key under the LDS image m of an RMI with L leaves (lm1 = L-1,
// rm1 = R-1).  Non-finite binary64 keys go to the first / last bucket by sign.
template <bool U64>
__device__ __forceinline__ uint32_t rmi_lds_bucket(const uint64_t* m, uint32_t L, uint32_t lm1, uint32_t rm1,
                                                   uint64_t raw) {
    const double* p = (const double*)(m + 4);
    const double x = U64 ? (double)raw : __longlong_as_double((long long)raw);
    const uint32_t j = min(cvt_sat_u32(__builtin_fma(p[0], x, p[1])), lm1);
    const double2 ab = *(const double2*)(m + RMI_PAIRS + 2 * j);
    const uint2 lh = *(const uint2*)(m + RMI_PAIRS + 2 * L + j);
    const uint32_t g = med3_u32(cvt_sat_u32(__builtin_fma(ab.x, x, ab.y)), lh.x, lh.y);
    if (U64) return g;
    const bool nf = __builtin_amdgcn_class(x, 0x003 | 0x004 | 0x200);  // NaN, -inf, +inf
    const uint32_t edge = (int32_t)(raw >> 32) < 0 ? 0u : rm1;
    return nf ? edge : g;
}

// The same bucket (at resolution R) evaluated on the stored form in global
// memory, for the few keys a search needs.
__device__ __forceinline__ uint32_t rmi_stored_bucket(const uint64_t* model, uint64_t raw, int u64) {
    const RmiModel* h = (const RmiModel*)model;
    const double* p = (const double*)(model + 4);
    const uint32_t rm1 = (uint32_t)(h->R - 1.0);
    const double x = u64 ? (double)raw : __longlong_as_double((long long)raw);
    if (!u64 && __builtin_amdgcn_class(x, 0x003 | 0x004 | 0x200)) return (int32_t)(raw >> 32) < 0 ? 0u : rm1;
    const uint32_t j = min(cvt_sat_u32(__builtin_fma(p[0], x, p[1])), h->L - 1);
    const double* q = p + 2 + 4 * j;
    uint32_t lo, hi;
    rmi_leaf_range(q[2], q[3], h->R - 1.0, lo, hi);
    return med3_u32(cvt_sat_u32(__builtin_fma(q[0], x, q[1])), lo, hi);
}

// Splitter tree (Sec. 2.4): k = #{u_i <= o} by branch-free binary lifting over
// the ascending splitters (the search a Super Scalar SampleSort decision tree
// performs), then the equality-bucket remap through lut[k] =
// (equality buckets before splitter k) << 1 | (splitter k-1 has one).
__device__ __forceinline__ uint32_t tree_bucket(const uint64_t* u, const uint16_t* lut, uint32_t m, uint32_t top,
                                                uint64_t o) {
    uint32_t k = 0;
    for (uint32_t s = top; s > 0; s >>= 1) {
        uint32_t nk = k + s;
        if (nk <= m && u[nk - 1] <= o) k = nk;
    }
    uint32_t e = lut[k];
    uint32_t id = k + (e >> 1);
    if ((e & 1u) && u[k - 1] == o) id -= 1;
    return id;
}

// Range radix: the top bits of (o - lo).
__device__ __forceinline__ uint32_t radix_bucket(uint64_t lo, uint32_t shift, uint64_t o) {
    return shift >= 64 ? 0u : (uint32_t)((o - lo) >> shift);
}

// Monotone MLP CDF in FP32 (1-16-16-1; non-negative effective weights;
// units 0..7 max(z,0), 8..15 min(z,0)); fmaf chains in index order.
__device__ __forceinline__ float mlp_eval(const float* w, float t) {
    float h1[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) {
        float z = __builtin_fmaf(w[OFF_V1 + i], t, w[OFF_B1 + i]);
        h1[i] = i < MLP_HALF ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
    }
    float out = w[OFF_B3];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) {
        float z = w[OFF_B2 + i];
#pragma unroll
        for (int k = 0; k < MLP_H; k++) z = __builtin_fmaf(w[OFF_V2 + MLP_H * i + k], h1[k], z);
        float h = i < MLP_HALF ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
        // The output layer consumes h2 in index order, so it can be folded in
        // here without changing the operation sequence.
        out = __builtin_fmaf(w[OFF_V3 + i], h, out);
    }
    return fminf(fmaxf(out, 0.0f), 1.0f);
}

__device__ __forceinline__ float mlp_input(double x, double lo, double inv) {
    double t = (x - lo) * inv;
    t = fmin(fmax(t, 0.0), 1.0);
    return (float)t;
}

// K keys per thread through the network at once: the same operation
// sequence per key as mlp_eval, with each weight read from LDS once for all
// K keys (the weights are uniform across the wave, so their reads are
// broadcasts; K amortises them against the ~300 FMAs per key).
template <int K>
__device__ __forceinline__ void mlp_eval_multi(const float* w, const float (&t)[K], float (&F)[K]) {
    float h1[K][MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) {
        const float v = w[OFF_V1 + i], b = w[OFF_B1 + i];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const float z = __builtin_fmaf(v, t[k], b);
            h1[k][i] = i < MLP_HALF ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
        }
    }
    float out[K];
#pragma unroll
    for (int k = 0; k < K; k++) out[k] = w[OFF_B3];
    // layer 2, max units then min units; not unrolled over units, so that
    // only one unit's 16 weights are live at a time
#pragma unroll
    for (int half = 0; half < 2; half++) {
#pragma unroll 1
        for (int i = half * MLP_HALF; i < (half + 1) * MLP_HALF; i++) {
            float z[K];
#pragma unroll
            for (int k = 0; k < K; k++) z[k] = w[OFF_B2 + i];
#pragma unroll
            for (int j = 0; j < MLP_H; j++) {
                const float v = w[OFF_V2 + MLP_H * i + j];
#pragma unroll
                for (int k = 0; k < K; k++) z[k] = __builtin_fmaf(v, h1[k][j], z[k]);
            }
            const float v3 = w[OFF_V3 + i];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const float h = half == 0 ? fmaxf(z[k], 0.0f) : fminf(z[k], 0.0f);
                out[k] = __builtin_fmaf(v3, h, out[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; k++) F[k] = fminf(fmaxf(out[k], 0.0f), 1.0f);
}

// Two-level model with the MLP as its root (Sec. 2.1 stages): the leaf is
// j = min(floor(F * L), L - 1) in fp32 from the clamped network output F,
// then leaf j's clamped line at total resolution R as in rmi_eval.  F is
// non-decreasing in x, so j is, and the clamp chain keeps g monotone.
// Non-finite keys go to 0 (negative) or R - 1.
template <int K>
__device__ __forceinline__ void mlp_root_buckets(const float* w, const double* leaves, double lo, double inv, float Lf,
                                                 double Rm1, const uint64_t (&raw)[K], int u64, uint32_t (&g)[K]) {
    double x[K];
    int nf[K];
    float t[K], F[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        nf[k] = key_x(raw[k], u64, x[k]);
        t[k] = nf[k] ? 0.0f : mlp_input(x[k], lo, inv);
    }
    mlp_eval_multi<K>(w, t, F);
#pragma unroll
    for (int k = 0; k < K; k++) {
        const float j = fminf(floorf(F[k] * Lf), Lf - 1.0f);
        const double* q = leaves + 4 * (int)j;
        double u = __builtin_fma(q[0], x[k], q[1]);
        u = fmin(fmax(u, q[2]), q[3]);
        double gg = floor(u);
        gg = fmin(fmax(gg, 0.0), Rm1);
        g[k] = nf[k] ? (nf[k] < 0 ? 0u : (uint32_t)Rm1) : (uint32_t)gg;
    }
}

// The network alone as a CDF at resolution R (fp32).
template <int K>
__device__ __forceinline__ void mlp_buckets_multi(const float* w, double lo, double inv, float Rf,
                                                  const uint64_t (&raw)[K], int u64, uint32_t (&g)[K]) {
    double x[K];
    int nf[K];
    float t[K], F[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        nf[k] = key_x(raw[k], u64, x[k]);
        t[k] = nf[k] ? 0.0f : mlp_input(x[k], lo, inv);
    }
    mlp_eval_multi<K>(w, t, F);
#pragma unroll
    for (int k = 0; k < K; k++) {
        const float gg = fminf(floorf(F[k] * Rf), Rf - 1.0f);
        g[k] = nf[k] ? (nf[k] < 0 ? 0u : (uint32_t)(Rf - 1.0f)) : (uint32_t)gg;
    }
}

// Keeps the compiler from hoisting LDS weight reads out of a loop (which
// would pin all 321 weights in registers and leave one wave per SIMD).
__device__ __forceinline__ void lds_reload_fence() { __asm__ volatile("" ::: "memory"); }

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Value of lane (lane ^ s) for s in {1, 2, 4, 8, 16, 32}, without LDS: DPP
// quad permutes for 1 and 2, row rotates for 4 and 8 (16-lane rows), and the
// gfx950 permlane swaps for 16 and 32.  Every lane must be active.  s must
// be a compile-time constant after unrolling.
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v, int s, uint32_t lane) {
    switch (s) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    case 4: {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12C, 0xF, 0xF, false);  // row_ror 12: lane+4
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, false);  // row_ror 4: lane-4
        return (lane & 4) ? dn : up;
    }
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror 8
    case 16: {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    default: {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
    }
}

__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, int s, uint32_t lane) {
    const uint32_t lo = xor_lane32((uint32_t)v, s, lane), hi = xor_lane32((uint32_t)(v >> 32), s, lane);
    return ((uint64_t)hi << 32) | lo;
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Lanes of the active set whose value v equals this lane's (v < 2^bits):
// one ballot per bit (wave64 has no native match instruction).
__device__ __forceinline__ uint64_t match_peers(uint32_t v, int bits) {
    uint64_t peers = __ballot(1);
    for (int i = 0; i < bits; i++) {
        uint32_t bit = (v >> i) & 1u;
        uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// ===========================================================================
// Block-level reductions and scans (deterministic: fixed combination order)
// ===========================================================================

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T y = __shfl_xor(v, o);
        v = y > v ? y : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T y = __shfl_xor(v, o);
        v = y < v ? y : v;
    }
    return v;
}

// Sum over the block; every thread gets the total. sh: >= NT/64 entries.
template <int NT, typename T>
__device__ T block_sum(T v, T* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    T t = 0;
    for (int i = 0; i < NT / 64; i++) t += sh[i];
    __syncthreads();
    return t;
}

template <int NT, typename T>
__device__ T block_max(T v, T* sh) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    T t = sh[0];
    for (int i = 1; i < NT / 64; i++) t = sh[i] > t ? sh[i] : t;
    __syncthreads();
    return t;
}

template <int NT, typename T>
__device__ T block_min(T v, T* sh) {
    v = wave_min(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    T t = sh[0];
    for (int i = 1; i < NT / 64; i++) t = sh[i] < t ? sh[i] : t;
    __syncthreads();
    return t;
}

// Exclusive prefix sum of one value per thread; *total gets the sum.
template <int NT, typename T>
__device__ T block_excl_scan(T v, T* sh, T* total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) sh[w] = x;
    __syncthreads();
    T before = 0, all = 0;
    for (int i = 0; i < NT / 64; i++) {
        if (i < w) before += sh[i];
        all += sh[i];
    }
    __syncthreads();
    if (total) *total = all;
    return before + x - v;
}

// Inclusive prefix maximum of one double per thread.
template <int NT>
__device__ double block_incl_max(double v, double* sh) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        double y = __shfl_up(x, o);
        if (lane >= o) x = y > x ? y : x;
    }
    __syncthreads();
    if (lane == 63) sh[w] = x;
    __syncthreads();
    double before = -INFINITY;
    for (int i = 0; i < w; i++) before = sh[i] > before ? sh[i] : before;
    __syncthreads();
    return before > x ? before : x;
}

__device__ __forceinline__ uint32_t ceil_log2(uint32_t v) {  // smallest b with 2^b >= v
    return v <= 1 ? 0 : 32 - __clz(v - 1);
}
__device__ __forceinline__ uint32_t floor_pow2(uint32_t v) { return v ? 1u << (31 - __clz(v)) : 0; }

// In-LDS bitonic sort (Batcher 1968) of P (power of two) ordered keys.
template <int NT>
__device__ void bitonic_keys(uint64_t* a, uint32_t P) {
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = threadIdx.x; q < P / 2; q += NT) {
                uint32_t i = ((q & ~(j - 1)) << 1) | (q & (j - 1));  // j is a power of two
                uint32_t l = i + j;
                bool up = (i & k) == 0;
                uint64_t x = a[i], y = a[l];
                if ((x > y) == up) { a[i] = y; a[l] = x; }
            }
            __syncthreads();
        }
    }
}

// Same on (key, index) pairs, ordered lexicographically (stable tie-break).
template <int NT>
__device__ void bitonic_pairs(uint64_t* a, uint16_t* ix, uint32_t P) {
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = threadIdx.x; q < P / 2; q += NT) {
                uint32_t i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                uint32_t l = i + j;
                bool up = (i & k) == 0;
                uint64_t x = a[i], y = a[l];
                uint16_t xi = ix[i], yi = ix[l];
                bool gt = x > y || (x == y && xi > yi);
                if (gt == up) { a[i] = y; a[l] = x; ix[i] = yi; ix[l] = xi; }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Group sort (keys only): one wavefront sorts 64/G independent sub-arrays at
// once, G = 2^LG lanes each (G <= 64), E = 2^LE keys per lane.
// Element i of a sub-array sits in lane (group base + i / E), register i % E:
// the low LE index bits are register bits, so most comparators of the
// network join two registers of one lane.  The network is the bitonic sort
// in its flip form: phase p merges sorted runs of 2^(p-1) by comparing i with
// i ^ (2^p - 1), then half-cleans with i ^ 2^c for c = p-2 .. 0; every
// comparator puts the smaller key at the lower index, so there are no
// direction bits.  Lane partners come from dpp_t: the flip's partner lane is
// a mirror, a half-cleaner's a lane xor.
//   T = double: finite or infinite binary64 keys without NaN and without
//   -0.0 (callers check), compared as numbers (v_min_f64 / v_max_f64);
//   T = uint64_t: ordered keys compared as integers.
// ---------------------------------------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wavefront in six DPP adds (no
// LDS): shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the last lane
// of row 0 / 2 added to rows 1 / 3 and that of row 1 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr 1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr 2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr 4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr 8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast 15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast 31
    return x;
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Partner value across lanes: OP s (0..5) is lane ^ 2^s, OP 8 + s is the
// mirror lane ^ (2^(s+1) - 1).  Inside a row of 16 lanes DPP does it (one
// move per word, two for lane ^ 4); lane bits 4 and 5 go through the
// permlane swaps (xor_lane64).
template <int OP, typename T>
__device__ __forceinline__ T dpp_t(T v, uint32_t lane) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    if constexpr (OP == 0) u = dpp_u64<0xB1>(u);                  // lane ^ 1
    else if constexpr (OP == 1) u = dpp_u64<0x4E>(u);             // lane ^ 2
    else if constexpr (OP == 2) u = dpp_u64<0x1B>(dpp_u64<0x141>(u));  // lane ^ 4 = (lane ^ 7) ^ 3
    else if constexpr (OP == 3) u = dpp_u64<0x128>(u);            // lane ^ 8
    else if constexpr (OP == 4) u = xor_lane64(u, 16, lane);      // lane ^ 16
    else if constexpr (OP == 5) u = xor_lane64(u, 32, lane);      // lane ^ 32
    else if constexpr (OP == 8) u = dpp_u64<0xB1>(u);             // lane ^ 1  (mirror of 2 lanes)
    else if constexpr (OP == 9) u = dpp_u64<0x1B>(u);             // lane ^ 3  (mirror of 4)
    else if constexpr (OP == 10) u = dpp_u64<0x141>(u);           // lane ^ 7  (mirror of 8)
    else if constexpr (OP == 11) u = dpp_u64<0x140>(u);           // lane ^ 15 (mirror of 16)
    else if constexpr (OP == 12) u = xor_lane64(dpp_u64<0x140>(u), 16, lane);                       // lane ^ 31
    else u = xor_lane64(xor_lane64(dpp_u64<0x140>(u), 16, lane), 32, lane);                         // lane ^ 63
    return __builtin_bit_cast(T, u);
}

// Comparator inside a lane: a <- min, b <- max.
__device__ __forceinline__ void cx_reg(double& a, double& b) {
    const double lo = __builtin_fmin(a, b), hi = __builtin_fmax(a, b);
    a = lo;
    b = hi;
}
__device__ __forceinline__ void cx_reg(uint64_t& a, uint64_t& b) {
    const bool lt = a < b;
    const uint64_t lo = lt ? a : b, hi = lt ? b : a;
    a = lo;
    b = hi;
}

// Lane-pair comparator: the lane holding the higher index (keep_max) keeps
// the larger key of the pair, its partner the smaller.
template <typename T>
__device__ __forceinline__ T cx_lane(T mine, T other, bool keep_max) {
    return ((other < mine) != keep_max) ? other : mine;
}

// Index with a 0 bit inserted at position c: the q-th register whose bit c is 0.
__device__ __forceinline__ constexpr int ins0(int q, int c) { return ((q >> c) << (c + 1)) | (q & ((1 << c) - 1)); }

// Scheduling window: a fence every GW comparators keeps the scheduler from
// overlapping a whole stage's comparators, each of which holds a temporary
// register pair while in flight.
constexpr int GW = 4;
__device__ __forceinline__ void cx_window(int q) {
    if ((q % GW) == GW - 1) __builtin_amdgcn_sched_barrier(0);
}

// One stage of the network, B the index bit it compares across; FLIP: the
// merge's first stage (partner i ^ (2^(B+1) - 1)), else a half-cleaner
// (partner i ^ 2^B).  Stages and phases are unrolled by template recursion,
// so every register index and lane exchange is a compile-time constant.
template <typename T, int LE, int B, bool FLIP>
__device__ __forceinline__ void group_stage(T (&k)[1 << LE], int lane) {
    constexpr int E = 1 << LE;
    if constexpr (B < LE) {  // inside the lane
#pragma unroll
        for (int q = 0; q < E / 2; q++) {
            const int r = ins0(q, B);
            cx_reg(k[r], k[FLIP ? r ^ ((2 << B) - 1) : r | (1 << B)]);
            cx_window(q);
        }
    } else if constexpr (FLIP && E == 1) {  // one register: the mirror lane's
        constexpr int S = B - LE;
        const bool km = (lane >> S) & 1;
        k[0] = cx_lane(k[0], dpp_t<8 + S>(k[0], (uint32_t)lane), km);
    } else if constexpr (FLIP) {  // partner lane ^ (2^(s+1) - 1), register E-1-r
        constexpr int S = B - LE;
        const bool km = (lane >> S) & 1;
#pragma unroll
        for (int r = 0; r < E / 2; r++) {
            const T y0 = dpp_t<8 + S>(k[E - 1 - r], (uint32_t)lane), y1 = dpp_t<8 + S>(k[r], (uint32_t)lane);
            k[r] = cx_lane(k[r], y0, km);
            k[E - 1 - r] = cx_lane(k[E - 1 - r], y1, km);
            cx_window(r);
        }
    } else {
        constexpr int S = B - LE;
        const bool km = (lane >> S) & 1;
#pragma unroll
        for (int r = 0; r < E; r++) {
            k[r] = cx_lane(k[r], dpp_t<S>(k[r], (uint32_t)lane), km);
            cx_window(r);
        }
    }
}

template <typename T, int LE, int C>
__device__ __forceinline__ void group_clean(T (&k)[1 << LE], int lane) {
    if constexpr (C >= 0) {
        group_stage<T, LE, C, false>(k, lane);
        group_clean<T, LE, C - 1>(k, lane);
    }
}

template <typename T, int LE, int LG, int PH>
__device__ __forceinline__ void group_phases(T (&k)[1 << LE], int lane) {
    if constexpr (PH <= LE + LG) {
        group_stage<T, LE, PH - 1, true>(k, lane);
        group_clean<T, LE, PH - 2>(k, lane);
        group_phases<T, LE, LG, PH + 1>(k, lane);
    }
}

template <typename T, int LE, int LG>
__device__ __forceinline__ void group_bitonic(T (&k)[1 << LE], int lane) {
    static_assert(LG <= 6, "lane groups within one wavefront");
    group_phases<T, LE, LG, 1>(k, lane);
}

// The same network over (key, index) pairs, ordered by key, then index
// (indices are distinct: a total order, so the result is the stable order):
// 2^LE pairs per lane, element i = lane * 2^LE + register, 2^LG lanes.
template <int OP>
__device__ __forceinline__ uint32_t dpp32(uint32_t v, uint32_t lane) {
    auto m = [](uint32_t x, auto ctrl) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, decltype(ctrl)::value, 0xF, 0xF, false);
    };
    using C0 = std::integral_constant<int, 0xB1>;
    using C1 = std::integral_constant<int, 0x4E>;
    using C3 = std::integral_constant<int, 0x1B>;
    using C7 = std::integral_constant<int, 0x141>;
    using C8 = std::integral_constant<int, 0x128>;
    using C15 = std::integral_constant<int, 0x140>;
    if constexpr (OP == 0 || OP == 8) return m(v, C0{});
    else if constexpr (OP == 1) return m(v, C1{});
    else if constexpr (OP == 2) return m(m(v, C7{}), C3{});
    else if constexpr (OP == 3) return m(v, C8{});
    else if constexpr (OP == 4) return xor_lane32(v, 16, lane);
    else if constexpr (OP == 5) return xor_lane32(v, 32, lane);
    else if constexpr (OP == 9) return m(v, C3{});
    else if constexpr (OP == 10) return m(v, C7{});
    else if constexpr (OP == 11) return m(v, C15{});
    else if constexpr (OP == 12) return xor_lane32(m(v, C15{}), 16, lane);
    else return xor_lane32(xor_lane32(m(v, C15{}), 16, lane), 32, lane);
}

__device__ __forceinline__ bool pair_lt(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

template <int LE, int B, bool FLIP>
__device__ __forceinline__ void pair_stage(uint64_t (&k)[1 << LE], uint32_t (&x)[1 << LE], int lane) {
    constexpr int E = 1 << LE;
    if constexpr (B < LE) {  // inside the lane
#pragma unroll
        for (int q = 0; q < E / 2; q++) {
            const int r = ins0(q, B), s = FLIP ? r ^ ((2 << B) - 1) : r | (1 << B);
            const bool lt = pair_lt(k[r], x[r], k[s], x[s]);
            const uint64_t k0 = lt ? k[r] : k[s], k1 = lt ? k[s] : k[r];
            const uint32_t x0 = lt ? x[r] : x[s], x1 = lt ? x[s] : x[r];
            k[r] = k0; k[s] = k1; x[r] = x0; x[s] = x1;
            cx_window(q);
        }
    } else {
        constexpr int S = B - LE;
        const bool km = (lane >> S) & 1;
        // the lane holding the higher element keeps the larger pair
        auto take = [&](int r, uint64_t ky, uint32_t iy) {
            const bool t = pair_lt(ky, iy, k[r], x[r]) != km;
            k[r] = t ? ky : k[r];
            x[r] = t ? iy : x[r];
        };
        if constexpr (FLIP && E == 1) {  // one register: the mirror lane's
            take(0, dpp_t<8 + S>(k[0], (uint32_t)lane), dpp32<8 + S>(x[0], (uint32_t)lane));
        } else if constexpr (FLIP) {  // partner lane ^ (2^(S+1) - 1), register E-1-r
#pragma unroll
            for (int r = 0; r < E / 2; r++) {
                const uint64_t y0 = dpp_t<8 + S>(k[E - 1 - r], (uint32_t)lane), y1 = dpp_t<8 + S>(k[r], (uint32_t)lane);
                const uint32_t j0 = dpp32<8 + S>(x[E - 1 - r], (uint32_t)lane), j1 = dpp32<8 + S>(x[r], (uint32_t)lane);
                take(r, y0, j0);
                take(E - 1 - r, y1, j1);
                cx_window(r);
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; r++) {
                const uint64_t y = dpp_t<S>(k[r], (uint32_t)lane);
                const uint32_t j = dpp32<S>(x[r], (uint32_t)lane);
                take(r, y, j);
                cx_window(r);
            }
        }
    }
}

template <int LE, int C>
__device__ __forceinline__ void pair_clean(uint64_t (&k)[1 << LE], uint32_t (&x)[1 << LE], int lane) {
    if constexpr (C >= 0) {
        pair_stage<LE, C, false>(k, x, lane);
        pair_clean<LE, C - 1>(k, x, lane);
    }
}

template <int LE, int LG, int PH>
__device__ __forceinline__ void pair_phases(uint64_t (&k)[1 << LE], uint32_t (&x)[1 << LE], int lane) {
    if constexpr (PH <= LE + LG) {
        pair_stage<LE, PH - 1, true>(k, x, lane);
        pair_clean<LE, PH - 2>(k, x, lane);
        pair_phases<LE, LG, PH + 1>(k, x, lane);
    }
}

template <int LE, int LG>
__device__ __forceinline__ void pair_bitonic(uint64_t (&k)[1 << LE], uint32_t (&x)[1 << LE], int lane) {
    static_assert(LG <= 6, "lane groups within one wavefront");
    pair_phases<LE, LG, 1>(k, x, lane);
}

// Bitonic sort of NT*E (key[, index]) pairs by a workgroup of NT threads,
// thread t holding elements t*E .. t*E+E-1 in registers.  Stages with
// distance j < E stay in registers, E <= j < 64E exchange through cross-lane
// shuffles, and only j >= 64E go through LDS (column layout ex[e*NT + t], so
// a wavefront's accesses are conflict-free).  exk / exi: NT*E entries of LDS.
template <int NT, int E, bool PAIRS>
__device__ void block_bitonic(uint64_t (&k)[E], uint32_t (&ix)[E], uint64_t* exk, uint32_t* exi) {
    constexpr int N = NT * E;
    const int t = threadIdx.x;
    for (int kk = 2; kk <= N; kk <<= 1) {
        int j = kk >> 1;
        for (; j >= 64 * E; j >>= 1) {  // partner in another wavefront: through LDS
            const int s = j / E;
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; e++) {
                exk[e * NT + t] = k[e];
                if (PAIRS) exi[e * NT + t] = ix[e];
            }
            __syncthreads();
            const bool keep_max = (((t * E) & kk) == 0) != ((t & s) == 0);
#pragma unroll
            for (int e = 0; e < E; e++) {
                const uint64_t y = exk[e * NT + (t ^ s)];
                const uint32_t iy = PAIRS ? exi[e * NT + (t ^ s)] : 0u;
                const bool lt = y < k[e] || (PAIRS && y == k[e] && iy < ix[e]);
                if (lt != keep_max) {
                    k[e] = y;
                    if (PAIRS) ix[e] = iy;
                }
            }
        }
        for (; j >= E; j >>= 1) {  // partner in the same wavefront: shuffle
            const int s = j / E;
            const bool keep_max = (((t * E) & kk) == 0) != ((t & s) == 0);
#pragma unroll
            for (int e = 0; e < E; e++) {
                const uint64_t y = __shfl_xor(k[e], s);
                const uint32_t iy = PAIRS ? __shfl_xor(ix[e], s) : 0u;
                const bool lt = y < k[e] || (PAIRS && y == k[e] && iy < ix[e]);
                if (lt != keep_max) {
                    k[e] = y;
                    if (PAIRS) ix[e] = iy;
                }
            }
        }
#pragma unroll
        for (int jj = E / 2; jj > 0; jj >>= 1) {  // partner in the same thread
            if (jj <= j) {
#pragma unroll
                for (int e = 0; e < E; e++) {
                    if ((e & jj) == 0) {
                        const int f = e | jj;
                        const bool up = ((t * E + e) & kk) == 0;
                        const bool gt = k[e] > k[f] || (PAIRS && k[e] == k[f] && ix[e] > ix[f]);
                        if (gt == up) {
                            uint64_t tmp = k[e]; k[e] = k[f]; k[f] = tmp;
                            if (PAIRS) { uint32_t u = ix[e]; ix[e] = ix[f]; ix[f] = u; }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
}

// ===========================================================================
// Model views in LDS
// ===========================================================================

struct View {
    uint32_t kind, nb, win, log2B2;
    uint32_t L, lm1, rm1;  // RMI: leaves, L - 1, R - 1
    uint32_t m, top;     // tree
    uint64_t lo;         // radix
    uint32_t shift;
};

// Partition models evaluated inside the partition kernels.  The MLP-rooted
// model is not among them: k_mlp_ids first stores every key's bucket id of
// such a level, so that its ~300 FMAs per key are paid once, not twice.
__device__ __forceinline__ View make_view(const uint64_t* mdl, uint32_t kind, uint32_t nb, uint32_t win) {
    View v{};
    v.kind = kind; v.nb = nb; v.win = win;
    if (kind == K_RMI || kind == K_RMI_FINE) {
        const RmiModel* h = (const RmiModel*)mdl;
        v.L = h->L; v.lm1 = h->L - 1; v.rm1 = (uint32_t)(h->R - 1.0); v.log2B2 = h->log2B2;
    } else if (kind == K_TREE || kind == K_TREE_FORCED) {
        const TreeModel* h = (const TreeModel*)mdl;
        v.m = h->m; v.top = h->top;
    } else if (kind == K_RADIX) {
        const RadixModel* h = (const RadixModel*)mdl;
        v.lo = h->lo; v.shift = h->shift;
    }
    return v;
}

// Model of a segment into the LDS of a partition kernel: the RMI's LDS
// image, a tree or radix model as stored; nothing for the stored-id kinds
// (their bucket ids come from k_mlp_ids).
__device__ __forceinline__ void load_model_lds(uint64_t* dst, const uint64_t* src, uint32_t kind, uint32_t words,
                                               int tid, int nt) {
    if (kind == K_RMI || kind == K_RMI_FINE) {
        rmi_to_lds(dst, src, tid, nt);
    } else if (kind == K_TREE || kind == K_TREE_FORCED || kind == K_RADIX) {
        const uint32_t w = words < (uint32_t)LDS_MODEL_WORDS ? words : (uint32_t)LDS_MODEL_WORDS;
        for (uint32_t i = tid; i < w; i += nt) dst[i] = src[i];
    }
}

// Bucket of the key at absolute position pos (stash: precomputed id), the
// model being in LDS (load_model_lds).
__device__ __forceinline__ uint32_t view_bucket(const View& v, const uint64_t* mdl, uint64_t raw, int u64,
                                                const uint16_t* ids, uint64_t pos) {
    switch (v.kind) {
    case K_RMI:
    case K_RMI_FINE: {
        const uint32_t g = u64 ? rmi_lds_bucket<true>(mdl, v.L, v.lm1, v.rm1, raw)
                               : rmi_lds_bucket<false>(mdl, v.L, v.lm1, v.rm1, raw);
        return v.kind == K_RMI ? g >> v.log2B2 : g - v.win;
    }
    case K_TREE:
    case K_TREE_FORCED:
        return tree_bucket(mdl + 2, (const uint16_t*)(mdl + 2 + v.m), v.m, v.top, key_ord(raw, u64));
    case K_RADIX: return radix_bucket(v.lo, v.shift, key_ord(raw, u64));
    default: return ids[pos];  // K_MLP, K_MLP_FINE: ids stored by k_mlp_ids
    }
}

// view_bucket with the kind fixed at compile time (KIND: K_RMI, K_RMI_FINE,
// each with or without KIND_U64 for uint64 keys, K_TREE for both tree kinds,
// K_RADIX, K_MLP for both stored-id kinds), so that a loop over keys carries
// no per-key dispatch; KIND 0 dispatches at run time (one copy of the loop).
constexpr int KIND_U64 = 0x100;

template <int KIND>
__device__ __forceinline__ uint32_t kind_bucket(const View& v, const uint64_t* mdl, uint64_t raw, int u64,
                                                const uint16_t* ids, uint64_t pos) {
    constexpr int K = KIND & 0xff;
    constexpr bool U = (KIND & KIND_U64) != 0;
    if constexpr (KIND == 0) return view_bucket(v, mdl, raw, u64, ids, pos);
    else if constexpr (K == K_RMI) return rmi_lds_bucket<U>(mdl, v.L, v.lm1, v.rm1, raw) >> v.log2B2;
    else if constexpr (K == K_RMI_FINE) return rmi_lds_bucket<U>(mdl, v.L, v.lm1, v.rm1, raw) - v.win;
    else if constexpr (K == K_TREE)
        return tree_bucket(mdl + 2, (const uint16_t*)(mdl + 2 + v.m), v.m, v.top, key_ord(raw, u64));
    else if constexpr (K == K_RADIX) return radix_bucket(v.lo, v.shift, key_ord(raw, u64));
    else return ids[pos];
}

// Calls f(std::integral_constant<int, KIND>) for the kind of a view and the
// key type (with KIND 0, the run-time dispatch, when SPECIALISE is false).
template <bool SPECIALISE = true, typename F>
__device__ __forceinline__ void with_kind(uint32_t kind, int u64, F&& f) {
    if (!SPECIALISE) {
        f(std::integral_constant<int, 0>{});
        return;
    }
    switch (kind) {
    case K_RMI:
        if (u64) f(std::integral_constant<int, K_RMI | KIND_U64>{});
        else f(std::integral_constant<int, K_RMI>{});
        break;
    case K_RMI_FINE:
        if (u64) f(std::integral_constant<int, K_RMI_FINE | KIND_U64>{});
        else f(std::integral_constant<int, K_RMI_FINE>{});
        break;
    case K_TREE:
    case K_TREE_FORCED: f(std::integral_constant<int, K_TREE>{}); break;
    case K_RADIX: f(std::integral_constant<int, K_RADIX>{}); break;
    default: f(std::integral_constant<int, K_MLP>{}); break;
    }
}

constexpr int M_THREADS = 1024;  // threads of a one-workgroup model builder

// Bytes of arena a model takes (16-byte multiple).
__device__ __forceinline__ uint32_t rmi_words(uint32_t L) { return 4 + 2 + 4 * L; }
__device__ __forceinline__ uint32_t tree_words(uint32_t m) { return 2 + m + (m + 1 + 3) / 4; }

// Splitters of a sorted sample (ordered keys) -> TreeModel at dst.
// Candidate i = smp[floor((i+1) S / B)], de-duplicated; repeated candidates
// get equality buckets (Sec. 2.4).  Returns the bucket count.
template <typename Get>
__device__ uint32_t build_tree_block(Get get, uint32_t S, uint32_t B, uint64_t* dst, uint32_t* scratch32,
                                     uint64_t* red64) {
    const int tid = threadIdx.x;
    const uint32_t nc = B - 1;
    uint64_t cand = 0, prev = 0;
    uint32_t isnew = 0;
    if ((uint32_t)tid < nc) {
        uint64_t r = ((uint64_t)(tid + 1) * S) / B;
        if (r >= S) r = S - 1;
        cand = get(r);
        if (tid > 0) {
            uint64_t rp = ((uint64_t)tid * S) / B;
            if (rp >= S) rp = S - 1;
            prev = get(rp);
        }
        isnew = (tid == 0) || (cand != prev);
    }
    uint64_t tot;
    uint64_t idx = block_excl_scan<M_THREADS, uint64_t>((uint64_t)isnew, red64, &tot);  // unique index if new
    const uint32_t m = (uint32_t)tot;
    uint32_t* eqf = scratch32;  // m flags
    for (uint32_t i = tid; i <= m; i += M_THREADS) eqf[i] = 0;
    __syncthreads();
    uint64_t* u = dst + 2;
    if ((uint32_t)tid < nc) {
        if (isnew) u[idx] = cand;
        else eqf[idx - 1] = 1;  // idx counts new candidates before this one
    }
    __syncthreads();
    uint32_t f = (uint32_t)tid < m ? eqf[tid] : 0;
    uint64_t neq;
    uint64_t pe = block_excl_scan<M_THREADS, uint64_t>((uint64_t)f, red64, &neq);
    uint16_t* lut = (uint16_t*)(dst + 2 + m);
    // lut[k] for k = 1..m from splitter k-1; lut[0] = 0
    if ((uint32_t)tid < m) lut[tid + 1] = (uint16_t)(((pe + f) << 1) | f);
    if (tid == 0) {
        lut[0] = 0;
        TreeModel* h = (TreeModel*)dst;
        h->m = m; h->nb = m + 1 + (uint32_t)neq; h->top = floor_pow2(m); h->pad = 0;
    }
    __syncthreads();
    return m + 1 + (uint32_t)neq;
}

}  // namespace ls
