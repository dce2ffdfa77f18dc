// lsort_basemodel.hip -- model-based counting-sort base case (LearnedSort's
// base case, Sec. 2.2: the model places each key directly and a final pass
// repairs what the model could not separate).
//
// A base-case item that comes from a bucket of the first level's RMI covers a
// known range [g0, g0 + w) of the model's fine ids (w = 1 for a bucket of the
// reused model's second level, w = 2^log2B2 for a first-level bucket).  The
// RMI's clamped leaf line t(x) (Sec. 2.1 formula at total resolution R;
// monotone across leaves by the clamp chain of Sec. 4) lies in that range for
// every key of the item, so
//     bin(x) = min(floor((t(x) - g0) * M / w), M - 1),   M = bins >= size
// is a non-decreasing function of the key: a counting sort by bin leaves the
// item sorted except inside bins.  Each key's final place is its bin's start
// plus the number of keys of its bin that precede it in (ordered key,
// original index) order -- a stable result, unique, whatever the model's
// rounding.  Bins are about one key on average; an item whose largest bin
// exceeds MB_BIN_LIMIT keys (a flat stretch of the model, or many equal
// keys) is handed to the comparison sort of k_base_mid instead.
//
// One wavefront per item (64 .. 1024 keys), every exchange through its own
// LDS region; the keys are written out in order, coalesced.
#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {

constexpr int MB_THREADS = 256;
constexpr int MB_W = MB_THREADS / WAVE;
constexpr int MB_E = (int)(MB_MAX / WAVE);      // keys per lane
constexpr uint32_t MB_BIN_LIMIT = 24;

__device__ __forceinline__ void mb_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(MB_THREADS) void k_base_model(Params P) {
    __shared__ uint64_t skey[MB_W][MB_MAX];
    __shared__ uint16_t sidx[MB_W][MB_MAX];
    __shared__ uint32_t scnt[MB_W][MB_MAX + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * MB_W, wid = (uint64_t)blockIdx.x * MB_W + wv;
    const uint64_t nit = min<unsigned long long>(P.ctl->nitems_m, P.item_m_cap);
    const uint64_t* mdl = P.fmodel;
    if (!mdl || wid >= nit) return;  // no workgroup barrier below: every exchange is wave-local
    const RmiModel* h = (const RmiModel*)mdl;
    const double* p = (const double*)(mdl + 4);
    const double ar = p[0], br = p[1];
    const uint32_t lm1 = h->L - 1;
    const int u64 = P.u64;
    uint64_t* K = skey[wv];
    uint16_t* I = sidx[wv];
    uint32_t* C = scnt[wv];
    for (uint64_t it = wid; it < nit; it += waves) {
        const uint64_t wd = P.items_m[2 * it], wg = P.items_m[2 * it + 1];
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        const double g0 = (double)(uint32_t)wg;
        const int log2w = (int)(wg >> 32);
        uint32_t M = WAVE;
        while (M < size) M <<= 1;
        const double scale = __builtin_ldexp((double)M, -log2w);  // M / w, exact
        const double mtop = (double)(M - 1);
        const uint64_t* src = P.keys[srcb] + off;
        for (uint32_t b = lane; b <= M; b += WAVE) C[b] = 0;
        mb_wave_sync();
        uint64_t k[MB_E];
        uint32_t sb[MB_E], rk[MB_E];
#pragma unroll
        for (int e = 0; e < MB_E; e++) {
            const uint32_t i = e * WAVE + lane;
            const bool valid = i < size;
            const uint64_t raw = valid ? src[i] : 0ull;
            k[e] = key_ord(raw, u64);
            double x;
            const int nf = key_x(raw, u64, x);
            uint32_t s;
            if (nf) {
                s = nf < 0 ? 0u : M - 1;
            } else {
                const uint32_t j = min(cvt_sat_u32(__builtin_fma(ar, x, br)), lm1);
                const double* q = p + 2 + 4 * j;
                double c = q[2], d = q[3];
                if (c != c) c = -INFINITY;
                if (d != d) d = INFINITY;
                if (c > d) c = d;
                const double t = fmin(fmax(__builtin_fma(q[0], x, q[1]), c), d);
                // truncation of a non-negative value is its floor; negative -> 0
                s = (uint32_t)fmin((double)cvt_sat_u32((t - g0) * scale), mtop);
            }
            sb[e] = s;
            rk[e] = valid ? atomicAdd(&C[s], 1u) : 0u;
        }
        mb_wave_sync();
        // bin starts: lane l owns bins [l * per, (l + 1) * per)
        const uint32_t per = M / WAVE;
        uint32_t loc = 0, mx = 0;
        for (uint32_t u = 0; u < per; u++) {
            const uint32_t c = C[lane * per + u];
            loc += c;
            mx = c > mx ? c : mx;
        }
        const uint32_t incl = wave_incl_sum(loc);
        uint32_t run = incl - loc;
        for (uint32_t u = 0; u < per; u++) {
            const uint32_t c = C[lane * per + u];
            C[lane * per + u] = run;
            run += c;
        }
        if (lane == WAVE - 1) C[M] = incl;
        mx = wave_max(mx);
        mb_wave_sync();
        if (mx > MB_BIN_LIMIT) {  // the model cannot separate these keys: comparison sort
            if (lane == 0) {
                const uint64_t b = atomicAdd(&P.ctl->nbig, 1ull);
                atomicAdd(&P.ctl->nmoved, 1ull);
                if (b < P.big_cap) P.bigs[b] = wd;
                else atomicOr(&P.ctl->overflow, OVF_ITEM);
            }
            continue;
        }
        // counting-sort placement
#pragma unroll
        for (int e = 0; e < MB_E; e++) {
            const uint32_t i = e * WAVE + lane;
            if (i < size) {
                const uint32_t slot = C[sb[e]] + rk[e];
                K[slot] = k[e];
                I[slot] = (uint16_t)i;
            }
        }
        mb_wave_sync();
        // repair inside each bin: final place = bin start + keys of the bin
        // before this one in (ordered key, original index) order
        uint32_t pos[MB_E];
#pragma unroll
        for (int e = 0; e < MB_E; e++) {
            const uint32_t i = e * WAVE + lane;
            pos[e] = 0;
            if (i < size) {
                const uint32_t s0 = C[sb[e]], s1 = C[sb[e] + 1];
                uint32_t r = 0;
                for (uint32_t q = s0; q < s1; q++) {
                    const uint64_t kq = K[q];
                    r += (kq < k[e] || (kq == k[e] && (uint32_t)I[q] < i)) ? 1u : 0u;
                }
                pos[e] = s0 + r;
            }
        }
        mb_wave_sync();
#pragma unroll
        for (int e = 0; e < MB_E; e++) {
            const uint32_t i = e * WAVE + lane;
            if (i < size) {
                K[pos[e]] = k[e];
                I[pos[e]] = (uint16_t)i;
            }
        }
        mb_wave_sync();
        uint64_t* dst = P.keys[0] + off;
        for (uint32_t i = lane; i < size; i += WAVE) dst[i] = key_unord(K[i], u64);
        if (P.has_pay) {
            // the payload moves through LDS: every read of the item's payload
            // is complete before the first write (source and destination may
            // be the same buffer)
            const uint32_t* pin = P.pay[srcb] + off;
            uint32_t* pout = P.pay[0] + off;
            for (uint32_t i = lane; i < size; i += WAVE) C[i] = pin[I[i]];
            mb_wave_sync();
            for (uint32_t i = lane; i < size; i += WAVE) pout[i] = C[i];
        }
        mb_wave_sync();  // the next item rewrites the region
    }
}

hipError_t launch_base_model(const Params& P, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_base_model, dim3(grid), dim3(MB_THREADS), 0, st, P);
    return hipGetLastError();
}

}  // namespace ls
