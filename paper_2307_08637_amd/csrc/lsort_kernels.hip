// lsort_kernels.hip -- HIP kernels of the learned sample sort for gfx950.
//
// One partition level over a list of sub-arrays ("segments") runs as
//   k_model   -> k_hist -> k_scan -> k_scatter
// and after the last level the base-case kernels (lsort_base.hip) sort every
// small bucket.  Segments
// of one level share every launch (the batched form is the same code with
// more segments).  Buffers ping-pong between the caller's keys (index 0) and
// a temporary (index 1): level l reads buffer l&1 and writes buffer (l+1)&1;
// the base case always writes the caller's buffer.
#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {


// ===========================================================================
// Call set-up
// ===========================================================================

// Zero the per-call control block and advance the look-back epoch.
__global__ void k_reset(Params P, uint64_t* persist) {
    uint32_t* c = (uint32_t*)P.ctl;
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) c[i] = 0;
    if (threadIdx.x == 0) {
        uint64_t e = persist[0] + 1;
        uint32_t clear = 0;
        if ((e + 1) * MAXL >= (1ull << ST_TAG_BITS)) { e = 1; clear = 1; }
        persist[0] = e;
        persist[1] = clear;
    }
}

// Seed level 0 from the caller's segments; clear the status pool on epoch wrap.
// List slots are reserved with one atomicAdd per workgroup; every slot below
// a list's capacity is written by its owner, so consumers never meet a stale
// entry (slots at or above capacity are dropped and flagged as overflow).
__global__ __launch_bounds__(256) void k_seed(Params P, const uint64_t* offsets, uint64_t m, uint64_t n_single,
                                              uint32_t prebuilt, const uint64_t* persist) {
    __shared__ uint64_t red64[256 / 64];
    __shared__ uint64_t base[8];
    if (persist[1]) {
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.status_cap;
             i += (uint64_t)gridDim.x * blockDim.x)
            P.status[i] = 0;
    }
    const uint64_t rounds = (m + 255) / 256;
    for (uint64_t rb = blockIdx.x; rb < rounds; rb += gridDim.x) {
        const uint64_t s = rb * 256 + threadIdx.x;
        uint64_t lo = 0, n = 0;
        if (s < m) {
            lo = offsets ? offsets[s] : 0;
            n = offsets ? offsets[s + 1] - lo : n_single;
        }
        // prebuilt: the caller supplied the first level's model; always partition
        const bool item = s < m && !prebuilt && n >= 2 && n <= P.cutoff;
        // keys only: up to GROUP_LARGE_MAX keys still go to k_base_small
        const bool small = item && (n <= SMALL_MAX || (n <= GROUP_WAVE_MAX && !P.has_pay));
        const int cls = !small ? 3 : n <= GROUP_SMALL_MAX ? 0 : n <= GROUP_MAX ? 1 : n <= SMALL_MAX ? 2
                      : n <= GROUP_LARGE_MAX ? 4 : 5;
        const bool seg = s < m && (prebuilt ? n >= 1 : n > P.cutoff);
        // an array small enough for one workgroup is sorted whole by k_resident
        const bool resident = seg && !prebuilt && n <= RES_MAX;
        // a single array of at most SMALL_UNIT_N keys at the default unit:
        // one-tile units, so that its first level spreads over the CUs
        const uint32_t us = m == 1 && !prebuilt && n <= SMALL_UNIT_N && P.unit0_shift == 0 ? USHIFT_TILE : P.unit0_shift;
        const uint64_t unit0 = us == USHIFT_TILE ? (uint64_t)TILE : (uint64_t)UNIT << us;
        const uint32_t nt = seg && !resident ? (uint32_t)((n + unit0 - 1) / unit0) : 0;
        {
            const uint32_t nr = (uint32_t)__popcll(__ballot(resident));
            if ((threadIdx.x & 63) == 0 && nr) atomicAdd(&P.ctl->nres[0], nr);
        }
        uint64_t itot, wtot, gtot, ktot, ctot, btot, stot, ttot;
        const uint64_t iex = block_excl_scan<256, uint64_t>(item && cls == 0 ? 1 : 0, red64, &itot);
        const uint64_t gex = block_excl_scan<256, uint64_t>(item && cls == 1 ? 1 : 0, red64, &gtot);
        const uint64_t wex = block_excl_scan<256, uint64_t>(item && cls == 2 ? 1 : 0, red64, &wtot);
        const uint64_t kex = block_excl_scan<256, uint64_t>(item && cls == 4 ? 1 : 0, red64, &ktot);
        const uint64_t cex = block_excl_scan<256, uint64_t>(item && cls == 5 ? 1 : 0, red64, &ctot);
        const uint64_t bex = block_excl_scan<256, uint64_t>(item && !small ? 1 : 0, red64, &btot);
        const uint64_t sex = block_excl_scan<256, uint64_t>(seg ? 1 : 0, red64, &stot);
        const uint64_t tex = block_excl_scan<256, uint64_t>(nt, red64, &ttot);
        const uint64_t sk = block_sum<256, uint64_t>(small ? n : 0, red64);
        const uint64_t gk = block_sum<256, uint64_t>(item && !small ? n : 0, red64);
        if (threadIdx.x == 0) {
            base[0] = itot ? atomicAdd(&P.ctl->nitems, (unsigned long long)itot) : 0;
            base[1] = stot ? atomicAdd(&P.ctl->nseg[0], (uint32_t)stot) : 0;
            base[2] = ttot ? atomicAdd(&P.ctl->ntile[0], (uint32_t)ttot) : 0;
            base[3] = btot ? atomicAdd(&P.ctl->nbig, (unsigned long long)btot) : 0;
            base[4] = wtot ? atomicAdd(&P.ctl->nitems_w, (unsigned long long)wtot) : 0;
            base[5] = gtot ? atomicAdd(&P.ctl->nitems_b, (unsigned long long)gtot) : 0;
            base[6] = ktot ? atomicAdd(&P.ctl->nitems_k, (unsigned long long)ktot) : 0;
            base[7] = ctot ? atomicAdd(&P.ctl->nitems_c, (unsigned long long)ctot) : 0;
            if (sk) atomicAdd(&P.ctl->small_keys, (unsigned long long)sk);
            if (gk) atomicAdd(&P.ctl->big_keys, (unsigned long long)gk);
        }
        __syncthreads();
        if (item) {
            const uint64_t it = cls == 0 ? base[0] + iex : cls == 1 ? base[5] + gex : cls == 2 ? base[4] + wex
                              : cls == 4 ? base[6] + kex : cls == 5 ? base[7] + cex : base[3] + bex;
            const uint64_t cap = cls == 1 || cls == 4 ? P.item_b_cap : cls == 3 ? P.big_cap
                               : cls == 5 ? P.item_c_cap : P.item_cap;
            uint64_t* list = cls == 1 || cls == 4 ? P.items_b : cls == 3 ? P.bigs : cls == 5 ? P.items_c : P.items;
            // lists 2 and 4 fill their arrays from the back
            if (it < cap) list[cls == 2 || cls == 4 ? cap - 1 - it : it] = item_pack(lo, 0, 0, (uint32_t)n);
            else atomicOr(&P.ctl->overflow, OVF_ITEM);
        }
        if (seg) {
            const uint64_t si = base[1] + sex, t0 = base[2] + tex;
            if (si >= P.seg_cap) {
                atomicOr(&P.ctl->overflow, OVF_SEG);
            } else {
                Seg sg{};
                sg.off = lo; sg.n = n; sg.kind = K_FRESH; sg.tile0 = (uint32_t)t0; sg.ntiles = nt;
                sg.flags = (prebuilt ? SEG_PREBUILT : (resident ? SEG_RESIDENT : 0)) | (us << SEG_USHIFT_POS);
                if (t0 + nt > P.tile_cap) { atomicOr(&P.ctl->overflow, OVF_TILE); sg.flags |= SEG_FAILED; }
                if (prebuilt) {  // the first level's model and kind were written into segs[1][0]
                    Seg pb = P.segs[1][0];
                    sg.kind = pb.kind; sg.nb = pb.nb; sg.model = pb.model; sg.flags |= pb.flags & 0xffff0000u;
                }
                P.segs[0][si] = sg;
            }
        }
        __syncthreads();
    }
}

// ===========================================================================
// k_model: build each segment's partition model (one workgroup per segment)
// ===========================================================================


__device__ uint64_t arena_alloc(Params& P, uint32_t words, uint64_t* sh) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t bytes = ((uint64_t)words * 8 + 15) & ~15ull;
        uint64_t o = atomicAdd(&P.ctl->arena_used[P.level & 1], (unsigned long long)bytes);
        if (o + bytes > P.arena_cap) {
            atomicOr(&P.ctl->overflow, OVF_ARENA);
            sh[0] = 0;
        } else {
            sh[0] = (uint64_t)(P.arena[P.level & 1] + o);
        }
    }
    __syncthreads();
    uint64_t r = sh[0];
    __syncthreads();
    return r;
}

// Fit the monotone RMI on the sorted sample smp[0..S) (ordered keys, all
// finite) and write it at model address `dst` (RmiModel + 2 + 4L doubles).
// Least squares on (x_i, i/S): root over all points, leaf j over the points
// the pre-scaled root sends to j; slopes clamped >= 0; clamp intervals
// c_j = clip01(max(pmin_j, d_{j-1})), d_j = clip01(max(pmax_j, d_{j-1}))
// computed with a prefix maximum (Sec. 2.1, Sec. 2.2 training, Sec. 4).
__device__ void fit_rmi_block(const uint64_t* smp, uint32_t S, int u64, uint32_t L, uint32_t B1, uint32_t log2B2,
                              double* dst, uint32_t* lstart, double* red) {
    const int tid = threadIdx.x;
    const double Sd = (double)S;
    // root: two passes
    double sx = 0;
    for (uint32_t i = tid; i < S; i += M_THREADS) {
        double x; key_x(key_unord(smp[i], u64), u64, x); sx += x;
    }
    double mx = block_sum<M_THREADS>(sx, red) / Sd;
    double my = (Sd - 1.0) / (2.0 * Sd);
    double sxx = 0, sxy = 0;
    for (uint32_t i = tid; i < S; i += M_THREADS) {
        double x; key_x(key_unord(smp[i], u64), u64, x);
        double dx = x - mx, dy = (double)i / Sd - my;
        sxx += dx * dx; sxy += dx * dy;
    }
    sxx = block_sum<M_THREADS>(sxx, red);
    sxy = block_sum<M_THREADS>(sxy, red);
    double ar = sxx > 0 ? sxy / sxx : 0.0;
    if (ar < 0) ar = 0;
    double br = my - ar * mx;
    const double alpha_r = (double)L * ar, beta_r = (double)L * br;
    const double Lm1 = (double)L - 1.0;
    // leaf ranges: leaf index is non-decreasing along the sorted sample
    for (uint32_t i = tid; i < S; i += M_THREADS) {
        double x; key_x(key_unord(smp[i], u64), u64, x);
        uint32_t j = (uint32_t)fmin(fmax(floor(__builtin_fma(alpha_r, x, beta_r)), 0.0), Lm1);
        int jp = -1;
        if (i > 0) {
            double xp; key_x(key_unord(smp[i - 1], u64), u64, xp);
            jp = (int)fmin(fmax(floor(__builtin_fma(alpha_r, xp, beta_r)), 0.0), Lm1);
        }
        for (int q = jp + 1; q <= (int)j; q++) lstart[q] = i;
        if (i == S - 1)
            for (uint32_t q = j + 1; q <= L; q++) lstart[q] = S;
    }
    __syncthreads();
    // per-leaf least squares: two threads per leaf (even and odd points, the
    // partial sums combined through a lane swap), so that a leaf the root
    // clamps a tail into is walked in half the time; a leaf of more than
    // FB_HEAVY points (a distribution whose mass the linear root sends to a
    // few leaves) is summed by a whole wavefront instead, below.  The raw
    // line and its ends go to the leaf's model slots and are read back below.
    constexpr uint32_t FB_HEAVY = 128;
    const double invS = 1.0 / Sd;  // i / S as i * (1 / S): no division per point
    for (uint32_t j0 = 0; j0 < L; j0 += M_THREADS / 2) {
        const uint32_t j = j0 + ((uint32_t)tid >> 1), half = (uint32_t)tid & 1u;
        const uint32_t jl = j < L ? j : L - 1;
        const uint32_t lo = lstart[jl];
        const uint32_t hi = j < L && lstart[jl + 1] - lo <= FB_HEAVY ? lstart[jl + 1] : lo;
        const double cnt = (double)(hi - lo);
        double s = 0;
        for (uint32_t i = lo + half; i < hi; i += 2) { double x; key_x(key_unord(smp[i], u64), u64, x); s += x; }
        s += __shfl_xor(s, 1);
        const double lmx = hi > lo ? s / cnt : 0.0;
        const double lmy = ((double)lo + (double)hi - 1.0) / (2.0 * Sd);
        double lxx = 0, lxy = 0;
        for (uint32_t i = lo + half; i < hi; i += 2) {
            double x; key_x(key_unord(smp[i], u64), u64, x);
            const double dx = x - lmx, dy = (double)i * invS - lmy;
            lxx += dx * dx; lxy += dx * dy;
        }
        lxx += __shfl_xor(lxx, 1);
        lxy += __shfl_xor(lxy, 1);
        if (j < L && hi > lo && half == 0) {
            double a = lxx > 0 ? lxy / lxx : 0.0;
            if (a < 0) a = 0;
            const double b = lmy - a * lmx;
            double x0, x1;
            key_x(key_unord(smp[lo], u64), u64, x0);
            key_x(key_unord(smp[hi - 1], u64), u64, x1);
            double* q = dst + 4 + 2 + 4 * j;
            q[0] = a; q[1] = b; q[2] = a * x0 + b; q[3] = a * x1 + b;
        }
    }
    {  // leaves of more than FB_HEAVY points: one wavefront each, dealt to the
       // wavefronts in leaf order; lanes stride the points, sums in a fixed order
        constexpr uint32_t NW = M_THREADS / 64;
        const uint32_t wv = (uint32_t)tid >> 6, lane = (uint32_t)tid & 63u;
        uint32_t seen = 0;
        for (uint32_t c0 = 0; c0 < L; c0 += 64) {
            const uint32_t jj = c0 + lane;
            uint64_t m = __ballot(jj < L && lstart[jj + 1] - lstart[jj] > FB_HEAVY);
            while (m) {
                const uint32_t j = c0 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
                m &= m - 1;
                if (seen++ % NW != wv) continue;
                const uint32_t lo = lstart[j], hi = lstart[j + 1];
                const double cnt = (double)(hi - lo);
                double s = 0;
                for (uint32_t i = lo + lane; i < hi; i += 64) { double x; key_x(key_unord(smp[i], u64), u64, x); s += x; }
                s = wave_sum(s);
                const double lmx = s / cnt;
                const double lmy = ((double)lo + (double)hi - 1.0) / (2.0 * Sd);
                double lxx = 0, lxy = 0;
                for (uint32_t i = lo + lane; i < hi; i += 64) {
                    double x; key_x(key_unord(smp[i], u64), u64, x);
                    const double dx = x - lmx, dy = (double)i * invS - lmy;
                    lxx += dx * dx; lxy += dx * dy;
                }
                lxx = wave_sum(lxx);
                lxy = wave_sum(lxy);
                if (lane == 0) {
                    double a = lxx > 0 ? lxy / lxx : 0.0;
                    if (a < 0) a = 0;
                    const double b = lmy - a * lmx;
                    double x0, x1;
                    key_x(key_unord(smp[lo], u64), u64, x0);
                    key_x(key_unord(smp[hi - 1], u64), u64, x1);
                    double* q = dst + 4 + 2 + 4 * j;
                    q[0] = a; q[1] = b; q[2] = a * x0 + b; q[3] = a * x1 + b;
                }
            }
        }
    }
    __syncthreads();
    double a = 0, b = 0, pmin = 0, pmax = -INFINITY;
    uint32_t lo = 0, hi = 0;
    if ((uint32_t)tid < L) {
        lo = lstart[tid]; hi = lstart[tid + 1];
        if (hi > lo) {
            const double* q = dst + 4 + 2 + 4 * tid;
            a = q[0]; b = q[1]; pmin = q[2]; pmax = q[3];
        }
    }
    // d_j = clip01(max(0, prefix max of pmax over non-empty leaves))
    double incl = block_incl_max<M_THREADS>(pmax, red);
    double excl = __shfl_up(incl, 1);
    __shared__ double wave_last[M_THREADS / 64];
    if ((tid & 63) == 63) wave_last[tid >> 6] = incl;
    __syncthreads();
    if ((tid & 63) == 0) excl = tid == 0 ? -INFINITY : wave_last[(tid >> 6) - 1];
    __syncthreads();
    if ((uint32_t)tid < L) {
        double dprev = fmin(fmax(excl, 0.0), 1.0);
        double c, d;
        if (hi > lo) {
            c = fmin(fmax(fmax(pmin, dprev), 0.0), 1.0);
            d = fmin(fmax(fmax(pmax, c), 0.0), 1.0);
        } else {
            a = 0; b = dprev; c = dprev; d = dprev;
        }
        double R = (double)((uint64_t)B1 << log2B2);
        double* q = dst + 4 + 2 + 4 * tid;
        q[0] = R * a; q[1] = R * b; q[2] = R * c; q[3] = R * d;
    }
    if (tid == 0) {
        RmiModel* h = (RmiModel*)dst;
        h->L = L; h->B1 = B1; h->log2B2 = log2B2; h->pad = 0;
        h->R = (double)((uint64_t)B1 << log2B2);
        h->pad2 = 0;
        dst[4] = alpha_r; dst[5] = beta_r;
    }
}

// Gather sample k -> element k of the sort (padding with the largest key),
// sort M_THREADS * E of them in registers, leave the result in smp[].
template <int E>
__device__ void sample_sort(uint64_t* smp, const uint64_t* src, uint64_t off, uint64_t n, uint32_t S, uint64_t seed,
                            int u64) {
    uint64_t k[E];
    uint32_t ix[E];
    const int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = t * E + e;
        k[e] = i < S ? key_ord(src[off + sample_index(seed, i, n)], u64) : ~0ull;
        ix[e] = 0;
    }
    block_bitonic<M_THREADS, E, false>(k, ix, smp, nullptr);
#pragma unroll
    for (int e = 0; e < E; e++) smp[t * E + e] = k[e];
    __syncthreads();
}

// The one-workgroup fit on its own (the fit every small segment's model
// gets): a sorted sample of S <= S_LDS raw keys into LDS as ordered keys,
// then fit_rmi_block at total resolution B1 (log2B2 = 0) into dst.
__global__ __launch_bounds__(M_THREADS) void k_fit_block(const uint64_t* s, uint32_t S, int u64, uint32_t L,
                                                         uint32_t B1, double* dst) {
    __shared__ uint64_t smp[S_LDS];
    __shared__ uint32_t lstart[L_MAX + 1];
    __shared__ double red[M_THREADS / 64];
    for (uint32_t i = threadIdx.x; i < S; i += M_THREADS) smp[i] = key_ord(s[i], u64);
    __syncthreads();
    fit_rmi_block(smp, S, u64, L, B1, 0, dst, lstart, red);
}

// The first-level sample's keys in parent bucket b (the run
// [bstart[b], bstart[b+1]) that k_fit_bstart found), as ordered keys in smp[]
// (evenly thinned to S_LDS when more); returns their number.
__device__ uint32_t sample_slice(uint64_t* smp, const uint64_t* fs, uint64_t S, const uint64_t* bstart, uint32_t b,
                                 int u64) {
    const uint64_t lo = min(bstart[b], S), hi = min(bstart[b + 1], S);
    const uint64_t cnt = hi > lo ? hi - lo : 0;
    const uint32_t m = (uint32_t)min<uint64_t>(cnt, S_LDS);
    for (uint32_t k = threadIdx.x; k < m; k += M_THREADS)
        smp[k] = key_ord(fs[lo + (cnt > S_LDS ? (uint64_t)k * cnt / S_LDS : k)], u64);
    __syncthreads();
    return m;
}

// A segment whose model exists already (a fine window of its parent's, or
// the caller's): no sample, only the bookkeeping below.
__device__ __forceinline__ bool model_given(const Seg& sg) {
    return (sg.flags & SEG_PREBUILT) || sg.kind == K_RMI_FINE || sg.kind == K_MLP_FINE;
}

// Bookkeeping of one segment, by one wavefront: the one-tile re-cut (a level
// of few work units), counts and look-back reservations, the descriptor,
// cleared counts and the unit list.  The same steps as the workgroup form at
// the end of k_model, for a segment whose model is given.
__device__ __forceinline__ void model_book_wave(Params& P, int lvl, uint32_t s, Seg sg, int lane) {
    const uint32_t nb = sg.nb, words = sg.flags >> 16;
    if (P.split && sg.ntiles && !(sg.flags & (SEG_FAILED | SEG_RESIDENT))) {
        const uint32_t nt2 = (uint32_t)((sg.n + TILE - 1) / TILE);
        uint32_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(&P.ctl->nsplit[lvl], nt2);
        sg.tile0 = __shfl(t0, 0);
        sg.ntiles = nt2;
        sg.flags = (sg.flags & ~(7u << SEG_USHIFT_POS)) | (USHIFT_TILE << SEG_USHIFT_POS);
        if ((uint64_t)sg.tile0 + nt2 > P.tile_cap) {
            if (lane == 0) atomicOr(&P.ctl->overflow, OVF_TILE);
            sg.flags |= SEG_FAILED;
        }
    }
    uint64_t cb = 0, sb = 0;
    uint32_t fl = (sg.flags & 0xffffu) | (words << 16);
    if (lane == 0) {
        if (!(fl & SEG_FAILED)) {
            cb = atomicAdd(&P.ctl->counts_used, 2ull * nb);
            sb = atomicAdd(&P.ctl->status_used, (unsigned long long)sg.ntiles * nb);
            if (cb + 2ull * nb > P.counts_cap) { atomicOr(&P.ctl->overflow, OVF_COUNTS); fl |= SEG_FAILED; cb = 0; }
            if (sb + (uint64_t)sg.ntiles * nb > P.status_cap) {
                atomicOr(&P.ctl->overflow, OVF_STATUS); fl |= SEG_FAILED; sb = 0;
            }
        }
        if (!sg.model) fl |= SEG_FAILED;
        Seg& o = P.segs[lvl & 1][s];
        o.cbase = cb; o.sbase = sb; o.flags = fl;
        o.tile0 = sg.tile0; o.ntiles = sg.ntiles;
        if (P.flags & FLAG_STATS) {
            LevelStats& st = P.ctl->lv[lvl];
            const uint32_t kind = sg.kind;
            if (kind == K_RMI || kind == K_RMI_FINE || kind == K_MLP || kind == K_MLP_FINE) atomicAdd(&st.learned, 1ull);
            else if (kind == K_RADIX) atomicAdd(&st.radix, 1ull);
            else atomicAdd(&st.tree, 1ull);
        }
    }
    cb = __shfl(cb, 0);
    fl = __shfl(fl, 0);
    if (!(fl & (SEG_FAILED | SEG_RESIDENT)))  // k_resident writes its counts whole
        for (uint32_t b = lane; b < nb; b += WAVE) P.counts[cb + b] = 0;
    for (uint32_t i = lane; i < sg.ntiles; i += WAVE)
        if ((uint64_t)sg.tile0 + i < P.tile_cap) P.tiles[lvl & 1][sg.tile0 + i] = Tile{s, i};
}

__global__ __launch_bounds__(M_THREADS) void k_model(Params P) {
    __shared__ uint64_t smp[S_LDS];
    __shared__ uint32_t lstart[L_MAX + 1];
    __shared__ double red[M_THREADS / 64];
    __shared__ uint64_t red64[M_THREADS / 64];
    __shared__ uint64_t shv[4];
    const int tid = threadIdx.x;
    const int lvl = P.level;
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    const uint64_t* src = P.keys[lvl & 1];
    const int u64 = P.u64;
    // segments whose model is given: one wavefront each (a level of ~1000
    // fine windows is bookkeeping only, and a workgroup per segment would
    // hold a CU's LDS for each)
    {
        constexpr int MW = M_THREADS / WAVE;
        const int lane = tid & (WAVE - 1);
        for (uint32_t s = blockIdx.x * MW + (tid >> 6); s < nseg; s += gridDim.x * MW) {
            const Seg sg = P.segs[lvl & 1][s];
            if (model_given(sg)) model_book_wave(P, lvl, s, sg, lane);
        }
    }
    for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        Seg sg = P.segs[lvl & 1][s];
        if (model_given(sg)) continue;  // done above (uniform over the workgroup)
        uint32_t kind = sg.kind, nb = sg.nb, words = sg.flags >> 16;
        uint64_t model = sg.model;
        if (kind == K_RADIX) {
            uint64_t lo = ~0ull, hi = 0;
            for (uint64_t i = tid; i < sg.n; i += M_THREADS) {
                uint64_t o = key_ord(src[sg.off + i], u64);
                lo = o < lo ? o : lo;
                hi = o > hi ? o : hi;
            }
            lo = block_min<M_THREADS, uint64_t>(lo, red64);
            hi = block_max<M_THREADS, uint64_t>(hi, red64);
            uint32_t shift = 0;
            if (hi > lo) {
                uint64_t span = hi - lo;
                uint32_t bits = 64 - __clzll(span);
                uint32_t lb = 8;
                while (lb > 1 && (sg.n >> (lb + 2)) == 0) lb--;  // keep nb <= n/4
                shift = bits > lb ? bits - lb : 0;
                nb = (uint32_t)(span >> shift) + 1;
            } else {
                nb = 1;
            }
            words = 2;
            model = arena_alloc(P, words, shv);
            if (tid == 0 && model) {
                RadixModel* h = (RadixModel*)model;
                h->lo = lo; h->shift = hi > lo ? shift : 64; h->nb = nb;
            }
        } else {
            // sample (Sec. 2.2: ~1% random sample; Alg. 5 Sample) and sort it
            const uint64_t n = sg.n;
            uint32_t Bt = min(P.tree_buckets, max(2u, floor_pow2((uint32_t)min<uint64_t>(n / 16, 1u << 30))));
            // children that would be base-case items of more than
            // GROUP_LARGE_MAX keys: twice the fan-out (up to 512), so that they
            // fall into the cheaper register classes
            if (Bt == P.tree_buckets && Bt < 512 && n / Bt > (uint64_t)GROUP_LARGE_MAX && n / Bt <= (uint64_t)BIG_MAX &&
                2ull * Bt <= n / 16)
                Bt *= 2;
            uint64_t want = (uint64_t)ceil(P.sample_frac * (double)n);
            uint64_t floor_s = min<uint64_t>(n, 8ull * Bt);  // 8 sample keys per bucket at least
            uint32_t S = (uint32_t)min<uint64_t>(S_LDS, max<uint64_t>(want, max<uint64_t>(floor_s, 2)));
            // a fallback child of a large array's first level: the first-level
            // sample's keys in the parent bucket are already a sorted random
            // sample of this segment (about 1% of it)
            const uint32_t Sf = (sg.flags & SEG_FROM_SAMPLE) && P.fsample && P.fbstart
                                    ? sample_slice(smp, P.fsample, P.fS, P.fbstart, sg.win, u64)
                                    : 0u;
            if (Sf >= 2) {
                S = Sf;
            } else {
                const uint32_t P2 = 1u << ceil_log2(S);
                const uint64_t sseed = splitmix64_at(P.seed, (sg.off << 6) | (uint64_t)lvl);
                // gather and sort in registers; the sorted sample lands in smp[]
                if (P2 <= 1024) sample_sort<1>(smp, src, sg.off, n, S, sseed, u64);
                else if (P2 <= 2048) sample_sort<2>(smp, src, sg.off, n, S, sseed, u64);
                else if (P2 <= 4096) sample_sort<4>(smp, src, sg.off, n, S, sseed, u64);
                else if (P2 <= 8192) sample_sort<8>(smp, src, sg.off, n, S, sseed, u64);
                else sample_sort<16>(smp, src, sg.off, n, S, sseed, u64);
            }
            // duplicates and finiteness (Alg. 5; Sec. 4: more than 10% duplicates -> tree)
            uint64_t dup = 0;
            for (uint32_t j = 1 + tid; j < S; j += M_THREADS) dup += smp[j] == smp[j - 1];
            dup = block_sum<M_THREADS, uint64_t>(dup, red64);
            double x0, x1;
            int nf0 = key_x(key_unord(smp[0], u64), u64, x0);
            int nf1 = key_x(key_unord(smp[S - 1], u64), u64, x1);
            bool learned = kind == K_FRESH && P.model != 3 /* SPLITTER */ && (double)n >= 1e5 &&
                           (double)dup <= 0.10 * (double)(S - 1) && !nf0 && !nf1 && x1 > x0;
            if (learned) {
                uint32_t L = min(P.leaves, max(2u, S / 8));
                uint64_t half = max(1u, P.cutoff / 2);
                uint32_t B1 = (uint32_t)min<uint64_t>(P.buckets, max<uint64_t>(2, (n + half - 1) / half));
                B1 = (uint32_t)min<uint64_t>(B1, max<uint64_t>(2, n / 4));
                uint32_t log2B2 = 0;
                uint64_t per = n / B1;
                if (per > P.cutoff) log2B2 = min(10u, ceil_log2((uint32_t)min<uint64_t>((per + half - 1) / half, 1u << 20)));
                words = rmi_words(L);
                model = arena_alloc(P, words, shv);
                if (model) fit_rmi_block(smp, S, u64, L, B1, log2B2, (double*)model, lstart, red);
                kind = K_RMI;
                nb = B1;
            }
            if (!learned) {
                uint32_t mmax = Bt - 1;
                words = tree_words(mmax);
                model = arena_alloc(P, words, shv);
                if (model) {
                    nb = build_tree_block([&](uint64_t r) { return smp[r]; }, S, Bt, (uint64_t*)model, lstart, red64);
                } else {
                    nb = 1;
                }
                kind = kind == K_TREE_FORCED ? K_TREE_FORCED : K_TREE;
                // actual words for loading
                if (model) words = tree_words(((TreeModel*)model)->m);
            }
        }
        __syncthreads();
        // a level with fewer work units than CUs: this segment's units are
        // cut again into one-tile units (from a fresh count), so that the
        // level's histogram and scatter spread over the CUs
        if (P.split && sg.ntiles && !(sg.flags & (SEG_FAILED | SEG_RESIDENT))) {
            const uint32_t nt2 = (uint32_t)((sg.n + TILE - 1) / TILE);
            if (tid == 0) shv[3] = atomicAdd(&P.ctl->nsplit[lvl], nt2);
            __syncthreads();
            sg.tile0 = (uint32_t)shv[3];
            sg.ntiles = nt2;
            sg.flags = (sg.flags & ~(7u << SEG_USHIFT_POS)) | (USHIFT_TILE << SEG_USHIFT_POS);
            if ((uint64_t)sg.tile0 + nt2 > P.tile_cap) {
                if (tid == 0) atomicOr(&P.ctl->overflow, OVF_TILE);
                sg.flags |= SEG_FAILED;
            }
            __syncthreads();  // shv is rewritten below
        }
        // bucket counts and look-back words
        if (tid == 0) {
            uint32_t fl = (sg.flags & 0xffffu) | (words << 16);
            uint64_t cb = 0, sb = 0;
            if (!(fl & SEG_FAILED)) {
                cb = atomicAdd(&P.ctl->counts_used, 2ull * nb);
                sb = atomicAdd(&P.ctl->status_used, (unsigned long long)sg.ntiles * nb);
                if (cb + 2ull * nb > P.counts_cap) { atomicOr(&P.ctl->overflow, OVF_COUNTS); fl |= SEG_FAILED; cb = 0; }
                if (sb + (uint64_t)sg.ntiles * nb > P.status_cap) {
                    atomicOr(&P.ctl->overflow, OVF_STATUS); fl |= SEG_FAILED; sb = 0;
                }
            }
            if (!model) fl |= SEG_FAILED;
            shv[0] = cb; shv[1] = sb; shv[2] = fl;
            Seg& o = P.segs[lvl & 1][s];
            o.kind = kind; o.nb = nb; o.model = model; o.cbase = cb; o.sbase = sb; o.flags = fl;
            o.tile0 = sg.tile0; o.ntiles = sg.ntiles;
            LevelStats& st = P.ctl->lv[lvl];
            if (P.flags & FLAG_STATS) {
                if (kind == K_RMI || kind == K_RMI_FINE || kind == K_MLP || kind == K_MLP_FINE) atomicAdd(&st.learned, 1ull);
                else if (kind == K_RADIX) atomicAdd(&st.radix, 1ull);
                else atomicAdd(&st.tree, 1ull);
            }
        }
        __syncthreads();
        if (!(shv[2] & (SEG_FAILED | SEG_RESIDENT)))  // k_resident writes its counts whole
            for (uint32_t b = tid; b < nb; b += M_THREADS) P.counts[shv[0] + b] = 0;
        // this segment's tile descriptors (every reserved slot below capacity)
        for (uint32_t i = tid; i < sg.ntiles; i += M_THREADS)
            if ((uint64_t)sg.tile0 + i < P.tile_cap) P.tiles[lvl & 1][sg.tile0 + i] = Tile{s, i};
        __syncthreads();
    }
}

// ===========================================================================
// k_hist: model evaluation fused with an LDS-private bucket histogram, one
// work unit (32768 keys) at a time.  Each unit's per-bucket counts are
// published as the aggregate words of the decoupled look-back and added to
// the segment's bucket totals.
// ===========================================================================

__device__ __forceinline__ uint64_t st_load(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store(unsigned long long* p, uint64_t v) {
    __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int HK = 8;  // keys per thread in flight in k_hist

__global__ __launch_bounds__(P_THREADS) void k_hist(Params P) {
    __shared__ __align__(16) uint64_t mdl[LDS_MODEL_WORDS];
    __shared__ uint32_t h[B_MAX];
    const int tid = threadIdx.x;
    const int lvl = P.level;
    const uint32_t nunit = level_units(P, lvl);
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    const uint64_t tag = ((uint64_t)(P.persist[0] * MAXL + lvl)) << ST_TAG_SHIFT;
    const uint64_t* src = P.keys[lvl & 1];
    const int u64 = P.u64;
    __shared__ uint32_t sh_t;
    uint64_t cur_model = 0;
    // units taken through a ticket: a workgroup that drew slow units (tree
    // models) takes fewer, so the launch ends evenly
    for (;;) {
        __syncthreads();  // the previous unit is done with mdl, h and sh_t
        if (tid == 0) sh_t = atomicAdd(&P.ctl->hticket[lvl], 1u);
        __syncthreads();
        const uint32_t t = sh_t;
        if (t >= nunit) break;
        const Tile td = P.tiles[lvl & 1][t];
        if (td.seg >= nseg) continue;
        const Seg sg = P.segs[lvl & 1][td.seg];
        if (sg.flags & SEG_FAILED) continue;
        if (sg.model != cur_model) {
            load_model_lds(mdl, (const uint64_t*)sg.model, sg.kind, sg.flags >> 16, tid, P_THREADS);
            cur_model = sg.model;
        }
        for (uint32_t b = tid; b < B_MAX; b += P_THREADS) h[b] = 0;
        __syncthreads();
        const View v = make_view(mdl, sg.kind, sg.nb, sg.win);
        const uint32_t U = seg_unit(sg.flags);
        const uint64_t base = sg.off + (uint64_t)td.idx * U;
        const uint32_t un = (uint32_t)min<uint64_t>(U, sg.n - (uint64_t)td.idx * U);
        const int bits = ceil_log2(sg.nb);
        with_kind(v.kind, u64, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            // trees and radix put runs of equal keys into one bucket: add per
            // distinct bucket of the wave
            constexpr bool aggregate = KIND == K_TREE || KIND == K_RADIX;
            auto add = [&](uint32_t b, bool in) {
                if (aggregate) {
                    if (in) {
                        const uint64_t peers = match_peers(b, bits);
                        if (mask_rank(peers) == 0) atomicAdd(&h[b], (uint32_t)__popcll(peers));
                    }
                } else if (in) {
                    const uint32_t b0 = __builtin_amdgcn_readfirstlane(b);
                    const uint64_t act = __ballot(1), same = __ballot(b == b0);
                    if (same == act) {
                        if (mask_rank(act) == 0) atomicAdd(&h[b0], (uint32_t)__popcll(act));
                    } else {
                        atomicAdd(&h[b], 1u);
                    }
                }
            };
            constexpr uint32_t RND = P_THREADS * HK;  // keys per round
            if (un == U) {
                // full unit: no bounds checks; the next round's HK keys are
                // loaded (unconditionally: the last round reloads itself)
                // while this round's are bucketed
                uint64_t kk[HK], kn[HK];
#pragma unroll
                for (int r = 0; r < HK; r++) kk[r] = src[base + r * P_THREADS + tid];
                for (uint32_t i0 = 0; i0 < U; i0 += RND) {
                    const uint32_t nx = i0 + RND < U ? i0 + RND : i0;
#pragma unroll
                    for (int r = 0; r < HK; r++) kn[r] = src[base + nx + r * P_THREADS + tid];
#pragma unroll
                    for (int r = 0; r < HK; r++)
                        add(kind_bucket<KIND>(v, mdl, kk[r], u64, P.ids, base + i0 + r * P_THREADS + tid), true);
#pragma unroll
                    for (int r = 0; r < HK; r++) kk[r] = kn[r];
                }
                return;
            }
            // HK keys per thread are loaded before any is used, so that every
            // wave keeps HK loads in flight (the unit is read exactly once)
            for (uint32_t i0 = 0; i0 < un; i0 += RND) {
                uint64_t kk[HK];
#pragma unroll
                for (int r = 0; r < HK; r++) {
                    const uint32_t i = i0 + r * P_THREADS + tid;
                    kk[r] = i < un ? src[base + i] : 0;
                }
#pragma unroll
                for (int r = 0; r < HK; r++) {
                    const uint32_t i = i0 + r * P_THREADS + tid;
                    if (i0 + r * P_THREADS >= un) break;  // uniform: no key of this round in range
                    const bool in = i < un;
                    add(in ? kind_bucket<KIND>(v, mdl, kk[r], u64, P.ids, base + i) : 0u, in);
                }
            }
        });
        __syncthreads();
        unsigned long long* row = P.status + sg.sbase + (uint64_t)td.idx * sg.nb;
        for (uint32_t b = tid; b < sg.nb; b += P_THREADS) {
            const uint32_t c = h[b];
            st_store(row + b, tag | ST_AGG | c);
            if (c) atomicAdd(&P.counts[sg.cbase + b], (unsigned long long)c);
        }
    }
}

// ===========================================================================
// k_scan: bucket starts and classification of every bucket (one WG / segment)
// ===========================================================================

constexpr int S_THREADS = 256;
constexpr int S_BPT = B_MAX / S_THREADS;  // buckets per thread

// Per-bucket decision (Sec. 2.2 homogeneity check, Sec. 4 base case, the 2x
// fallback rule): 0 nothing, 1 copy run, 2 base case, 3 range radix child,
// 4 fine child (same model), 5 splitter-tree child (fallback), 6 fresh child.
// A child segment small enough for one workgroup goes to k_resident (no
// work units); children of the MLP-rooted model stay on the unit path, whose
// k_mlp_ids supplies their bucket ids.
__device__ __forceinline__ bool child_resident(uint32_t parent_kind, uint32_t act, uint64_t n) {
    return n <= RES_MAX && !(act == 4 && parent_kind == K_MLP);
}

struct Decision {
    uint32_t act;
    uint64_t stat;  // 12-bit fields: empty, equality, base, recurse
};

__device__ __forceinline__ Decision decide(const Params& P, int lvl, uint32_t q, uint64_t c, bool single_value,
                                           bool fine_ok, uint32_t log2B2, double expected) {
    Decision d{0, 0};
    if (c == 0) { d.stat = 1; return d; }
    if (single_value || c == 1) {
        d.stat = 1ull << 12;
        // finished; only a run left in the temporary moves (one key: a trivial sort)
        d.act = q == 1 ? (c == 1 ? 2u : 1u) : 0u;
        return d;
    }
    const bool oversized = (double)c > P.fallback_ratio * expected;
    const bool fine = fine_ok && !(P.flags & FLAG_REFIT) && !oversized && (4ull << log2B2) <= c &&
                      (uint32_t)lvl + 1 < P.max_levels;
    // The base case takes a bucket at or below the cutoff, and any bucket it
    // can hold (BIG_MAX): sorting it directly is one pass, another level is at
    // least a partition pass plus the fixed work of a segment.  At the depth
    // cap this leaves range radix (8 bits per level) only buckets of more
    // than BIG_MAX keys.
    if (c <= P.cutoff || c <= (uint64_t)BIG_MAX) { d.stat = 1ull << 24; d.act = 2; return d; }
    d.stat = 1ull << 36;
    if ((uint32_t)lvl + 1 >= P.max_levels) d.act = 3;
    else if (fine) d.act = 4;
    else if (oversized && !(P.flags & 0x1u)) d.act = 5;
    else d.act = 6;
    return d;
}

__global__ __launch_bounds__(S_THREADS) void k_scan(Params P) {
    __shared__ uint64_t red64[S_THREADS / 64];
    __shared__ uint8_t eqb[B_MAX];
    __shared__ uint64_t resv[10];
    const int tid = threadIdx.x;
    const int lvl = P.level;
    if (blockIdx.x == 0 && tid == 0) {  // pools of the next level (this level's data stays readable)
        P.ctl->counts_used = 0;
        P.ctl->status_used = 0;
        P.ctl->arena_used[(lvl + 1) & 1] = 0;
    }
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    const uint32_t q = (lvl + 1) & 1;  // buffer the children live in
    LevelStats& st = P.ctl->lv[lvl];
    for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        const Seg sg = P.segs[lvl & 1][s];
        if (sg.flags & SEG_FAILED) continue;
        const uint32_t nb = sg.nb;
        // this thread's buckets: S_BPT * tid + i
        uint64_t c[S_BPT], local = 0, cmax = 0;
#pragma unroll
        for (int i = 0; i < S_BPT; i++) {
            const uint32_t b = S_BPT * tid + i;
            c[i] = b < nb ? P.counts[sg.cbase + b] : 0;
            local += c[i];
            cmax = c[i] > cmax ? c[i] : cmax;
        }
        uint64_t tot;
        uint64_t run = sg.off + block_excl_scan<S_THREADS, uint64_t>(local, red64, &tot);
        uint64_t start[S_BPT];
#pragma unroll
        for (int i = 0; i < S_BPT; i++) {
            const uint32_t b = S_BPT * tid + i;
            start[i] = run;
            run += c[i];
            if (b < nb) P.counts[sg.cbase + nb + b] = start[i];
        }
        // which buckets hold a single value
        for (uint32_t b = tid; b < B_MAX; b += S_THREADS) eqb[b] = 0;
        __syncthreads();
        uint32_t log2B2 = 0;
        bool fine_ok = false;
        if (sg.kind == K_TREE || sg.kind == K_TREE_FORCED) {
            const TreeModel* h = (const TreeModel*)sg.model;
            const uint16_t* lut = (const uint16_t*)((const uint64_t*)sg.model + 2 + h->m);
            for (uint32_t u = tid; u < h->m; u += S_THREADS) {
                const uint16_t e = lut[u + 1];
                if (e & 1) eqb[(u + 1) + (e >> 1) - 1] = 1;
            }
        } else if (sg.kind == K_RADIX) {
            const RadixModel* h = (const RadixModel*)sg.model;
            if (h->shift == 0 || h->shift == 64)
                for (uint32_t b = tid; b < nb; b += S_THREADS) eqb[b] = 1;
        } else if (sg.kind == K_RMI) {
            log2B2 = ((const RmiModel*)sg.model)->log2B2;
            fine_ok = log2B2 > 0;
        } else if (sg.kind == K_MLP) {
            log2B2 = ((const MlpModel*)sg.model)->log2B2;
            fine_ok = log2B2 > 0;
        }
        __syncthreads();
        const double expected = (double)sg.n / (double)nb;
        // base-case items of the first level's RMI can be placed by the model
        // (k_base_model): its fine ids of an item are [g0, g0 + w)
        const bool mbase = (P.flags & FLAG_MODEL_BASE) && P.fmodel && sg.model == (uint64_t)P.fmodel &&
                           (sg.kind == K_RMI || sg.kind == K_RMI_FINE);
        uint32_t act[S_BPT];
        uint64_t la = 0, lb = 0, lc = 0, lstat = 0, lsk = 0, lgk = 0, lcp = 0, lfb = 0, ld = 0, lmk = 0, lm = 0;
#pragma unroll
        for (int i = 0; i < S_BPT; i++) {
            const uint32_t b = S_BPT * tid + i;
            act[i] = 0;
            if (b >= nb) continue;
            const Decision d = decide(P, lvl, q, c[i], eqb[b] != 0, fine_ok, log2B2, expected);
            act[i] = d.act;
            lstat += d.stat;
            const bool mb = mbase && d.act == 2 && c[i] >= MB_MIN && c[i] <= MB_MAX;
            ld += mb ? 1 : 0;
            lmk += mb ? c[i] : 0;
            const uint64_t nsm = d.act == 2 && !mb && (c[i] <= SMALL_MAX || (c[i] <= GROUP_WAVE_MAX && !P.has_pay)) ? 1 : 0;
            const uint64_t nsp = d.act == 2 && !mb && !nsm ? split_chunks(c[i], P.has_pay) : 0;
            const uint64_t ng0 = nsm && c[i] <= GROUP_SMALL_MAX ? 1 : 0;
            const uint64_t ng1 = nsm && !ng0 && c[i] <= GROUP_MAX ? 1 : 0;
            const uint64_t ng3 = nsm && c[i] > SMALL_MAX && c[i] <= GROUP_LARGE_MAX ? 1 : 0;
            const uint64_t ng4 = nsm && c[i] > GROUP_LARGE_MAX ? 1 : 0;
            const uint64_t nbg = d.act == 1 ? (c[i] + COPY_CHUNK - 1) / COPY_CHUNK : (d.act == 2 && !nsm && !mb && !nsp ? 1 : 0);
            const uint64_t ntl = d.act >= 3 && !child_resident(sg.kind, d.act, c[i]) ? (c[i] + UNIT - 1) / UNIT : 0;
            // packed counters: items <= 128 keys | children << 16 | large items << 32,
            // units | items of 129..256 keys << 32 | items of 257..512 keys << 48
            la += ng0 | ((uint64_t)(d.act >= 3) << 16) | (nbg << 32);
            lb += ntl | (ng1 << 32) | ((nsm - ng0 - ng1 - ng3 - ng4) << 48);
            lc += ng3 | ((ng4 + nsp) << 32);
            lm += nsp > 1 ? 1 | (nsp << 16) | (c[i] << 32) : 0;  // merged items (one chunk: none)
            // fallbacks | merged items of more than GROUP_WAVE_MAX keys << 16 |
            // of more than twice that << 32 (each at most B_MAX per segment)
            static_assert(B_MAX < (1 << 16), "16-bit count fields");
            lfb += (d.act == 5 ? 1 : 0) | (nsp > 1 && c[i] > GROUP_WAVE_MAX ? 1ull << 16 : 0) |
                   (nsp > 1 && c[i] > 2 * GROUP_WAVE_MAX ? 1ull << 32 : 0);
            lsk += nsm || nsp ? c[i] : 0;
            lgk += nbg ? c[i] : 0;
            lcp += d.act == 1 ? nbg : 0;
        }
        // one reservation per list for the whole workgroup
        uint64_t ta, tb;
        uint64_t xa = block_excl_scan<S_THREADS, uint64_t>(la, red64, &ta);
        uint64_t xb = block_excl_scan<S_THREADS, uint64_t>(lb, red64, &tb);
        uint64_t tc, td;
        uint64_t xc = block_excl_scan<S_THREADS, uint64_t>(lc, red64, &tc);
        uint64_t xd = block_excl_scan<S_THREADS, uint64_t>(ld, red64, &td);
        uint64_t tm;  // merged items | their chunks << 16 | their keys << 32
        uint64_t xm = block_excl_scan<S_THREADS, uint64_t>(lm, red64, &tm);
        const uint64_t mk = block_sum<S_THREADS, uint64_t>(lmk, red64);
        const uint64_t sk = block_sum<S_THREADS, uint64_t>(lsk, red64);
        const uint64_t gk = block_sum<S_THREADS, uint64_t>(lgk, red64);
        const uint64_t ncp = block_sum<S_THREADS, uint64_t>(lcp, red64);
        const uint64_t sc = block_sum<S_THREADS, uint64_t>(lstat, red64);
        const uint64_t fbm = block_sum<S_THREADS, uint64_t>(lfb, red64);
        const uint64_t nfb = fbm & 0xffff;
        const uint64_t mx = block_max<S_THREADS, uint64_t>(cmax, red64);
        if (tid < WAVE) {
            // the reservations: one device-scope atomic per lane, issued as one
            // instruction per width, so that their round trips overlap
            const uint64_t itot = ta & 0xffff, ctot = (ta >> 16) & 0xffff, gtot = ta >> 32, ttot = tb & 0xffffffffull;
            const uint64_t btot = (tb >> 32) & 0xffff, wtot = tb >> 48;
            const int l = tid;
            unsigned long long* p64 = l == 0 ? &P.ctl->nitems : l == 1 ? &P.ctl->nitems_w : l == 2 ? &P.ctl->nitems_b
                                    : l == 3 ? &P.ctl->nitems_k : l == 4 ? &P.ctl->nitems_c : l == 5 ? &P.ctl->nbig
                                    : l == 6 ? &P.ctl->ncopy : l == 7 ? &P.ctl->small_keys : l == 8 ? &P.ctl->big_keys
                                    : &st.keys;
            const uint64_t v64 = l == 0 ? itot : l == 1 ? wtot : l == 2 ? btot : l == 3 ? (tc & 0xffffffffull)
                               : l == 4 ? (tc >> 32) : l == 5 ? gtot : l == 6 ? ncp : l == 7 ? sk : l == 8 ? gk
                               : l == 9 ? sg.n : 0;  // st.keys always: per-level kernel timing reads it
            if (l < 10 && (v64 || l == 9)) {
                const uint64_t r = atomicAdd(p64, (unsigned long long)v64);
                const int slot = l == 0 ? 0 : l == 1 ? 4 : l == 2 ? 5 : l == 3 ? 6 : l == 4 ? 7 : l == 5 ? 3 : -1;
                if (slot >= 0) resv[slot] = r;
            } else if (l < 6) {
                const int slot = l == 0 ? 0 : l == 1 ? 4 : l == 2 ? 5 : l == 3 ? 6 : l == 4 ? 7 : 3;
                resv[slot] = 0;
            }
            const uint32_t v32 = l == 10 ? (uint32_t)ctot : l == 11 ? (uint32_t)ttot : 0u;
            if (l == 10 || l == 11) {
                resv[l - 9] = v32 ? atomicAdd(l == 10 ? &P.ctl->nseg[lvl + 1] : &P.ctl->ntile[lvl + 1], v32) : 0u;
            }
            if (l == 12) resv[8] = td ? atomicAdd(&P.ctl->nitems_m, (unsigned long long)td) : 0ull;
            if (l == 13 && mk) atomicAdd(&P.ctl->model_keys, (unsigned long long)mk);
            if (l == 14) resv[9] = (tm & 0xffff) ? atomicAdd(&P.ctl->nmerge, (unsigned long long)(tm & 0xffff)) : 0ull;
            if (l == 15 && (tm >> 32)) atomicAdd(&P.ctl->merge_keys, (unsigned long long)(tm >> 32));
            if (l == 16 && (tm & 0xffff)) atomicAdd(&P.ctl->nchunk, (unsigned long long)((tm >> 16) & 0xffff));
            const uint64_t mcl = l == 17 ? (fbm >> 16) & 0xffff : fbm >> 32;
            if ((l == 17 || l == 18) && mcl) atomicAdd(&P.ctl->nmerge_cls[l - 17], (unsigned long long)mcl);
        }
        if (tid == 0) {
            const uint64_t m12 = 4095;
            if (P.flags & FLAG_STATS) {
                atomicAdd(&st.segments, 1ull);
                atomicAdd(&st.buckets, (unsigned long long)nb);
                atomicMax(&st.max_bucket, (unsigned long long)mx);
                atomicMax(&st.max_ratio_x1000, (unsigned long long)(1000.0 * (double)mx / expected));
                atomicAdd(&st.empty, (unsigned long long)(sc & m12));
                atomicAdd(&st.equality, (unsigned long long)((sc >> 12) & m12));
                atomicAdd(&st.base, (unsigned long long)((sc >> 24) & m12));
                atomicAdd(&st.recurse, (unsigned long long)((sc >> 36) & m12));
                atomicAdd(&st.fallback, (unsigned long long)nfb);
            }
        }
        __syncthreads();
        uint32_t nresc = 0;
#pragma unroll
        for (int i = 0; i < S_BPT; i++) {
            const uint32_t b = S_BPT * tid + i;
            const uint32_t a = act[i];
            const uint64_t ci = c[i];
            const bool mb = mbase && a == 2 && ci >= MB_MIN && ci <= MB_MAX;
            const uint64_t nsm = a == 2 && !mb && (ci <= SMALL_MAX || (ci <= GROUP_WAVE_MAX && !P.has_pay)) ? 1 : 0;
            const uint64_t nsp = a == 2 && !mb && !nsm ? split_chunks(ci, P.has_pay) : 0;
            const uint64_t nbg = a == 1 ? (ci + COPY_CHUNK - 1) / COPY_CHUNK : (a == 2 && !nsm && !mb && !nsp ? 1 : 0);
            if (mb) {
                const uint64_t it = resv[8] + xd;
                if (it < P.item_m_cap) {
                    const bool fine = sg.kind == K_RMI_FINE;
                    P.items_m[2 * it] = item_pack(start[i], q, 0u, (uint32_t)ci);
                    P.items_m[2 * it + 1] = (uint64_t)(fine ? sg.win + b : b << log2B2) |
                                            ((uint64_t)(fine ? 0u : log2B2) << 32);
                } else {
                    atomicOr(&P.ctl->overflow, OVF_ITEM);
                }
            }
            const uint64_t ntl = a >= 3 && !child_resident(sg.kind, a, ci) ? (ci + UNIT - 1) / UNIT : 0;
            const uint64_t iex = xa & 0xffff, cex = (xa >> 16) & 0xffff, gex = xa >> 32, tex = xb & 0xffffffffull;
            const uint64_t bex = (xb >> 32) & 0xffff, wex = xb >> 48;
            const uint64_t ng0 = nsm && ci <= GROUP_SMALL_MAX ? 1 : 0;
            const uint64_t ng1 = nsm && !ng0 && ci <= GROUP_MAX ? 1 : 0;
            const uint64_t ng3 = nsm && ci > SMALL_MAX && ci <= GROUP_LARGE_MAX ? 1 : 0;
            const uint64_t ng4 = nsm && ci > GROUP_LARGE_MAX ? 1 : 0;
            if (nsm) {
                // lists: <= 128 front of items, 129..256 front of items_b,
                // 257..512 back of items, 513..1024 back of items_b,
                // 1025..2048 items_c
                const uint64_t it = ng0 ? resv[0] + iex : ng1 ? resv[5] + bex : ng3 ? resv[6] + (xc & 0xffffffffull)
                                  : ng4 ? resv[7] + (xc >> 32) : resv[4] + wex;
                const bool inb = ng1 || ng3;
                const uint64_t cap = inb ? P.item_b_cap : ng4 ? P.item_c_cap : P.item_cap;
                uint64_t* list = inb ? P.items_b : ng4 ? P.items_c : P.items;
                if (it < cap) list[ng0 || ng1 || ng4 ? it : cap - 1 - it] = item_pack(start[i], q, 0u, (uint32_t)ci);
                else atomicOr(&P.ctl->overflow, OVF_ITEM);
            }
            if (nsp) {
                // chunks (the last one shorter) sorted as items of their own,
                // then, for more than one, a merge of the whole bucket
                const uint64_t ch = chunk_keys(P.has_pay);
                for (uint64_t k = 0; k < nsp; k++) {
                    const uint64_t it = resv[7] + (xc >> 32) + k;
                    if (it >= P.item_c_cap) { atomicOr(&P.ctl->overflow, OVF_ITEM); break; }
                    const uint64_t sz = min<uint64_t>(ch, ci - k * ch);
                    P.items_c[it] = item_pack(start[i] + k * ch, q, 0u, (uint32_t)sz);
                }
                if (nsp > 1) {
                    const uint64_t it = resv[9] + (xm & 0xffff);
                    if (it < P.merge_cap) P.merges[it] = item_pack(start[i], 0u, 0u, (uint32_t)ci);
                    else atomicOr(&P.ctl->overflow, OVF_ITEM);
                }
            }
            for (uint64_t k = 0; k < nbg; k++) {
                const uint64_t it = resv[3] + gex + k;
                if (it >= P.big_cap) { atomicOr(&P.ctl->overflow, OVF_ITEM); break; }
                const uint64_t sz = a == 1 ? min<uint64_t>(COPY_CHUNK, ci - k * COPY_CHUNK) : ci;
                P.bigs[it] = item_pack(start[i] + k * COPY_CHUNK, a == 1 ? 1u : q, a == 1 ? 1u : 0u, (uint32_t)sz);
            }
            nresc += a >= 3 && child_resident(sg.kind, a, ci) ? 1u : 0u;
            if (a >= 3) {
                const uint64_t si = resv[1] + cex, t0 = resv[2] + tex;
                if (si < P.seg_cap) {
                    Seg ch{};
                    ch.off = start[i]; ch.n = ci; ch.ntiles = (uint32_t)ntl; ch.tile0 = (uint32_t)t0;
                    ch.kind = a == 3 ? K_RADIX : a == 4 ? (sg.kind == K_RMI ? K_RMI_FINE : K_MLP_FINE)
                            : a == 5 ? K_TREE_FORCED : K_FRESH;
                    if (child_resident(sg.kind, a, ci)) ch.flags = SEG_RESIDENT;
                    if (a == 5 && lvl == 0 && sg.kind == K_RMI && (sg.flags & SEG_PREBUILT) && P.fsample) {
                        ch.flags |= SEG_FROM_SAMPLE;  // the tree's sample: the first-level sample in bucket b
                        ch.model = sg.model;
                        ch.win = b;
                    }
                    if (a == 4) {
                        ch.model = sg.model;
                        ch.nb = 1u << log2B2;
                        ch.win = b << log2B2;
                        ch.flags |= sg.flags & 0xffff0000u;  // model words
                    }
                    if (t0 + ntl > P.tile_cap) { atomicOr(&P.ctl->overflow, OVF_TILE); ch.flags |= SEG_FAILED; }
                    P.segs[q][si] = ch;  // k_model of the next level writes its unit descriptors
                } else {
                    atomicOr(&P.ctl->overflow, OVF_SEG);
                    for (uint32_t u = 0; u < ntl; u++)  // keep the unit list free of stale slots
                        if (t0 + u < P.tile_cap) P.tiles[q][t0 + u] = Tile{0xffffffffu, 0};
                }
            }
            xd += mb ? 1 : 0;
            xa += ng0 | ((uint64_t)(a >= 3) << 16) | (nbg << 32);
            xb += ntl | (ng1 << 32) | ((nsm - ng0 - ng1 - ng3 - ng4) << 48);
            xc += ng3 | ((ng4 + nsp) << 32);
            xm += nsp > 1 ? 1 | (nsp << 16) | (ci << 32) : 0;
        }
        {  // resident children, one atomic per wavefront that has any
            const uint32_t wt = wave_incl_sum(nresc);
            if ((tid & 63) == 63 && wt) atomicAdd(&P.ctl->nres[lvl + 1], wt);
        }
        __syncthreads();
    }
}

// ===========================================================================
// k_scatter<PAY>: one work unit (4 tiles of 8192 keys) per iteration, units taken
// in order through a ticket.  First the unit's exclusive prefix per bucket
// comes from a decoupled look-back (Merrill & Garland) over the preceding
// units of its segment: every such word already holds at least the unit's
// aggregate (written by k_hist), so the walk never waits -- it stops at the
// first inclusive prefix or at the segment's first unit -- and the unit
// publishes its own inclusive prefix at once.  Then each tile: in-tile rank,
// tile-local bucket starts, keys staged in LDS grouped by bucket and written
// as contiguous runs.  The next tile's keys are loaded while the current one
// is ranked.
//   PAY = true: the rank is stable (wave match over the bucket bits and
//   per-wave counters), so a payload keeps the input order of equal keys.
//   PAY = false: keys only.  Order inside a bucket is not observable -- the
//   bucket is sorted later and equal keys are identical -- so the rank is one
//   LDS atomic per key.  A tile writes each bucket's keys only up to the last
//   64-byte boundary they reach and carries the rest (at most 7 keys, in the
//   registers of the bucket's thread) into the unit's next tile, which writes
//   them in front of its own: a tile's run of a bucket is ~8 keys at 1000
//   buckets, and output segments shared by two tiles written at different
//   times cost the memory system about twice the bytes of whole ones.
// ===========================================================================

// Keys only, per bucket: keys held back from one tile for the next (a partial
// 64-byte output segment has at most 7).
constexpr int CARRY = 7;

// Barrier for LDS hand-offs only: global loads in flight stay in flight.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <bool PAY, int NT>
__global__ __launch_bounds__(NT) void k_scatter(Params P) {
    constexpr int SW = NT / WAVE;        // waves
    constexpr int SK = TILE / NT;        // keys per thread per tile
    constexpr int SWK = WAVE * SK;       // keys per wave per tile
    constexpr int SB = B_MAX / NT;       // buckets per thread in the tile scan
    static_assert(SK * NT == TILE && SB * NT == B_MAX, "tile and bucket range split evenly");
    static_assert(PAY || SB == 1, "keys only: thread j owns bucket j (its carry and output cursor)");
    __shared__ __align__(16) uint64_t mdl[LDS_MODEL_WORDS];
    __shared__ uint64_t stage[TILE];
    __shared__ uint16_t sbid[TILE];
    __shared__ uint16_t wcnt[PAY ? SW : 1][PAY ? B_MAX : 1];
    __shared__ uint32_t tcnt[B_MAX];
    __shared__ uint16_t tstart[B_MAX];
    __shared__ uint64_t run[PAY ? B_MAX : 1];    // payload: output position of the tile's run of each bucket
    // keys only: output position of staging slot 0 for each bucket's slots, in
    // the low 48 bits; the end of the bucket's slots written this tile, above
    __shared__ uint64_t delta[PAY ? 1 : B_MAX];
    __shared__ uint32_t sh_t;
    __shared__ uint64_t red64[SW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lvl = P.level;
    const uint32_t nunit = level_units(P, lvl);
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    const uint64_t tag = ((uint64_t)(P.persist[0] * MAXL + lvl)) << ST_TAG_SHIFT;
    const uint64_t* src = P.keys[lvl & 1];
    uint64_t* dst = P.keys[(lvl + 1) & 1];
    const uint32_t* psrc = P.pay[lvl & 1];
    uint32_t* pdst = P.pay[(lvl + 1) & 1];
    const int u64 = P.u64;
    constexpr bool has_pay = PAY;
    uint64_t cur_model = 0;
    for (;;) {
        if (tid == 0) sh_t = atomicAdd(&P.ctl->ticket[lvl], 1u);
        __syncthreads();
        const uint32_t t = sh_t;
        if (t >= nunit) break;
        const Tile td = P.tiles[lvl & 1][t];
        if (td.seg >= nseg) { __syncthreads(); continue; }
        const Seg sg = P.segs[lvl & 1][td.seg];
        if (sg.flags & SEG_FAILED) { __syncthreads(); continue; }
        if (sg.model != cur_model) {
            load_model_lds(mdl, (const uint64_t*)sg.model, sg.kind, sg.flags >> 16, tid, NT);
            cur_model = sg.model;
        }
        const uint32_t nb = sg.nb;
        // keys only, thread j for bucket j: the output cursor and the carry,
        // the keys of the bucket's last partial 64-byte segment held back for
        // the unit's next tile (at most CARRY of them)
        uint64_t acur = 0;
        uint32_t kcar = 0;
        uint64_t car[CARRY];
#pragma unroll
        for (int c = 0; c < CARRY; c++) car[c] = 0;
        // ---- look-back: exclusive prefix of this unit for every bucket ----
        {
            unsigned long long* row = P.status + sg.sbase + (uint64_t)td.idx * nb;
            uint32_t bad = 0;
            for (uint32_t j = tid; j < nb; j += NT) {
                const uint64_t own = st_load(row + j);
                uint64_t excl = 0;
                for (int64_t pk = (int64_t)td.idx - 1; pk >= 0; pk--) {
                    const uint64_t wv = st_load(P.status + sg.sbase + (uint64_t)pk * nb + j);
                    const uint64_t hdr = wv & ~ST_LOW_MASK;
                    if (hdr != (tag | ST_AGG) && hdr != (tag | ST_PREFIX)) { bad = 1; break; }
                    excl += wv & ST_VALUE_MASK;
                    if (hdr == (tag | ST_PREFIX)) break;
                }
                if ((own & ~ST_LOW_MASK) != (tag | ST_AGG) && (own & ~ST_LOW_MASK) != (tag | ST_PREFIX)) bad = 1;
                st_store(row + j, tag | ST_PREFIX | (excl + (own & ST_VALUE_MASK)));
                if (PAY) run[j] = P.counts[sg.cbase + nb + j] + excl;
                else acur = P.counts[sg.cbase + nb + j] + excl;
                if (!PAY) tcnt[j] = 0;  // the first tile's counters (later tiles: in the scan)
            }
            if (__syncthreads_or(bad)) {  // never expected: refuse to write anything for this unit
                if (tid == 0) atomicOr(&P.ctl->overflow, OVF_STATE);
                __syncthreads();
                continue;
            }
        }
        const View v = make_view(mdl, sg.kind, sg.nb, sg.win);
        const int bits = ceil_log2(nb);
        const uint32_t U = seg_unit(sg.flags);
        const uint64_t ubase = sg.off + (uint64_t)td.idx * U;
        const uint32_t un = (uint32_t)min<uint64_t>(U, sg.n - (uint64_t)td.idx * U);
        const uint32_t ntl = (un + TILE - 1) / TILE;
        // the payload variant keeps one copy of the tile loop (registers)
        with_kind<!PAY>(v.kind, u64, [&](auto kc) {
        constexpr int KIND = decltype(kc)::value;
        // wave w owns keys [w*1024, (w+1)*1024) of a tile, 64 per round.
        // Keys only: every global load and store of the tile loop is issued
        // unconditionally (indices clamp into the tile; a lane past the end
        // repeats the tile's last load or store, same address and value), so
        // the compiler's vector-memory wait counts stay exact and the next
        // tile's loads stay in flight across this tile's stores.
        uint64_t k[SK], kn[SK];
        uint32_t pl[SK], pn[SK];
#pragma unroll
        for (int r = 0; r < SK; r++) {
            const uint32_t i = w * SWK + r * WAVE + lane;
            if (PAY) {
                k[r] = i < un ? src[ubase + i] : 0;
                pl[r] = i < un ? psrc[ubase + i] : 0;
            } else {
                k[r] = __builtin_nontemporal_load(src + ubase + min(i, un - 1));
            }
        }
        // the first tile's keys have arrived before the loop, so that inside
        // it only the prefetched keys are waited for, never this tile's stores
        if (!PAY) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        for (uint32_t tt = 0; tt < ntl; tt++) {
            const uint64_t base = ubase + (uint64_t)tt * TILE;
            const uint32_t tn = min<uint32_t>(TILE, un - tt * TILE);
            if (PAY && tt + 1 < ntl) {  // prefetch the next tile
                const uint32_t nn = min<uint32_t>(TILE, un - (tt + 1) * TILE);
#pragma unroll
                for (int r = 0; r < SK; r++) {
                    const uint32_t i = w * SWK + r * WAVE + lane;
                    kn[r] = i < nn ? src[base + TILE + i] : 0;
                    pn[r] = i < nn ? psrc[base + TILE + i] : 0;
                }
            }
            uint32_t b[SK], rk[SK];
            if (PAY) {
                for (uint32_t j = lane; j < nb; j += WAVE) wcnt[w][j] = 0;
            }
#pragma unroll
            for (int r = 0; r < SK; r++) {
                const uint32_t i = w * SWK + r * WAVE + lane;
                if (PAY) {
                    b[r] = i < tn ? kind_bucket<KIND>(v, mdl, k[r], u64, P.ids, base + i) : 0;
                } else {
                    const uint32_t bk = kind_bucket<KIND>(v, mdl, k[r], u64, P.ids, base + min(i, tn - 1));
                    b[r] = i < tn ? bk : 0;
                }
            }
            if (!PAY) {  // prefetch the next tile (after the last one: one line, in bounds, no branch)
                const bool more = tt + 1 < ntl;
                const uint32_t nn = more ? min<uint32_t>(TILE, un - (tt + 1) * TILE) : 1u;
                const uint32_t lim = more ? nn - 1 : 0u;
#pragma unroll
                for (int r = 0; r < SK; r++) kn[r] = __builtin_nontemporal_load(src + base + (more ? TILE : 0) + min<uint32_t>(w * SWK + r * WAVE + lane, lim));
            }
            if (PAY) {
                // stable rank within the wave: rounds in key order, lanes in key order
#pragma unroll
                for (int r = 0; r < SK; r++) {
                    const uint32_t i = w * SWK + r * WAVE + lane;
                    rk[r] = 0;
                    if (i < tn) {
                        const uint64_t peers = match_peers(b[r], bits);
                        const uint32_t below = mask_rank(peers);
                        const uint32_t before = wcnt[w][b[r]];
                        if (below == 0) wcnt[w][b[r]] = (uint16_t)(before + __popcll(peers));
                        rk[r] = before + below;
                    }
                }
                lds_barrier();
                // per bucket: exclusive prefix over waves (in place) and tile count
                for (uint32_t j = tid; j < nb; j += NT) {
                    uint32_t acc = 0;
#pragma unroll
                    for (int x = 0; x < SW; x++) {
                        const uint32_t c = wcnt[x][j];
                        wcnt[x][j] = (uint16_t)acc;
                        acc += c;
                    }
                    tcnt[j] = acc;
                }
            } else {
                // any order inside a bucket: one LDS atomic per key (one per wave
                // when the whole wave falls into a single bucket)
#pragma unroll
                for (int r = 0; r < SK; r++) {
                    const uint32_t i = w * SWK + r * WAVE + lane;
                    rk[r] = 0;
                    if (i < tn) {
                        const uint32_t b0 = __builtin_amdgcn_readfirstlane(b[r]);
                        const uint64_t act = __ballot(1), same = __ballot(b[r] == b0);
                        if (same == act) {
                            uint32_t bs = 0;
                            if (mask_rank(act) == 0) bs = atomicAdd(&tcnt[b0], (uint32_t)__popcll(act));
                            rk[r] = __shfl(bs, __ffsll((unsigned long long)act) - 1) + mask_rank(act);
                        } else {
                            rk[r] = atomicAdd(&tcnt[b[r]], 1u);
                        }
                    }
                }
            }
            lds_barrier();
            // keys only, thread j for bucket j: keys written this tile (twr) of the
            // carry + this tile's keys of the bucket (tm), and the bucket's
            // first staging slot (tex)
            uint32_t twr = 0, tm = 0, tex = 0;
            {  // tile-local bucket starts: exclusive scan over buckets, SB per thread
                uint32_t c[SB], lane_sum = 0;
#pragma unroll
                for (int q = 0; q < SB; q++) {
                    const uint32_t j = SB * tid + q;
                    c[q] = j < nb ? tcnt[j] : 0u;
                    // keys only: bucket j's counter is read by thread j alone, so
                    // it is cleared for the next tile here (the barriers before
                    // the next tile's atomics order the two)
                    if (!PAY && j < nb) tcnt[j] = 0;
                    lane_sum += c[q];
                }
                const uint32_t x = wave_incl_sum(lane_sum);
                if (lane == 63) red64[w] = x;
                lds_barrier();
                uint32_t ex = x - lane_sum;
#pragma unroll
                for (int q = 0; q < SW; q++) ex += q < w ? (uint32_t)red64[q] : 0u;
#pragma unroll
                for (int q = 0; q < SB; q++) {
                    const uint32_t j = SB * tid + q;
                    if (j < nb) {
                        tstart[j] = (uint16_t)ex;
                        if (!PAY) {
                            // the carry, then this tile's keys, go out from acur up to
                            // the last 64-byte boundary they reach (all of them in the
                            // unit's last tile); the rest is carried.  Once past the
                            // unit's first write, acur stays on a boundary, so every
                            // 64-byte segment inside the unit's run of the bucket is
                            // written whole, by one tile.
                            const uint32_t m = kcar + c[q];
                            uint32_t wr = m;
                            if (tt + 1 < ntl) {
                                const uint64_t e = (acur + m) & ~7ull;
                                wr = e > acur ? (uint32_t)(e - acur) : 0u;  // 0, or more than kcar
                            }
                            // staging slot p (new keys only) goes to (delta & MASK48) + p
                            // while p < delta >> 48
                            const uint32_t wend = ex + (wr > 0 ? wr - kcar : 0u);
                            delta[j] = (acur + kcar - ex) | ((uint64_t)wend << 48);
                            twr = wr; tm = m; tex = ex;
                        }
                    }
                    ex += c[q];
                }
            }
            lds_barrier();
            // stage keys grouped by bucket (stable positions)
            uint32_t pos[SK];
#pragma unroll
            for (int r = 0; r < SK; r++) {
                const uint32_t i = w * SWK + r * WAVE + lane;
                pos[r] = 0xffffffffu;
                if (i < tn) {
                    const uint32_t p = tstart[b[r]] + (PAY ? (uint32_t)wcnt[w][b[r]] : 0u) + rk[r];
                    pos[r] = p;
                    stage[p] = k[r];
                    sbid[p] = (uint16_t)b[r];
                }
            }
            lds_barrier();
            if (!PAY) {
                // the next tile's keys are taken now, before this tile's stores
                // are issued: the wait for them then never waits for stores
#pragma unroll
                for (int r = 0; r < SK; r++) k[r] = kn[r];
                uint32_t bq[SK];
                uint64_t vq[SK];
#pragma unroll
                for (int q = 0; q < SK; q++) {
                    const uint32_t p = min<uint32_t>(tid + q * NT, tn - 1);
                    bq[q] = sbid[p];
                    vq[q] = stage[p];
                }
#pragma unroll
                for (int q = 0; q < SK; q++) {
                    const uint32_t p = min<uint32_t>(tid + q * NT, tn - 1);
                    const uint64_t dl = delta[bq[q]];
                    if (p < (uint32_t)(dl >> 48)) dst[(dl & 0xFFFFFFFFFFFFull) + p] = vq[q];
                }
                if ((uint32_t)tid < nb) {
                    // the carry goes out in front of the bucket's new keys, then the
                    // keys past the written part become the carry
                    if (twr > 0) {
#pragma unroll
                        for (int c = 0; c < CARRY; c++)
                            if ((uint32_t)c < kcar) dst[acur + c] = car[c];
                    }
                    const uint32_t nk = tm - twr;
                    const int32_t o0 = twr > 0 ? (int32_t)(twr - kcar) : -(int32_t)kcar;
#pragma unroll
                    for (int c = 0; c < CARRY; c++) {
                        const bool keep = twr == 0 && (uint32_t)c < kcar;
                        if (!keep && (uint32_t)c < nk) car[c] = stage[(int32_t)tex + o0 + c];
                    }
                    acur += twr;
                    kcar = nk;
                }
            } else {
                for (uint32_t p = tid; p < tn; p += NT) {
                    const uint32_t bb = sbid[p];
                    dst[run[bb] + (p - tstart[bb])] = stage[p];
                }
                lds_barrier();
                uint32_t* st32 = (uint32_t*)stage;
#pragma unroll
                for (int r = 0; r < SK; r++)
                    if (pos[r] != 0xffffffffu) st32[pos[r]] = pl[r];
                lds_barrier();
                for (uint32_t p = tid; p < tn; p += NT) {
                    const uint32_t bb = sbid[p];
                    pdst[run[bb] + (p - tstart[bb])] = st32[p];
                }
                lds_barrier();
                for (uint32_t j = tid; j < nb; j += NT) run[j] += tcnt[j];
                lds_barrier();
            }
            // keys only: no barrier here; the next tile's first LDS writes
            // (its bucket counters) are not read by this write-out, and the
            // barrier after them orders everything else
            if (PAY) {
#pragma unroll
                for (int r = 0; r < SK; r++) { k[r] = kn[r]; pl[r] = pn[r]; }
            }
        }
        });
        __syncthreads();
    }
}

// ===========================================================================
// k_resident: one workgroup partitions a whole segment of at most RES_MAX
// keys (one work unit), with no look-back: it histograms the segment with
// its model, finds the bucket starts in LDS, scatters the keys into the
// other buffer, and writes the counts for k_scan, which classifies the
// buckets exactly as for any other segment.  The second read of the segment
// comes from the cache.
//   PAY: the scatter is stable (wave-match ranks and per-wave bucket
//   positions, tile by tile in key order), so a payload keeps the input
//   order of equal keys; without a payload one LDS atomic per key places it.
// ===========================================================================

constexpr int R_THREADS = 512;
constexpr int R_WAVES = R_THREADS / WAVE;
constexpr int RK = 8;                        // keys per thread per tile
constexpr int R_TILE = R_THREADS * RK;       // 4096 keys
constexpr int R_WKEYS = WAVE * RK;           // keys per wave per tile

template <int KIND>
__device__ __forceinline__ uint32_t rbucket(const View& v, const uint64_t* mdl, uint64_t raw, int u64) {
    return kind_bucket<KIND>(v, mdl, raw, u64, nullptr, 0);
}

template <bool PAY>
struct ResLds {
    alignas(16) uint64_t mdl[LDS_MODEL_WORDS];
    uint32_t cnt[B_MAX];
    uint32_t start[B_MAX];
    uint32_t cur[B_MAX];
    uint32_t wpos[PAY ? R_WAVES : 1][PAY ? B_MAX : 1];
    uint64_t red[R_WAVES];
    uint32_t seg;
};

// Histogram, bucket starts and the scatter of one resident segment.
template <int KIND, bool PAY>
__device__ void res_partition(const Params& P, const Seg& sg, const View& v, ResLds<PAY>& L, int lvl) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t* src = P.keys[lvl & 1];
    uint64_t* dst = P.keys[(lvl + 1) & 1];
    const uint32_t* psrc = P.pay[lvl & 1];
    uint32_t* pdst = P.pay[(lvl + 1) & 1];
    const int u64 = P.u64;
    const uint32_t n = (uint32_t)sg.n, nb = sg.nb;
    const uint64_t off = sg.off;
    for (uint32_t b = tid; b < B_MAX; b += R_THREADS) L.cnt[b] = 0;
    __syncthreads();
    // histogram
    for (uint32_t t0 = 0; t0 < n; t0 += R_TILE) {
        uint64_t k[RK];
#pragma unroll
        for (int r = 0; r < RK; r++) {
            const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
            k[r] = i < n ? src[off + i] : 0;
        }
#pragma unroll
        for (int r = 0; r < RK; r++) {
            const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
            if (i < n) atomicAdd(&L.cnt[rbucket<KIND>(v, L.mdl, k[r], u64)], 1u);
        }
    }
    __syncthreads();
    // bucket starts: exclusive scan, 2 buckets per thread
    {
        const uint32_t j0 = 2 * tid, j1 = 2 * tid + 1;
        const uint32_t c0 = j0 < nb ? L.cnt[j0] : 0u, c1 = j1 < nb ? L.cnt[j1] : 0u;
        uint64_t tot;
        const uint32_t ex = (uint32_t)block_excl_scan<R_THREADS, uint64_t>((uint64_t)(c0 + c1), L.red, &tot);
        if (j0 < nb) { L.start[j0] = ex; L.cur[j0] = ex; }
        if (j1 < nb) { L.start[j1] = ex + c0; L.cur[j1] = ex + c0; }
    }
    __syncthreads();
    // scatter into the other buffer
    const int bits = ceil_log2(nb);
    for (uint32_t t0 = 0; t0 < n; t0 += R_TILE) {
        uint64_t k[RK];
        uint32_t pl[RK], b[RK];
#pragma unroll
        for (int r = 0; r < RK; r++) {
            const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
            k[r] = i < n ? src[off + i] : 0;
            pl[r] = (PAY && i < n) ? psrc[off + i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < RK; r++) {
            const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
            b[r] = i < n ? rbucket<KIND>(v, L.mdl, k[r], u64) : 0u;
        }
        if constexpr (!PAY) {
#pragma unroll
            for (int r = 0; r < RK; r++) {
                const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
                if (i < n) dst[off + atomicAdd(&L.cur[b[r]], 1u)] = k[r];
            }
        } else {
            // stable: ranks within the wave in key order, then positions per
            // (wave, bucket) from the running cursors
            for (uint32_t j = lane; j < nb; j += WAVE) L.wpos[w][j] = 0;
            uint32_t rk[RK];
#pragma unroll
            for (int r = 0; r < RK; r++) {
                const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
                rk[r] = 0;
                if (i < n) {
                    const uint64_t peers = match_peers(b[r], bits);
                    const uint32_t below = mask_rank(peers);
                    const uint32_t before = L.wpos[w][b[r]];
                    if (below == 0) L.wpos[w][b[r]] = before + (uint32_t)__popcll(peers);
                    rk[r] = before + below;
                }
            }
            __syncthreads();
            for (uint32_t j = tid; j < nb; j += R_THREADS) {
                uint32_t acc = L.cur[j];
#pragma unroll
                for (int x = 0; x < R_WAVES; x++) {
                    const uint32_t c = L.wpos[x][j];
                    L.wpos[x][j] = acc;
                    acc += c;
                }
                L.cur[j] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < RK; r++) {
                const uint32_t i = t0 + w * R_WKEYS + r * WAVE + lane;
                if (i < n) {
                    const uint32_t pos = L.wpos[w][b[r]] + rk[r];
                    dst[off + pos] = k[r];
                    pdst[off + pos] = pl[r];
                }
            }
            __syncthreads();
        }
    }
}

template <bool PAY>
__global__ __launch_bounds__(R_THREADS) void k_resident(Params P) {
    __shared__ ResLds<PAY> L;
    const int tid = threadIdx.x;
    const int lvl = P.level;
    if (P.ctl->nres[lvl] == 0) return;  // no segment of this level is resident
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    uint64_t cur_model = 0;
    for (;;) {
        if (tid == 0) L.seg = atomicAdd(&P.ctl->rticket[lvl], 1u);
        __syncthreads();
        const uint32_t s = L.seg;
        if (s >= nseg) break;
        const Seg sg = P.segs[lvl & 1][s];
        if (!(sg.flags & SEG_RESIDENT) || (sg.flags & SEG_FAILED)) {
            __syncthreads();
            continue;
        }
        if (sg.model != cur_model) {
            load_model_lds(L.mdl, (const uint64_t*)sg.model, sg.kind, sg.flags >> 16, tid, R_THREADS);
            cur_model = sg.model;
        }
        __syncthreads();
        const View v = make_view(L.mdl, sg.kind, sg.nb, sg.win);
        switch (sg.kind) {
        case K_RMI:
            if (P.u64) res_partition<K_RMI | KIND_U64, PAY>(P, sg, v, L, lvl);
            else res_partition<K_RMI, PAY>(P, sg, v, L, lvl);
            break;
        case K_RMI_FINE:
            if (P.u64) res_partition<K_RMI_FINE | KIND_U64, PAY>(P, sg, v, L, lvl);
            else res_partition<K_RMI_FINE, PAY>(P, sg, v, L, lvl);
            break;
        case K_TREE:
        case K_TREE_FORCED: res_partition<K_TREE, PAY>(P, sg, v, L, lvl); break;
        default: res_partition<K_RADIX, PAY>(P, sg, v, L, lvl); break;
        }
        for (uint32_t b = tid; b < sg.nb; b += R_THREADS) P.counts[sg.cbase + b] = L.cnt[b];
        __syncthreads();
    }
}

}  // namespace ls

namespace ls {

#define LAUNCH(kernel, grid, block, stream, ...)                                     \
    do {                                                                             \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_reset(const Params& P, uint64_t* persist, hipStream_t st) { LAUNCH(k_reset, 1, 256, st, P, persist); }
hipError_t launch_seed(const Params& P, const uint64_t* offsets, uint64_t m, uint64_t n_single, uint32_t prebuilt,
                       const uint64_t* persist, uint32_t grid, hipStream_t st) {
    LAUNCH(k_seed, grid, 256, st, P, offsets, m, n_single, prebuilt, persist);
}
hipError_t launch_model(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_model, grid, M_THREADS, st, P); }
hipError_t launch_fit_block(const uint64_t* s, uint32_t S, int u64, uint32_t L, uint32_t B1, double* dst,
                            hipStream_t st) {
    LAUNCH(k_fit_block, 1, M_THREADS, st, s, S, u64, L, B1, dst);
}
hipError_t launch_hist(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_hist, grid, P_THREADS, st, P); }
hipError_t launch_scan(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_scan, grid, S_THREADS, st, P); }
constexpr int SC_THREADS = 1024;  // threads of a scatter workgroup (16 waves, 8 keys each per tile)

hipError_t launch_scatter(const Params& P, uint32_t grid, hipStream_t st) {
    if (P.has_pay) LAUNCH((k_scatter<true, SC_THREADS>), grid, SC_THREADS, st, P);
    LAUNCH((k_scatter<false, SC_THREADS>), grid, SC_THREADS, st, P);
}
hipError_t launch_resident(const Params& P, uint32_t grid, hipStream_t st) {
    if (P.has_pay) LAUNCH(k_resident<true>, grid, R_THREADS, st, P);
    LAUNCH(k_resident<false>, grid, R_THREADS, st, P);
}


}  // namespace ls
