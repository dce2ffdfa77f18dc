// lsort_kernels.hip -- HIP kernels of the learned sample sort for gfx950.
//
// One partition level over a list of sub-arrays ("segments") runs as
//   k_model   -> k_hist -> k_scan -> k_scatter
// and after the last level k_base sorts every small bucket in LDS.  Segments
// of one level share every launch (the batched form is the same code with
// more segments).  Buffers ping-pong between the caller's keys (index 0) and
// a temporary (index 1): level l reads buffer l&1 and writes buffer (l+1)&1;
// the base case always writes the caller's buffer.
#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {

__device__ __forceinline__ void load_model(uint64_t* dst, const uint64_t* src, uint32_t words, int tid, int nt) {
    for (uint32_t i = tid; i < words; i += nt) dst[i] = src[i];
}

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
    __shared__ uint64_t base[3];
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
        const bool seg = s < m && (prebuilt ? n >= 1 : n > P.cutoff);
        const uint32_t nt = seg ? (uint32_t)((n + TILE - 1) / TILE) : 0;
        uint64_t itot, stot, ttot;
        const uint64_t iex = block_excl_scan<256, uint64_t>(item ? 1 : 0, red64, &itot);
        const uint64_t sex = block_excl_scan<256, uint64_t>(seg ? 1 : 0, red64, &stot);
        const uint64_t tex = block_excl_scan<256, uint64_t>(nt, red64, &ttot);
        if (threadIdx.x == 0) {
            base[0] = itot ? atomicAdd(&P.ctl->nitems, (unsigned long long)itot) : 0;
            base[1] = stot ? atomicAdd(&P.ctl->nseg[0], (uint32_t)stot) : 0;
            base[2] = ttot ? atomicAdd(&P.ctl->ntile[0], (uint32_t)ttot) : 0;
        }
        __syncthreads();
        if (item) {
            uint64_t it = base[0] + iex;
            if (it < P.item_cap) {
                P.items[it] = item_pack(lo, 0, 0, (uint32_t)n);
                atomicAdd(&P.ctl->base_keys, (unsigned long long)n);
            } else {
                atomicOr(&P.ctl->overflow, OVF_ITEM);
            }
        }
        if (seg) {
            uint64_t si = base[1] + sex, t0 = base[2] + tex;
            if (si >= P.seg_cap) {
                atomicOr(&P.ctl->overflow, OVF_SEG);
            } else {
                Seg sg{};
                sg.off = lo; sg.n = n; sg.kind = K_FRESH; sg.tile0 = (uint32_t)t0; sg.ntiles = nt;
                sg.flags = prebuilt ? SEG_PREBUILT : 0;
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
    // per-leaf least squares (thread j)
    double a = 0, b = 0, pmin = 0, pmax = -INFINITY;
    uint32_t lo = 0, hi = 0;
    if ((uint32_t)tid < L) {
        lo = lstart[tid]; hi = lstart[tid + 1];
        if (hi > lo) {
            double cnt = (double)(hi - lo), s = 0;
            for (uint32_t i = lo; i < hi; i++) { double x; key_x(key_unord(smp[i], u64), u64, x); s += x; }
            double lmx = s / cnt;
            double lmy = ((double)lo + (double)hi - 1.0) / (2.0 * Sd);
            double lxx = 0, lxy = 0;
            for (uint32_t i = lo; i < hi; i++) {
                double x; key_x(key_unord(smp[i], u64), u64, x);
                double dx = x - lmx, dy = (double)i / Sd - lmy;
                lxx += dx * dx; lxy += dx * dy;
            }
            a = lxx > 0 ? lxy / lxx : 0.0;
            if (a < 0) a = 0;
            b = lmy - a * lmx;
            double x0, x1;
            key_x(key_unord(smp[lo], u64), u64, x0);
            key_x(key_unord(smp[hi - 1], u64), u64, x1);
            pmin = a * x0 + b;
            pmax = a * x1 + b;
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
    for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        Seg sg = P.segs[lvl & 1][s];
        uint32_t kind = sg.kind, nb = sg.nb, words = sg.flags >> 16;
        uint64_t model = sg.model;
        const bool have = (sg.flags & SEG_PREBUILT) || kind == K_RMI_FINE || kind == K_MLP_FINE;
        if (!have && kind == K_RADIX) {
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
        } else if (!have) {
            // sample (Sec. 2.2: ~1% random sample; Alg. 5 Sample) and sort it
            const uint64_t n = sg.n;
            uint32_t Bt = min(P.tree_buckets, max(2u, floor_pow2((uint32_t)min<uint64_t>(n / 16, 1u << 30))));
            uint64_t want = (uint64_t)ceil(P.sample_frac * (double)n);
            uint64_t floor_s = min<uint64_t>(n, 16ull * Bt);
            uint32_t S = (uint32_t)min<uint64_t>(S_LDS, max<uint64_t>(want, max<uint64_t>(floor_s, 2)));
            uint32_t P2 = 1u << ceil_log2(S);
            const uint64_t sseed = splitmix64_at(P.seed, (sg.off << 6) | (uint64_t)lvl);
            for (uint32_t k = tid; k < P2; k += M_THREADS)
                smp[k] = k < S ? key_ord(src[sg.off + sample_index(sseed, k, n)], u64) : ~0ull;
            __syncthreads();
            bitonic_keys<M_THREADS>(smp, P2);
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
            } else {
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
            LevelStats& st = P.ctl->lv[lvl];
            if (kind == K_RMI || kind == K_RMI_FINE || kind == K_MLP || kind == K_MLP_FINE) atomicAdd(&st.learned, 1ull);
            else if (kind == K_RADIX) atomicAdd(&st.radix, 1ull);
            else atomicAdd(&st.tree, 1ull);
        }
        __syncthreads();
        if (!(shv[2] & SEG_FAILED))
            for (uint32_t b = tid; b < nb; b += M_THREADS) P.counts[shv[0] + b] = 0;
        // this segment's tile descriptors (every reserved slot below capacity)
        for (uint32_t i = tid; i < sg.ntiles; i += M_THREADS)
            if ((uint64_t)sg.tile0 + i < P.tile_cap) P.tiles[lvl & 1][sg.tile0 + i] = Tile{s, i};
        __syncthreads();
    }
}

// ===========================================================================
// k_hist: model evaluation fused with an LDS-private bucket histogram
// ===========================================================================

__global__ __launch_bounds__(P_THREADS) void k_hist(Params P) {
    __shared__ uint64_t mdl[MODEL_WORDS];
    __shared__ uint32_t h[B_MAX];
    const int tid = threadIdx.x, lane = tid & 63;
    const int lvl = P.level;
    const uint32_t ntile = min(P.ctl->ntile[lvl], (uint32_t)P.tile_cap);
    const uint32_t chunk = (ntile + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * chunk, t1 = min(t0 + chunk, ntile);
    const uint64_t* src = P.keys[lvl & 1];
    const int u64 = P.u64;
    uint32_t cur = 0xffffffffu;
    uint64_t cur_model = 0;
    Seg sg{};
    View v{};
    bool skip = false;
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    for (uint32_t t = t0; t < t1; t++) {
        Tile td = P.tiles[lvl & 1][t];
        if (td.seg >= nseg) continue;
        if (td.seg != cur) {
            if (cur != 0xffffffffu && !skip) {
                __syncthreads();
                for (uint32_t b = tid; b < sg.nb; b += P_THREADS)
                    if (h[b]) atomicAdd(&P.counts[sg.cbase + b], (unsigned long long)h[b]);
            }
            __syncthreads();
            sg = P.segs[lvl & 1][td.seg];
            cur = td.seg;
            skip = (sg.flags & SEG_FAILED) != 0;
            if (!skip && sg.model != cur_model) {
                load_model(mdl, (const uint64_t*)sg.model, sg.flags >> 16, tid, P_THREADS);
                cur_model = sg.model;
            }
            for (uint32_t b = tid; b < B_MAX; b += P_THREADS) h[b] = 0;
            __syncthreads();
            v = make_view(mdl, sg.kind, sg.nb, sg.win);
        }
        if (skip) continue;
        const uint64_t base = sg.off + (uint64_t)td.idx * TILE;
        const uint64_t tn = min<uint64_t>(TILE, sg.n - (uint64_t)td.idx * TILE);
        const bool aggregate = v.kind == K_TREE || v.kind == K_TREE_FORCED || v.kind == K_RADIX;
        const int bits = ceil_log2(sg.nb);
#pragma unroll 4
        for (int r = 0; r < KPT; r++) {
            uint32_t i = r * P_THREADS + tid;
            if (i < tn) {
                uint32_t b = view_bucket(v, mdl, src[base + i], u64, P.ids, base + i);
                if (aggregate) {
                    // wave-aggregated: one LDS add per distinct bucket in the wave
                    uint64_t peers = match_peers(b, bits);
                    if (mask_rank(peers) == 0) atomicAdd(&h[b], (uint32_t)__popcll(peers));
                } else {
                    uint32_t b0 = __builtin_amdgcn_readfirstlane(b);
                    uint64_t act = __ballot(1), same = __ballot(b == b0);
                    if (same == act) {
                        if (mask_rank(act) == 0) atomicAdd(&h[b0], (uint32_t)__popcll(act));
                    } else {
                        atomicAdd(&h[b], 1u);
                    }
                }
            }
        }
        (void)lane;
    }
    if (cur != 0xffffffffu && !skip) {
        __syncthreads();
        for (uint32_t b = tid; b < sg.nb; b += P_THREADS)
            if (h[b]) atomicAdd(&P.counts[sg.cbase + b], (unsigned long long)h[b]);
    }
}

// ===========================================================================
// k_scan: bucket starts and classification of every bucket (one WG / segment)
// ===========================================================================

constexpr int S_THREADS = 1024;

__global__ __launch_bounds__(S_THREADS) void k_scan(Params P) {
    __shared__ uint64_t red64[S_THREADS / 64];
    __shared__ uint8_t eqb[B_MAX];
    __shared__ uint64_t resv[3];
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
        uint64_t c = (uint32_t)tid < nb ? P.counts[sg.cbase + tid] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan<S_THREADS, uint64_t>(c, red64, &tot);
        uint64_t start = sg.off + ex;
        if ((uint32_t)tid < nb) P.counts[sg.cbase + nb + tid] = start;
        // which buckets hold a single value
        eqb[tid] = 0;
        __syncthreads();
        uint32_t log2B2 = 0;
        bool fine_ok = false;
        if (sg.kind == K_TREE || sg.kind == K_TREE_FORCED) {
            const TreeModel* h = (const TreeModel*)sg.model;
            const uint16_t* lut = (const uint16_t*)((const uint64_t*)sg.model + 2 + h->m);
            for (uint32_t u = tid; u < h->m; u += S_THREADS) {
                uint16_t e = lut[u + 1];
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
        // action of this bucket: 0 nothing, 1 copy items, 2 base item, 3..6 child of kind
        // K_RADIX / fine / K_TREE_FORCED / K_FRESH
        uint32_t act = 0;
        uint64_t stat = 0;  // 12-bit fields: empty, equality, base, recurse
        if ((uint32_t)tid < nb && c > 0) {
            if (eqb[tid] || c == 1) {
                stat = 1ull << 12;
                act = q == 1 ? 1 : 0;  // finished; only a run left in the temporary moves
            } else if (c <= P.cutoff || ((uint32_t)lvl + 1 >= P.max_levels && c <= (uint64_t)C_MAX)) {
                // at the depth cap every bucket the base case can hold goes there,
                // so range-radix levels only ever see more than C_MAX keys (8 bits each)
                stat = 1ull << 24;
                act = 2;
            } else {
                const bool oversized = (double)c > P.fallback_ratio * expected;
                stat = 1ull << 36;
                if ((uint32_t)lvl + 1 >= P.max_levels) act = 3;
                else if (fine_ok && !oversized && (4ull << log2B2) <= c) act = 4;
                else if (oversized && !(P.flags & 0x1u)) act = 5;
                else act = 6;
            }
        } else if ((uint32_t)tid < nb) {
            stat = 1ull;
        }
        const uint64_t nitem = act == 1 ? (c + COPY_CHUNK - 1) / COPY_CHUNK : (act == 2 ? 1 : 0);
        const uint32_t ntl = act >= 3 ? (uint32_t)((c + TILE - 1) / TILE) : 0;
        // one reservation per list for the whole workgroup
        uint64_t itot, ctot, ttot;
        const uint64_t iex = block_excl_scan<S_THREADS, uint64_t>(nitem, red64, &itot);
        const uint64_t cex = block_excl_scan<S_THREADS, uint64_t>(act >= 3 ? 1 : 0, red64, &ctot);
        const uint64_t tex = block_excl_scan<S_THREADS, uint64_t>(ntl, red64, &ttot);
        const uint64_t ck = block_sum<S_THREADS, uint64_t>(act == 1 ? c : 0, red64);
        const uint64_t bk = block_sum<S_THREADS, uint64_t>(act == 2 ? c : 0, red64);
        const uint64_t nfb = block_sum<S_THREADS, uint64_t>(act == 5 ? 1 : 0, red64);
        const uint64_t ncp = block_sum<S_THREADS, uint64_t>(act == 1 ? nitem : 0, red64);
        if (tid == 0) {
            resv[0] = itot ? atomicAdd(&P.ctl->nitems, (unsigned long long)itot) : 0;
            resv[1] = ctot ? atomicAdd(&P.ctl->nseg[lvl + 1], (uint32_t)ctot) : 0;
            resv[2] = ttot ? atomicAdd(&P.ctl->ntile[lvl + 1], (uint32_t)ttot) : 0;
            if (ck) {
                atomicAdd(&P.ctl->copy_keys, (unsigned long long)ck);
                atomicAdd(&P.ctl->ncopy, (unsigned long long)ncp);
            }
            if (bk) atomicAdd(&P.ctl->base_keys, (unsigned long long)bk);
        }
        __syncthreads();
        for (uint64_t k = 0; k < nitem; k++) {
            const uint64_t it = resv[0] + iex + k;
            if (it >= P.item_cap) { atomicOr(&P.ctl->overflow, OVF_ITEM); break; }
            const uint64_t sz = act == 1 ? min<uint64_t>(COPY_CHUNK, c - k * COPY_CHUNK) : c;
            P.items[it] = item_pack(start + k * COPY_CHUNK, act == 1 ? 1u : q, act == 1 ? 1u : 0u, (uint32_t)sz);
        }
        if (act >= 3) {
            const uint64_t si = resv[1] + cex, t0 = resv[2] + tex;
            if (si < P.seg_cap) {
                Seg ch{};
                ch.off = start; ch.n = c; ch.ntiles = ntl; ch.tile0 = (uint32_t)t0;
                ch.kind = act == 3 ? K_RADIX : act == 4 ? (sg.kind == K_RMI ? K_RMI_FINE : K_MLP_FINE)
                        : act == 5 ? K_TREE_FORCED : K_FRESH;
                if (act == 4) {
                    ch.model = sg.model;
                    ch.nb = 1u << log2B2;
                    ch.win = (uint32_t)tid << log2B2;
                    ch.flags = sg.flags & 0xffff0000u;  // model words
                }
                if (t0 + ntl > P.tile_cap) { atomicOr(&P.ctl->overflow, OVF_TILE); ch.flags |= SEG_FAILED; }
                P.segs[q][si] = ch;  // k_model of the next level writes its tile descriptors
            } else {
                atomicOr(&P.ctl->overflow, OVF_SEG);
                for (uint32_t i = 0; i < ntl; i++)  // keep the tile list free of stale slots
                    if (t0 + i < P.tile_cap) P.tiles[q][t0 + i] = Tile{0xffffffffu, 0};
            }
        }
        // statistics
        const uint64_t sc = block_sum<S_THREADS, uint64_t>(stat, red64);
        uint64_t mx = block_max<S_THREADS, uint64_t>(c, red64);
        if (tid == 0) {
            const uint64_t m12 = 4095;
            atomicAdd(&st.segments, 1ull);
            atomicAdd(&st.keys, (unsigned long long)sg.n);
            atomicAdd(&st.buckets, (unsigned long long)nb);
            atomicMax(&st.max_bucket, (unsigned long long)mx);
            atomicMax(&st.max_ratio_x1000, (unsigned long long)(1000.0 * (double)mx / expected));
            atomicAdd(&st.empty, (unsigned long long)(sc & m12));
            atomicAdd(&st.equality, (unsigned long long)((sc >> 12) & m12));
            atomicAdd(&st.base, (unsigned long long)((sc >> 24) & m12));
            atomicAdd(&st.recurse, (unsigned long long)((sc >> 36) & m12));
            atomicAdd(&st.fallback, (unsigned long long)nfb);
        }
        __syncthreads();
    }
}

// ===========================================================================
// k_scatter: stable in-tile rank, decoupled look-back over tiles, LDS-staged
// coalesced write of each bucket's run (one tile of 8192 keys per iteration)
// ===========================================================================

__device__ __forceinline__ uint64_t st_load(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store(unsigned long long* p, uint64_t v) {
    __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(P_THREADS) void k_scatter(Params P) {
    __shared__ uint64_t mdl[MODEL_WORDS];
    __shared__ uint64_t stage[TILE];
    __shared__ uint16_t sbid[TILE];
    __shared__ uint16_t wcnt[P_WAVES][B_MAX];
    __shared__ uint16_t tcnt[B_MAX];
    __shared__ uint16_t tstart[B_MAX];
    __shared__ uint64_t goff[B_MAX];
    __shared__ uint32_t sh_t;
    __shared__ uint64_t red64[P_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lvl = P.level;
    const uint32_t ntile = min(P.ctl->ntile[lvl], (uint32_t)P.tile_cap);
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    const uint64_t tag = ((uint64_t)(P.persist[0] * MAXL + lvl)) << ST_TAG_SHIFT;
    const uint64_t* src = P.keys[lvl & 1];
    uint64_t* dst = P.keys[(lvl + 1) & 1];
    const uint32_t* psrc = P.pay[lvl & 1];
    uint32_t* pdst = P.pay[(lvl + 1) & 1];
    const int u64 = P.u64, has_pay = P.has_pay;
    uint64_t cur_model = 0;
    for (;;) {
        if (tid == 0) sh_t = atomicAdd(&P.ctl->ticket[lvl], 1u);
        __syncthreads();
        const uint32_t t = sh_t;
        if (t >= ntile) break;
        const Tile td = P.tiles[lvl & 1][t];
        if (td.seg >= nseg) { __syncthreads(); continue; }
        const Seg sg = P.segs[lvl & 1][td.seg];
        if (sg.flags & SEG_FAILED) { __syncthreads(); continue; }
        if (sg.model != cur_model) {
            load_model(mdl, (const uint64_t*)sg.model, sg.flags >> 16, tid, P_THREADS);
            cur_model = sg.model;
            __syncthreads();
        }
        const View v = make_view(mdl, sg.kind, sg.nb, sg.win);
        const uint32_t nb = sg.nb;
        const int bits = ceil_log2(nb);
        const uint64_t base = sg.off + (uint64_t)td.idx * TILE;
        const uint32_t tn = (uint32_t)min<uint64_t>(TILE, sg.n - (uint64_t)td.idx * TILE);
        // load: wave w owns keys [w*1024, (w+1)*1024) of the tile, 64 per round
        uint64_t k[KPT];
        uint32_t b[KPT];
        uint32_t pl[KPT];
#pragma unroll
        for (int r = 0; r < KPT; r++) {
            uint32_t i = w * WAVE_KEYS + r * WAVE + lane;
            k[r] = i < tn ? src[base + i] : 0;
            pl[r] = (has_pay && i < tn) ? psrc[base + i] : 0;
        }
        for (uint32_t j = lane; j < nb; j += WAVE) wcnt[w][j] = 0;
#pragma unroll
        for (int r = 0; r < KPT; r++) {
            uint32_t i = w * WAVE_KEYS + r * WAVE + lane;
            b[r] = i < tn ? view_bucket(v, mdl, k[r], u64, P.ids, base + i) : 0;
        }
        // stable rank within the wave: rounds in key order, lanes in key order
        uint32_t rk[KPT];
#pragma unroll
        for (int r = 0; r < KPT; r++) {
            uint32_t i = w * WAVE_KEYS + r * WAVE + lane;
            rk[r] = 0;
            if (i < tn) {
                uint64_t peers = match_peers(b[r], bits);
                uint32_t below = mask_rank(peers);
                uint32_t before = wcnt[w][b[r]];
                if (below == 0) wcnt[w][b[r]] = (uint16_t)(before + __popcll(peers));
                rk[r] = before + below;
            }
        }
        __syncthreads();
        // per bucket: exclusive prefix over waves (in place) and tile count
        for (uint32_t j = tid; j < nb; j += P_THREADS) {
            uint32_t run = 0;
#pragma unroll
            for (int x = 0; x < P_WAVES; x++) {
                uint32_t c = wcnt[x][j];
                wcnt[x][j] = (uint16_t)run;
                run += c;
            }
            tcnt[j] = (uint16_t)run;
        }
        __syncthreads();
        // tile-local bucket starts: exclusive scan over buckets, 2 per thread
        {
            uint32_t j0 = 2 * tid, j1 = 2 * tid + 1;
            uint64_t c0 = j0 < nb ? tcnt[j0] : 0, c1 = j1 < nb ? tcnt[j1] : 0;
            uint64_t ex = block_excl_scan<P_THREADS, uint64_t>(c0 + c1, red64, nullptr);
            if (j0 < nb) tstart[j0] = (uint16_t)ex;
            if (j1 < nb) tstart[j1] = (uint16_t)(ex + c0);
        }
        // decoupled look-back (Merrill & Garland): publish this tile's counts
        // for every bucket first, then add predecessors' aggregates until an
        // inclusive prefix is found.  The first tile of a segment publishes
        // its inclusive prefix at once, so every wait ends.
        unsigned long long* row = P.status + sg.sbase + (uint64_t)td.idx * nb;
        for (uint32_t j = tid; j < nb; j += P_THREADS)
            st_store(row + j, tag | (td.idx == 0 ? ST_PREFIX : ST_AGG) | (uint64_t)tcnt[j]);
        for (uint32_t j = tid; j < nb; j += P_THREADS) {
            uint64_t excl = 0;
            if (td.idx > 0) {
                int64_t pk = (int64_t)td.idx - 1;
                for (;;) {
                    uint64_t wv = st_load(P.status + sg.sbase + (uint64_t)pk * nb + j);
                    uint64_t hdr = wv & ~ST_LOW_MASK;
                    if (hdr == (tag | ST_PREFIX)) { excl += wv & ST_VALUE_MASK; break; }
                    if (hdr == (tag | ST_AGG)) { excl += wv & ST_VALUE_MASK; pk--; continue; }
                    __builtin_amdgcn_s_sleep(1);
                }
                st_store(row + j, tag | ST_PREFIX | (excl + tcnt[j]));
            }
            goff[j] = P.counts[sg.cbase + nb + j] + excl;
        }
        __syncthreads();
        // stage keys grouped by bucket (stable positions)
        uint32_t pos[KPT];
#pragma unroll
        for (int r = 0; r < KPT; r++) {
            uint32_t i = w * WAVE_KEYS + r * WAVE + lane;
            pos[r] = 0xffffffffu;
            if (i < tn) {
                uint32_t p = tstart[b[r]] + wcnt[w][b[r]] + rk[r];
                pos[r] = p;
                stage[p] = k[r];
                sbid[p] = (uint16_t)b[r];
            }
        }
        __syncthreads();
        for (uint32_t p = tid; p < tn; p += P_THREADS) {
            uint32_t bb = sbid[p];
            dst[goff[bb] + (p - tstart[bb])] = stage[p];
        }
        if (has_pay) {
            __syncthreads();
            uint32_t* st32 = (uint32_t*)stage;
#pragma unroll
            for (int r = 0; r < KPT; r++)
                if (pos[r] != 0xffffffffu) st32[pos[r]] = pl[r];
            __syncthreads();
            for (uint32_t p = tid; p < tn; p += P_THREADS) {
                uint32_t bb = sbid[p];
                pdst[goff[bb] + (p - tstart[bb])] = st32[p];
            }
        }
        __syncthreads();
    }
}

// ===========================================================================
// k_base: in-LDS stable sort of every small bucket; copies of finished runs
// ===========================================================================

constexpr int BASE_THREADS = 256;

__global__ __launch_bounds__(BASE_THREADS) void k_base(Params P) {
    __shared__ uint64_t sk[C_MAX];
    __shared__ uint16_t si[C_MAX];
    __shared__ uint32_t sp[C_MAX];
    const int tid = threadIdx.x;
    const uint64_t nitems = min<unsigned long long>(P.ctl->nitems, P.item_cap);
    const int u64 = P.u64, has_pay = P.has_pay;
    uint64_t* out = P.keys[0];
    uint32_t* pout = P.pay[0];
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint64_t wd = P.items[it];
        const uint64_t off = wd >> 18;
        const uint32_t srcb = (wd >> 17) & 1u, copy = (wd >> 16) & 1u;
        const uint32_t size = (uint32_t)(wd & 0xffffu) + 1;
        const uint64_t* in = P.keys[srcb];
        const uint32_t* pin = P.pay[srcb];
        if (copy) {
            if (srcb)
                for (uint32_t i = tid; i < size; i += BASE_THREADS) {
                    out[off + i] = in[off + i];
                    if (has_pay) pout[off + i] = pin[off + i];
                }
            continue;
        }
        const uint32_t P2 = 1u << ceil_log2(size);
        for (uint32_t i = tid; i < P2; i += BASE_THREADS) {
            sk[i] = i < size ? key_ord(in[off + i], u64) : ~0ull;
            if (has_pay) {
                si[i] = (uint16_t)i;
                if (i < size) sp[i] = pin[off + i];
            }
        }
        __syncthreads();
        if (has_pay) bitonic_pairs<BASE_THREADS>(sk, si, P2);
        else bitonic_keys<BASE_THREADS>(sk, P2);
        for (uint32_t i = tid; i < size; i += BASE_THREADS) {
            out[off + i] = key_unord(sk[i], u64);
            if (has_pay) pout[off + i] = sp[si[i]];
        }
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
hipError_t launch_hist(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_hist, grid, P_THREADS, st, P); }
hipError_t launch_scan(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_scan, grid, S_THREADS, st, P); }
hipError_t launch_scatter(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_scatter, grid, P_THREADS, st, P); }
hipError_t launch_base(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_base, grid, BASE_THREADS, st, P); }

}  // namespace ls
