// lsort_api.hip -- host planner and C ABI of liblsort.
//
// The planner lays out one workspace per call (temporary key/payload
// buffers, per-level segment and tile lists, base-case items, bucket counts,
// look-back status words, model arenas), enqueues the fixed kernel sequence
// of each partition level on the caller's stream and, unless asked to launch
// a fixed number of levels, reads back one counter per level to stop when no
// sub-array needs another level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lsort.h"
#include "lsort_internal.hpp"
#include "lsort_kernels.hpp"

namespace ls {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err = "";

static ls_status fail(ls_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(LS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------
struct Opts {
    uint32_t model, buckets, leaves, tree_buckets, cutoff, max_levels, flags;
    double sample_frac, fallback_ratio;
    uint64_t seed;
    uint32_t mlp_steps, mlp_sample;
    float mlp_lr;
    uint32_t tile;   // keys per work unit of the first level's partition passes
    uint32_t balance_pct;  // large array's first level: tree instead of the RMI when oversized buckets hold
                           // more than this share of the sample (100: never)
};

// ---------------------------------------------------------------------------
// tuning table (ls_autotune / ls_load_tuning): per size class -- the decimal
// order of magnitude of the average array size n / m -- the bucket count,
// base-case cutoff and splitter fan-out that ran fastest on this device
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

int report_error(int status, const char* msg) { return fail((ls_status)status, msg); }

void tuning_install(const std::vector<TuneEntry>& t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = t;
}

static int size_class(uint64_t n, uint64_t m) {
    const double avg = (double)n / (double)std::max<uint64_t>(m, 1);
    return (int)std::floor(std::log10(std::max(avg, 1.0)) + 1e-9);
}

// Fields the caller left zero take the table's values for the call's class
// (the nearest class in the table when its own is missing; ties go to the
// smaller class).
static void apply_tuning(const ls_options* o, Opts& r, uint64_t n, uint64_t m) {
    if (n == 0 || (o && !(o->flags & LS_FLAG_TUNED))) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return;
    const int c = size_class(n, m);
    const TuneEntry* best = &g_tune[0];
    for (const TuneEntry& e : g_tune)
        if (std::abs(e.cls - c) < std::abs(best->cls - c)) best = &e;
    if (!o || !o->buckets) r.buckets = best->buckets;
    if (!o || !o->cutoff) r.cutoff = best->cutoff;
    if (!o || !o->tree_buckets) r.tree_buckets = best->tree_buckets;
    if (!o || !o->tile) r.tile = best->tile;
}

static ls_status normalize(const ls_options* o, Opts& r, uint64_t n = 0, uint64_t m = 0) {
    // cutoff: measured on 1e8-key arrays, 1024 (two-level buckets of ~400 keys,
    // 16-lane group sorts) beats 512 by 1.5 %; on the 10,000-array segmented
    // workload 512 is 5 % faster
    r.model = LS_MODEL_AUTO; r.buckets = 1000; r.leaves = 1000; r.tree_buckets = 256; r.cutoff = m > 1 ? 512 : 1024;
    r.max_levels = 16; r.flags = LS_FLAG_SYNC_LEVELS; r.sample_frac = 0.01; r.fallback_ratio = 2.0; r.seed = 0x5EED;
    r.mlp_steps = 200; r.mlp_sample = 1000000; r.mlp_lr = 3e-3f;
    r.tile = UNIT;
    // the balance judge: on every law measured at 1e8 keys it changes nothing
    // but the 70/20/10 piecewise law's first level, which the tree takes
    // (3.4 ms instead of 4.2 ms; at 1e9 keys 32.9 ms against 33.1 ms)
    r.balance_pct = 50;
    if (!o) {
        apply_tuning(o, r, n, m);
        return LS_OK;
    }
    if (o->struct_size != sizeof(ls_options)) return fail(LS_EINVAL, "ls_options.struct_size mismatch");
    if (o->model > LS_MODEL_SPLITTER) return fail(LS_EINVAL, "unknown model");
    r.model = o->model;
    if (o->buckets) r.buckets = o->buckets;
    if (o->leaves) r.leaves = o->leaves;
    if (o->tree_buckets) r.tree_buckets = o->tree_buckets;
    if (o->cutoff) r.cutoff = o->cutoff;
    if (o->max_levels) r.max_levels = o->max_levels;
    if (o->flags) r.flags = o->flags;
    if (o->sample_frac > 0) r.sample_frac = o->sample_frac;
    if (o->fallback_ratio > 0) r.fallback_ratio = o->fallback_ratio;
    if (o->seed) r.seed = o->seed;
    if (o->mlp_steps) r.mlp_steps = o->mlp_steps;
    if (o->mlp_sample) r.mlp_sample = o->mlp_sample;
    if (o->mlp_lr > 0) r.mlp_lr = o->mlp_lr;
    if (o->tile) r.tile = o->tile;
    if (o->balance_pct) r.balance_pct = o->balance_pct;
    if (r.balance_pct > 100) return fail(LS_EINVAL, "balance_pct must be in [1, 100]");
    apply_tuning(o, r, n, m);
    {
        bool ok = false;
        for (uint32_t s = 0; s <= USHIFT_MAX; s++) ok |= r.tile == ((uint32_t)UNIT << s);
        if (!ok) return fail(LS_EINVAL, "tile must be 32768 << k keys, k in [0, 4]");
    }
    if (r.buckets < 2 || r.buckets > B_MAX) return fail(LS_EINVAL, "buckets must be in [2, 1024]");
    if (r.leaves < 2 || r.leaves > L_MAX) return fail(LS_EINVAL, "leaves must be in [2, 1024]");
    if (r.tree_buckets < 2 || r.tree_buckets > 512 || (r.tree_buckets & (r.tree_buckets - 1)))
        return fail(LS_EINVAL, "tree_buckets must be a power of two in [2, 512]");
    if (r.cutoff < 1 || r.cutoff > C_MAX) return fail(LS_EINVAL, "cutoff must be in [1, 4096]");
    if (r.max_levels < 1 || r.max_levels > MAXL - 9) return fail(LS_EINVAL, "max_levels must be in [1, 23]");
    if (r.sample_frac > 1.0) return fail(LS_EINVAL, "sample_frac must be in (0, 1]");
    if (r.mlp_steps > 100000) return fail(LS_EINVAL, "mlp_steps must be at most 100000");
    return LS_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static inline uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

struct Layout {
    uint64_t n, m;
    int has_pay;
    uint64_t seg_cap, tile_cap, item_cap, big_cap, counts_cap, status_cap, arena_cap, item_b_cap, item_c_cap, merge_cap;
    uint64_t item_m_cap = 0, o_items_m = 0;  // model-based counting-sort items (large single array)
    uint64_t o_persist, o_ctl, o_tmp, o_tmppay, o_ids, o_segs[2], o_tiles[2], o_items, o_bigs, o_items_b, o_items_c, o_merges, o_counts, o_status,
        o_arena[2], o_bigmodel, o_part, o_leaf, o_flag, o_sample, o_nested, o_mlp, o_mlp_t, o_mlp_y, o_bstart;
    uint64_t S_big;       // large-path sample size (0: none)
    uint64_t mlp_S;       // MLP training-set size (0: no MLP training)
    uint64_t mlp_stride;  // training set = every mlp_stride-th point of the sorted sample
    uint64_t bytes;
    std::vector<Layout> nested;  // sorting the large-path sample
    // key types / payload width mapped onto the engine's (lsort_types.hip):
    // widened float32 keys, original indices, saved 64-bit payload
    uint64_t o_wide = 0, o_idx = 0, o_save = 0;
    // MLP training by regions: prefix moments of the training set, block totals
    uint64_t o_mlp_mom = 0, o_mlp_bsum = 0;
};

// Prefix moments of an MLP training set of S points at the end of a layout.
static void plan_mlp_moments(Layout& L, uint64_t S, uint64_t& o_) {
    L.o_mlp_mom = o_;
    o_ += align256((S + 1) * MOM_W * 16);
    L.o_mlp_bsum = o_;
    o_ += align256(((S + MOM_BLOCK - 1) / MOM_BLOCK) * MOM_W * 16);
}

// The MLP-rooted model is built only on the large-array path, and there for
// any array the policy could give a learned model (n >= 1e5).
static bool mlp_first_level(uint64_t n, uint64_t m, const Opts& o) {
    return o.model == LS_MODEL_MLP && m == 1 && n >= 100000;
}

static uint64_t big_sample_size(uint64_t n, uint64_t m, const Opts& o) {
    if (m != 1) return 0;
    uint64_t S = (uint64_t)std::ceil(o.sample_frac * (double)n);
    if (mlp_first_level(n, m, o)) return std::min<uint64_t>(n, std::max<uint64_t>(S, 4096));
    return S > (uint64_t)S_LDS ? S : 0;
}

// Optimiser state of MLP training inside the workspace area o_mlp.
struct MlpState {
    float *p, *m, *v, *best, *scale, *partial, *best_loss;
    unsigned int* done;
    double* lo_inv;
};
constexpr uint64_t MLP_VEC_BYTES = 4ull * (MLP_NP + 3);  // 324 floats: 16-byte multiple
constexpr uint64_t MLP_STATE_BYTES = 5 * MLP_VEC_BYTES + 4ull * MLP_G * MLP_ACC + 64;
static MlpState mlp_state(uint8_t* base, const Layout& L) {
    uint8_t* b = base + L.o_mlp;
    const uint64_t tail = 5 * MLP_VEC_BYTES + 4ull * MLP_G * MLP_ACC;  // 8-byte aligned
    MlpState s;
    s.p = (float*)b;
    s.m = (float*)(b + MLP_VEC_BYTES);
    s.v = (float*)(b + 2 * MLP_VEC_BYTES);
    s.best = (float*)(b + 3 * MLP_VEC_BYTES);
    s.scale = (float*)(b + 4 * MLP_VEC_BYTES);
    s.partial = (float*)(b + 5 * MLP_VEC_BYTES);
    s.done = (unsigned int*)(b + tail);
    s.best_loss = (float*)(b + tail + 4);
    s.lo_inv = (double*)(b + tail + 16);
    return s;
}

// Extra regions at the end of a sort's workspace for the key types and the
// payload width the engine does not handle natively.
static void plan_types(Layout& L, uint64_t n, ls_dtype dtype, int pay64) {
    if (dtype == LS_F32) { L.o_wide = L.bytes; L.bytes += align256(n * 8); }
    if (pay64) {
        L.o_idx = L.bytes; L.bytes += align256(n * 4);
        L.o_save = L.bytes; L.bytes += align256(n * 8);
    }
}

// Options of the engine run that sorts a large first level's sample.  The
// sample's own model only has to split the sample: a 0.4% sub-sample (4096
// keys for a 1e6-key sample) keeps its one-workgroup sort short.
static Opts nested_opts(const Opts& o) {
    Opts r = o;
    r.flags = (o.flags & LS_FLAG_FIXED_LEVELS) ? o.flags : ((o.flags & ~(uint32_t)LS_FLAG_FIXED_LEVELS) | LS_FLAG_SYNC_LEVELS);
    r.model = o.model == LS_MODEL_SPLITTER ? LS_MODEL_SPLITTER : LS_MODEL_AUTO;
    r.sample_frac = 0.002;
    r.tile = UNIT;
    return r;
}

static Layout plan(uint64_t n, uint64_t m, int has_pay, const Opts& o) {
    Layout L{};
    L.n = n; L.m = m; L.has_pay = has_pay;
    const uint64_t C = o.cutoff;
    L.seg_cap = std::max<uint64_t>(m, n / (C + 1)) + 16;
    // (a single array of at most SMALL_UNIT_N keys: units of one tile)
    const uint64_t small_units = m == 1 && n <= SMALL_UNIT_N ? n / TILE + 1 : 0;
    L.tile_cap = n / UNIT + small_units + L.seg_cap + 16;
    L.item_cap = n + m + 64;        // small items hold >= 1 key
    L.big_cap = n / 2 + m + 64;     // large items > 512 keys, copy runs >= 2 keys
    L.item_b_cap = n / (GROUP_SMALL_MAX + 1) + m + 64;  // items of 129..256 keys and of 513..1024
    // keys only: items of 1025..2048 keys, and the 2048-key chunks of items of
    // 2049..8192 (at most 2 per 2049 keys: <= n / 1024); with a payload:
    // items and 1024-key chunks of 513..8192-key items (<= n / 512)
    L.item_c_cap = n / SMALL_MAX + m + 64;
    L.merge_cap = n / (PAIR_CHUNK + 1) + m + 64;  // items of more than one chunk
    // Bucket counts per level: a segment gets at most n_seg / 4 buckets (at
    // least 2), except one first-level segment whose model the caller gives
    // (up to B_MAX).  Look-back words: tiles x buckets of each segment.
    L.counts_cap = 2 * (n / 4 + 2 * L.seg_cap + B_MAX) + 64;
    L.status_cap = (n / UNIT + small_units) * B_MAX + n / 4 + 2 * L.seg_cap + 2 * B_MAX + 64;
    L.arena_cap = (n / 100000 + m + 2) * (8ull * MODEL_WORDS + 16) + (uint64_t)(0.7 * (double)n) + L.seg_cap * 32 + 65536;
    uint64_t o_ = 0;
    auto take = [&](uint64_t bytes) { uint64_t r = o_; o_ += align256(bytes); return r; };
    L.o_persist = take(256);
    L.o_ctl = take(sizeof(Ctl));
    L.o_tmp = take(n * 8);
    L.o_tmppay = has_pay ? take(n * 4) : 0;
    L.o_ids = 0;
    L.o_segs[0] = take(L.seg_cap * sizeof(Seg));
    L.o_segs[1] = take(L.seg_cap * sizeof(Seg));
    L.o_tiles[0] = take(L.tile_cap * sizeof(Tile));
    L.o_tiles[1] = take(L.tile_cap * sizeof(Tile));
    L.o_items = take(L.item_cap * 8);
    L.o_bigs = take(L.big_cap * 8);
    L.o_items_b = take(L.item_b_cap * 8);
    L.o_items_c = take(L.item_c_cap * 8);
    L.o_merges = take(L.merge_cap * 8);
    L.o_counts = take(L.counts_cap * 8);
    L.o_status = take(L.status_cap * 8);
    L.o_arena[0] = take(L.arena_cap);
    L.o_arena[1] = take(L.arena_cap);
    L.o_bigmodel = take(8ull * std::max(MODEL_WORDS, MLP_MODEL_WORDS) + 64);
    L.o_part = take(FIT_G * 8 * 8);
    // leaf lines, leaf boundaries, then the leaf least squares' piece sums
    L.o_leaf = take(L_MAX * 8 * 8 + (L_MAX + 1) * 8 + (L_MAX + FIT_PIECES + 2) * 4 * 8);
    L.o_flag = take(256);
    L.o_mlp = take(MLP_STATE_BYTES);
    L.S_big = big_sample_size(n, m, o);
    if (L.S_big) {
        L.item_m_cap = n / MB_MIN + 64;
        L.o_items_m = take(L.item_m_cap * 16);
        L.o_sample = take(L.S_big * 8);
        L.o_bstart = take((B_MAX + 1) * 8);
        L.nested.push_back(plan(L.S_big, 1, 0, nested_opts(o)));
        L.o_nested = take(L.nested[0].bytes);
    }
    if (L.S_big && mlp_first_level(n, m, o)) {
        L.mlp_stride = std::max<uint64_t>(1, (L.S_big + o.mlp_sample - 1) / o.mlp_sample);
        L.mlp_S = (L.S_big + L.mlp_stride - 1) / L.mlp_stride;
        L.o_mlp_t = take(L.mlp_S * 4);
        L.o_mlp_y = take(L.mlp_S * 4);
        plan_mlp_moments(L, L.mlp_S, o_);
        L.o_ids = take(n * 2);
    }
    L.bytes = o_;
    return L;
}

// ---------------------------------------------------------------------------
// library-owned workspace (per device, grow-only) and per-thread call state
// ---------------------------------------------------------------------------
struct DevPool {
    void* ptr = nullptr;
    size_t bytes = 0;
    void* user = nullptr;
    size_t user_bytes = 0;
    hipEvent_t last = nullptr;
    hipStream_t last_stream = nullptr;
    uint64_t* pinned = nullptr;  // host read-back slots
    hipStream_t rb = nullptr;    // read-back stream: a level's counters copied while its scatter runs
    hipEvent_t scanned = nullptr;  // recorded after each level's k_scan
    int cus = 0;
    uint64_t sig = 0;            // layout of the last call (status pools valid for it)
};
static std::mutex g_mu;
static DevPool g_pool[64];

struct LastCall {
    Ctl* ctl = nullptr;
    hipStream_t st = nullptr;
    int dev = -1;
    bool valid = false;
};
static thread_local LastCall g_last;

// ---------------------------------------------------------------------------
// optional kernel timing: an event pair around each launch
// ---------------------------------------------------------------------------
enum KernelId {
    KI_RESET, KI_SEED, KI_MODEL, KI_HIST, KI_SCAN, KI_SCATTER, KI_BASE, KI_BASE_BIG, KI_GATHER, KI_FIT, KI_MLP_TRAIN,
    KI_MLP_IDS, KI_RESIDENT, KI_CONVERT, KI_BASE_MODEL, KI_BASE_MERGE, KI_N
};
static const char* KNAME[KI_N] = {"k_reset", "k_seed", "k_model", "k_hist", "k_scan", "k_scatter", "k_base_small",
                                  "k_base_big", "k_gather", "k_fit", "k_mlp_step", "k_mlp_ids", "k_resident",
                                  "k_convert", "k_base_model", "k_base_merge"};
struct TRec {
    int kid;
    hipEvent_t a, b;
    double keys;
};
static bool g_timing = false;
static thread_local bool t_untimed = false;  // this thread's call takes no timing records (ls_sort_noalloc)
static std::vector<TRec> g_trec;
static std::vector<hipEvent_t> g_evfree;

static hipEvent_t ev_get() {
    if (!g_evfree.empty()) {
        hipEvent_t e = g_evfree.back();
        g_evfree.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `expr` (a hipError_t expression); when timing, bracket it with events.
#define TIMED(kid, st, expr)                                              \
    do {                                                                  \
        if (g_timing && !t_untimed) {                                     \
            TRec r_{(kid), ev_get(), ev_get(), 0.0};                      \
            if (r_.a) HIP_TRY(hipEventRecord(r_.a, (st)));                \
            HIP_TRY(expr);                                                \
            if (r_.b) HIP_TRY(hipEventRecord(r_.b, (st)));                \
            g_trec.push_back(r_);                                         \
        } else {                                                          \
            HIP_TRY(expr);                                                \
        }                                                                 \
    } while (0)

static uint64_t layout_sig(const Layout& L) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    mix(L.o_persist); mix(L.o_status); mix(L.status_cap); mix(L.bytes);
    for (const Layout& c : L.nested) { mix(c.o_status); mix(c.status_cap); mix(c.bytes); }
    return h;
}

// The look-back words of a workspace are only valid against the history of
// that same layout: when the layout changes, clear them (and the epoch).
static ls_status prepare_status(DevPool* pool, uint8_t* base, const Layout& L, hipStream_t st) {
    uint64_t sig = layout_sig(L);
    if (sig == pool->sig) return LS_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(LS_EINVAL, "first call with this size must run outside stream capture (workspace set-up)");
    std::vector<std::pair<uint8_t*, const Layout*>> todo{{base, &L}};
    while (!todo.empty()) {
        auto [b, l] = todo.back();
        todo.pop_back();
        HIP_TRY(hipMemsetAsync(b + l->o_persist, 0, 256, st));
        HIP_TRY(hipMemsetAsync(b + l->o_status, 0, l->status_cap * 8, st));
        for (const Layout& c : l->nested) todo.push_back({b + l->o_nested, &c});
    }
    pool->sig = sig;
    return LS_OK;
}

// Per-device set-up: compute-unit count, the ordering event, pinned read-back
// slots.  Runs outside stream capture (ls_set_workspace or the first call).
static ls_status pool_init(int dev, DevPool*& pool) {
    if (dev < 0 || dev >= 64) return fail(LS_EINVAL, "device index out of range");
    pool = &g_pool[dev];
    if (!pool->cus) {
        HIP_TRY(hipDeviceGetAttribute(&pool->cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIP_TRY(hipEventCreateWithFlags(&pool->last, hipEventDisableTiming));
        HIP_TRY(hipHostMalloc((void**)&pool->pinned, std::max<size_t>(4096, sizeof(Ctl)), hipHostMallocDefault));
        HIP_TRY(hipStreamCreateWithFlags(&pool->rb, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&pool->scanned, hipEventDisableTiming));
    }
    return LS_OK;
}

static ls_status capturing(hipStream_t st, bool& cap) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    cap = cs != hipStreamCaptureStatusNone;
    return LS_OK;
}

// The workspace of a call.  Under stream capture only a caller-owned
// workspace (ls_set_workspace) is used: the library's own pool is freed and
// reallocated when a later call needs more, which would leave a captured
// graph's kernel arguments pointing at freed memory.
static ls_status acquire(uint64_t bytes, const Layout& L, DevPool*& pool, uint8_t*& base, hipStream_t st) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    bool cap = false;
    ls_status s0 = capturing(st, cap);
    if (s0) return s0;
    if (cap && (dev < 0 || dev >= 64 || !g_pool[dev].user))
        return fail(LS_EINVAL, "a call under stream capture needs a caller-owned workspace: call ls_set_workspace "
                               "first (outside capture)");
    if ((s0 = pool_init(dev, pool))) return s0;
    if (pool->user) {
        if (bytes > pool->user_bytes)
            return fail(LS_ENOMEM, "workspace set by ls_set_workspace is too small: need " + std::to_string(bytes) +
                                       " bytes");
        base = (uint8_t*)pool->user;
        return LS_OK;
    }
    if (bytes > pool->bytes) {
        if (pool->ptr) HIP_TRY(hipFree(pool->ptr));
        pool->ptr = nullptr;
        pool->bytes = 0;
        pool->sig = 0;
        size_t want = (size_t)(bytes + bytes / 8 + (1 << 20));
        if (hipMalloc(&pool->ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            pool->ptr = nullptr;
            return fail(LS_ENOMEM, "cannot allocate a workspace of " + std::to_string(want) + " bytes");
        }
        pool->bytes = want;
        HIP_TRY(hipMemset(pool->ptr, 0, want));
    }
    base = (uint8_t*)pool->ptr;
    (void)L;
    return LS_OK;
}

// ---------------------------------------------------------------------------
// the engine
// ---------------------------------------------------------------------------
struct Call {
    uint64_t* keys;
    uint32_t* pay;
    uint64_t n;
    uint64_t m;
    const uint64_t* offsets;   // device, null for a single array
    int u64;
    Opts o;
    hipStream_t st;
    // first level given by the caller (single-step partition): model already
    // at layout.o_bigmodel and described in segs[1][0]; run one level only
    bool one_level = false;
    uint64_t* out_keys = nullptr;
    uint32_t* out_pay = nullptr;
};

static Params make_params(const Call& c, const Layout& L, uint8_t* base) {
    Params P{};
    P.keys[0] = c.keys;
    P.keys[1] = c.one_level ? c.out_keys : (uint64_t*)(base + L.o_tmp);
    P.pay[0] = c.pay;
    P.pay[1] = c.pay ? (c.one_level ? c.out_pay : (uint32_t*)(base + L.o_tmppay)) : nullptr;
    P.u64 = c.u64;
    P.has_pay = c.pay != nullptr;
    P.buckets = c.o.buckets; P.leaves = c.o.leaves; P.tree_buckets = c.o.tree_buckets; P.cutoff = c.o.cutoff;
    P.max_levels = c.o.max_levels; P.flags = c.o.flags; P.model = c.o.model;
    P.sample_frac = c.o.sample_frac; P.fallback_ratio = c.o.fallback_ratio; P.seed = c.o.seed;
    P.unit0_shift = 0;
    while (((uint32_t)UNIT << P.unit0_shift) < c.o.tile && P.unit0_shift < USHIFT_MAX) P.unit0_shift++;
    P.ctl = (Ctl*)(base + L.o_ctl);
    for (int i = 0; i < 2; i++) {
        P.segs[i] = (Seg*)(base + L.o_segs[i]);
        P.tiles[i] = (Tile*)(base + L.o_tiles[i]);
        P.arena[i] = base + L.o_arena[i];
    }
    P.items = (uint64_t*)(base + L.o_items);
    P.bigs = (uint64_t*)(base + L.o_bigs);
    P.items_b = (uint64_t*)(base + L.o_items_b);
    P.items_c = (uint64_t*)(base + L.o_items_c);
    P.merges = (uint64_t*)(base + L.o_merges);
    P.merge_cap = L.merge_cap;
    P.items_m = L.o_items_m ? (uint64_t*)(base + L.o_items_m) : nullptr;
    P.item_m_cap = L.item_m_cap;
    P.fmodel = L.S_big && !c.one_level ? (const uint64_t*)(base + L.o_bigmodel) : nullptr;
    P.counts = (unsigned long long*)(base + L.o_counts);
    P.status = (unsigned long long*)(base + L.o_status);
    P.ids = L.o_ids ? (uint16_t*)(base + L.o_ids) : nullptr;
    P.seg_cap = L.seg_cap; P.tile_cap = L.tile_cap; P.item_cap = L.item_cap; P.big_cap = L.big_cap; P.counts_cap = L.counts_cap;
    P.status_cap = L.status_cap; P.arena_cap = L.arena_cap; P.item_b_cap = L.item_b_cap; P.item_c_cap = L.item_c_cap;
    P.persist = (const uint64_t*)(base + L.o_persist);
    P.fsample = L.S_big ? (const uint64_t*)(base + L.o_sample) : nullptr;
    P.fbstart = L.S_big ? (const uint64_t*)(base + L.o_bstart) : nullptr;
    P.fS = L.S_big;
    P.level = 0;
    return P;
}

static std::string overflow_text(uint32_t f) {
    std::string s;
    if (f & OVF_SEG) s += " segments";
    if (f & OVF_TILE) s += " tiles";
    if (f & OVF_ITEM) s += " base-case items";
    if (f & OVF_COUNTS) s += " bucket counts";
    if (f & OVF_STATUS) s += " look-back words";
    if (f & OVF_ARENA) s += " model arena";
    if (f & OVF_STATE) s += " (internal: look-back word out of sequence)";
    return s;
}

static ls_status run(const Call& c, const Layout& L, uint8_t* base, DevPool* pool);

// Large first level: sample ~1% of the keys, sort the sample with the same
// engine, then fit the RMI (or build the splitter tree) over it with the
// multi-workgroup fit kernels (Alg. 5).  The model lands in o_bigmodel and its
// descriptor in segs[1][0] for k_seed to pick up.
static ls_status big_model(const Call& c, const Layout& L, uint8_t* base, DevPool* pool, const Params& P) {
    uint64_t* smp = (uint64_t*)(base + L.o_sample);
    const uint64_t sseed = 0;  // stream state for (offset 0, level 0): SplitMix64 output 0 of seed
    (void)sseed;
    // segment seed = splitmix64_at(seed, (off << 6) | level) with off = 0, level = 0
    uint64_t z = c.o.seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    TIMED(KI_GATHER, c.st, launch_gather(c.keys, c.n, z, L.S_big, smp, c.st));
    Call nc{};
    nc.keys = smp; nc.pay = nullptr; nc.n = L.S_big; nc.m = 1; nc.offsets = nullptr; nc.u64 = c.u64;
    nc.o = nested_opts(c.o);
    nc.st = c.st;
    ls_status s = run(nc, L.nested[0], base + L.o_nested, pool);
    if (s) return s;
    FitArgs A{};
    A.s = smp; A.S = L.S_big; A.n = c.n; A.u64 = c.u64;
    A.mode = c.o.model == LS_MODEL_SPLITTER ? 2 : 0;
    A.mlp = L.mlp_S ? 1 : 0;
    A.L = std::min<uint32_t>(c.o.leaves, std::max<uint32_t>(2, (uint32_t)std::min<uint64_t>(L.S_big / 8, L_MAX)));
    const uint64_t half = std::max<uint32_t>(1, c.o.cutoff / 2);
    uint64_t B1 = std::min<uint64_t>(c.o.buckets, std::max<uint64_t>(2, (c.n + half - 1) / half));
    B1 = std::min<uint64_t>(B1, std::max<uint64_t>(2, c.n / 4));
    uint32_t log2B2 = 0;
    uint64_t per = c.n / B1;
    if (per > c.o.cutoff) {
        uint64_t want = (per + half - 1) / half;
        while ((1ull << log2B2) < want && log2B2 < 10) log2B2++;
    }
    A.B1 = (uint32_t)B1; A.log2B2 = log2B2; A.R = (double)(B1 << log2B2);
    uint64_t nt = c.n / 16;
    uint32_t Bt = 2;
    while (Bt * 2 <= c.o.tree_buckets && Bt * 2 <= nt) Bt *= 2;
    A.Bt = Bt;
    A.G = FIT_G;
    A.part = (double*)(base + L.o_part);
    A.leaf = (double*)(base + L.o_leaf);
    A.model = (uint64_t*)(base + L.o_bigmodel);
    A.flag = (uint32_t*)(base + L.o_flag);
    A.seg = P.segs[1];
    A.first_mlp = &P.ctl->first_mlp;
    TIMED(KI_FIT, c.st, launch_fit1(A, c.st));
    TIMED(KI_FIT, c.st, launch_fit2(A, c.st));
    TIMED(KI_FIT, c.st, launch_fit_root(A, c.st));
    if (A.mlp) {
        // train the MLP root on (every stride-th point of) the sorted sample;
        // every kernel is gated on the policy's decision in A.flag
        const MlpState ms = mlp_state(base, L);
        float* t = (float*)(base + L.o_mlp_t);
        float* y = (float*)(base + L.o_mlp_y);
        TIMED(KI_FIT, c.st, launch_mlp_prep(smp, L.S_big, L.mlp_stride, c.u64, t, y, ms.lo_inv, A.flag, c.st));
        TIMED(KI_FIT, c.st, launch_mlp_setup(t, L.mlp_S, nullptr, 1e-3, ms.p, ms.m, ms.v, ms.best, ms.scale,
                                             ms.best_loss, ms.done, A.flag, c.st));
        // every Adam step of the training in one launch (gradients by activation regions)
        double* mom = (double*)(base + L.o_mlp_mom);
        TIMED(KI_MLP_TRAIN, c.st, launch_mlp_moments(t, y, L.mlp_S, (double*)(base + L.o_mlp_bsum), mom, A.flag,
                                                     c.st));
        MlpRegion R{};
        R.t = t; R.mom = mom; R.S = L.mlp_S; R.p = ms.p; R.m = ms.m; R.v = ms.v; R.scale = ms.scale;
        R.best = ms.best; R.best_loss = ms.best_loss; R.loss_pair = P.ctl->mlp_loss; R.gate = A.flag;
        R.steps = c.o.mlp_steps; R.lr = c.o.mlp_lr; R.b1 = 0.9f; R.b2 = 0.999f; R.eps = 1e-8f;
        TIMED(KI_MLP_TRAIN, c.st, launch_mlp_regions(R, c.st));
        TIMED(KI_FIT, c.st, launch_mlp_install(ms.best, ms.lo_inv, A.L, A.B1, A.log2B2, A.R, nullptr, A.flag, nullptr,
                                               A.model, c.st));
    }
    TIMED(KI_FIT, c.st, launch_fit_leaves(A, c.st));
    TIMED(KI_FIT, c.st, launch_fit_finish(A, c.st));
    A.bstart = (uint64_t*)(base + L.o_bstart);
    TIMED(KI_FIT, c.st, launch_fit_bstart(A, c.st));
    A.ratio = c.o.fallback_ratio;
    A.balance = (c.o.flags & LS_FLAG_NO_FALLBACK) ? 2.0 : (double)c.o.balance_pct / 100.0;
    TIMED(KI_FIT, c.st, launch_fit_balance(A, c.st));
    return LS_OK;
}

static ls_status run(const Call& c, const Layout& L, uint8_t* base, DevPool* pool) {
    Params P = make_params(c, L, base);
    uint64_t* persist = (uint64_t*)(base + L.o_persist);
    TIMED(KI_RESET, c.st, launch_reset(P, persist, c.st));
    uint32_t prebuilt = 0;
    if (c.one_level) {
        prebuilt = 1;
    } else if (L.S_big) {
        ls_status s = big_model(c, L, base, pool, P);
        if (s) return s;
        prebuilt = 1;
    }
    const uint32_t seed_grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>((c.m + 255) / 256, 256), 65535);
    TIMED(KI_SEED, c.st, launch_seed(P, c.offsets, c.m, c.n, prebuilt, persist, seed_grid, c.st));
    const uint32_t cus = (uint32_t)pool->cus;
    const bool fixed = (c.o.flags & LS_FLAG_FIXED_LEVELS) != 0;
    if (!fixed) {  // the read-backs between levels cannot be captured
        bool cap = false;
        ls_status s0 = capturing(c.st, cap);
        if (s0) return s0;
        if (cap) return fail(LS_EINVAL, "a call under stream capture needs LS_FLAG_FIXED_LEVELS");
    }
    const uint32_t max_run = c.one_level ? 1 : std::min<uint32_t>(MAXL - 1, c.o.max_levels + 9);
    uint32_t levels = 0;
    uint32_t next_res = 0;  // resident segments of the next level (read back)
    uint64_t nmerge = ~0ull;  // chunk-and-merge items (read back after the last level; unknown: fixed levels)
    uint32_t mclasses = 7;    // their size classes present (bits: up to 2048 keys, 2049..4096, 4097..8192)
    uint32_t split = 0;       // the next level has fewer work units than CUs (read back)
    for (uint32_t lvl = 0; lvl < max_run; lvl++) {
        P.level = (int)lvl;
        P.split = split;
        const size_t rec0 = g_trec.size();
        const uint32_t g0 = lvl == 0 ? (uint32_t)std::min<uint64_t>(std::max<uint64_t>(c.m, 1), 4096) : 1024;
        // k_model holds a CU's LDS per workgroup: after the first level (mostly
        // fine windows, a wavefront each) one workgroup per CU
        TIMED(KI_MODEL, c.st, launch_model(P, lvl == 0 ? g0 : cus, c.st));
        // (after the first level the read-back below says whether any segment is resident)
        if (!c.one_level && (lvl == 0 || fixed || next_res))
            TIMED(KI_RESIDENT, c.st, launch_resident(P, cus * (c.pay ? 2 : 3), c.st));
        if (P.ids && lvl <= 1) TIMED(KI_MLP_IDS, c.st, launch_mlp_ids(P, cus * 4, c.st));
        TIMED(KI_HIST, c.st, launch_hist(P, cus * 4, c.st));
        TIMED(KI_SCAN, c.st, launch_scan(P, g0, c.st));
        const bool readback = !c.one_level && !fixed;
        if (readback) HIP_TRY(hipEventRecord(pool->scanned, c.st));
        TIMED(KI_SCATTER, c.st, launch_scatter(P, cus, c.st));
        levels = lvl + 1;
        if (c.one_level) {
            HIP_TRY(hipMemcpyAsync(pool->pinned, &P.ctl->overflow, 4, hipMemcpyDeviceToHost, c.st));
            HIP_TRY(hipStreamSynchronize(c.st));
            uint32_t ovf = ((uint32_t*)pool->pinned)[0];
            if (ovf) return fail(LS_ENOMEM, "workspace capacity exceeded:" + overflow_text(ovf));
            continue;
        }
        if (fixed) continue;
        // read back the next level's work, the overflow flags and this level's
        // keys: the whole control block in one copy (one copy dispatch instead
        // of one per field).  Everything read here is final once k_scan is
        // done, so the copy runs on the read-back stream while k_scatter runs,
        // and the next level's launches queue behind the scatter before it
        // ends (the GPU does not idle through the host's round trip).  The
        // scatter's only flag (a look-back word without this level's tag,
        // never expected) is seen at the next read-back.
        HIP_TRY(hipStreamWaitEvent(pool->rb, pool->scanned, 0));
        HIP_TRY(hipMemcpyAsync(pool->pinned, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, pool->rb));
        HIP_TRY(hipStreamSynchronize(pool->rb));
        const Ctl* hc = (const Ctl*)pool->pinned;
        uint32_t next = hc->nseg[lvl + 1];
        uint32_t ovf = hc->overflow;
        double lkeys = (double)hc->lv[lvl].keys;
        next_res = hc->nres[lvl + 1];
        nmerge = hc->nmerge;
        // a launch per size class present; with fewer items than CUs x 4,
        // one launch for all (their merges are latency, not throughput)
        mclasses = nmerge < 4ull * cus ? 8u
                 : (nmerge > hc->nmerge_cls[0] ? 1u : 0u) | (hc->nmerge_cls[0] > hc->nmerge_cls[1] ? 2u : 0u) |
                       (hc->nmerge_cls[1] ? 4u : 0u);
        // a next level of few work units (a few small segments) is re-cut
        // into one-tile units, when the unit list has room for them
        const uint64_t nu = hc->ntile[lvl + 1];
        split = nu > 0 && nu < cus && 4 * nu + hc->nseg[lvl + 1] <= P.tile_cap ? 1u : 0u;
        for (size_t i = rec0; i < g_trec.size(); i++) g_trec[i].keys = lkeys;
        if (ovf) return fail(LS_ENOMEM, "workspace capacity exceeded:" + overflow_text(ovf));
        if (next == 0) break;
    }
    (void)levels;
    if (!c.one_level) {
        const size_t r0 = g_trec.size();
        TIMED(KI_BASE, c.st, launch_base_small(P, cus * 8, c.st));
        const bool mbase = (c.o.flags & LS_FLAG_MODEL_BASE) && P.fmodel;
        if (mbase) TIMED(KI_BASE_MODEL, c.st, launch_base_model(P, cus * 2, c.st));
        TIMED(KI_BASE_BIG, c.st, launch_base_big(P, cus * 2, c.st));
        // the items sorted above as chunks, merged (none: no launch)
        const bool merge = nmerge != 0;
        if (merge) TIMED(KI_BASE_MERGE, c.st, launch_base_merge(P, cus, mclasses, c.st));
        if (g_timing && !t_untimed && g_trec.size() > r0) {  // keys through each base-case kernel
            HIP_TRY(hipMemcpyAsync(pool->pinned, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c.st));
            HIP_TRY(hipStreamSynchronize(c.st));
            const Ctl* hc = (const Ctl*)pool->pinned;
            size_t r = r0;
            g_trec[r++].keys = (double)hc->small_keys;
            if (mbase) g_trec[r++].keys = (double)hc->model_keys;
            g_trec[r++].keys = (double)hc->big_keys;
            if (merge) g_trec[r++].keys = (double)hc->merge_keys;
        }
    }
    return LS_OK;
}

static ls_status check_keys(const void* keys, uint64_t n, ls_dtype dtype, const uint32_t* payload) {
    if (dtype != LS_F64 && dtype != LS_U64) return fail(LS_EINVAL, "dtype must be LS_F64 or LS_U64");
    if (n > 0 && !keys) return fail(LS_EINVAL, "keys is NULL");
    if (((uintptr_t)keys) & 7) return fail(LS_EINVAL, "keys must be 8-byte aligned");
    if (((uintptr_t)payload) & 3) return fail(LS_EINVAL, "payload must be 4-byte aligned");
    if (n >= (1ull << 45)) return fail(LS_EINVAL, "n too large");
    return LS_OK;
}

// Arguments of the sort entry points: every key type, uint32 or 64-bit payload.
static ls_status check_sort_args(const void* keys, uint64_t n, ls_dtype dtype, const void* payload, int pay64) {
    if (dtype != LS_F64 && dtype != LS_U64 && dtype != LS_I64 && dtype != LS_F32)
        return fail(LS_EINVAL, "dtype must be LS_F64, LS_U64, LS_I64 or LS_F32");
    if (n > 0 && !keys) return fail(LS_EINVAL, "keys is NULL");
    if (((uintptr_t)keys) & (dtype == LS_F32 ? 3 : 7))
        return fail(LS_EINVAL, dtype == LS_F32 ? "keys must be 4-byte aligned" : "keys must be 8-byte aligned");
    if (((uintptr_t)payload) & (pay64 ? 7 : 3))
        return fail(LS_EINVAL, pay64 ? "payload must be 8-byte aligned" : "payload must be 4-byte aligned");
    if (pay64 && n > 0 && !payload) return fail(LS_EINVAL, "payload is NULL");
    if (pay64 && n >= (1ull << 32)) return fail(LS_EINVAL, "64-bit payloads need fewer than 2^32 keys");
    if (n >= (1ull << 45)) return fail(LS_EINVAL, "n too large");
    return LS_OK;
}

// Before the engine runs: int64 keys flipped to uint64 order in place,
// float32 keys widened into the workspace (the engine then sorts those),
// 64-bit payloads saved and replaced by the original indices.
static ls_status types_before(Call& c, void* keys, void* payload, ls_dtype dtype, int pay64, const Layout& L,
                              uint8_t* base, uint32_t cus) {
    if (dtype == LS_I64) TIMED(KI_CONVERT, c.st, launch_flip_sign((uint64_t*)keys, c.n, cus, c.st));
    if (dtype == LS_F32) {
        c.keys = (uint64_t*)(base + L.o_wide);
        TIMED(KI_CONVERT, c.st, launch_widen((const uint32_t*)keys, c.keys, c.n, cus, c.st));
    }
    if (pay64) {
        c.pay = (uint32_t*)(base + L.o_idx);
        TIMED(KI_CONVERT, c.st, launch_index_save((const uint64_t*)payload, (uint64_t*)(base + L.o_save), c.pay,
                                                  c.n, cus, c.st));
    }
    return LS_OK;
}

// After it: the inverse maps, and the payload gathered through the indices.
static ls_status types_after(const Call& c, void* keys, void* payload, ls_dtype dtype, int pay64, const Layout& L,
                             uint8_t* base, uint32_t cus) {
    if (pay64)
        TIMED(KI_CONVERT, c.st, launch_gather64((const uint64_t*)(base + L.o_save), c.pay, (uint64_t*)payload, c.n,
                                                cus, c.st));
    if (dtype == LS_I64) TIMED(KI_CONVERT, c.st, launch_flip_sign((uint64_t*)keys, c.n, cus, c.st));
    if (dtype == LS_F32) TIMED(KI_CONVERT, c.st, launch_narrow(c.keys, (uint32_t*)keys, c.n, cus, c.st));
    return LS_OK;
}

static ls_status order_after_last(DevPool* pool, hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone && pool->last_stream != st && pool->last_stream != nullptr)
        HIP_TRY(hipStreamWaitEvent(st, pool->last, 0));
    return LS_OK;
}

static ls_status mark_done(DevPool* pool, hipStream_t st, Ctl* ctl) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) {
        HIP_TRY(hipEventRecord(pool->last, st));
        pool->last_stream = st;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    g_last.ctl = ctl; g_last.st = st; g_last.dev = dev; g_last.valid = true;
    return LS_OK;
}

static ls_status sort_common(void* keys, const uint64_t* offsets, uint64_t m, uint64_t n, ls_dtype dtype,
                             void* payload, int pay64, const ls_options* opt, void* stream) {
    ls_status s = check_sort_args(keys, n, dtype, payload, pay64);
    if (s) return s;
    Opts o;
    if ((s = normalize(opt, o, n, m))) return s;
    if (o.model == LS_MODEL_MLP && offsets)
        return fail(LS_EUNSUPPORTED, "the MLP model is available for single arrays (ls_sort) only");
    if (n <= 1 || m == 0) return LS_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Layout L = plan(n, m, payload != nullptr, o);
    plan_types(L, n, dtype, pay64);
    DevPool* pool;
    uint8_t* base;
    hipStream_t st = (hipStream_t)stream;
    if ((s = acquire(L.bytes, L, pool, base, st))) return s;
    if ((s = order_after_last(pool, st))) return s;
    if ((s = prepare_status(pool, base, L, st))) return s;
    Call c{};
    c.keys = (uint64_t*)keys; c.pay = (uint32_t*)payload; c.n = n; c.m = m; c.offsets = offsets;
    c.u64 = dtype == LS_U64 || dtype == LS_I64;
    c.o = o; c.st = st;
    if ((s = types_before(c, keys, payload, dtype, pay64, L, base, (uint32_t)pool->cus))) return s;
    if ((s = run(c, L, base, pool))) return s;
    if ((s = types_after(c, keys, payload, dtype, pay64, L, base, (uint32_t)pool->cus))) return s;
    return mark_done(pool, st, (Ctl*)(base + L.o_ctl));
}

// ---------------------------------------------------------------------------
// allocation-free sorting (ls_sort_noalloc)
//
// The workspace is `scratch`, a fixed-size device array of the library: each
// device the library runs on holds its own copy until the process ends.  In
// host code the array's name is only a host-side stand-in, so its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to the kernels and to memsets.
// The call launches a fixed number of levels (no host read-back: there is no
// pinned buffer to read into without allocating one), records no timing
// events, and is not ordered against other calls: calls that use the array
// of one device must not overlap in time.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[LS_NOALLOC_SCRATCH_BYTES];
static DevPool g_npool[64];  // per device: the array's device address (ptr), CU count, layout signature

static ls_status noalloc_pool(DevPool*& pool) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(LS_EINVAL, "device index out of range");
    pool = &g_npool[dev];
    if (!pool->ptr) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) return fail(LS_EHIP, "scratch array has no usable device address");
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        pool->cus = cus;
        pool->bytes = LS_NOALLOC_SCRATCH_BYTES;
        pool->sig = 0;
        pool->ptr = p;
    }
    return LS_OK;
}

static ls_status sort_noalloc(void* keys, uint64_t n, ls_dtype dtype, uint32_t* payload, const ls_options* opt,
                              void* stream) {
    ls_status s = check_sort_args(keys, n, dtype, payload, 0);
    if (s) return s;
    Opts o;
    if ((s = normalize(opt, o, n, 1))) return s;
    o.flags = (o.flags & ~(uint32_t)LS_FLAG_SYNC_LEVELS) | LS_FLAG_FIXED_LEVELS;
    if (n <= 1) return LS_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Layout L = plan(n, 1, payload != nullptr, o);
    plan_types(L, n, dtype, 0);
    if (L.bytes > LS_NOALLOC_SCRATCH_BYTES)
        return fail(LS_ENOMEM, "ls_sort_noalloc: " + std::to_string(n) + " keys need " + std::to_string(L.bytes) +
                                   " bytes of scratch; the fixed scratch array holds " +
                                   std::to_string((unsigned long long)LS_NOALLOC_SCRATCH_BYTES) + " (use ls_sort)");
    DevPool* pool = nullptr;
    if ((s = noalloc_pool(pool))) return s;
    hipStream_t st = (hipStream_t)stream;
    uint8_t* base = (uint8_t*)pool->ptr;
    // the look-back words and the call epoch start at zero for every new
    // layout (the array keeps the previous call's contents)
    if ((s = prepare_status(pool, base, L, st))) return s;
    Call c{};
    c.keys = (uint64_t*)keys; c.pay = payload; c.n = n; c.m = 1; c.offsets = nullptr;
    c.u64 = dtype == LS_U64 || dtype == LS_I64;
    c.o = o; c.st = st;
    t_untimed = true;
    s = types_before(c, keys, payload, dtype, 0, L, base, (uint32_t)pool->cus);
    if (!s) s = run(c, L, base, pool);
    if (!s) s = types_after(c, keys, payload, dtype, 0, L, base, (uint32_t)pool->cus);
    t_untimed = false;
    if (s) return s;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    g_last.ctl = (Ctl*)(base + L.o_ctl); g_last.st = st; g_last.dev = dev; g_last.valid = true;
    return LS_OK;
}

// Small scratch for the single-step entry points (model, fit partials).
static ls_status step_scratch(uint8_t*& base, DevPool*& pool, Layout& L, hipStream_t st, uint64_t mlp_S = 0) {
    Opts o;
    normalize(nullptr, o);
    L = plan(16, 1, 0, o);
    if (mlp_S) {  // training set of the single-step MLP entry points
        L.mlp_S = mlp_S;
        L.o_mlp_t = L.bytes;
        L.o_mlp_y = L.o_mlp_t + align256(mlp_S * 4);
        uint64_t o_ = L.o_mlp_y + align256(mlp_S * 4);
        plan_mlp_moments(L, mlp_S, o_);
        L.bytes = o_;
    }
    ls_status s = acquire(L.bytes, L, pool, base, st);
    if (!s) pool->sig = 0;  // this scratch may overlap another layout's look-back words
    return s;
}

}  // namespace ls

using namespace ls;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ls_last_error(void) { return g_err.c_str(); }

const char* ls_version(void) { return "lsort 0.1 gfx950"; }

ls_status ls_sort(void* keys, uint64_t n, ls_dtype dtype, uint32_t* payload, const ls_options* opt, void* stream) {
    return sort_common(keys, nullptr, 1, n, dtype, payload, 0, opt, stream);
}

ls_status ls_sort_payload64(void* keys, uint64_t n, ls_dtype dtype, uint64_t* payload, const ls_options* opt,
                            void* stream) {
    return sort_common(keys, nullptr, 1, n, dtype, payload, 1, opt, stream);
}

ls_status ls_sort_noalloc(void* keys, uint64_t n, ls_dtype dtype, uint32_t* payload, const ls_options* opt,
                          void* stream) {
    return sort_noalloc(keys, n, dtype, payload, opt, stream);
}

ls_status ls_sort_segmented(void* keys, const uint64_t* offsets, uint64_t m, uint64_t host_total, ls_dtype dtype,
                            uint32_t* payload, const ls_options* opt, void* stream) {
    if (m > 0 && !offsets) return fail(LS_EINVAL, "offsets is NULL");
    if (((uintptr_t)offsets) & 7) return fail(LS_EINVAL, "offsets must be 8-byte aligned");
    if (m >= (1ull << 32)) return fail(LS_EINVAL, "too many segments");
    return sort_common(keys, offsets, m, host_total, dtype, payload, 0, opt, stream);
}

ls_status ls_workspace_bytes(uint64_t n_total, uint64_t m, ls_dtype dtype, int has_payload, const ls_options* opt,
                             size_t* out) {
    if (!out) return fail(LS_EINVAL, "out is NULL");
    if (dtype != LS_F64 && dtype != LS_U64 && dtype != LS_I64 && dtype != LS_F32) return fail(LS_EINVAL, "bad dtype");
    if (has_payload < 0 || has_payload > 2) return fail(LS_EINVAL, "has_payload must be 0, 1 or 2");
    Opts o;
    ls_status s = normalize(opt, o, std::max<uint64_t>(n_total, 16), std::max<uint64_t>(m, 1));
    if (s) return s;
    const uint64_t nn = std::max<uint64_t>(n_total, 16);
    Layout L = plan(nn, std::max<uint64_t>(m, 1), has_payload != 0, o);
    plan_types(L, nn, dtype, has_payload == 2);
    *out = (size_t)L.bytes;
    return LS_OK;
}

ls_status ls_set_workspace(void* dev_ptr, size_t bytes, void* stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(LS_EHIP, "hipGetDevice failed");
    if (((uintptr_t)dev_ptr) & 255) return fail(LS_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    ls_status s = capturing(st, cap);
    if (s) return s;
    if (cap) return fail(LS_EINVAL, "ls_set_workspace must be called outside stream capture");
    std::lock_guard<std::mutex> lk(g_mu);
    DevPool* p = nullptr;
    if ((s = pool_init(dev, p))) return s;
    // earlier calls that used the previous workspace finish first; the
    // clearing is ordered before every later call by the pool's event
    if ((s = order_after_last(p, st))) return s;
    if (dev_ptr) HIP_TRY(hipMemsetAsync(dev_ptr, 0, bytes, st));
    HIP_TRY(hipEventRecord(p->last, st));
    p->last_stream = st;
    p->user = dev_ptr;
    p->user_bytes = dev_ptr ? bytes : 0;
    p->sig = 0;
    return LS_OK;
}

ls_status ls_get_stats(ls_stats* out) {
    if (!out) return fail(LS_EINVAL, "out is NULL");
    if (!g_last.valid) return fail(LS_EINVAL, "no completed call on this thread");
    HIP_TRY(hipStreamSynchronize(g_last.st));
    Ctl c;
    HIP_TRY(hipMemcpy(&c, g_last.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    uint32_t levels = 0;
    for (int l = 0; l < MAXL && l < LS_MAX_STAT_LEVELS; l++) {
        const LevelStats& s = c.lv[l];
        ls_level_stats& d = out->level[l];
        d.segments = s.segments; d.keys = s.keys; d.buckets = s.buckets; d.max_bucket = s.max_bucket;
        d.max_bucket_x1000_over_mean = s.max_ratio_x1000; d.empty = s.empty; d.equality = s.equality;
        d.base = s.base; d.recurse = s.recurse; d.fallback = s.fallback; d.learned = s.learned; d.tree = s.tree;
        d.radix = s.radix;
        if (s.segments) levels = l + 1;
    }
    out->levels = levels;
    out->first_model = c.first_mlp ? LS_MODEL_MLP
                       : c.lv[0].learned ? LS_MODEL_RMI : (c.lv[0].segments ? LS_MODEL_SPLITTER : LS_MODEL_AUTO);
    out->base_items = c.nitems + c.nitems_b + c.nitems_w + c.nitems_k + c.nitems_c - c.nchunk + c.nmerge + c.nitems_m +
                      c.nbig - c.ncopy - c.nmoved;
    out->copy_items = c.ncopy;
    out->mlp_loss_first = c.mlp_loss[0];
    out->mlp_loss_last = c.mlp_loss[1];
    out->overflow = c.overflow;
    out->merged_items = (uint32_t)std::min<uint64_t>(c.nmerge, 0xffffffffull);
    return LS_OK;
}

ls_status ls_timing(int enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (TRec& r : g_trec) {
        if (r.a) g_evfree.push_back(r.a);
        if (r.b) g_evfree.push_back(r.b);
    }
    g_trec.clear();
    g_timing = enable != 0;
    return LS_OK;
}

ls_status ls_timing_read(ls_kernel_timing* out, uint32_t cap, uint32_t* count) {
    if (!out || !count) return fail(LS_EINVAL, "out / count is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    ls_kernel_timing agg[KI_N];
    std::memset(agg, 0, sizeof(agg));
    for (const TRec& r : g_trec) {
        float ms = 0;
        if (r.a && r.b) {
            HIP_TRY(hipEventSynchronize(r.b));
            HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        }
        agg[r.kid].launches++;
        agg[r.kid].ms += ms;
        agg[r.kid].keys += r.keys;
    }
    uint32_t k = 0;
    for (int i = 0; i < KI_N && k < cap; i++) {
        if (!agg[i].launches) continue;
        out[k] = agg[i];
        std::snprintf(out[k].name, sizeof(out[k].name), "%s", KNAME[i]);
        k++;
    }
    *count = k;
    return LS_OK;
}

ls_status ls_timing_records(ls_kernel_timing* out, uint32_t cap, uint32_t* count) {
    if (!out || !count) return fail(LS_EINVAL, "out / count is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    uint32_t k = 0;
    for (const TRec& r : g_trec) {
        if (k >= cap) break;
        float ms = 0;
        if (r.a && r.b) {
            HIP_TRY(hipEventSynchronize(r.b));
            HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        }
        std::memset(&out[k], 0, sizeof(out[k]));
        out[k].launches = 1;
        out[k].ms = ms;
        out[k].keys = r.keys;
        std::snprintf(out[k].name, sizeof(out[k].name), "%s", KNAME[r.kid]);
        k++;
    }
    *count = k;
    return LS_OK;
}

ls_status ls_sample(const void* keys, uint64_t n, ls_dtype dtype, uint64_t seed, uint64_t S, void* out, void* stream) {
    ls_status s = check_keys(keys, n, dtype, nullptr);
    if (s) return s;
    if (S > 0 && (n == 0 || !out)) return fail(LS_EINVAL, "sampling needs n > 0 and an output");
    if (S == 0) return LS_OK;
    HIP_TRY(launch_gather((const uint64_t*)keys, n, seed, S, (uint64_t*)out, (hipStream_t)stream));
    return LS_OK;
}

ls_status ls_rmi_fit(const void* sorted_sample, uint64_t S, ls_dtype dtype, uint32_t L, double R, double* params,
                     void* stream) {
    ls_status s = check_keys(sorted_sample, S, dtype, nullptr);
    if (s) return s;
    if (S < 2 || L < 2 || L > L_MAX || !params || !(R >= 1.0) || R > 4294967296.0)
        return fail(LS_EINVAL, "ls_rmi_fit needs S >= 2, 2 <= L <= 1024, R >= 1, params");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    FitArgs A{};
    A.s = (const uint64_t*)sorted_sample; A.S = S; A.n = S; A.u64 = dtype == LS_U64; A.mode = 1;
    A.L = L; A.B1 = 1; A.log2B2 = 0; A.R = R; A.Bt = 2; A.G = FIT_G;
    A.part = (double*)(base + Lo.o_part);
    A.leaf = (double*)(base + Lo.o_leaf);
    A.model = (uint64_t*)(base + Lo.o_bigmodel);
    A.flag = (uint32_t*)(base + Lo.o_flag);
    A.seg = nullptr;
    HIP_TRY(launch_fit1(A, st));
    HIP_TRY(launch_fit2(A, st));
    HIP_TRY(launch_fit_root(A, st));
    HIP_TRY(launch_fit_leaves(A, st));
    HIP_TRY(launch_fit_finish(A, st));
    HIP_TRY(launch_copy_words(A.model + 4, (uint64_t*)params, 2 + 4ull * L, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_rmi_fit_block(const void* sorted_sample, uint64_t S, ls_dtype dtype, uint32_t L, double R,
                           double* params, void* stream) {
    ls_status s = check_keys(sorted_sample, S, dtype, nullptr);
    if (s) return s;
    if (S < 2 || S > (uint64_t)S_LDS || L < 2 || L > L_MAX || !params || !(R >= 1.0) || R > 4294967295.0 ||
        R != std::floor(R))
        return fail(LS_EINVAL, "ls_rmi_fit_block needs 2 <= S <= 16384, 2 <= L <= 1024, integer 1 <= R < 2^32, params");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    double* mdl = (double*)(base + Lo.o_bigmodel);
    HIP_TRY(launch_fit_block((const uint64_t*)sorted_sample, (uint32_t)S, dtype == LS_U64, L, (uint32_t)R, mdl, st));
    HIP_TRY(launch_copy_words((const uint64_t*)(mdl + 4), (uint64_t*)params, 2 + 4ull * L, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_rmi_buckets(const void* keys, uint64_t n, ls_dtype dtype, const double* params, uint32_t L, double R,
                         uint32_t* out, void* stream) {
    ls_status s = check_keys(keys, n, dtype, nullptr);
    if (s) return s;
    if (L < 2 || L > L_MAX || !params || !(R >= 1.0) || R > 4294967296.0 || (n && !out))
        return fail(LS_EINVAL, "ls_rmi_buckets needs 2 <= L <= 1024, 1 <= R <= 2^32, params, out");
    if (n == 0) return LS_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    uint64_t* mdl = (uint64_t*)(base + Lo.o_bigmodel);
    HIP_TRY(launch_install_rmi(params, L, R, 1, 0, mdl, st));
    HIP_TRY(launch_model_buckets(mdl, 6 + 4 * L, K_RMI_FINE, 0, 0, (const uint64_t*)keys, n, dtype == LS_U64, out, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_splitters(const void* sorted_sample, uint64_t S, ls_dtype dtype, uint32_t B, uint64_t* splitters,
                       uint8_t* eq, uint32_t* m, void* stream) {
    ls_status s = check_keys(sorted_sample, S, dtype, nullptr);
    if (s) return s;
    if (S < 1 || B < 2 || B > B_MAX || S >= (1ull << 32) || !splitters || !eq || !m)
        return fail(LS_EINVAL, "ls_splitters needs S >= 1, 2 <= B <= 1024 and outputs");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    HIP_TRY(launch_splitters((const uint64_t*)sorted_sample, S, dtype == LS_U64, B, (uint64_t*)(base + Lo.o_bigmodel),
                             splitters, eq, m, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_splitter_buckets(const void* keys, uint64_t n, ls_dtype dtype, const uint64_t* splitters, const uint8_t* eq,
                              uint32_t m, uint32_t* out, void* stream) {
    ls_status s = check_keys(keys, n, dtype, nullptr);
    if (s) return s;
    if (m < 1 || m >= B_MAX || !splitters || !eq || (n && !out))
        return fail(LS_EINVAL, "ls_splitter_buckets needs 1 <= m < 1024, splitters, eq, out");
    if (n == 0) return LS_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    uint64_t* mdl = (uint64_t*)(base + Lo.o_bigmodel);
    HIP_TRY(launch_install_tree(splitters, eq, m, mdl, st));
    uint32_t words = 2 + m + (m + 1 + 3) / 4;
    HIP_TRY(launch_model_buckets(mdl, words, K_TREE, 0, 0, (const uint64_t*)keys, n, dtype == LS_U64, out, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

static ls_status partition_one(const void* keys, const uint32_t* payload, uint64_t n, ls_dtype dtype, bool rmi,
                               const double* params, uint32_t L, double R, uint32_t nb, const uint64_t* splitters,
                               const uint8_t* eq, uint32_t m, void* out_keys, uint32_t* out_payload, uint64_t* counts,
                               void* stream) {
    ls_status s = check_keys(keys, n, dtype, payload);
    if (s) return s;
    if (n == 0) return LS_OK;
    if (!out_keys || !counts || (payload && !out_payload)) return fail(LS_EINVAL, "missing output");
    if (((uintptr_t)out_keys) & 7 || ((uintptr_t)out_payload) & 3) return fail(LS_EINVAL, "misaligned output");
    uint32_t log2B2 = 0;
    if (rmi) {
        if (L < 2 || L > L_MAX || !params || nb < 1 || nb > B_MAX || !(R >= nb)) return fail(LS_EINVAL, "bad RMI arguments");
        double ratio = R / nb;
        while ((double)(1u << log2B2) < ratio && log2B2 < 20) log2B2++;
        if ((double)(1u << log2B2) != ratio || (double)nb * (1u << log2B2) != R)
            return fail(LS_EINVAL, "R / nb must be a power of two");
    } else {
        if (m < 1 || m >= B_MAX / 2 || !splitters || !eq) return fail(LS_EINVAL, "bad splitter arguments");
    }
    Opts o;
    normalize(nullptr, o);
    std::lock_guard<std::mutex> lk(g_mu);
    Layout Lo = plan(n, 1, payload != nullptr, o);
    Lo.S_big = 0;
    DevPool* pool;
    uint8_t* base;
    hipStream_t st = (hipStream_t)stream;
    if ((s = acquire(Lo.bytes, Lo, pool, base, st))) return s;
    if ((s = order_after_last(pool, st))) return s;
    if ((s = prepare_status(pool, base, Lo, st))) return s;
    uint64_t* mdl = (uint64_t*)(base + Lo.o_bigmodel);
    Seg sg{};
    if (rmi) {
        HIP_TRY(launch_install_rmi(params, L, R, nb, log2B2, mdl, st));
        sg.kind = K_RMI; sg.nb = nb; sg.flags = SEG_PREBUILT | ((6 + 4 * L) << 16);
    } else {
        HIP_TRY(launch_install_tree(splitters, eq, m, mdl, st));
        sg.kind = K_TREE; sg.nb = 0;  // filled below from the flags
        sg.flags = SEG_PREBUILT | ((2 + m + (m + 1 + 3) / 4) << 16);
    }
    sg.model = (uint64_t)mdl;
    Call c{};
    c.keys = (uint64_t*)keys; c.pay = (uint32_t*)payload; c.n = n; c.m = 1; c.offsets = nullptr; c.u64 = dtype == LS_U64;
    c.o = o; c.st = st; c.one_level = true; c.out_keys = (uint64_t*)out_keys; c.out_pay = out_payload;
    Params P = make_params(c, Lo, base);
    if (!rmi) {
        // number of buckets = m + 1 + (flags set); read the flags once on the host
        std::vector<uint8_t> h(m);
        HIP_TRY(hipMemcpyAsync(h.data(), eq, m, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        uint32_t ne = 0;
        for (uint8_t f : h) ne += f ? 1 : 0;
        sg.nb = m + 1 + ne;
    }
    HIP_TRY(hipMemcpyAsync(P.segs[1], &sg, sizeof(Seg), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // sg lives on this stack frame
    if ((s = run(c, Lo, base, pool))) return s;
    HIP_TRY(launch_copy_words((const uint64_t*)P.counts, counts, sg.nb, st));  // segment 0 takes counts[0..nb)
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_partition_rmi(const void* keys, const uint32_t* payload, uint64_t n, ls_dtype dtype, const double* params,
                           uint32_t L, double R, uint32_t nb, void* out_keys, uint32_t* out_payload, uint64_t* counts,
                           void* stream) {
    return partition_one(keys, payload, n, dtype, true, params, L, R, nb, nullptr, nullptr, 0, out_keys, out_payload,
                         counts, stream);
}

ls_status ls_partition_splitters(const void* keys, const uint32_t* payload, uint64_t n, ls_dtype dtype,
                                 const uint64_t* splitters, const uint8_t* eq, uint32_t m, void* out_keys,
                                 uint32_t* out_payload, uint64_t* counts, void* stream) {
    return partition_one(keys, payload, n, dtype, false, nullptr, 0, 0, 0, splitters, eq, m, out_keys, out_payload,
                         counts, stream);
}

ls_status ls_mlp_loss_grad(const float* params, const float* t, const float* y, uint64_t S, float* grad, float* loss,
                           void* stream) {
    if (!params || !t || !y || S == 0 || (!grad && !loss))
        return fail(LS_EINVAL, "ls_mlp_loss_grad needs params, t, y, S >= 1 and an output");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    ls_status s = step_scratch(base, pool, Lo, (hipStream_t)stream);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    const MlpState ms = mlp_state(base, Lo);
    HIP_TRY(launch_mlp_setup(t, S, params, 0.0, ms.p, ms.m, ms.v, ms.best, ms.scale, ms.best_loss, ms.done, nullptr,
                             st));
    MlpStep A{};
    A.t = t; A.y = y; A.S = S; A.p = ms.p; A.m = ms.m; A.v = ms.v; A.partial = ms.partial; A.done = ms.done;
    A.grad_out = grad; A.loss_out = loss; A.step = 1; A.update = 0;
    HIP_TRY(launch_mlp_step(A, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_mlp_loss_grad_regions(const float* params, const float* t, const float* y, uint64_t S, float* grad,
                                   float* loss, void* stream) {
    if (!params || !t || !y || S == 0 || (!grad && !loss))
        return fail(LS_EINVAL, "ls_mlp_loss_grad_regions needs params, t, y, S >= 1 and an output");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    ls_status s = step_scratch(base, pool, Lo, (hipStream_t)stream, S);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    const MlpState ms = mlp_state(base, Lo);
    HIP_TRY(launch_mlp_setup(t, S, params, 0.0, ms.p, ms.m, ms.v, ms.best, ms.scale, ms.best_loss, ms.done, nullptr,
                             st));
    double* mom = (double*)(base + Lo.o_mlp_mom);
    HIP_TRY(launch_mlp_moments(t, y, S, (double*)(base + Lo.o_mlp_bsum), mom, nullptr, st));
    MlpRegion R{};
    R.t = t; R.mom = mom; R.S = S; R.p = ms.p; R.m = ms.m; R.v = ms.v; R.grad_out = grad; R.loss_out = loss;
    R.steps = 0;
    HIP_TRY(launch_mlp_regions(R, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_mlp_train(const void* sorted_sample, uint64_t S, ls_dtype dtype, const float* params_init, uint32_t steps,
                       float lr, float* params_out, double* lo_inv, float* losses, void* stream) {
    ls_status s = check_keys(sorted_sample, S, dtype, nullptr);
    if (s) return s;
    if (S < 2 || !params_out || !lo_inv || !(lr > 0.0f) || steps > 100000)
        return fail(LS_EINVAL, "ls_mlp_train needs S >= 2, lr > 0, steps <= 100000, params_out and lo_inv");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream, S))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    const MlpState ms = mlp_state(base, Lo);
    float* t = (float*)(base + Lo.o_mlp_t);
    float* y = (float*)(base + Lo.o_mlp_y);
    HIP_TRY(launch_mlp_prep((const uint64_t*)sorted_sample, S, 1, dtype == LS_U64, t, y, lo_inv, nullptr, st));
    HIP_TRY(launch_mlp_setup(t, S, params_init, 1e-3, ms.p, ms.m, ms.v, ms.best, ms.scale, ms.best_loss, ms.done,
                             nullptr, st));
    if (steps) {
        double* mom = (double*)(base + Lo.o_mlp_mom);
        HIP_TRY(launch_mlp_moments(t, y, S, (double*)(base + Lo.o_mlp_bsum), mom, nullptr, st));
        MlpRegion R{};
        R.t = t; R.mom = mom; R.S = S; R.p = ms.p; R.m = ms.m; R.v = ms.v; R.scale = ms.scale;
        R.best = ms.best; R.best_loss = ms.best_loss; R.losses = losses;
        R.steps = steps; R.lr = lr; R.b1 = 0.9f; R.b2 = 0.999f; R.eps = 1e-8f;
        HIP_TRY(launch_mlp_regions(R, st));
    }
    HIP_TRY(hipMemcpyAsync(params_out, ms.best, 4 * MLP_NP, hipMemcpyDeviceToDevice, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_mlp_buckets(const void* keys, uint64_t n, ls_dtype dtype, const float* params, const double* lo_inv,
                         uint32_t R, uint32_t* out, void* stream) {
    ls_status s = check_keys(keys, n, dtype, nullptr);
    if (s) return s;
    if (!params || !lo_inv || R < 1 || R > (1u << 24) || (n && !out))
        return fail(LS_EINVAL, "ls_mlp_buckets needs params, lo_inv, 1 <= R <= 2^24 and out");
    if (n == 0) return LS_OK;
    HIP_TRY(launch_mlp_buckets(params, lo_inv, R, (const uint64_t*)keys, n, dtype == LS_U64, out, (hipStream_t)stream));
    return LS_OK;
}

ls_status ls_mlp_rmi_fit(const void* sorted_sample, uint64_t S, ls_dtype dtype, const float* params,
                         const double* lo_inv, uint32_t L, double R, double* leaves, void* stream) {
    ls_status s = check_keys(sorted_sample, S, dtype, nullptr);
    if (s) return s;
    if (S < 2 || L < 2 || L > L_MAX || !params || !lo_inv || !leaves || !(R >= 1.0) || R > 4294967296.0)
        return fail(LS_EINVAL, "ls_mlp_rmi_fit needs S >= 2, 2 <= L <= 1024, 1 <= R <= 2^32 and all pointers");
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    FitArgs A{};
    A.s = (const uint64_t*)sorted_sample; A.S = S; A.n = S; A.u64 = dtype == LS_U64; A.mode = 1; A.mlp = 1;
    A.L = L; A.B1 = 1; A.log2B2 = 0; A.R = R; A.Bt = 2; A.G = FIT_G;
    A.part = (double*)(base + Lo.o_part);
    A.leaf = (double*)(base + Lo.o_leaf);
    A.model = (uint64_t*)(base + Lo.o_bigmodel);
    A.flag = (uint32_t*)(base + Lo.o_flag);
    HIP_TRY(launch_mlp_install(params, lo_inv, L, 1, 0, R, nullptr, nullptr, A.flag, A.model, st));
    HIP_TRY(launch_fit_leaves(A, st));
    HIP_TRY(launch_fit_finish(A, st));
    HIP_TRY(launch_copy_words(A.model + MLP_LEAF_WORD, (uint64_t*)leaves, 4ull * L, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

ls_status ls_mlp_rmi_buckets(const void* keys, uint64_t n, ls_dtype dtype, const float* params, const double* lo_inv,
                             const double* leaves, uint32_t L, double R, uint32_t* out, void* stream) {
    ls_status s = check_keys(keys, n, dtype, nullptr);
    if (s) return s;
    if (L < 2 || L > L_MAX || !params || !lo_inv || !leaves || !(R >= 1.0) || R > 4294967296.0 || (n && !out))
        return fail(LS_EINVAL, "ls_mlp_rmi_buckets needs 2 <= L <= 1024, 1 <= R <= 2^32 and all pointers");
    if (n == 0) return LS_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t* base;
    DevPool* pool;
    Layout Lo;
    if ((s = step_scratch(base, pool, Lo, (hipStream_t)stream))) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(pool, st))) return s;
    uint64_t* mdl = (uint64_t*)(base + Lo.o_bigmodel);
    HIP_TRY(launch_mlp_install(params, lo_inv, L, 1, 0, R, leaves, nullptr, nullptr, mdl, st));
    HIP_TRY(launch_mlp_rmi_buckets(mdl, (const uint64_t*)keys, n, dtype == LS_U64, out, st));
    return mark_done(pool, st, (Ctl*)(base + Lo.o_ctl));
}

static ls_status stream_args(const void* a, const void* b, uint64_t n, const char* name, uint32_t& cus) {
    if (n > 0 && (!a || !b)) return fail(LS_EINVAL, std::string(name) + ": NULL pointer with n > 0");
    if (((uintptr_t)a | (uintptr_t)b) & 7) return fail(LS_EINVAL, std::string(name) + ": pointers must be 8-byte aligned");
    if (n >= (1ull << 45)) return fail(LS_EINVAL, std::string(name) + ": n too large");
    int dev = 0, c = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    cus = (uint32_t)std::max(c, 1);
    return LS_OK;
}

ls_status ls_stream_copy(const void* src, void* dst, uint64_t n, void* stream) {
    if (n == 0) return LS_OK;
    uint32_t cus = 0;
    ls_status s = stream_args(src, dst, n, "ls_stream_copy", cus);
    if (s) return s;
    HIP_TRY(launch_stream_copy((const uint64_t*)src, (uint64_t*)dst, n, cus, (hipStream_t)stream));
    return LS_OK;
}

ls_status ls_stream_read(const void* src, uint64_t n, uint64_t* sum, void* stream) {
    uint32_t cus = 0;
    if (!sum) return fail(LS_EINVAL, "ls_stream_read: sum is NULL");
    ls_status s = stream_args(n ? src : sum, sum, n, "ls_stream_read", cus);
    if (s) return s;
    HIP_TRY(launch_stream_read((const uint64_t*)src, n, sum, cus, (hipStream_t)stream));
    return LS_OK;
}

ls_status ls_tuned_options(uint64_t n_total, uint64_t m, ls_options* out) {
    if (!out) return fail(LS_EINVAL, "out is NULL");
    Opts o;
    ls_status s = normalize(nullptr, o, std::max<uint64_t>(n_total, 1), std::max<uint64_t>(m, 1));
    if (s) return s;
    std::memset(out, 0, sizeof(*out));
    out->struct_size = sizeof(ls_options);
    out->model = o.model; out->buckets = o.buckets; out->leaves = o.leaves; out->tree_buckets = o.tree_buckets;
    out->cutoff = o.cutoff; out->max_levels = o.max_levels; out->flags = o.flags; out->sample_frac = o.sample_frac;
    out->fallback_ratio = o.fallback_ratio; out->seed = o.seed; out->mlp_steps = o.mlp_steps;
    out->mlp_sample = o.mlp_sample; out->mlp_lr = o.mlp_lr; out->tile = o.tile; out->balance_pct = o.balance_pct;
    return LS_OK;
}

}  // extern "C"
