// lsort_internal.hpp -- data layout shared by the HIP kernels and the host
// planner of liblsort (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ls {

// ---- sizes ---------------------------------------------------------------
constexpr int WAVE = 64;
constexpr int P_THREADS = 512;                 // threads of a partition workgroup (8 waves)
constexpr int P_WAVES = P_THREADS / WAVE;
constexpr int KPT = 16;                        // keys per thread per tile
constexpr int TILE = P_THREADS * KPT;          // 8192 keys: one pass of a partition workgroup
constexpr int UNIT_TILES = 4;
constexpr int UNIT = TILE * UNIT_TILES;        // 32768 keys: work unit of k_hist / k_scatter
constexpr int WAVE_KEYS = WAVE * KPT;          // 1024 keys per wave per tile
constexpr int B_MAX = 1024;                    // buckets of one partition
constexpr int L_MAX = 1024;                    // RMI leaves
constexpr int S_LDS = 16384;                   // largest sample one workgroup sorts in LDS
constexpr int C_MAX = 4096;                    // largest base-case cutoff an option may set
constexpr int BIG_MAX = 8192;                  // largest sub-array the base case takes (k_base_big)
constexpr int SMALL_MAX = 512;                 // largest sub-array one wavefront sorts in registers
constexpr int GROUP_MAX = 256;                 // largest sub-array a lane group sorts (4 per wavefront)
constexpr int GROUP_SMALL_MAX = 128;           // ... sorted by a smaller lane group (8 per wavefront)
constexpr int GROUP_LARGE_MAX = 1024;          // keys only: largest sub-array two per wavefront are sorted
constexpr int GROUP_WAVE_MAX = 2048;           // keys only: largest sub-array one wavefront sorts in registers
constexpr uint32_t MB_MIN = 64, MB_MAX = 1024;  // sub-arrays the model-based counting sort takes
constexpr int MAXL = 32;                       // partition levels (arrays)
constexpr int MODEL_WORDS = 4 + 2 + 4 * L_MAX; // 8-byte words of the largest model (RMI, L_MAX leaves)
constexpr int LDS_MODEL_WORDS = 4 + 2 + 3 * L_MAX;  // ... of its LDS image in the partition kernels
constexpr uint64_t COPY_CHUNK = 65536;         // keys per copy item

// ---- MLP parameter layout (321 floats) -------------------------------------
constexpr int MLP_H = 16, MLP_HALF = 8, MLP_NP = 321;
constexpr int OFF_V1 = 0, OFF_B1 = 16, OFF_V2 = 32, OFF_B2 = 288, OFF_V3 = 304, OFF_B3 = 320;

// ---- partition kinds -------------------------------------------------------
enum Kind : uint32_t {
    K_FRESH = 1,     // build a model from a sample of this segment (Alg. 5 policy)
    K_RMI = 2,       // RMI fitted for this segment; bucket = g >> log2(B2)
    K_RMI_FINE = 3,  // child of an RMI level: same model, bucket = g - win
    K_TREE = 4,      // splitter tree (fallback or policy)
    K_RADIX = 5,     // range radix (depth cap; guaranteed progress)
    K_MLP = 6,       // MLP CDF; bucket = g >> log2(B2)
    K_MLP_FINE = 7,  // child of an MLP level
    K_TREE_FORCED = 8,  // splitter tree requested by the fallback rule
};

// Model headers (8-byte aligned, followed by their payload in the arena).
struct RmiModel {     // 32 bytes, followed by double p[2 + 4L] (model word 4 on)
    uint32_t L, B1, log2B2, pad;
    double R;         // B1 << log2B2
    uint64_t pad2;
};
static_assert(sizeof(RmiModel) == 32, "RMI parameters start at model word 4");
struct TreeModel {    // 16 bytes, followed by uint64 u[m] then uint16 lut[m+1]
    uint32_t m, nb, top, pad;
};
static_assert(sizeof(TreeModel) == 16, "splitters start at model word 2");
struct RadixModel {
    uint64_t lo;
    uint32_t shift, nb;
};
static_assert(sizeof(RadixModel) == 16, "radix model is two words");
// Two-level model whose root is the monotone MLP: 48-byte header, the
// network's effective weights (|V|, biases) as float w[321] from model word
// MLP_W_WORD, then the pre-scaled leaves (alpha, beta, gamma, delta) x L as
// doubles from model word MLP_LEAF_WORD.
struct MlpModel {
    uint32_t L, B1, log2B2, pad;
    double lo, inv;   // model input t = clamp((x - lo) * inv, 0, 1)
    double R;         // B1 << log2B2
    uint64_t pad2;
};
static_assert(sizeof(MlpModel) == 48, "MLP weights start at model word 6");
constexpr int MLP_W_WORD = 6;
constexpr int MLP_LEAF_WORD = MLP_W_WORD + (MLP_NP + 1) / 2;  // 167
constexpr int MLP_MODEL_WORDS = MLP_LEAF_WORD + 4 * L_MAX;

// One sub-array partitioned at some level.
struct Seg {
    uint64_t off;     // absolute index of the first key
    uint64_t n;       // keys
    uint64_t model;   // device address of the model
    uint64_t cbase;   // bucket counts at counts[cbase..+nb), bucket starts at counts[cbase+nb..+nb)
    uint64_t sbase;   // look-back status words at status[sbase + unit * nb + b]
    uint32_t kind;    // Kind
    uint32_t nb;      // buckets
    uint32_t win;     // fine window base for *_FINE kinds
    uint32_t tile0;   // first work unit in the level's unit list
    uint32_t ntiles;  // work units (UNIT keys each, the last one partial)
    uint32_t flags;   // SEG_* bits; model size in 8-byte words in bits 16..31
};
static_assert(sizeof(Seg) == 64, "segment descriptor is 64 bytes");
constexpr uint32_t FLAG_STATS = 0x8u;   // LS_FLAG_COLLECT_STATS: per-level statistics wanted
constexpr uint32_t FLAG_REFIT = 0x20u;  // LS_FLAG_REFIT: children of learned buckets get fresh models
constexpr uint32_t FLAG_MODEL_BASE = 0x40u;  // LS_FLAG_MODEL_BASE: model-based counting-sort base case
constexpr uint32_t SEG_PREBUILT = 1u;  // model already built (large first level)
constexpr uint32_t SEG_FAILED = 2u;    // capacity exceeded; not partitioned
constexpr uint32_t SEG_RESIDENT = 4u;  // sorted by one workgroup (k_resident): no work units
constexpr uint32_t SEG_FROM_SAMPLE = 8u;  // fallback child of the first level: its tree's sample is the
                                          // first-level sample's run in its bucket (model = parent's, win = bucket)
constexpr uint64_t RES_MAX = 8192;     // largest segment a single workgroup takes (one work unit)
// Work units of a segment: UNIT << s keys, s in bits 8..10 of the flags (0
// for every segment below the first level).  k_scatter carries a bucket's
// last partial 64-byte segment from tile to tile within a unit, so larger
// units leave fewer partial segments in the output.
// Value 7 marks one-tile units (TILE keys): a single array of at most
// SMALL_UNIT_N keys, whose few units of UNIT keys would leave most CUs idle
// (the nested sort of a large array's sample is one).
constexpr uint32_t SEG_USHIFT_POS = 8, USHIFT_MAX = 4, USHIFT_TILE = 7;
constexpr uint64_t SMALL_UNIT_N = 1ull << 20;
__host__ __device__ inline uint32_t seg_unit(uint32_t flags) {
    const uint32_t s = (flags >> SEG_USHIFT_POS) & 7u;
    return s == USHIFT_TILE ? (uint32_t)TILE : (uint32_t)UNIT << s;
}

struct Tile {          // one work unit of UNIT keys
    uint32_t seg;     // index in the level's segment list
    uint32_t idx;     // unit number within the segment
};

// Base-case / copy work item packed in 64 bits:
// [63:18] offset, [17] source buffer (0 caller, 1 temp), [16] copy-only, [15:0] size - 1.
// Base-case items sorted as chunks of their own, then merged: keys only,
// items of GROUP_WAVE_MAX+1 .. BIG_MAX keys in chunks of GROUP_WAVE_MAX keys
// (the register group sort); with a payload, items of SMALL_MAX+1 .. BIG_MAX
// keys in chunks of PAIR_CHUNK keys (the wavefront pair sort; an item of one
// chunk needs no merge).  The number of chunks (the last one shorter), 0 for
// any other size.
constexpr int PAIR_CHUNK = 1024;
__host__ __device__ inline uint32_t chunk_keys(bool pay) { return pay ? (uint32_t)PAIR_CHUNK : (uint32_t)GROUP_WAVE_MAX; }
__host__ __device__ inline uint64_t split_chunks(uint64_t c, bool pay) {
    const uint64_t lo = pay ? (uint64_t)SMALL_MAX : (uint64_t)GROUP_WAVE_MAX, ch = chunk_keys(pay);
    return c > lo && c <= (uint64_t)BIG_MAX ? (c + ch - 1) / ch : 0;
}

__host__ __device__ inline uint64_t item_pack(uint64_t off, uint32_t src, uint32_t copy, uint32_t size) {
    return (off << 18) | ((uint64_t)src << 17) | ((uint64_t)copy << 16) | (uint64_t)(size - 1);
}

// Per-level statistics (device; mirrors ls_level_stats).
struct LevelStats {
    unsigned long long segments, keys, buckets, max_bucket, max_ratio_x1000, empty, equality, base, recurse,
        fallback, learned, tree, radix;
};

// Control block at the start of the workspace.
// Counters that every workgroup of a launch updates with device-scope atomics
// each sit in a 256-byte slot of their own: atomics on one address are
// serialised where they are performed, but different lines proceed in
// parallel (a level of ~1000 segments updates about ten of these counters per
// segment).
#define LS_HOT alignas(256)
struct Ctl {
    LS_HOT uint32_t nseg[MAXL + 1];         // segments at each level
    LS_HOT uint32_t ntile[MAXL + 1];        // tiles at each level
    LS_HOT uint32_t ticket[MAXL + 1];       // scatter unit tickets
    LS_HOT uint32_t rticket[MAXL + 1];      // k_resident segment tickets
    LS_HOT uint32_t hticket[MAXL + 1];      // k_hist unit tickets
    LS_HOT uint32_t nres[MAXL + 1];         // segments at each level that k_resident sorts whole
    LS_HOT uint32_t nsplit[MAXL + 1];       // work units of a level re-cut into one-tile units (Params::split)
    LS_HOT unsigned long long nitems;       // small base-case items of <= GROUP_SMALL_MAX keys (front of items)
    LS_HOT unsigned long long nitems_w;     // small base-case items of GROUP_MAX+1 .. SMALL_MAX keys (back of items)
    LS_HOT unsigned long long nitems_b;     // small base-case items of GROUP_SMALL_MAX+1 .. GROUP_MAX keys (items_b)
    LS_HOT unsigned long long nitems_k;     // keys only: items of SMALL_MAX+1 .. GROUP_LARGE_MAX keys (back of items_b)
    LS_HOT unsigned long long nitems_c;     // keys only: items of GROUP_LARGE_MAX+1 .. GROUP_WAVE_MAX keys (items_c)
    LS_HOT unsigned long long nbig;         // large base-case items and copy items
    LS_HOT unsigned long long nmoved;       // small items handed on to the large list (NaN / -0.0 tasks)
    LS_HOT unsigned long long nitems_m;     // items of the model-based counting sort (two words each)
    LS_HOT unsigned long long nmerge;       // items sorted as chunks, then merged (k_base_merge; split_chunks)
    LS_HOT unsigned long long merge_keys;   // keys in those items
    LS_HOT unsigned long long nmerge_cls[2];  // those of more than GROUP_WAVE_MAX keys, of more than 2 GROUP_WAVE_MAX
    LS_HOT unsigned long long nchunk;       // their chunks (in nitems_c)
    LS_HOT unsigned long long model_keys;   // keys in those items
    LS_HOT unsigned long long ncopy;
    LS_HOT unsigned long long small_keys;   // keys in small base-case items
    LS_HOT unsigned long long big_keys;     // keys in large base-case items and copy runs
    LS_HOT unsigned long long counts_used;  // bump allocators (reset per level)
    LS_HOT unsigned long long status_used;
    LS_HOT unsigned long long arena_used[2];
    LS_HOT uint32_t overflow;               // OVF_* bits
    uint32_t first_mlp;                     // the first level's model is the MLP-rooted one
    double mlp_loss[2];                     // MLP training loss at the first and the last step
    LS_HOT LevelStats lv[MAXL];
};
#undef LS_HOT
constexpr uint32_t OVF_SEG = 1, OVF_TILE = 2, OVF_ITEM = 4, OVF_COUNTS = 8, OVF_STATUS = 16, OVF_ARENA = 32,
                   OVF_STATE = 64;  // a look-back word without this level's tag (never expected)

// Everything a level's kernels need, passed by value.
struct Params {
    // buffers: index 0 = caller's keys, 1 = temporary
    uint64_t* keys[2];
    uint32_t* pay[2];               // null when there is no payload
    int u64;                        // dtype: 1 uint64, 0 float64
    int has_pay;
    // options
    uint32_t buckets, leaves, tree_buckets, cutoff, max_levels, flags, model;
    uint32_t unit0_shift;           // first-level segments: work units of UNIT << unit0_shift keys
    uint32_t split;                 // this level has fewer units than CUs: k_model re-cuts every segment
                                    // into one-tile units, counted in ctl->nsplit
    double sample_frac, fallback_ratio;
    uint64_t seed;
    // workspace
    Ctl* ctl;
    Seg* segs[2];
    Tile* tiles[2];
    uint64_t* items;                // small base-case items: <= GROUP_SMALL_MAX keys from the front,
                                    // GROUP_MAX+1 .. SMALL_MAX keys from the back
    uint64_t* items_b;              // small base-case items of GROUP_SMALL_MAX+1 .. GROUP_MAX keys from the
                                    // front, keys only SMALL_MAX+1 .. GROUP_LARGE_MAX from the back
    uint64_t* bigs;                 // large base-case items and copy items
    unsigned long long* counts;
    unsigned long long* status;
    uint8_t* arena[2];
    uint16_t* ids;                  // per-key bucket ids of MLP levels (absolute positions)
    uint64_t* items_c;              // keys only: items of GROUP_LARGE_MAX+1 .. GROUP_WAVE_MAX keys and the
                                    // chunks of larger ones; with a payload: items and chunks of
                                    // SMALL_MAX+1 .. PAIR_CHUNK keys (k_base_pairs)
    uint64_t* items_m;              // model-based counting-sort items: (item word, g0 | log2(w) << 32)
    uint64_t item_m_cap;
    uint64_t* merges;               // items whose chunks are merged (k_base_merge)
    uint64_t merge_cap;
    const uint64_t* fmodel;         // the first level's prebuilt model (large single array), or null
    uint64_t seg_cap, tile_cap, item_cap, big_cap, counts_cap, status_cap, arena_cap, item_b_cap, item_c_cap;
    const uint64_t* persist;        // [0] call epoch, [1] clear-status request (survives calls)
    const uint64_t* fsample;        // sorted first-level sample of a large array (raw keys), or null
    const uint64_t* fbstart;        // [B1 + 1]: first sample index of each first-level bucket
    uint64_t fS;                    // its size
    int level;
};

// Work units of the level the kernels run on (k_model re-cut them when split).
__device__ __forceinline__ uint32_t level_units(const Params& P, int lvl) {
    return min(P.split ? P.ctl->nsplit[lvl] : P.ctl->ntile[lvl], (uint32_t)P.tile_cap);
}

// Status word of the decoupled look-back:
// [63:38] tag = call epoch * MAXL + level (never 0), [37:36] flag
// (1 aggregate, 2 inclusive prefix), [35:0] value.
constexpr int ST_TAG_BITS = 26;
constexpr int ST_TAG_SHIFT = 38;
constexpr uint64_t ST_VALUE_MASK = (1ull << 36) - 1;
constexpr uint64_t ST_LOW_MASK = ST_VALUE_MASK;
constexpr uint64_t ST_AGG = 1ull << 36, ST_PREFIX = 2ull << 36;

}  // namespace ls
