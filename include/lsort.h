/*
 * lsort.h -- C ABI of liblsort: a learned sample sort for AMD MI355X (gfx950).
 *
 * Method: "LearnedSort as a learning-augmented SampleSort" (Carvalho &
 * Lawrence, SSDBM 2023).  A CDF model fitted on a random sample maps each key
 * to a bucket (Sec. 2.2, bucket = floor(B * F(x))); buckets are histogrammed,
 * prefix-summed and scattered; large buckets recurse, buckets whose keys are
 * all equal stop (Sec. 2.2 homogeneity check; Sec. 2.4 equality buckets) and
 * small ones get a base-case sort (Sec. 4).  The model is a monotone
 * two-level linear RMI (Sec. 2.1; monotone constraint of Sec. 4), optionally
 * with a monotone FP32 MLP as its root, or -- when the input is small or
 * duplicate-heavy (Alg. 5)
 * and whenever a bucket comes out more than twice its expected size -- a
 * splitter tree (Sec. 2.4).
 *
 * Conventions for every entry point:
 *   - Pointers to keys, payloads, offsets and outputs are DEVICE pointers
 *     (memory from hipMalloc / torch on the current device) unless a
 *     parameter says "host".  The library never frees caller memory.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without waiting, except where noted.
 *   - Return value: LS_OK (0) or a negative ls_status; ls_last_error() then
 *     holds a message (thread-local).  Nothing aborts or throws across the
 *     ABI.
 *   - Keys are float64 ordered by IEEE-754 totalOrder
 *     (-NaN < -inf < ... < -0.0 < +0.0 < ... < +inf < +NaN) or uint64 in
 *     numeric order.  Sorting is stable: a uint32 payload follows its key and
 *     equal keys keep their input order.
 *   - Calls that share a workspace (the library's own, per device, unless
 *     ls_set_workspace gave one) must not overlap in time: the library
 *     serialises them on one stream per call; two threads that sort on two
 *     streams at once must each set their own workspace.
 */
#ifndef LSORT_H
#define LSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types.  The partition engine works on 8-byte words in the order of
 * float64 totalOrder or uint64; the other two are mapped onto those around
 * the engine by order-preserving bijections: int64 by flipping the sign bit
 * (in place, undone afterwards), float32 by widening to the float64 of the
 * same value (NaNs keep sign and payload) in the workspace, 8 bytes per key,
 * and narrowing back bit for bit.  The single-step entry points take
 * LS_F64 / LS_U64 only. */
typedef enum { LS_F64 = 0, LS_U64 = 1, LS_I64 = 2, LS_F32 = 3 } ls_dtype;

typedef enum {
    LS_OK = 0,
    LS_EINVAL = -1,       /* bad argument: null pointer with n > 0, bad dtype, misalignment, bad option */
    LS_ENOMEM = -2,       /* workspace could not be allocated or is too small */
    LS_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
    LS_EUNSUPPORTED = -4  /* option combination not implemented */
} ls_status;

/* Partition model of the first level (Alg. 5 decides under LS_MODEL_AUTO). */
typedef enum {
    LS_MODEL_AUTO = 0,     /* RMI if n >= 1e5 and <= 10% sample duplicates, else splitter tree */
    LS_MODEL_RMI = 1,      /* same as AUTO (the policy may still pick the tree) */
    LS_MODEL_MLP = 2,      /* first level: two-level model whose root is a monotone 1-16-16-1 FP32 MLP
                              trained on the GPU, with linear leaves; deeper levels as AUTO.  Single
                              arrays of n >= 1e5 keys (smaller ones sort as AUTO) */
    LS_MODEL_SPLITTER = 3  /* classic SampleSort: splitter tree at every level */
} ls_model;

/* Option flags. */
#define LS_FLAG_NO_FALLBACK   0x1u  /* never replace an oversized learned bucket's model by a splitter tree */
#define LS_FLAG_SYNC_LEVELS   0x2u  /* (host) read back the work count after each level to stop early; default on */
#define LS_FLAG_FIXED_LEVELS  0x4u  /* no host read-back: launch every level the depth cap allows,
                                       min(max_levels + 9, 31) (max_levels model-based levels, then up to
                                       8 range-radix levels and one more), each exiting at once when it
                                       has no work; needed for stream capture (a call under capture
                                       without it returns LS_EINVAL).  The host cannot see a
                                       workspace overflow then: read ls_get_stats().overflow after the
                                       call (or after a graph replay); nonzero means the output is
                                       invalid */
#define LS_FLAG_COLLECT_STATS 0x8u  /* record per-level statistics (read with ls_get_stats) */
#define LS_FLAG_TUNED         0x10u /* take buckets / cutoff / tree_buckets left 0 from the loaded tuning table */
#define LS_FLAG_REFIT         0x20u /* a learned bucket that needs another level gets a model of its own (a
                                       fresh sample and fit under the Alg. 5 policy, as AIPS2o trains per
                                       call, Sec. 5.1) instead of the parent's model evaluated at a finer
                                       resolution (LearnedSort's reuse, Sec. 3.3); default off */
#define LS_FLAG_MODEL_BASE    0x40u /* base case of a large single array's RMI buckets (64..1024 keys): the
                                       model places each key (a counting sort on its fine position inside
                                       the bucket) and each key's rank among the few keys of its bin
                                       finishes the sort (LearnedSort's base case, Sec. 2.2); items the
                                       model cannot spread go to the comparison sort */

/* Options.  Zero-initialise and set struct_size = sizeof(ls_options); every
 * zero field takes its default. */
typedef struct {
    uint32_t struct_size;
    uint32_t model;          /* ls_model; default AUTO */
    uint32_t buckets;        /* B of a learned level; default 1000 (Sec. 2.1/2.2); 2..1024 */
    uint32_t leaves;         /* RMI leaves L; default 1000 (Sec. 2.1); 2..1024 */
    uint32_t tree_buckets;   /* splitter-tree fan-out; default 256 (Sec. 4); power of two 2..512 */
    uint32_t cutoff;         /* base case at or below this many keys (and the fine resolution of a reused
                                model: sub-buckets of about cutoff/2 keys); default 1024 for a single array,
                                512 for the segmented form (the paper's CPU base case takes 4096, Sec. 4);
                                1..4096 */
    uint32_t max_levels;     /* model-based levels before range radix (8 bits per level) takes over; default 16; 1..23 */
    uint32_t flags;          /* LS_FLAG_* */
    double sample_frac;      /* sample size as a fraction of n; default 0.01 (Sec. 2.2) */
    double fallback_ratio;   /* oversized bucket threshold, x expected; default 2.0 */
    uint64_t seed;           /* sampling seed; default 0x5EED */
    uint32_t mlp_steps;      /* MLP Adam steps; default 200; at most 100000 */
    uint32_t mlp_sample;     /* MLP training-set size: every k-th point of the sorted sample so that at
                                most this many remain; default 1e6 */
    float mlp_lr;            /* MLP Adam learning rate; default 3e-3 */
    uint32_t tile;           /* keys per work unit of the first level's histogram and scatter passes:
                                32768 << k, k in [0, 4]; the scatter writes each bucket's share of a unit
                                in whole 64-byte segments except its first and last; default 32768 */
    uint32_t balance_pct;    /* large single array: when the first level's fitted RMI puts more than this
                                percentage of its sample into buckets above fallback_ratio x expected,
                                the first level takes the splitter tree instead (the tree as judge of the
                                model's balance); 100 = never; default 50 (measured at 1e8 keys: no change
                                on the smooth and duplicate-heavy laws; the 70/20/10 piecewise law 3.4 ms
                                instead of 4.2 ms, at 1e9 keys 32.9 instead of 33.1 ms) */
    uint32_t reserved[3];
} ls_options;

/* Per-call statistics (LS_FLAG_COLLECT_STATS). */
#define LS_MAX_STAT_LEVELS 32
typedef struct {
    uint64_t segments;       /* sub-arrays partitioned at this level */
    uint64_t keys;           /* keys partitioned at this level */
    uint64_t buckets;        /* buckets produced (sum over segments) */
    uint64_t max_bucket;     /* largest bucket */
    uint64_t max_bucket_x1000_over_mean; /* max over segments of 1000 * max bucket / (n_seg / B_seg) */
    uint64_t empty;          /* empty buckets */
    uint64_t equality;       /* equality buckets (or single-value buckets) finished here */
    uint64_t base;           /* buckets sent to the base case */
    uint64_t recurse;        /* buckets partitioned again */
    uint64_t fallback;       /* oversized buckets re-partitioned by a splitter tree */
    uint64_t learned;        /* segments partitioned by a learned model (RMI or MLP) */
    uint64_t tree;           /* segments partitioned by a splitter tree */
    uint64_t radix;          /* segments partitioned by range radix */
} ls_level_stats;

typedef struct {
    uint32_t levels;         /* partition levels run */
    uint32_t first_model;    /* ls_model actually used by the first level of the first segment */
    uint64_t base_items;     /* base-case sub-arrays sorted */
    uint64_t copy_items;     /* finished runs copied back to the caller's buffer */
    double mlp_loss_first;   /* MLP training: loss at step 1 and at the last step */
    double mlp_loss_last;
    uint32_t overflow;       /* nonzero: a workspace capacity was exceeded and some sub-arrays were left
                                unsorted (the call returned LS_ENOMEM, or with LS_FLAG_FIXED_LEVELS could
                                not tell); bits: 1 segments, 2 work units, 4 base-case items, 8 bucket
                                counts, 16 look-back words, 32 model arena, 64 look-back sequence */
    uint32_t merged_items;   /* of base_items: sub-arrays sorted as chunks, then merged (keys only: 2049..8192
                                keys in chunks of 2048; with a payload: 1025..8192 keys in chunks of 1024) */
    ls_level_stats level[LS_MAX_STAT_LEVELS];
} ls_stats;

/* ---- Sorting -------------------------------------------------------------- */

/* Sort keys[0..n) in place (stable), permuting payload (nullable) with them
 * (Sec. 2.2 partitioning into buckets, Sec. 2.4 recursion and equality
 * buckets, Alg. 5 model choice; the result is the unique stable sort).
 * keys: device, n keys of `dtype`, 8-byte aligned (4-byte for LS_F32).
 * payload: device, 4-byte aligned, n entries, or NULL.  opt: NULL for
 * defaults.  n = 0 or 1 is a no-op.  Errors: LS_EINVAL (null keys with n > 0,
 * bad dtype, misalignment, option out of range), LS_ENOMEM, LS_EHIP. */
ls_status ls_sort(void *keys, uint64_t n, ls_dtype dtype, uint32_t *payload,
                  const ls_options *opt, void *stream);

/* ls_sort with a 64-bit payload (device, 8-byte aligned, n entries, not
 * NULL; any 8-byte values, e.g. row ids or pointers).  The engine sorts the
 * keys with their original 32-bit indices (stable) and the payload is then
 * gathered through them, which needs n < 2^32 and 12 more workspace bytes
 * per key (the indices and a saved copy of the payload).  Errors as ls_sort;
 * LS_EINVAL also for n >= 2^32. */
ls_status ls_sort_payload64(void *keys, uint64_t n, ls_dtype dtype, uint64_t *payload,
                            const ls_options *opt, void *stream);

/* Allocation-free ls_sort, for callers that cannot allocate device or host
 * memory during the call (tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as ls_sort, except:
 *   - the scratch memory is a fixed device array inside the library,
 *     LS_NOALLOC_SCRATCH_BYTES per device, held from the library's first use
 *     of a device until the process ends; a call whose workspace
 *     (ls_workspace_bytes with LS_FLAG_FIXED_LEVELS) exceeds it returns
 *     LS_ENOMEM without enqueuing anything (about 2.2e6 float64 keys without
 *     a payload, 1.9e6 with one, at the default options);
 *   - no hipMalloc, hipHostMalloc, hipFree or event creation, ever (the
 *     first call on a device looks up the array's device address);
 *   - LS_FLAG_FIXED_LEVELS is always in effect: no host read-back, so the
 *     call cannot see a workspace overflow; ls_get_stats().overflow after
 *     it tells (nonzero: output invalid);
 *   - not ordered against other calls: every call on a device shares its
 *     array, so calls on one device that overlap in time race (serialise
 *     them on one stream); no timing records are taken;
 *   - the array keeps the last call's contents; what must start at zero is
 *     cleared by the call itself. */
#define LS_NOALLOC_SCRATCH_BYTES (64ull << 20)
ls_status ls_sort_noalloc(void *keys, uint64_t n, ls_dtype dtype, uint32_t *payload,
                          const ls_options *opt, void *stream);

/* Sort each segment [offsets[i], offsets[i+1]) of keys independently, in
 * place, in one batched pass (all segments share every kernel launch; the
 * counterpart of the paper's task scheduler, Sec. 2.4).
 * offsets: DEVICE array of m + 1 non-decreasing uint64 values; offsets[m] is
 * the total length.  host_total: offsets[m] as known by the host (sizes the
 * workspace; must be >= offsets[m]).  Malformed offsets are undefined
 * behaviour.  Errors as ls_sort; LS_EUNSUPPORTED for LS_MODEL_MLP. */
ls_status ls_sort_segmented(void *keys, const uint64_t *offsets, uint64_t m, uint64_t host_total,
                            ls_dtype dtype, uint32_t *payload, const ls_options *opt, void *stream);

/* Bytes of workspace a call with these sizes needs (written to *out, host).
 * has_payload: 0 none, 1 uint32 payload, 2 64-bit payload. */
ls_status ls_workspace_bytes(uint64_t n_total, uint64_t m, ls_dtype dtype, int has_payload,
                             const ls_options *opt, size_t *out);

/* Use caller memory (device, 256-byte aligned) as the workspace of later
 * calls on this device; dev_ptr = NULL returns to the library's own pool.
 * The memory is cleared on `stream` (after every earlier call that used the
 * previous workspace), and later calls on any stream are ordered after that.
 * The library never allocates while a workspace is set: a call that needs
 * more than `bytes` fails with LS_ENOMEM.  Required before stream capture: a
 * call made while its stream is capturing fails with LS_EINVAL unless a
 * workspace is set (the library's own pool may be reallocated by a later
 * eager call, which a captured graph would not see).  The caller keeps the
 * memory alive while any graph captured with it exists; a replay must not
 * overlap another call that uses the same workspace.  Must itself be called
 * outside capture.  Errors: LS_EINVAL, LS_EHIP. */
ls_status ls_set_workspace(void *dev_ptr, size_t bytes, void *stream);

/* Statistics of the last call on this thread (per-level counts only when it
 * set LS_FLAG_COLLECT_STATS; `overflow` always), read from its workspace, so
 * after a graph replay they are the replay's.  Waits for that call's stream.
 * out: host. */
ls_status ls_get_stats(ls_stats *out);

/* Message for the last non-OK status on this thread (never NULL). */
const char *ls_last_error(void);

/* ---- Tuning (batched and single-array form) -------------------------------- */
/* Autotuner: on the current device, for each size class -- the decimal order
 * of magnitude of the average array size n / m, 1e3 .. 1e8 -- time every
 * candidate (buckets in {256, 512, 1000, 1024}, cutoff in {256, 512, 1024},
 * tree_buckets in {128, 256}; from 1e6 keys per array also the first-level
 * work unit, tile in {32768, 65536, 131072}) on synthetic arrays it generates on the device
 * (uniform, normal and lognormal laws; ~2e7 keys in arrays log-uniform over
 * [avg / 4, 4 avg) for the batched classes, one array of 1e7 or 1e8 keys for
 * the others), keep the fastest, write a JSON table to table_path (host
 * path) keyed by the device's architecture and compute-unit count, and load
 * it.  Synchronous; allocates its own buffers; takes about a minute.
 * Errors: LS_EINVAL (path), LS_EHIP, and those of ls_sort. */
ls_status ls_autotune(const char *table_path);

/* Load a table written by ls_autotune (NULL: unload).  Afterwards a call
 * with opt == NULL, or with LS_FLAG_TUNED set, takes buckets, cutoff,
 * tree_buckets and tile that it leaves 0 from the entry of its size class (the
 * nearest class present; ties go to the smaller class).  Errors: LS_EINVAL
 * (unreadable, malformed, out of range, or made on a different device
 * architecture / CU count). */
ls_status ls_load_tuning(const char *table_path);

/* The options a call over n_total keys in m arrays with opt == NULL would
 * use (defaults, or the loaded table's entry).  out: host. */
ls_status ls_tuned_options(uint64_t n_total, uint64_t m, ls_options *out);

/* Library version string, e.g. "lsort 0.1 gfx950". */
const char *ls_version(void);

/* ---- Kernel timing (measurement tools) ------------------------------------ */

/* Per-kernel totals over the calls made while timing was on.  keys: keys the
 * launches processed (hist/scatter: keys of the level; base: keys in base-case
 * and copy items; other kernels 0) -- the unit a kernel's algorithmic bytes
 * are counted per. */
typedef struct {
    char name[32];
    uint64_t launches;
    double ms;               /* summed launch durations (HIP events on the call's stream) */
    double keys;
} ls_kernel_timing;

/* Start (enable = 1) or stop (0) recording; starting clears earlier records.
 * While on, every launch is bracketed by two events on its stream and each
 * call waits for its last kernel before returning. */
ls_status ls_timing(int enable);

/* Totals per kernel name (host array of cap entries); *count gets the number
 * of names written.  Waits for the recorded work to finish. */
ls_status ls_timing_read(ls_kernel_timing *out, uint32_t cap, uint32_t *count);

/* The recorded launches one by one, in launch order (launches = 1 each;
 * keys = the keys of the level the launch belongs to).  Host array of cap
 * entries; *count gets the number written. */
ls_status ls_timing_records(ls_kernel_timing *out, uint32_t cap, uint32_t *count);

/* ---- Single steps (exposed so each step can be checked on its own) -------- */

/* Random sample with replacement (Sec. 2.2: the model is trained on a ~1%
 * sample; Alg. 5 Sample): out[k] = keys[idx_k], idx_k = high 64 bits of
 * SplitMix64(seed, k) * n (SplitMix64 of Steele, Lea & Flood, output k =
 * finaliser(seed + (k+1) * 0x9E3779B97F4A7C15)).  keys, out: device. */
ls_status ls_sample(const void *keys, uint64_t n, ls_dtype dtype, uint64_t seed, uint64_t S,
                    void *out, void *stream);

/* Fit the monotone two-level linear RMI (Sec. 2.1; monotone clamp of Sec. 4)
 * on a SORTED sample of S keys (device).  Writes 2 + 4L doubles to params
 * (device): alpha_r = L*a_root, beta_r = L*b_root, then for each leaf j
 * R*(a_j, b_j, c_j, d_j), where leaf j's line a_j x + b_j is the least-squares
 * fit to (x_i, i/S) over the sample points the root sends to leaf j (slope
 * clamped >= 0), and [c_j, d_j] is its monotone clamp interval
 * (c_j = clip01(max(line(min_j), d_{j-1})), d_j = clip01(max(line(max_j), c_j)),
 * d_{-1} = 0; an empty leaf is the flat line at d_{j-1}).  R: total bucket
 * resolution the scaled leaf parameters target.  Requires finite keys,
 * S >= 2, 2 <= L <= 1024. */
ls_status ls_rmi_fit(const void *sorted_sample, uint64_t S, ls_dtype dtype, uint32_t L, double R,
                     double *params, void *stream);

/* The same fit (Sec. 2.1 RMI, Sec. 4 monotone clamp) by the one-workgroup
 * kernel that builds the model of every segment whose sample fits on chip:
 * the sample is held in LDS, sums run in a workgroup's reduction order.
 * Same output layout as ls_rmi_fit.  Requires 2 <= S <= 16384, 2 <= L <= 1024
 * and an integer R in [1, 2^32).  sorted_sample, params: device.
 * Errors: LS_EINVAL, LS_ENOMEM, LS_EHIP. */
ls_status ls_rmi_fit_block(const void *sorted_sample, uint64_t S, ls_dtype dtype, uint32_t L, double R,
                           double *params, void *stream);

/* Bucket ids of keys under RMI params (the layout ls_rmi_fit writes):
 * j = clamp(floor(fma(alpha_r, x, beta_r)), 0, L-1),
 * g = clamp(floor(clamp(fma(alpha_j, x, beta_j), gamma_j, delta_j)), 0, R-1)
 * (Sec. 2.2 bucket formula; Alg. 4 line computing g).  Non-finite float64
 * keys: bucket 0 for negative sign, R-1 otherwise.  out: device uint32[n]. */
ls_status ls_rmi_buckets(const void *keys, uint64_t n, ls_dtype dtype, const double *params,
                         uint32_t L, double R, uint32_t *out, void *stream);

/* Splitters of a SORTED sample (Sec. 2.4): candidate i = sample[floor((i+1)S/B)],
 * i < B-1, de-duplicated; a repeated candidate gets an equality bucket.
 * Writes m unique splitters in ordered-key form (device uint64[B-1]),
 * equality flags (device uint8[B-1]) and m (device uint32[1]). */
ls_status ls_splitters(const void *sorted_sample, uint64_t S, ls_dtype dtype, uint32_t B,
                       uint64_t *splitters, uint8_t *eq, uint32_t *m, void *stream);

/* Bucket ids under splitters: with k = #{splitters <= key}, buckets run in
 * key order -- the range below splitter 0, then per splitter its equality
 * bucket (if flagged) and the range above it.  m: host.  out: device. */
ls_status ls_splitter_buckets(const void *keys, uint64_t n, ls_dtype dtype, const uint64_t *splitters,
                              const uint8_t *eq, uint32_t m, uint32_t *out, void *stream);

/* One stable partition level (Sec. 2.2 partitioning): bucket ids from the RMI
 * params at resolution R with every R/nb consecutive fine buckets merged into
 * one (nb divides R), histogram, prefix sum (decoupled look-back), stable
 * scatter of keys (and payload) into out_keys / out_payload.  counts: device
 * uint64[nb] (bucket sizes).  All arrays device; payload nullable. */
ls_status ls_partition_rmi(const void *keys, const uint32_t *payload, uint64_t n, ls_dtype dtype,
                           const double *params, uint32_t L, double R, uint32_t nb,
                           void *out_keys, uint32_t *out_payload, uint64_t *counts, void *stream);

/* Same with the splitter-tree bucket function (m host, splitters/eq device). */
ls_status ls_partition_splitters(const void *keys, const uint32_t *payload, uint64_t n, ls_dtype dtype,
                                 const uint64_t *splitters, const uint8_t *eq, uint32_t m,
                                 void *out_keys, uint32_t *out_payload, uint64_t *counts, void *stream);

/* ---- Monotone MLP CDF (1-16-16-1, FP32) ----------------------------------- */
/* Parameter vector: 321 floats V1[16] b1[16] V2[16x16] (row = output unit)
 * b2[16] V3[16] b3[1]; effective weights |V|; hidden units 0..7 use
 * max(z,0), 8..15 use min(z,0); so the network is non-decreasing in its
 * input (Sec. 3.1 monotone CDF).  Input t = clamp((x - lo) * inv, 0, 1) in
 * fp64 rounded to fp32, with lo_inv = {lo, inv} (device double[2]) taken
 * from a sorted sample: lo = smallest key, inv = 1 / (largest - smallest).
 * Every function here runs on the GPU; all pointers are device pointers. */

/* Mean squared error of the unclamped output against targets y and its
 * gradient over the 321 parameters, in FP32: per-sample terms summed in
 * sample order within each of up to 256 workgroups, then the workgroup
 * partials in workgroup order (deterministic).  t, y: float[S].  params:
 * float[321].  grad: float[321] (nullable).  loss: float[1] (nullable; one
 * of grad / loss required).  Errors: LS_EINVAL. */
ls_status ls_mlp_loss_grad(const float *params, const float *t, const float *y, uint64_t S,
                           float *grad, float *loss, void *stream);

/* The same loss and gradient computed by activation regions, the way the
 * training runs: t must be non-decreasing (a sorted training set).  Every
 * hidden pre-activation is non-decreasing in t, so each hidden unit switches
 * on or off once along the training set; the 32 switch indices (found by
 * binary search of the pre-activations, in FP64) cut it into at most 33 regions on which
 * the network is affine in t, and each gradient entry is a combination of
 * the regions' moments (count, sums of t, t^2, y, t y, y^2) from FP64 prefix
 * sums -- the per-sample gradient summed over every sample in another order,
 * in FP64 from the FP32 parameters, returned in FP32.  Errors: LS_EINVAL. */
ls_status ls_mlp_loss_grad_regions(const float *params, const float *t, const float *y, uint64_t S,
                                   float *grad, float *loss, void *stream);

/* Train on a SORTED sample of S keys: t from the sample's own lo_inv
 * (written to lo_inv), targets y_i = i / S, full-batch Adam (Kingma & Ba
 * 2015; betas 0.9 / 0.999, eps 1e-8, learning rate lr) for `steps` steps
 * from params_init (float[321]) or, if NULL, the start point that makes the
 * network the piecewise-linear interpolant of the sample CDF through its
 * octiles.  Adam runs on q = p / s: s = 1 / max(1, |V1_k| + |b1_k|) (at the
 * start point) for the layer-2 weights of input unit k, 1 otherwise, so that
 * no step moves a pre-activation by much more than lr.  Every step's gradient
 * and loss are computed by activation regions (as ls_mlp_loss_grad_regions),
 * all steps in one launch.  The loss is evaluated at the start of every step; params_out
 * (float[321]) receives the parameters with the lowest of those losses (the
 * start point when steps == 0) and losses (float[steps], nullable) the
 * losses.
 * Errors: LS_EINVAL (S < 2, lr <= 0, steps > 100000, missing output). */
ls_status ls_mlp_train(const void *sorted_sample, uint64_t S, ls_dtype dtype, const float *params_init,
                       uint32_t steps, float lr, float *params_out, double *lo_inv, float *losses,
                       void *stream);

/* The network alone as a CDF: g = min(floor(F * R), R - 1) in fp32 with
 * F = clamp(net(t), 0, 1), every product-sum an fmaf chain in index order;
 * non-finite keys go to 0 (negative) or R - 1.  out: uint32[n].
 * Errors: LS_EINVAL (R outside [1, 2^24]). */
ls_status ls_mlp_buckets(const void *keys, uint64_t n, ls_dtype dtype, const float *params,
                         const double *lo_inv, uint32_t R, uint32_t *out, void *stream);

/* Two-level model with the MLP as its root (Sec. 2.1 stages; the model
 * LS_MODEL_MLP uses): leaf j = min(floor(F * L), L - 1) in fp32; leaves are
 * the RMI's monotone least-squares lines (Sec. 2.1, Sec. 4).  Fits the L
 * leaves on a SORTED sample and writes them pre-scaled by R as
 * leaves[4L] = (alpha_j, beta_j, gamma_j, delta_j) (device doubles).
 * Errors: LS_EINVAL. */
ls_status ls_mlp_rmi_fit(const void *sorted_sample, uint64_t S, ls_dtype dtype, const float *params,
                         const double *lo_inv, uint32_t L, double R, double *leaves, void *stream);

/* Bucket ids at total resolution R under that model:
 * g = clamp(floor(clamp(fma(alpha_j, x, beta_j), gamma_j, delta_j)), 0, R-1)
 * with j from the network; non-finite keys as for the RMI.  out: uint32[n].
 * Errors: LS_EINVAL. */
ls_status ls_mlp_rmi_buckets(const void *keys, uint64_t n, ls_dtype dtype, const float *params,
                             const double *lo_inv, const double *leaves, uint32_t L, double R,
                             uint32_t *out, void *stream);

/* Reference streams (not steps of the sort): the practical ceilings that the
 * sort's passes are measured against.  ls_stream_copy copies n 8-byte words
 * from src to dst (one read and one write per word, as in a partition
 * scatter or the base case); ls_stream_read reads n words and writes their
 * wrapping sum (mod 2^64) to *sum (one read per word, as in the histogram
 * pass; *sum is 0 when n == 0; a copy of n == 0 words does nothing).
 * src, dst: device, 8-byte aligned, not overlapping; sum: device uint64.
 * Asynchronous on `stream`; nothing is allocated.
 * Errors: LS_EINVAL (NULL pointer with n > 0, misalignment, n >= 2^45). */
ls_status ls_stream_copy(const void *src, void *dst, uint64_t n, void *stream);
ls_status ls_stream_read(const void *src, uint64_t n, uint64_t *sum, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LSORT_H */
