/*
 * lsort_oracle.c -- plain, slow, single-threaded CPU oracle for the learned
 * sample sort ("LearnedSort as a learning-augmented SampleSort", Carvalho &
 * Lawrence, SSDBM 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) includes, links or calls this file.  It is used by the
 * tests, by the smoke check and by the CPU-baseline leg of the benchmark.  It
 * shares no header, helper, table or constant generator with the GPU code.
 *
 * Floating point: fp64 for model evaluation (the same operation sequence the
 * method defines: fma, floor, min/max), `long double` for least-squares sums.
 * Build with -O2 -ffp-contract=off and without fast-math so that the compiler
 * neither fuses nor reorders what is written here.
 *
 * Contents (each function cites the passage it follows):
 *   1. key order and model input          (Sec. 5 key extractor; Sec. 3.1 monotonicity);
 *      float64, uint64, int64 and float32 keys
 *   2. the sort itself: stable merge sort  (Sec. 2.1 sorted position; Sec. 2.2 sortedness)
 *   3. sampling                            (Sec. 2.2 "1% sample"; Alg. 5 Sample)
 *   4. duplicate fraction and policy       (Alg. 5; Sec. 4 constants)
 *   5. two-level RMI: fit and bucket       (Sec. 2.1 RMI formula; Sec. 2.2 bucket formula;
 *                                           Sec. 4 monotone constraint)
 *   6. splitter tree with equality buckets (Sec. 2.4 SampleSort, equality buckets)
 *   7. range-radix bucket (depth cap)      (Sec. 2.4 IPS2Ra MSD radix idea)
 *   8. one partition level                 (Sec. 2.2 partitioning into buckets)
 *   9. monotone FP32 MLP CDF: fp64 forward/backward, Adam, the scaled
 *      training rule with best-loss selection, start point, fp32 inference,
 *      and the MLP as the root of a two-level model
 *                                          (Sec. 3.1 CDF-model properties;
 *                                           Sec. 2.1 RMI stages)
 *  10. pivot quality and implicit pivots   (Sec. 3.3 Alg. 4; Sec. 3.4 Table 1 metric)
 *
 * Every function below is pinned by a CPU test (tests/test_oracle_*.py)
 * against something other than itself: closed forms, brute force, library
 * routines, exact rational arithmetic or hand-counted values.  Only the
 * paper's own Table 1 numbers are parity unpinned: the paper states neither
 * IPS4o's sample size nor the exact RMI behind them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_F64 0
#define ORC_U64 1
#define ORC_I64 2   /* two's-complement int64, numeric order */
#define ORC_F32 3   /* binary32, IEEE-754 totalOrder; 4-byte keys */

/* ------------------------------------------------------------------------ */
/* 1. Key order and model input                                             */
/* ------------------------------------------------------------------------ */

/* Order-preserving map of a key's bits to an unsigned integer (Sec. 5: the
 * float-to-integer key extractor used to radix-sort doubles).  For binary64
 * the result orders keys by IEEE-754 totalOrder:
 * -NaN < -inf < ... < -0.0 < +0.0 < ... < +inf < +NaN.
 * Negative values have every bit flipped, non-negative ones the sign bit set.
 * For uint64 keys the map is the identity.  For int64 keys it moves the
 * range [-2^63, 2^63) onto [0, 2^64) by adding 2^63 (mod 2^64), which is the
 * same as flipping the sign bit.  binary32 keys (the low 32 bits of `raw`)
 * take the binary64 rule on their own 32 bits; the result fits in 32 bits. */
uint64_t orc_ord(uint64_t raw, int dtype)
{
    if (dtype == ORC_U64) return raw;
    if (dtype == ORC_I64) return raw + 0x8000000000000000ull;
    if (dtype == ORC_F32) {
        uint32_t b = (uint32_t)raw;
        return (b >> 31) ? (uint32_t)~b : (b | 0x80000000u);
    }
    if (raw >> 63) return ~raw;
    return raw | 0x8000000000000000ull;
}

uint64_t orc_unord(uint64_t ord, int dtype)
{
    if (dtype == ORC_U64) return ord;
    if (dtype == ORC_I64) return ord - 0x8000000000000000ull;
    if (dtype == ORC_F32) {
        uint32_t o = (uint32_t)ord;
        return (o >> 31) ? (o & 0x7fffffffu) : (uint32_t)~o;
    }
    if (ord >> 63) return ord & 0x7fffffffffffffffull;
    return ~ord;
}

/* The real number a CDF model is evaluated at.  Returns 0 for a finite input
 * and writes x; returns +1 / -1 for a non-finite binary64 key of positive /
 * negative sign (those are routed to the last / first bucket, which keeps the
 * bucket function monotone in totalOrder).  uint64 keys convert with
 * round-to-nearest, a non-decreasing map. */
int orc_model_x(uint64_t raw, int dtype, double *x)
{
    if (dtype == ORC_U64) { *x = (double)raw; return 0; }
    if (((raw >> 52) & 0x7ff) == 0x7ff) return (raw >> 63) ? -1 : 1;
    double d; memcpy(&d, &raw, 8); *x = d; return 0;
}

/* ------------------------------------------------------------------------ */
/* 2. The sort: stable bottom-up merge sort on (ordered key, index)          */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t k; uint64_t i; } orc_pair;

static void merge_pass(const orc_pair *src, orc_pair *dst, uint64_t n, uint64_t w)
{
    for (uint64_t lo = 0; lo < n; lo += 2 * w) {
        uint64_t mid = lo + w < n ? lo + w : n;
        uint64_t hi = lo + 2 * w < n ? lo + 2 * w : n;
        uint64_t a = lo, b = mid, o = lo;
        while (a < mid && b < hi) {
            /* take from the left run on ties: this is what makes it stable */
            if (src[b].k < src[a].k) dst[o++] = src[b++];
            else dst[o++] = src[a++];
        }
        while (a < mid) dst[o++] = src[a++];
        while (b < hi) dst[o++] = src[b++];
    }
}

/* The definition the method must reach (Sec. 2.1: a key's place in the sorted
 * array is given by how many keys precede it; Sec. 2.2: the output must be
 * sorted whatever the model does).  Ties keep input order, so with a payload
 * the result is the unique stable sort.  keys[] holds n keys of `dtype` (8
 * bytes each, 4 for ORC_F32); payload[] (nullable) n values of pwidth bytes
 * (4 or 8).  On return keys[] is sorted, payload[] is permuted with it, and
 * perm[] (nullable) holds, for each output slot, the input index it came
 * from.  Returns 0, or -1 when out of memory or on a bad width. */
int orc_sort(void *keys, void *payload, int pwidth, uint64_t *perm, uint64_t n, int dtype)
{
    if (n == 0) return 0;
    if (payload && pwidth != 4 && pwidth != 8) return -1;
    const int kw = dtype == ORC_F32 ? 4 : 8;
    orc_pair *a = (orc_pair *)malloc(n * sizeof(orc_pair));
    orc_pair *b = (orc_pair *)malloc(n * sizeof(orc_pair));
    if (!a || !b) { free(a); free(b); return -1; }
    for (uint64_t i = 0; i < n; i++) {
        uint64_t raw = 0;
        memcpy(&raw, (const char *)keys + i * kw, kw);
        a[i].k = orc_ord(raw, dtype);
        a[i].i = i;
    }
    for (uint64_t w = 1; w < n; w *= 2) {
        merge_pass(a, b, n, w);
        orc_pair *t = a; a = b; b = t;
    }
    char *pl = NULL;
    if (payload) {
        pl = (char *)malloc(n * pwidth);
        if (!pl) { free(a); free(b); return -1; }
        memcpy(pl, payload, n * pwidth);
    }
    for (uint64_t i = 0; i < n; i++) {
        uint64_t raw = orc_unord(a[i].k, dtype);
        memcpy((char *)keys + i * kw, &raw, kw);
        if (payload) memcpy((char *)payload + i * pwidth, pl + a[i].i * pwidth, pwidth);
        if (perm) perm[i] = a[i].i;
    }
    free(pl); free(a); free(b);
    return 0;
}

/* Segment i is [off[i], off[i+1]); each is sorted on its own. */
int orc_sort_segmented(void *keys, void *payload, int pwidth, const uint64_t *off, uint64_t m, int dtype)
{
    const int kw = dtype == ORC_F32 ? 4 : 8;
    for (uint64_t s = 0; s < m; s++) {
        uint64_t lo = off[s], hi = off[s + 1];
        if (hi <= lo) continue;
        if (orc_sort((char *)keys + lo * kw, payload ? (char *)payload + lo * pwidth : NULL, pwidth, NULL,
                     hi - lo, dtype))
            return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3. Sampling                                                               */
/* ------------------------------------------------------------------------ */

/* Output number k (k = 0, 1, ...) of the SplitMix64 generator of Steele, Lea
 * and Flood (OOPSLA 2014) started from state `seed`: the state advances by
 * the golden-ratio increment before each output, and the output is the
 * state passed through the variant-13 finaliser. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Sample index k of a range of n keys: the high 64 bits of the 128-bit
 * product of a uniform 64-bit word and n (Lemire's multiply-shift map,
 * without the rejection step). Sampling is with replacement; the paper only
 * asks for a random sample of about 1% (Sec. 2.2; Alg. 5 Sample). */
uint64_t orc_sample_index(uint64_t seed, uint64_t k, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)orc_splitmix64_at(seed, k) * n) >> 64);
}

void orc_sample(const uint64_t *keys, uint64_t n, uint64_t seed, uint64_t S, uint64_t *out)
{
    for (uint64_t k = 0; k < S; k++) out[k] = keys[orc_sample_index(seed, k, n)];
}

/* ------------------------------------------------------------------------ */
/* 4. Duplicate fraction and the model policy                                */
/* ------------------------------------------------------------------------ */

/* Fraction of adjacent equal keys in a sorted sample: the "too many
 * duplicates" test of Alg. 5 reads it against 10% (Sec. 4). */
double orc_dup_fraction(const uint64_t *sorted_raw, uint64_t S, int dtype)
{
    if (S < 2) return 0.0;
    uint64_t d = 0;
    for (uint64_t j = 1; j < S; j++)
        d += orc_ord(sorted_raw[j], dtype) == orc_ord(sorted_raw[j - 1], dtype);
    return (double)d / (double)(S - 1);
}

/* Alg. 5 BuildPartitionModel: the RMI when the input is large (at least
 * 1e5 keys, Sec. 4) and the first sample has at most 10% duplicates,
 * otherwise the branchless decision tree.  A learned model also needs a
 * finite, non-degenerate key range in the sample.  Returns 1 for RMI,
 * 0 for the splitter tree. */
int orc_policy_learned(uint64_t n, const uint64_t *sorted_raw, uint64_t S, int dtype,
                       double large_n, double dup_limit)
{
    if ((double)n < large_n || S < 2) return 0;
    if (orc_dup_fraction(sorted_raw, S, dtype) > dup_limit) return 0;
    double x0, x1;
    if (orc_model_x(sorted_raw[0], dtype, &x0) || orc_model_x(sorted_raw[S - 1], dtype, &x1)) return 0;
    return x1 > x0;
}

/* ------------------------------------------------------------------------ */
/* 5. Two-level RMI                                                          */
/* ------------------------------------------------------------------------ */

/* Least squares line through (x_i, i/S) for i in [lo, hi) of a sorted
 * sample, two-pass and mean-centred in long double.  The slope is clamped at
 * 0 so that every line is non-decreasing (Sec. 3.1: a CDF model must be
 * monotone).  With one distinct x the line is flat at the mean target. */
static void lsq_line(const double *x, uint64_t lo, uint64_t hi, uint64_t S,
                     long double *a, long double *b)
{
    long double m = (long double)(hi - lo);
    long double sx = 0, sy = 0;
    for (uint64_t i = lo; i < hi; i++) { sx += x[i]; sy += (long double)i / (long double)S; }
    long double mx = sx / m, my = sy / m;
    long double sxx = 0, sxy = 0;
    for (uint64_t i = lo; i < hi; i++) {
        long double dx = (long double)x[i] - mx;
        long double dy = (long double)i / (long double)S - my;
        sxx += dx * dx; sxy += dx * dy;
    }
    long double slope = sxx > 0 ? sxy / sxx : 0;
    if (slope < 0) slope = 0;
    *a = slope;
    *b = my - slope * mx;
}

static double clip01(long double v)
{
    if (v < 0) return 0.0;
    if (v > 1) return 1.0;
    return (double)v;
}

/* Root-model leaf index of x: L * f1(x) floored and clamped to [0, L-1]
 * (Sec. 2.1 RMI: floor(B * f1(x)) selects the second-level model; here
 * alpha_r = L * a_root and beta_r = L * b_root are pre-scaled). */
uint32_t orc_rmi_leaf(double alpha_r, double beta_r, uint32_t L, double x)
{
    double r = floor(fma(alpha_r, x, beta_r));
    r = fmin(fmax(r, 0.0), (double)L - 1.0);
    return (uint32_t)r;
}

/* Fit the two-level linear RMI on a sorted sample x[0..S) (Sec. 2.1, Sec. 2.2
 * LearnedSort training: linear root, L linear leaves, targets i/S) and make it
 * monotone (Sec. 4): leaf j's output is clamped to [c_j, d_j] with
 *   c_j = clip01(max(a_j * min_j + b_j, d_{j-1})),   d_{-1} = 0,
 *   d_j = clip01(max(a_j * max_j + b_j, c_j)),
 * so max over leaf j never exceeds min over leaf j+1; an empty leaf is the
 * flat line at d_{j-1}.
 *
 * Leaf membership uses the pre-scaled root evaluated exactly as at sort
 * time.  If root_in is non-NULL it supplies that pre-scaled root (alpha_r,
 * beta_r) instead of the one fitted here, so a leaf fit can be checked
 * against another implementation's root.
 *
 * Outputs (all nullable):
 *   raw[2 + 4L]   : a_root, b_root, then (a_j, b_j, c_j, d_j) unscaled;
 *   scaled[2 + 4L]: alpha_r = L a_root, beta_r = L b_root, then
 *                   R * (a_j, b_j, c_j, d_j), rounded once to double --
 *                   the parameters orc_rmi_bucket evaluates at total
 *                   resolution R.
 *   counts[L]     : sample points per leaf. */
/* Leaf lines of a two-level model over a sorted sample, for any
 * non-decreasing root: leaf_of(ctx, x) gives the leaf of sample point x, so
 * the points of leaf j form one contiguous run.  Each run gets its
 * least-squares line (targets i/S) and the monotone clamp chain above;
 * outputs as for orc_rmi_fit, leaf part only (4 entries per leaf). */
typedef uint32_t (*leaf_fn)(const void *ctx, double x);

static void fit_leaves(const double *x, uint64_t S, uint32_t L, double R, leaf_fn leaf_of, const void *ctx,
                       double *raw, double *scaled, uint64_t *counts)
{
    uint64_t lo = 0;
    double dprev = 0.0;
    for (uint32_t j = 0; j < L; j++) {
        uint64_t hi = lo;
        while (hi < S && leaf_of(ctx, x[hi]) == j) hi++;
        long double a = 0, b;
        double c, d;
        if (hi == lo) {
            b = dprev;
            c = dprev; d = dprev;
        } else {
            lsq_line(x, lo, hi, S, &a, &b);
            long double pmin = a * (long double)x[lo] + b;
            long double pmax = a * (long double)x[hi - 1] + b;
            long double cc = pmin > dprev ? pmin : dprev;
            c = clip01(cc);
            long double dd = pmax > c ? pmax : c;
            d = clip01(dd);
        }
        if (raw) { raw[4 * j] = (double)a; raw[1 + 4 * j] = (double)b; raw[2 + 4 * j] = c; raw[3 + 4 * j] = d; }
        if (scaled) {
            long double Rl = R;
            scaled[4 * j] = (double)(Rl * a);
            scaled[1 + 4 * j] = (double)(Rl * b);
            scaled[2 + 4 * j] = (double)(Rl * (long double)c);
            scaled[3 + 4 * j] = (double)(Rl * (long double)d);
        }
        if (counts) counts[j] = hi - lo;
        dprev = d;
        lo = hi;
    }
}

struct linear_root { double alpha_r, beta_r; uint32_t L; };

static uint32_t linear_leaf(const void *ctx, double x)
{
    const struct linear_root *r = (const struct linear_root *)ctx;
    return orc_rmi_leaf(r->alpha_r, r->beta_r, r->L, x);
}

void orc_rmi_fit(const double *x, uint64_t S, uint32_t L, double R, const double *root_in,
                 double *raw, double *scaled, uint64_t *counts)
{
    long double ar, br;
    lsq_line(x, 0, S, S, &ar, &br);
    double alpha_r = (double)((long double)L * ar);
    double beta_r = (double)((long double)L * br);
    if (root_in) { alpha_r = root_in[0]; beta_r = root_in[1]; }
    if (raw) { raw[0] = (double)ar; raw[1] = (double)br; }
    if (scaled) { scaled[0] = alpha_r; scaled[1] = beta_r; }
    struct linear_root root = {alpha_r, beta_r, L};
    fit_leaves(x, S, L, R, linear_leaf, &root, raw ? raw + 2 : NULL, scaled ? scaled + 2 : NULL, counts);
}

/* Bucket of a key at total resolution R (Sec. 2.2: b = floor(B * F(x));
 * Alg. 4: g = floor(F(A[w]) * B)), with the monotone clamp of Sec. 4:
 *   j = clamp(floor(fma(alpha_r, x, beta_r)), 0, L-1)
 *   t = clamp(fma(alpha_j, x, beta_j), gamma_j, delta_j)
 *   g = clamp(floor(t), 0, R-1).
 * Non-finite binary64 keys go to bucket 0 (negative sign) or R-1. */
uint32_t orc_rmi_bucket(const double *scaled, uint32_t L, double R, uint64_t raw, int dtype)
{
    double x;
    int nf = orc_model_x(raw, dtype, &x);
    if (nf < 0) return 0;
    if (nf > 0) return (uint32_t)(R - 1.0);
    uint32_t j = orc_rmi_leaf(scaled[0], scaled[1], L, x);
    const double *q = scaled + 2 + 4 * (uint64_t)j;
    double t = fma(q[0], x, q[1]);
    t = fmin(fmax(t, q[2]), q[3]);
    double g = floor(t);
    g = fmin(fmax(g, 0.0), R - 1.0);
    return (uint32_t)g;
}

void orc_rmi_buckets(const double *scaled, uint32_t L, double R, const uint64_t *raw, uint64_t n,
                     int dtype, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_rmi_bucket(scaled, L, R, raw[i], dtype);
}

/* ------------------------------------------------------------------------ */
/* 6. Splitter tree with equality buckets                                    */
/* ------------------------------------------------------------------------ */

/* SampleSort splitters (Sec. 2.4): with a sorted sample s[0..S) and B
 * buckets, candidate i (i = 0..B-2) is s[floor((i+1) S / B)], compared as
 * ordered keys.  Candidates are de-duplicated; a value that was a candidate
 * more than once is a repeated splitter and gets an equality bucket holding
 * exactly the keys equal to it (Sec. 2.4, IPS4o equality buckets).
 * Writes the m unique splitters (ordered-key form, ascending) and their
 * equality flags; returns m. */
uint32_t orc_splitters(const uint64_t *sorted_raw, uint64_t S, uint32_t B, int dtype,
                       uint64_t *split_ord, uint8_t *eq)
{
    uint32_t m = 0;
    for (uint32_t i = 0; i + 1 < B; i++) {
        uint64_t r = (uint64_t)(((unsigned __int128)(i + 1) * S) / B);
        if (r >= S) r = S - 1;
        uint64_t v = orc_ord(sorted_raw[r], dtype);
        if (m > 0 && split_ord[m - 1] == v) { eq[m - 1] = 1; continue; }
        split_ord[m] = v; eq[m] = 0; m++;
    }
    return m;
}

/* Bucket of a key under m ascending splitters u with equality flags.
 * k = #{i : u_i <= key} (an upper bound).  Buckets are numbered in key order:
 * the range bucket below u_0, then for each splitter u_i its equality bucket
 * (if flagged) followed by the range bucket above it.  A key equal to a
 * flagged splitter goes to that splitter's equality bucket; a key equal to
 * an unflagged splitter joins the range bucket that starts at it.
 * Total buckets: m + 1 + (number of flags). */
uint32_t orc_splitter_bucket(const uint64_t *u, const uint8_t *eq, uint32_t m, uint64_t raw, int dtype)
{
    uint64_t o = orc_ord(raw, dtype);
    uint32_t k = 0;
    while (k < m && u[k] <= o) k++;
    uint32_t before = 0;
    for (uint32_t i = 0; i < k; i++) before += eq[i];
    if (k > 0 && eq[k - 1] && u[k - 1] == o) return k + before - 1;
    return k + before;
}

/* ------------------------------------------------------------------------ */
/* 7. Range-radix bucket                                                     */
/* ------------------------------------------------------------------------ */

/* Guaranteed-progress partition of a segment whose ordered keys span
 * [lo, hi], hi > lo: the top log2(B) significant bits of (key - lo), as in an
 * MSD radix pass over the key range (Sec. 2.4, IPS2Ra).  Each application
 * shrinks the range by a factor B, so a segment becomes homogeneous after at
 * most ceil(64 / log2 B) levels. */
uint32_t orc_radix_shift(uint64_t lo, uint64_t hi, uint32_t log2B)
{
    uint64_t span = hi - lo;
    uint32_t bits = 0;
    while (bits < 64 && (span >> bits) != 0) bits++;
    return bits > log2B ? bits - log2B : 0;
}

uint32_t orc_radix_bucket(uint64_t lo, uint32_t shift, uint64_t raw, int dtype)
{
    return (uint32_t)((orc_ord(raw, dtype) - lo) >> shift);
}

/* ------------------------------------------------------------------------ */
/* 8. One partition level                                                    */
/* ------------------------------------------------------------------------ */

/* Put every key into its bucket, buckets in increasing order, keys of one
 * bucket in input order (Sec. 2.2 partitioning into buckets; stable for the
 * payload).  This is a counting sort by bucket id: histogram, exclusive
 * prefix sum, scatter.  counts[B] and starts[B] are outputs (nullable). */
void orc_partition(const uint64_t *keys, const uint32_t *payload, const uint32_t *bucket,
                   uint64_t n, uint32_t B, uint64_t *out_keys, uint32_t *out_payload,
                   uint64_t *counts, uint64_t *starts)
{
    uint64_t *c = (uint64_t *)calloc(B, sizeof(uint64_t));
    uint64_t *p = (uint64_t *)calloc(B, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) c[bucket[i]]++;
    uint64_t run = 0;
    for (uint32_t b = 0; b < B; b++) { p[b] = run; run += c[b]; }
    if (counts) memcpy(counts, c, B * sizeof(uint64_t));
    if (starts) memcpy(starts, p, B * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) {
        uint64_t d = p[bucket[i]]++;
        out_keys[d] = keys[i];
        if (payload && out_payload) out_payload[d] = payload[i];
    }
    free(c); free(p);
}

/* ------------------------------------------------------------------------ */
/* 9. Monotone MLP CDF (1-16-16-1)                                           */
/* ------------------------------------------------------------------------ */
/* Parameter vector layout (321 entries):
 *   V1[16] b1[16] V2[16*16] (row i = output unit, column k = input) b2[16]
 *   V3[16] b3[1].
 * Effective weights are |V| (non-negative), biases are free.  In each hidden
 * layer units 0..7 use max(z, 0) and units 8..15 use min(z, 0); both are
 * non-decreasing, so with non-negative weights the network is non-decreasing
 * in its input -- the monotonicity a CDF model needs (Sec. 3.1).  The output
 * F is clamped to [0, 1] when used as a CDF; training uses the unclamped
 * output.  Loss: mean squared error to the targets i/S. */

#define MLP_H 16
#define MLP_HALF 8
#define MLP_NP 321
#define OFF_V1 0
#define OFF_B1 16
#define OFF_V2 32
#define OFF_B2 288
#define OFF_V3 304
#define OFF_B3 320

static double act(int unit, double z) { return unit < MLP_HALF ? (z > 0 ? z : 0) : (z < 0 ? z : 0); }
static double dact(int unit, double z) { return unit < MLP_HALF ? (z > 0 ? 1.0 : 0.0) : (z < 0 ? 1.0 : 0.0); }
static double sgn(double v) { return v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0); }

/* Forward pass in fp64 for one input t; returns the unclamped output and
 * (nullable) the pre-activations z1, z2 and activations h1, h2. */
double orc_mlp_forward(const double *p, double t, double *z1, double *h1, double *z2, double *h2)
{
    double lz1[MLP_H], lh1[MLP_H], lz2[MLP_H], lh2[MLP_H];
    for (int i = 0; i < MLP_H; i++) {
        lz1[i] = fabs(p[OFF_V1 + i]) * t + p[OFF_B1 + i];
        lh1[i] = act(i, lz1[i]);
    }
    for (int i = 0; i < MLP_H; i++) {
        double s = p[OFF_B2 + i];
        for (int k = 0; k < MLP_H; k++) s += fabs(p[OFF_V2 + MLP_H * i + k]) * lh1[k];
        lz2[i] = s;
        lh2[i] = act(i, s);
    }
    double out = p[OFF_B3];
    for (int k = 0; k < MLP_H; k++) out += fabs(p[OFF_V3 + k]) * lh2[k];
    if (z1) memcpy(z1, lz1, sizeof lz1);
    if (h1) memcpy(h1, lh1, sizeof lh1);
    if (z2) memcpy(z2, lz2, sizeof lz2);
    if (h2) memcpy(h2, lh2, sizeof lh2);
    return out;
}

/* Mean squared error over (t_i, y_i) and its gradient with respect to the 321
 * parameters, by the chain rule through |V| (d|v|/dv = sign v, 0 at 0) and
 * through the two activations (derivative 0 at z = 0).  fp64 throughout. */
double orc_mlp_loss_grad(const double *p, const double *t, const double *y, uint64_t S, double *grad)
{
    if (grad) memset(grad, 0, MLP_NP * sizeof(double));
    double loss = 0;
    for (uint64_t s = 0; s < S; s++) {
        double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H];
        double out = orc_mlp_forward(p, t[s], z1, h1, z2, h2);
        double e = out - y[s];
        loss += e * e;
        if (!grad) continue;
        double dout = 2.0 * e / (double)S;
        grad[OFF_B3] += dout;
        double dz2[MLP_H];
        for (int k = 0; k < MLP_H; k++) {
            grad[OFF_V3 + k] += dout * h2[k] * sgn(p[OFF_V3 + k]);
            dz2[k] = dout * fabs(p[OFF_V3 + k]) * dact(k, z2[k]);
        }
        double dh1[MLP_H] = {0};
        for (int i = 0; i < MLP_H; i++) {
            grad[OFF_B2 + i] += dz2[i];
            for (int k = 0; k < MLP_H; k++) {
                grad[OFF_V2 + MLP_H * i + k] += dz2[i] * h1[k] * sgn(p[OFF_V2 + MLP_H * i + k]);
                dh1[k] += dz2[i] * fabs(p[OFF_V2 + MLP_H * i + k]);
            }
        }
        for (int k = 0; k < MLP_H; k++) {
            double dz1 = dh1[k] * dact(k, z1[k]);
            grad[OFF_V1 + k] += dz1 * t[s] * sgn(p[OFF_V1 + k]);
            grad[OFF_B1 + k] += dz1;
        }
    }
    return loss / (double)S;
}

/* One Adam step (Kingma & Ba, ICLR 2015) at step number `step` (1-based):
 *   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   p <- p - lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
void orc_adam_step(double *p, double *m, double *v, const double *g, uint64_t np, uint64_t step,
                   double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (uint64_t i = 0; i < np; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Per-parameter optimiser step scale at the start point p0: a layer-2 weight
 * that reads hidden unit k gets s = 1 / max(1, |V1_k| + |b1_k|), the bound of
 * that unit's activation over t in [0, 1]; every other parameter gets 1.
 * (The paper trains no network; this is the reading the MLP CDF uses so that
 * a training step moves no layer-2 pre-activation by much more than the
 * learning rate, however steep a first-layer ramp is.) */
void orc_mlp_step_scale(const double *p0, double *s)
{
    for (int i = 0; i < MLP_NP; i++) s[i] = 1.0;
    for (int k = 0; k < MLP_H; k++) {
        double bound = fabs(p0[OFF_V1 + k]) + fabs(p0[OFF_B1 + k]);
        if (bound < 1.0) bound = 1.0;
        for (int i = 0; i < MLP_H; i++) s[OFF_V2 + MLP_H * i + k] = 1.0 / bound;
    }
}

/* Full-batch training on the mean squared error over (t_i, y_i), fp64.
 * Step k = 1..steps: the loss L_k and gradient g at the current p (from
 * orc_mlp_loss_grad), then one Adam step (orc_adam_step, betas 0.9 / 0.999,
 * eps 1e-8) on q = p / s with gradient s * g, and p = q * s, with
 * s = orc_mlp_step_scale(p0).  losses[k-1] = L_k (nullable).  p_out gets the
 * parameters at which the lowest L_k was taken (the earliest on ties; p0
 * when steps == 0), or with final != 0 the parameters after the last step. */
void orc_mlp_train(const double *t, const double *y, uint64_t S, const double *p0, uint32_t steps, double lr,
                   int final, double *p_out, double *losses)
{
    double p[MLP_NP], q[MLP_NP], sc[MLP_NP], g[MLP_NP], m[MLP_NP], v[MLP_NP], best[MLP_NP];
    double best_loss = INFINITY;
    memcpy(p, p0, sizeof p);
    memcpy(best, p0, sizeof best);
    orc_mlp_step_scale(p0, sc);
    memset(m, 0, sizeof m);
    memset(v, 0, sizeof v);
    for (uint32_t k = 1; k <= steps; k++) {
        double loss = orc_mlp_loss_grad(p, t, y, S, g);
        if (losses) losses[k - 1] = loss;
        if (loss < best_loss) {
            best_loss = loss;
            memcpy(best, p, sizeof best);
        }
        for (int i = 0; i < MLP_NP; i++) {
            q[i] = p[i] / sc[i];
            g[i] *= sc[i];
        }
        orc_adam_step(q, m, v, g, MLP_NP, k, lr, 0.9, 0.999, 1e-8);
        for (int i = 0; i < MLP_NP; i++) p[i] = q[i] * sc[i];
    }
    memcpy(p_out, final ? p : best, sizeof p);
}

/* Model input of the MLP: t = clamp((x - lo) * inv, 0, 1) in fp64, rounded to
 * fp32 (a non-decreasing map of x).  lo is the smallest sample key, inv is
 * 1 / (largest - smallest). */
float orc_mlp_input(double x, double lo, double inv)
{
    double t = (x - lo) * inv;
    t = fmin(fmax(t, 0.0), 1.0);
    return (float)t;
}

/* FP32 inference with a fixed operation order: every product-sum is an fmaf
 * chain over inputs in index order starting from the bias.  w holds the
 * effective (absolute) weights in the layout above, as float.  Each step is
 * non-decreasing in each input, so F is non-decreasing in t. */
float orc_mlp_eval_f32(const float *w, float t)
{
    float h1[MLP_H], h2[MLP_H];
    for (int i = 0; i < MLP_H; i++) {
        float z = fmaf(w[OFF_V1 + i], t, w[OFF_B1 + i]);
        h1[i] = i < MLP_HALF ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
    }
    for (int i = 0; i < MLP_H; i++) {
        float z = w[OFF_B2 + i];
        for (int k = 0; k < MLP_H; k++) z = fmaf(w[OFF_V2 + MLP_H * i + k], h1[k], z);
        h2[i] = i < MLP_HALF ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
    }
    float z = w[OFF_B3];
    for (int k = 0; k < MLP_H; k++) z = fmaf(w[OFF_V3 + k], h2[k], z);
    return fminf(fmaxf(z, 0.0f), 1.0f);
}

/* Bucket of a key under the MLP CDF at resolution R (Sec. 2.2 bucket formula):
 * g = min(floor(F * R), R - 1) computed in fp32.  Non-finite keys as for the
 * RMI. */
uint32_t orc_mlp_bucket(const float *w, double lo, double inv, uint32_t R, uint64_t raw, int dtype)
{
    double x;
    int nf = orc_model_x(raw, dtype, &x);
    if (nf < 0) return 0;
    if (nf > 0) return R - 1;
    float F = orc_mlp_eval_f32(w, orc_mlp_input(x, lo, inv));
    float g = floorf(F * (float)R);
    g = fminf(g, (float)R - 1.0f);
    return (uint32_t)g;
}

/* Data-dependent starting point of training.  With knots k_m = t[floor(mS/8)]
 * (m = 0..7) and k_8 = t[S-1] of the sorted inputs, widths
 * w_m = max(k_{m+1} - k_m, 1e-6):
 *   layer 1, units m = 0..7 (max):   V = 1 / w_m, b = -k_m / w_m, so
 *                                     h = max((t - k_m) / w_m, 0);
 *   layer 1, units 8 + m (min):       V = 1, b = -(m + 0.5) / 8;
 *   layer 2, unit 8 + m (min):        V[8+m][m] = 1, b = -1, so
 *                                     h = min(h_m, 1) - 1;
 *   every other layer-2 weight:       eps / max(1, |V1_k| + |b1_k|) (column k),
 *                                     biases of units 0..7 zero;
 *   output:                           V3 = eps (units 0..7), 1/8 (units 8..15), b3 = 1.
 * With eps = 0 the network is exactly sum_m min(max((t - k_m) / w_m, 0), 1) / 8,
 * the piecewise-linear interpolant of the sample CDF through (k_m, m / 8);
 * eps > 0 keeps the other weights trainable (the gradient of |V| vanishes at
 * V = 0).  fp64 throughout; the GPU rounds the same values to fp32. */
void orc_mlp_init(const double *t, uint64_t S, double eps, double *p)
{
    double M[MLP_H];
    for (int m = 0; m < MLP_HALF; m++) {
        double k = t[(uint64_t)m * S / 8];
        double kn = m == MLP_HALF - 1 ? t[S - 1] : t[(uint64_t)(m + 1) * S / 8];
        double w = kn - k;
        if (w < 1e-6) w = 1e-6;
        p[OFF_V1 + m] = 1.0 / w;
        p[OFF_B1 + m] = -k / w;
        p[OFF_V1 + MLP_HALF + m] = 1.0;
        p[OFF_B1 + MLP_HALF + m] = -((double)m + 0.5) / 8.0;
    }
    for (int k = 0; k < MLP_H; k++) {
        double bound = fabs(p[OFF_V1 + k]) + fabs(p[OFF_B1 + k]);
        M[k] = bound > 1.0 ? bound : 1.0;
    }
    for (int i = 0; i < MLP_H; i++)
        for (int k = 0; k < MLP_H; k++)
            p[OFF_V2 + MLP_H * i + k] = (i >= MLP_HALF && k == i - MLP_HALF) ? 1.0 : eps / M[k];
    for (int i = 0; i < MLP_H; i++) {
        p[OFF_B2 + i] = i < MLP_HALF ? 0.0 : -1.0;
        p[OFF_V3 + i] = i < MLP_HALF ? eps : 1.0 / 8.0;
    }
    p[OFF_B3] = 1.0;
}

/* Effective fp32 weights of a parameter vector: |V| for the weights, the
 * biases as they are, rounded to fp32 (the form the inference evaluates). */
void orc_mlp_effective(const double *p, float *w)
{
    for (int i = 0; i < MLP_NP; i++) {
        int weight = (i >= OFF_V1 && i < OFF_B1) || (i >= OFF_V2 && i < OFF_B2) || (i >= OFF_V3 && i < OFF_B3);
        w[i] = (float)(weight ? fabs(p[i]) : p[i]);
    }
}

/* Input range of the MLP from a sorted sample of finite keys: lo = the
 * smallest model input, inv = 1 / (largest - smallest), 0 when they are
 * equal. */
void orc_mlp_lo_inv(const uint64_t *sorted_raw, uint64_t S, int dtype, double *lo_inv)
{
    double x0, x1;
    orc_model_x(sorted_raw[0], dtype, &x0);
    orc_model_x(sorted_raw[S - 1], dtype, &x1);
    lo_inv[0] = x0;
    lo_inv[1] = x1 > x0 ? 1.0 / (x1 - x0) : 0.0;
}

void orc_mlp_inputs(const uint64_t *raw, uint64_t n, int dtype, double lo, double inv, float *t)
{
    for (uint64_t i = 0; i < n; i++) {
        double x;
        orc_model_x(raw[i], dtype, &x);
        t[i] = orc_mlp_input(x, lo, inv);
    }
}

/* The MLP as the first stage of a two-level model (Sec. 2.1 RMI with a
 * non-linear root): leaf j = min(floor(F * L), L - 1) in fp32, F the clamped
 * network output; leaves are the monotone linear lines of orc_rmi_fit.
 * Because F is non-decreasing, so is j, and the clamp chain keeps the whole
 * model monotone (Sec. 4). */
struct mlp_root { const float *w; double lo, inv; uint32_t L; };

uint32_t orc_mlp_leaf(const float *w, double lo, double inv, uint32_t L, double x)
{
    float F = orc_mlp_eval_f32(w, orc_mlp_input(x, lo, inv));
    float j = floorf(F * (float)L);
    j = fminf(j, (float)L - 1.0f);
    return (uint32_t)j;
}

static uint32_t mlp_leaf_fn(const void *ctx, double x)
{
    const struct mlp_root *r = (const struct mlp_root *)ctx;
    return orc_mlp_leaf(r->w, r->lo, r->inv, r->L, x);
}

/* Leaf fit under an MLP root on a sorted sample of model inputs x[0..S):
 * scaled[4L] = R * (a_j, b_j, c_j, d_j) as orc_rmi_fit. */
void orc_mlp_rmi_fit(const double *x, uint64_t S, const float *w, double lo, double inv, uint32_t L, double R,
                     double *raw, double *scaled, uint64_t *counts)
{
    struct mlp_root root = {w, lo, inv, L};
    fit_leaves(x, S, L, R, mlp_leaf_fn, &root, raw, scaled, counts);
}

/* Bucket at total resolution R: j from the MLP, then
 * t = clamp(fma(alpha_j, x, beta_j), gamma_j, delta_j), g = clamp(floor(t), 0, R-1);
 * non-finite keys as for the RMI. */
uint32_t orc_mlp_rmi_bucket(const float *w, double lo, double inv, const double *scaled, uint32_t L, double R,
                            uint64_t raw, int dtype)
{
    double x;
    int nf = orc_model_x(raw, dtype, &x);
    if (nf < 0) return 0;
    if (nf > 0) return (uint32_t)(R - 1.0);
    uint32_t j = orc_mlp_leaf(w, lo, inv, L, x);
    const double *q = scaled + 4 * (uint64_t)j;
    double t = fma(q[0], x, q[1]);
    t = fmin(fmax(t, q[2]), q[3]);
    double g = floor(t);
    g = fmin(fmax(g, 0.0), R - 1.0);
    return (uint32_t)g;
}

void orc_mlp_rmi_buckets(const float *w, double lo, double inv, const double *scaled, uint32_t L, double R,
                         const uint64_t *raw, uint64_t n, int dtype, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_mlp_rmi_bucket(w, lo, inv, scaled, L, R, raw[i], dtype);
}

/* ------------------------------------------------------------------------ */
/* 10. Implicit pivots and pivot quality                                     */
/* ------------------------------------------------------------------------ */

/* Alg. 4: for every bucket g the implicit pivot is the largest key (ordered
 * form) that falls in it; has[g] = 0 for an empty bucket. */
void orc_implicit_pivots(const uint64_t *raw, const uint32_t *bucket, uint64_t n, uint32_t B, int dtype,
                         uint64_t *pivot_ord, uint8_t *has)
{
    memset(has, 0, B);
    for (uint64_t i = 0; i < n; i++) {
        uint64_t o = orc_ord(raw[i], dtype);
        uint32_t g = bucket[i];
        if (!has[g] || o > pivot_ord[g]) { pivot_ord[g] = o; has[g] = 1; }
    }
}

/* Table 1 metric (Sec. 3.4): sum over i of |P(A <= p_i) - (i+1)/B| for
 * B-1 pivots p_0..p_{B-2}, with P taken from the sorted data (ordered keys,
 * ascending). */
double orc_pivot_quality(const uint64_t *sorted_ord, uint64_t n, const uint64_t *pivot_ord, uint32_t B)
{
    double q = 0;
    for (uint32_t i = 0; i + 1 < B; i++) {
        uint64_t lo = 0, hi = n;   /* first index with value > pivot */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (sorted_ord[mid] <= pivot_ord[i]) lo = mid + 1; else hi = mid;
        }
        q += fabs((double)lo / (double)n - (double)(i + 1) / (double)B);
    }
    return q;
}

/* ------------------------------------------------------------------------ */
/* Array forms of the element-wise functions above (same arithmetic).        */
/* ------------------------------------------------------------------------ */

/* Model inputs of n keys (orc_model_x); a non-finite key gives NaN. */
void orc_model_x_array(const uint64_t *raw, uint64_t n, int dtype, double *out)
{
    for (uint64_t i = 0; i < n; i++)
        if (orc_model_x(raw[i], dtype, &out[i])) out[i] = NAN;
}

void orc_ord_array(const uint64_t *raw, uint64_t n, int dtype, uint64_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_ord(raw[i], dtype);
}

void orc_splitter_buckets(const uint64_t *u, const uint8_t *eq, uint32_t m, const uint64_t *raw, uint64_t n,
                          int dtype, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_splitter_bucket(u, eq, m, raw[i], dtype);
}

void orc_radix_buckets(uint64_t lo, uint32_t shift, const uint64_t *raw, uint64_t n, int dtype, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_radix_bucket(lo, shift, raw[i], dtype);
}

void orc_mlp_buckets(const float *w, double lo, double inv, uint32_t R, const uint64_t *raw, uint64_t n,
                     int dtype, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_mlp_bucket(w, lo, inv, R, raw[i], dtype);
}
