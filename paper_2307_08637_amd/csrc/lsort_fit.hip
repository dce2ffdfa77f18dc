// lsort_fit.hip -- model construction over a large sorted sample (the first
// level of a big array, where the ~1% sample does not fit one workgroup's
// LDS), and the kernels behind the single-step entry points.
#include <algorithm>

#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {

// Random sample with replacement (Sec. 2.2: ~1% sample; Alg. 5 Sample).
__global__ void k_gather(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t S, uint64_t* out) {
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S; k += (uint64_t)gridDim.x * blockDim.x)
        out[k] = __builtin_nontemporal_load(keys + sample_index(seed, k, n));
}

// ---------------------------------------------------------------------------
// Least-squares passes over a sorted sample s[0..S) in global memory.
// part[g*8 + 0..4]: sum x, adjacent duplicates, non-finite keys, centred
// sum (x - mean)^2, centred sum (x - mean)(y - mean y).
// ---------------------------------------------------------------------------

// In every pass below a thread visits its indices i0, i0 + T, i0 + 2T, ... in
// that order (T: threads of the workgroup) and adds in that order; FIT_LU of
// its keys are loaded before any of them is used.
constexpr int FIT_LU = 8;

__global__ __launch_bounds__(FIT_T) void k_fit1(FitArgs A) {
    __shared__ double red[FIT_T / 64];
    __shared__ uint64_t red64[FIT_T / 64];
    const uint64_t chunk = (A.S + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = blockIdx.x * chunk, hi = min(A.S, lo + chunk);
    double sx = 0;
    uint64_t dup = 0, nf = 0;
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)FIT_T * FIT_LU) {
        uint64_t r[FIT_LU], rp[FIT_LU];
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) {
            const uint64_t i = i0 + (uint64_t)u * FIT_T;
            r[u] = i < hi ? A.s[i] : 0;
            rp[u] = i < hi && i > 0 ? A.s[i - 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) {
            const uint64_t i = i0 + (uint64_t)u * FIT_T;
            if (i >= hi) continue;
            double x;
            if (key_x(r[u], A.u64, x)) nf++;
            else sx += x;
            if (i > 0) dup += key_ord(r[u], A.u64) == key_ord(rp[u], A.u64);
        }
    }
    sx = block_sum<FIT_T, double>(sx, red);
    dup = block_sum<FIT_T, uint64_t>(dup, red64);
    nf = block_sum<FIT_T, uint64_t>(nf, red64);
    if (threadIdx.x == 0) {
        A.part[blockIdx.x * 8 + 0] = sx;
        A.part[blockIdx.x * 8 + 1] = (double)dup;
        A.part[blockIdx.x * 8 + 2] = (double)nf;
    }
}

__global__ __launch_bounds__(FIT_T) void k_fit2(FitArgs A) {
    __shared__ double red[FIT_T / 64];
    // total of the first pass, combined in the same order by every workgroup
    double sxt = 0;
    for (uint32_t g = threadIdx.x; g < gridDim.x; g += FIT_T) sxt += A.part[g * 8 + 0];
    sxt = block_sum<FIT_T, double>(sxt, red);
    const double Sd = (double)A.S;
    const double mx = sxt / Sd, my = (Sd - 1.0) / (2.0 * Sd);
    const uint64_t chunk = (A.S + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = blockIdx.x * chunk, hi = min(A.S, lo + chunk);
    double sxx = 0, sxy = 0;
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)FIT_T * FIT_LU) {
        uint64_t r[FIT_LU];
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) r[u] = i0 + (uint64_t)u * FIT_T < hi ? A.s[i0 + (uint64_t)u * FIT_T] : 0;
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) {
            const uint64_t i = i0 + (uint64_t)u * FIT_T;
            double x;
            if (i >= hi || key_x(r[u], A.u64, x)) continue;
            double dx = x - mx, dy = (double)i / Sd - my;
            sxx += dx * dx;
            sxy += dx * dy;
        }
    }
    sxx = block_sum<FIT_T, double>(sxx, red);
    sxy = block_sum<FIT_T, double>(sxy, red);
    if (threadIdx.x == 0) {
        A.part[blockIdx.x * 8 + 3] = sxx;
        A.part[blockIdx.x * 8 + 4] = sxy;
    }
}

// Root line, the Alg. 5 policy, and (when the policy says so) the splitter
// tree.  One workgroup.
__global__ __launch_bounds__(M_THREADS) void k_fit_root(FitArgs A) {
    __shared__ uint32_t scratch[B_MAX + 1];
    __shared__ uint64_t red64[M_THREADS / 64];
    __shared__ double redd[M_THREADS / 64];
    double sx = 0, dup = 0, nf = 0, sxx = 0, sxy = 0;
    for (uint32_t g = threadIdx.x; g < A.G; g += M_THREADS) {
        sx += A.part[g * 8 + 0];
        dup += A.part[g * 8 + 1];
        nf += A.part[g * 8 + 2];
        sxx += A.part[g * 8 + 3];
        sxy += A.part[g * 8 + 4];
    }
    sx = block_sum<M_THREADS, double>(sx, redd);
    dup = block_sum<M_THREADS, double>(dup, redd);
    nf = block_sum<M_THREADS, double>(nf, redd);
    sxx = block_sum<M_THREADS, double>(sxx, redd);
    sxy = block_sum<M_THREADS, double>(sxy, redd);
    const double Sd = (double)A.S;
    double x0, x1;
    int nf0 = key_x(A.s[0], A.u64, x0), nf1 = key_x(A.s[A.S - 1], A.u64, x1);
    bool learned;
    if (A.mode == 1) learned = true;
    else if (A.mode == 2) learned = false;
    else learned = (double)A.n >= 1e5 && dup <= 0.10 * (Sd - 1.0) && nf == 0 && !nf0 && !nf1 && x1 > x0;
    uint64_t* dst = A.model;
    uint32_t nb, words, kind;
    if (learned && A.mlp) {
        // the MLP root is trained next; its header, weights and leaves are
        // written by the MLP kernels and the leaf fit
        nb = A.B1;
        words = 0;  // per-key ids are stored by k_mlp_ids: nothing to load
        kind = K_MLP;
    } else if (learned) {
        double mx = sx / Sd, my = (Sd - 1.0) / (2.0 * Sd);
        double a = sxx > 0 ? sxy / sxx : 0.0;
        if (a < 0) a = 0;
        double b = my - a * mx;
        if (threadIdx.x == 0) {
            RmiModel* h = (RmiModel*)dst;
            h->L = A.L; h->B1 = A.B1; h->log2B2 = A.log2B2; h->pad = 0;
            h->R = A.R; h->pad2 = 0;
            ((double*)dst)[4] = (double)A.L * a;
            ((double*)dst)[5] = (double)A.L * b;
        }
        nb = A.B1;
        words = rmi_words(A.L);
        kind = K_RMI;
    } else {
        const uint64_t* s = A.s;
        const int u64 = A.u64;
        nb = build_tree_block([&](uint64_t r) { return key_ord(s[r], u64); }, (uint32_t)min<uint64_t>(A.S, 0xffffffffull),
                              A.Bt, dst, scratch, red64);
        words = tree_words(((TreeModel*)dst)->m);
        kind = K_TREE;
    }
    if (threadIdx.x == 0) {
        A.flag[0] = learned ? 1u : 0u;
        if (A.first_mlp) A.first_mlp[0] = learned && A.mlp ? 1u : 0u;
        if (A.seg) {
            Seg sg{};
            sg.kind = kind; sg.nb = nb; sg.model = (uint64_t)dst;
            sg.flags = SEG_PREBUILT | (words << 16);
            *A.seg = sg;
        }
    }
}

// Leaf lines: one wave per leaf.  Leaf j covers the sample points the
// pre-scaled root sends to j (a contiguous range, found by binary search).
// leaf[j*8 + 0..4] = a, b, line(min), line(max), non-empty.
__device__ __forceinline__ uint32_t root_leaf(double ar, double br, double Lm1, uint64_t raw, int u64) {
    double x;
    key_x(raw, u64, x);
    return (uint32_t)fmin(fmax(floor(__builtin_fma(ar, x, br)), 0.0), Lm1);
}

// Leaf boundaries: the root's leaf index is non-decreasing along the sorted
// sample, so leaf j covers [bounds[j], bounds[j+1]).  Each sample point
// writes the starts of the leaves that begin at it.
__device__ __forceinline__ void write_bounds(const FitArgs& A, uint64_t i, uint32_t j, int64_t jp) {
    uint64_t* bounds = (uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
    for (int64_t q = jp + 1; q <= (int64_t)j; q++) bounds[q] = i;
    if (i == A.S - 1)
        for (uint32_t q = j + 1; q <= A.L; q++) bounds[q] = A.S;
}

__global__ __launch_bounds__(FIT_T) void k_fit_bounds(FitArgs A) {
    if (A.flag[0] == 0) return;
    const double ar = ((const double*)A.model)[4], br = ((const double*)A.model)[5];
    const double Lm1 = (double)A.L - 1.0;
    for (uint64_t i = (uint64_t)blockIdx.x * FIT_T + threadIdx.x; i < A.S; i += (uint64_t)gridDim.x * FIT_T) {
        const uint32_t j = root_leaf(ar, br, Lm1, A.s[i], A.u64);
        const int64_t jp = i > 0 ? (int64_t)root_leaf(ar, br, Lm1, A.s[i - 1], A.u64) : -1;
        write_bounds(A, i, j, jp);
    }
}

// The same for the MLP root: leaf = min(floor(F L), L - 1) in fp32 (the
// sample is finite: the policy admits no learned model otherwise).
__global__ __launch_bounds__(FIT_T) void k_fit_bounds_mlp(FitArgs A) {
    __shared__ float w[MLP_NP];
    if (A.flag[0] == 0) return;
    const float* ws = (const float*)(A.model + MLP_W_WORD);
    for (int i = threadIdx.x; i < MLP_NP; i += FIT_T) w[i] = ws[i];
    __syncthreads();
    const MlpModel* h = (const MlpModel*)A.model;
    const double lo = h->lo, inv = h->inv;
    const float Lf = (float)A.L;
    for (uint64_t i = (uint64_t)blockIdx.x * FIT_T + threadIdx.x; i < A.S; i += (uint64_t)gridDim.x * FIT_T) {
        lds_reload_fence();
        float t[2], F[2];
        double x;
        key_x(A.s[i], A.u64, x);
        t[0] = mlp_input(x, lo, inv);
        key_x(A.s[i > 0 ? i - 1 : 0], A.u64, x);
        t[1] = mlp_input(x, lo, inv);
        mlp_eval_multi<2>(w, t, F);
        const uint32_t j = (uint32_t)fminf(floorf(F[0] * Lf), Lf - 1.0f);
        const int64_t jp = i > 0 ? (int64_t)fminf(floorf(F[1] * Lf), Lf - 1.0f) : -1;
        write_bounds(A, i, j, jp);
    }
}

// Leaf least squares, two passes per leaf (the mean, then centred sums).  A
// leaf is cut into pieces of A.piece sample points, one workgroup of FIT_LT
// threads each, so that a leaf holding most of the sample (a distribution
// whose mass sits in a small part of its key range: the linear root sends it
// to a few leaves) is summed by many workgroups; a leaf of at most one piece
// is summed exactly as by a single workgroup.  Pass one writes each piece's
// sum of x (leaves of several pieces only: a one-piece leaf's workgroup in
// pass two sums its own x first); pass two adds a leaf's piece sums in piece
// order (the mean) and writes each piece's centred sums; k_fit_finish adds
// those in piece order.
// Workgroup w takes the piece numbered w (numbering below).
// The rank term i / S is taken as i * (1 / S) (a rounding apart from the
// quotient).
constexpr int FIT_LT = 1024;
static_assert(FIT_LT >= L_MAX && M_THREADS >= L_MAX, "one thread per leaf in the piece numbering");

__device__ __forceinline__ uint64_t leaf_pieces(uint64_t c, uint64_t piece) { return c > piece ? (c + piece - 1) / piece : 1; }

// Piece numbering: piece 0 of leaf j is number j; pieces 1.. of the leaves of
// several pieces follow from L on, leaf by leaf: piece q >= 1 of leaf j is
// L + ex_j + q - 1, ex_j = sum over i < j of (pieces of i - 1).
__device__ __forceinline__ uint64_t piece_slot(uint32_t L, uint32_t j, uint64_t ex, uint64_t q) {
    return q == 0 ? j : L + ex + q - 1;
}

// Thread j (< L): its leaf's piece count, and ex_j (returned).
template <int NT>
__device__ __forceinline__ uint64_t extra_table(const FitArgs& A, uint64_t& np, uint64_t* red64) {
    const uint64_t* bounds = (const uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
    const uint32_t j = threadIdx.x;
    np = j < A.L ? leaf_pieces(bounds[j + 1] - bounds[j], A.piece) : 1;
    uint64_t tot;
    return block_excl_scan<NT, uint64_t>(np - 1, red64, &tot);
}

// This workgroup's piece: leaf j, index q within it, the leaf's piece count
// and ex_j (the extra-piece table is built only where it is needed: a leaf
// of several pieces, or a workgroup past the first L); false past the last.
__device__ bool my_piece(const FitArgs& A, uint32_t& j, uint64_t& q, uint64_t& ex, uint64_t& np, uint64_t* red64,
                         uint64_t* sh) {
    const uint64_t* bounds = (const uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
    const uint64_t w = blockIdx.x;
    if (w < A.L) {
        j = (uint32_t)w;
        q = 0;
        np = leaf_pieces(bounds[j + 1] - bounds[j], A.piece);
        ex = 0;
        if (np > 1) {  // uniform: the workgroup's leaf
            uint64_t npt;
            const uint64_t ext = extra_table<FIT_LT>(A, npt, red64);
            if (threadIdx.x == j) sh[0] = ext;
            __syncthreads();
            ex = sh[0];
        }
        return true;
    }
    uint64_t npt;
    const uint64_t ext = extra_table<FIT_LT>(A, npt, red64);
    if (threadIdx.x == 0) sh[0] = ~0ull;
    __syncthreads();
    const uint64_t e = w - A.L;
    if (threadIdx.x < A.L && npt > 1 && e >= ext && e < ext + npt - 1) {
        sh[0] = threadIdx.x; sh[1] = e - ext + 1; sh[2] = ext; sh[3] = npt;
    }
    __syncthreads();
    if (sh[0] == ~0ull) return false;
    j = (uint32_t)sh[0]; q = sh[1]; ex = sh[2]; np = sh[3];
    return true;
}

__global__ __launch_bounds__(FIT_LT) void k_fit_lsum(FitArgs A) {
    __shared__ double red[FIT_LT / 64];
    __shared__ uint64_t red64[FIT_LT / 64];
    __shared__ uint64_t sh[4];
    if (A.flag[0] == 0) return;
    uint32_t j;
    uint64_t q, ex, np;
    if (!my_piece(A, j, q, ex, np, red64, sh) || np == 1) return;
    const uint64_t* bounds = (const uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
    const uint64_t lo = bounds[j] + q * A.piece, hi = min(bounds[j + 1], lo + A.piece);
    double s = 0;
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)FIT_LT * FIT_LU) {
        uint64_t r[FIT_LU];
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) r[u] = i0 + (uint64_t)u * FIT_LT < hi ? A.s[i0 + (uint64_t)u * FIT_LT] : 0;
#pragma unroll
        for (int u = 0; u < FIT_LU; u++)
            if (i0 + (uint64_t)u * FIT_LT < hi) { double x; key_x(r[u], A.u64, x); s += x; }
    }
    s = block_sum<FIT_LT, double>(s, red);
    if (threadIdx.x == 0) A.lpart[blockIdx.x * 4 + 0] = s;
}

// Leaves of at most FIT_SMALL_LEAF points (most of them: a leaf holds ~S / L
// points), four per workgroup, a quarter of 256 threads each: the mean of x,
// then the centred sums, into the leaf's slot (piece 0 is slot j).  Larger
// leaves (the end leaves of a law's tails, and the leaves of several pieces)
// keep a whole workgroup per piece in k_fit_leaves.
constexpr int FIT_Q = FIT_LT / 4;
constexpr uint64_t FIT_SMALL_LEAF = 2ull * FIT_Q * FIT_LU;  // two rounds of loads per thread
static_assert(FIT_SMALL_LEAF < FIT_PIECE, "a small leaf is one piece");
__device__ __forceinline__ double quarter_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, q0 = (threadIdx.x / FIT_Q) * (FIT_Q / 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int i = 0; i < FIT_Q / 64; i++) t += red[q0 + i];
    return t;
}

__global__ __launch_bounds__(FIT_LT) void k_fit_leaves1(FitArgs A) {
    __shared__ double red[FIT_LT / 64];
    if (A.flag[0] == 0) return;
    const uint32_t j = blockIdx.x * 4 + threadIdx.x / FIT_Q, t = threadIdx.x % FIT_Q;
    const uint64_t* bounds = (const uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
    uint64_t lo = 0, hi = 0;
    if (j < A.L) {
        lo = bounds[j];
        hi = bounds[j + 1];
        if (hi - lo > FIT_SMALL_LEAF) hi = lo;  // k_fit_leaves' leaf (of one piece or several)
    }
    const double Sd = (double)A.S, invS = 1.0 / Sd;
    double s = 0;
    for (uint64_t i0 = lo + t; i0 < hi; i0 += (uint64_t)FIT_Q * FIT_LU) {
        uint64_t r[FIT_LU];
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) r[u] = i0 + (uint64_t)u * FIT_Q < hi ? A.s[i0 + (uint64_t)u * FIT_Q] : 0;
#pragma unroll
        for (int u = 0; u < FIT_LU; u++)
            if (i0 + (uint64_t)u * FIT_Q < hi) { double x; key_x(r[u], A.u64, x); s += x; }
    }
    s = quarter_sum(s, red);
    const double mx = hi > lo ? s / (double)(hi - lo) : 0.0, my = ((double)lo + (double)hi - 1.0) / (2.0 * Sd);
    double sxx = 0, sxy = 0;
    for (uint64_t i0 = lo + t; i0 < hi; i0 += (uint64_t)FIT_Q * FIT_LU) {
        uint64_t r[FIT_LU];
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) r[u] = i0 + (uint64_t)u * FIT_Q < hi ? A.s[i0 + (uint64_t)u * FIT_Q] : 0;
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) {
            const uint64_t i = i0 + (uint64_t)u * FIT_Q;
            if (i < hi) {
                double x; key_x(r[u], A.u64, x);
                double dx = x - mx, dy = (double)i * invS - my;
                sxx += dx * dx; sxy += dx * dy;
            }
        }
    }
    sxx = quarter_sum(sxx, red);
    sxy = quarter_sum(sxy, red);
    if (t == 0 && j < A.L && (hi > lo || bounds[j + 1] == bounds[j])) {  // this kernel's leaf
        A.lpart[j * 4 + 0] = s;
        A.lpart[j * 4 + 1] = sxx;
        A.lpart[j * 4 + 2] = sxy;
    }
}

__global__ __launch_bounds__(FIT_LT) void k_fit_leaves(FitArgs A) {
    __shared__ double red[FIT_LT / 64];
    __shared__ uint64_t red64[FIT_LT / 64];
    __shared__ uint64_t sh[4];
    __shared__ double sh_mx;
    if (A.flag[0] == 0) return;
    uint32_t j;
    uint64_t q, ex, np;
    if (!my_piece(A, j, q, ex, np, red64, sh)) return;
    const uint64_t* bounds = (const uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
    const uint64_t llo = bounds[j], lhi = bounds[j + 1];
    if (np == 1 && lhi - llo <= FIT_SMALL_LEAF) return;  // k_fit_leaves1
    const uint64_t lo = llo + q * A.piece, hi = min(lhi, lo + A.piece);
    const double Sd = (double)A.S, invS = 1.0 / Sd;
    if (np == 1) {  // the whole leaf: its own sum of x
        double s = 0;
        for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)FIT_LT * FIT_LU) {
            uint64_t r[FIT_LU];
#pragma unroll
            for (int u = 0; u < FIT_LU; u++) r[u] = i0 + (uint64_t)u * FIT_LT < hi ? A.s[i0 + (uint64_t)u * FIT_LT] : 0;
#pragma unroll
            for (int u = 0; u < FIT_LU; u++)
                if (i0 + (uint64_t)u * FIT_LT < hi) { double x; key_x(r[u], A.u64, x); s += x; }
        }
        s = block_sum<FIT_LT, double>(s, red);
        if (threadIdx.x == 0) {
            A.lpart[blockIdx.x * 4 + 0] = s;
            sh_mx = hi > lo ? s / (double)(hi - lo) : 0.0;
        }
    } else if (threadIdx.x == 0) {
        double s = 0;
        for (uint64_t r = 0; r < np; r++) s += A.lpart[piece_slot(A.L, j, ex, r) * 4 + 0];
        sh_mx = lhi > llo ? s / (double)(lhi - llo) : 0.0;
    }
    __syncthreads();
    const double mx = sh_mx, my = ((double)llo + (double)lhi - 1.0) / (2.0 * Sd);
    double sxx = 0, sxy = 0;
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)FIT_LT * FIT_LU) {
        uint64_t r[FIT_LU];
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) r[u] = i0 + (uint64_t)u * FIT_LT < hi ? A.s[i0 + (uint64_t)u * FIT_LT] : 0;
#pragma unroll
        for (int u = 0; u < FIT_LU; u++) {
            const uint64_t i = i0 + (uint64_t)u * FIT_LT;
            if (i < hi) {
                double x; key_x(r[u], A.u64, x);
                double dx = x - mx, dy = (double)i * invS - my;
                sxx += dx * dx; sxy += dx * dy;
            }
        }
    }
    sxx = block_sum<FIT_LT, double>(sxx, red);
    sxy = block_sum<FIT_LT, double>(sxy, red);
    if (threadIdx.x == 0) {
        A.lpart[blockIdx.x * 4 + 1] = sxx;
        A.lpart[blockIdx.x * 4 + 2] = sxy;
    }
}

// Where each first-level bucket starts in the sorted sample: bstart[b] = the
// first i with bucket(s[i]) >= b (S if none), for b in [0, B1].  The buckets
// of the sorted sample do not decrease (monotone model), so each entry is
// written once, by the sample key at which the bucket sequence passes b.
// Only for the RMI chosen by the policy (the fallback trees of its buckets
// take their samples from these runs).
__global__ __launch_bounds__(FIT_T) void k_fit_bstart(FitArgs A) {
    if (!A.bstart || A.flag[0] == 0 || (A.first_mlp && *A.first_mlp)) return;
    const uint32_t sh2 = A.log2B2;
    for (uint64_t i = (uint64_t)blockIdx.x * FIT_T + threadIdx.x; i < A.S; i += (uint64_t)gridDim.x * FIT_T) {
        const uint32_t g = rmi_stored_bucket(A.model, A.s[i], A.u64) >> sh2;
        const int64_t gp = i ? (int64_t)(rmi_stored_bucket(A.model, A.s[i - 1], A.u64) >> sh2) : -1;
        for (int64_t b = gp + 1; b <= (int64_t)g; b++) A.bstart[b] = i;
        if (i == A.S - 1)
            for (uint32_t b = g + 1; b <= A.B1; b++) A.bstart[b] = A.S;
    }
}

// The splitter tree as judge of the fitted RMI's balance, on the sample:
// the share of the sorted sample in first-level buckets above ratio x the
// expected size (bstart gives every bucket's sample count).  Each such bucket
// would be re-partitioned by a splitter tree at the next level (the 2x
// fallback rule), so when they hold more than `balance` of the sample the
// whole first level takes the splitter tree over the same sample instead.
__global__ __launch_bounds__(M_THREADS) void k_fit_balance(FitArgs A) {
    __shared__ uint32_t scratch[B_MAX + 1];
    __shared__ uint64_t red64[M_THREADS / 64];
    if (!A.bstart || A.flag[0] == 0 || (A.first_mlp && *A.first_mlp) || A.mode == 1 || !(A.balance < 1.0)) return;
    const double expected = (double)A.S / (double)A.B1;
    uint64_t over = 0;
    for (uint32_t b = threadIdx.x; b < A.B1; b += M_THREADS) {
        const uint64_t c = A.bstart[b + 1] - A.bstart[b];
        if ((double)c > A.ratio * expected) over += c;
    }
    over = block_sum<M_THREADS, uint64_t>(over, red64);
    if ((double)over <= A.balance * (double)A.S) return;
    const uint64_t* s = A.s;
    const int u64 = A.u64;
    const uint32_t nb = build_tree_block([&](uint64_t r) { return key_ord(s[r], u64); },
                                         (uint32_t)min<uint64_t>(A.S, 0xffffffffull), A.Bt, A.model, scratch, red64);
    if (threadIdx.x == 0) {
        A.flag[0] = 0;
        if (A.seg) {
            Seg sg{};
            sg.kind = K_TREE; sg.nb = nb; sg.model = (uint64_t)A.model;
            sg.flags = SEG_PREBUILT | (tree_words(((TreeModel*)A.model)->m) << 16);
            *A.seg = sg;
        }
    }
}

// Monotone clamp intervals (Sec. 4) via a prefix maximum, then pre-scaling
// by the total resolution R.  One workgroup of 1024 threads (L <= 1024).
__global__ __launch_bounds__(M_THREADS) void k_fit_finish(FitArgs A) {
    __shared__ double red[M_THREADS / 64];
    __shared__ double wave_last[M_THREADS / 64];
    __shared__ uint64_t red64[M_THREADS / 64];
    if (A.flag[0] == 0) return;
    const int tid = threadIdx.x;
    const bool in = (uint32_t)tid < A.L;
    // leaf line from its pieces' sums, added in piece order (as the mean in
    // k_fit_leaves)
    uint64_t np;
    const uint64_t ex = extra_table<M_THREADS>(A, np, red64);
    double a = 0, b = 0, pmin = 0, pmax = 0;
    bool ne = false;
    if (in) {
        const uint64_t* bounds = (const uint64_t*)(A.leaf + (uint64_t)L_MAX * 8);
        const uint64_t lo = bounds[tid], hi = bounds[tid + 1];
        if (hi > lo) {
            double s = 0, sxx = 0, sxy = 0;
            for (uint64_t r = 0; r < np; r++) s += A.lpart[piece_slot(A.L, tid, ex, r) * 4 + 0];
            for (uint64_t r = 0; r < np; r++) {
                sxx += A.lpart[piece_slot(A.L, tid, ex, r) * 4 + 1];
                sxy += A.lpart[piece_slot(A.L, tid, ex, r) * 4 + 2];
            }
            const double Sd = (double)A.S;
            const double mx = s / (double)(hi - lo), my = ((double)lo + (double)hi - 1.0) / (2.0 * Sd);
            a = sxx > 0 ? sxy / sxx : 0.0;
            if (a < 0) a = 0;
            b = my - a * mx;
            double x0, x1;
            key_x(A.s[lo], A.u64, x0);
            key_x(A.s[hi - 1], A.u64, x1);
            pmin = a * x0 + b;
            pmax = a * x1 + b;
            ne = true;
        }
    }
    double v = ne ? pmax : -INFINITY;
    double incl = block_incl_max<M_THREADS>(v, red);
    double excl = __shfl_up(incl, 1);
    if ((tid & 63) == 63) wave_last[tid >> 6] = incl;
    __syncthreads();
    if ((tid & 63) == 0) excl = tid == 0 ? -INFINITY : wave_last[(tid >> 6) - 1];
    if (in) {
        double dprev = fmin(fmax(excl, 0.0), 1.0);
        double c, d;
        if (ne) {
            c = fmin(fmax(fmax(pmin, dprev), 0.0), 1.0);
            d = fmin(fmax(fmax(pmax, c), 0.0), 1.0);
        } else {
            a = 0; b = dprev; c = dprev; d = dprev;
        }
        double* o = (double*)A.model + (A.mlp ? MLP_LEAF_WORD : 6) + 4 * tid;
        o[0] = A.R * a; o[1] = A.R * b; o[2] = A.R * c; o[3] = A.R * d;
    }
}

// ---------------------------------------------------------------------------
// Single-step kernels
// ---------------------------------------------------------------------------

// Bucket ids of keys under a model in global memory (copied into LDS).
__global__ __launch_bounds__(256) void k_model_buckets(const uint64_t* model, uint32_t words, uint32_t kind, uint32_t nb,
                                                       uint32_t win, const uint64_t* keys, uint64_t n, int u64,
                                                       uint32_t* out) {
    __shared__ __align__(16) uint64_t mdl[LDS_MODEL_WORDS];
    load_model_lds(mdl, model, kind, words, threadIdx.x, 256);
    __syncthreads();
    const View v = make_view(mdl, kind, nb, win);
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        out[i] = view_bucket(v, mdl, keys[i], u64, nullptr, 0);
}

// RMI model header + parameters from a caller's parameter array.
__global__ void k_install_rmi(const double* params, uint32_t L, double R, uint32_t B1, uint32_t log2B2, uint64_t* dst) {
    for (uint32_t i = threadIdx.x; i < 2 + 4 * L; i += blockDim.x) ((double*)dst)[4 + i] = params[i];
    if (threadIdx.x == 0) {
        RmiModel* h = (RmiModel*)dst;
        h->L = L; h->B1 = B1; h->log2B2 = log2B2; h->pad = 0; h->R = R; h->pad2 = 0;
    }
}

// Splitter-tree model from caller splitters (ordered keys) and flags.
__global__ __launch_bounds__(M_THREADS) void k_install_tree(const uint64_t* u, const uint8_t* eq, uint32_t m, uint64_t* dst) {
    __shared__ uint64_t red64[M_THREADS / 64];
    const int tid = threadIdx.x;
    for (uint32_t i = tid; i < m; i += M_THREADS) dst[2 + i] = u[i];
    uint32_t f = (uint32_t)tid < m ? (eq[tid] ? 1u : 0u) : 0u;
    uint64_t neq;
    uint64_t pe = block_excl_scan<M_THREADS, uint64_t>((uint64_t)f, red64, &neq);
    uint16_t* lut = (uint16_t*)(dst + 2 + m);
    if ((uint32_t)tid < m) lut[tid + 1] = (uint16_t)(((pe + f) << 1) | f);
    if (tid == 0) {
        lut[0] = 0;
        TreeModel* h = (TreeModel*)dst;
        h->m = m; h->nb = m + 1 + (uint32_t)neq; h->top = floor_pow2(m); h->pad = 0;
    }
}

// Splitters of a sorted sample (ordered keys) through the tree builder,
// exported as (unique splitters, equality flags, m).
__global__ __launch_bounds__(M_THREADS) void k_splitters(const uint64_t* s, uint64_t S, int u64, uint32_t B,
                                                         uint64_t* scratch_model, uint64_t* u_out, uint8_t* eq_out,
                                                         uint32_t* m_out) {
    __shared__ uint32_t scratch[B_MAX + 1];
    __shared__ uint64_t red64[M_THREADS / 64];
    build_tree_block([&](uint64_t r) { return key_ord(s[r], u64); }, (uint32_t)S, B, scratch_model, scratch, red64);
    const TreeModel* h = (const TreeModel*)scratch_model;
    const uint32_t m = h->m;
    const uint16_t* lut = (const uint16_t*)(scratch_model + 2 + m);
    for (uint32_t i = threadIdx.x; i < m; i += M_THREADS) {
        u_out[i] = scratch_model[2 + i];
        eq_out[i] = (uint8_t)(lut[i + 1] & 1u);
    }
    if (threadIdx.x == 0) *m_out = m;
}

// Copy n words (parameter export).
__global__ void k_copy_words(const uint64_t* src, uint64_t* dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
#define LAUNCH(kernel, grid, block, stream, ...)                                  \
    do {                                                                          \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
        return hipGetLastError();                                                 \
    } while (0)

hipError_t launch_gather(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t S, uint64_t* out, hipStream_t st) {
    uint32_t grid = (uint32_t)std::min<uint64_t>((S + 255) / 256, 4096ull);
    LAUNCH(k_gather, grid ? grid : 1, 256, st, keys, n, seed, S, out);
}
hipError_t launch_fit1(const FitArgs& A, hipStream_t st) { LAUNCH(k_fit1, A.G, FIT_T, st, A); }
hipError_t launch_fit2(const FitArgs& A, hipStream_t st) { LAUNCH(k_fit2, A.G, FIT_T, st, A); }
hipError_t launch_fit_root(const FitArgs& A, hipStream_t st) { LAUNCH(k_fit_root, 1, M_THREADS, st, A); }
// The piece size (at least FIT_PIECE points, larger for samples of more than
// FIT_PIECES * FIT_PIECE, so that the pieces never exceed L + FIT_PIECES) and
// the piece sums' place after the leaf boundaries.
static FitArgs with_pieces(const FitArgs& A) {
    FitArgs B = A;
    B.piece = std::max<uint64_t>(FIT_PIECE, (A.S + FIT_PIECES - 1) / FIT_PIECES);
    B.lpart = A.leaf + (uint64_t)L_MAX * 8 + (L_MAX + 1);
    return B;
}
hipError_t launch_fit_leaves(const FitArgs& A0, hipStream_t st) {
    const FitArgs A = with_pieces(A0);
    const uint32_t grid = (uint32_t)std::min<uint64_t>((A.S + FIT_T - 1) / FIT_T, 2048ull);
    if (A.mlp) hipLaunchKernelGGL(k_fit_bounds_mlp, dim3(grid ? grid : 1), dim3(FIT_T), 0, st, A);
    else hipLaunchKernelGGL(k_fit_bounds, dim3(grid ? grid : 1), dim3(FIT_T), 0, st, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t pieces = A.L + (uint32_t)((A.S + A.piece - 1) / A.piece);  // bounds every leaf's piece count
    hipLaunchKernelGGL(k_fit_lsum, dim3(pieces), dim3(FIT_LT), 0, st, A);
    hipLaunchKernelGGL(k_fit_leaves1, dim3((A.L + 3) / 4), dim3(FIT_LT), 0, st, A);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    LAUNCH(k_fit_leaves, pieces, FIT_LT, st, A);
}
hipError_t launch_fit_finish(const FitArgs& A, hipStream_t st) { LAUNCH(k_fit_finish, 1, M_THREADS, st, with_pieces(A)); }
hipError_t launch_fit_balance(const FitArgs& A, hipStream_t st) { LAUNCH(k_fit_balance, 1, M_THREADS, st, A); }
hipError_t launch_fit_bstart(const FitArgs& A, hipStream_t st) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>((A.S + FIT_T - 1) / FIT_T, 2048ull);
    LAUNCH(k_fit_bstart, grid ? grid : 1, FIT_T, st, A);
}
hipError_t launch_model_buckets(const uint64_t* model, uint32_t words, uint32_t kind, uint32_t nb, uint32_t win,
                                const uint64_t* keys, uint64_t n, int u64, uint32_t* out, hipStream_t st) {
    uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 2048ull);
    LAUNCH(k_model_buckets, grid ? grid : 1, 256, st, model, words, kind, nb, win, keys, n, u64, out);
}
hipError_t launch_install_rmi(const double* params, uint32_t L, double R, uint32_t B1, uint32_t log2B2, uint64_t* dst,
                              hipStream_t st) {
    LAUNCH(k_install_rmi, 1, 256, st, params, L, R, B1, log2B2, dst);
}
hipError_t launch_install_tree(const uint64_t* u, const uint8_t* eq, uint32_t m, uint64_t* dst, hipStream_t st) {
    LAUNCH(k_install_tree, 1, M_THREADS, st, u, eq, m, dst);
}
hipError_t launch_splitters(const uint64_t* s, uint64_t S, int u64, uint32_t B, uint64_t* scratch, uint64_t* u_out,
                            uint8_t* eq_out, uint32_t* m_out, hipStream_t st) {
    LAUNCH(k_splitters, 1, M_THREADS, st, s, S, u64, B, scratch, u_out, eq_out, m_out);
}
hipError_t launch_copy_words(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t st) {
    uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096ull);
    LAUNCH(k_copy_words, grid ? grid : 1, 256, st, src, dst, n);
}

}  // namespace ls
