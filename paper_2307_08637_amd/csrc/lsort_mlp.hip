// lsort_mlp.hip -- the monotone FP32 MLP CDF: training on the GPU (start
// point, forward, backward, Adam), the MLP-rooted two-level model, and the
// per-key bucket ids of levels partitioned by it.
//
// Network (a CDF model must be non-decreasing, Sec. 3.1): 1-16-16-1 with
// effective weights |V| >= 0; in each hidden layer units 0..7 use max(z, 0)
// and units 8..15 use min(z, 0), both non-decreasing.  Input
// t = clamp((x - lo) * inv, 0, 1) rounded to fp32; output clamped to [0, 1]
// when used as a CDF.  Training fits the unclamped output to the rank
// fractions of a sorted sample by mean squared error with full-batch Adam
// (Kingma & Ba 2015).  Parameter layout (321 floats): V1[16] b1[16]
// V2[16x16] (row = output unit) b2[16] V3[16] b3[1].
//
// As a partition model the network is the root of a two-level model
// (Sec. 2.1): it picks one of L linear leaves, fitted exactly as the RMI's.
#include <algorithm>

#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {

__host__ __device__ constexpr bool mlp_is_weight(int p) {
    return p < OFF_B1 || (p >= OFF_V2 && p < OFF_B2) || (p >= OFF_V3 && p < OFF_B3);
}

// ---------------------------------------------------------------------------
// Training set from a sorted sample s[0..S) of raw keys: every stride-th
// point, t = model input, y = its rank fraction i / S.  lo = smallest key,
// inv = 1 / (largest - smallest) (0 when all keys are equal or not finite).
// ---------------------------------------------------------------------------
__global__ void k_mlp_prep(const uint64_t* s, uint64_t S, uint64_t stride, int u64, float* t, float* y, double* lo_inv,
                           const uint32_t* gate) {
    if (gate && gate[0] == 0) return;
    double x0, x1;
    const int nf0 = key_x(s[0], u64, x0), nf1 = key_x(s[S - 1], u64, x1);
    const bool ok = !nf0 && !nf1 && x1 > x0;
    const double inv = ok ? 1.0 / (x1 - x0) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lo_inv[0] = ok ? x0 : 0.0;
        lo_inv[1] = inv;
    }
    const uint64_t Sp = (S + stride - 1) / stride;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Sp; i += (uint64_t)gridDim.x * blockDim.x) {
        double x;
        key_x(s[i * stride], u64, x);
        t[i] = ok ? mlp_input(x, x0, inv) : 0.0f;
        y[i] = (float)((double)(i * stride) / (double)S);
    }
}

// Start point (or the caller's parameters) and zeroed optimiser state.  The
// start point is the piecewise-linear interpolant of the sample CDF through
// its octiles: knots k_m = t[floor(m S / 8)], k_8 = t[S - 1], widths
// w_m = max(k_{m+1} - k_m, 1e-6); layer-1 max units ramp from k_m over w_m,
// layer-2 min units cap each ramp at 1 (V = 1, b = -1), the output averages
// the eight capped ramps (V3 = 1/8, b3 = 1).  Every other weight is
// eps / max(1, |V1_k| + |b1_k|) (column k) so that it stays trainable; the
// layer-1 min units start as unit-slope hinges at (m + 0.5) / 8.  Computed
// in fp64, rounded once to fp32.
constexpr int MLP_SETUP_T = 512;

__global__ __launch_bounds__(MLP_SETUP_T) void k_mlp_setup(const float* t, uint64_t S, const float* init, double eps,
                                                           float* p, float* m, float* v, float* best, float* scale,
                                                           float* best_loss, unsigned int* done,
                                                           const uint32_t* gate) {
    if (gate && gate[0] == 0) return;
    __shared__ double v1[MLP_H], b1[MLP_H];
    const int tid = threadIdx.x;
    if (init && tid < MLP_H) {
        v1[tid] = (double)init[OFF_V1 + tid];
        b1[tid] = (double)init[OFF_B1 + tid];
    }
    if (!init && tid < MLP_HALF) {
        const int q = tid;
        const double k = (double)t[(uint64_t)q * S / 8];
        const double kn = q == MLP_HALF - 1 ? (double)t[S - 1] : (double)t[(uint64_t)(q + 1) * S / 8];
        double w = kn - k;
        if (w < 1e-6) w = 1e-6;
        v1[q] = 1.0 / w;
        b1[q] = -k / w;
        v1[MLP_HALF + q] = 1.0;
        b1[MLP_HALF + q] = -((double)q + 0.5) / 8.0;
    }
    __syncthreads();
    for (int i = tid; i < MLP_NP; i += MLP_SETUP_T) {
        double val;
        if (init) {
            val = 0.0;
        } else if (i < OFF_B1) {
            val = v1[i - OFF_V1];
        } else if (i < OFF_V2) {
            val = b1[i - OFF_B1];
        } else if (i < OFF_B2) {
            const int r = (i - OFF_V2) / MLP_H, c = (i - OFF_V2) % MLP_H;
            const double bound = fabs(v1[c]) + fabs(b1[c]);
            val = (r >= MLP_HALF && c == r - MLP_HALF) ? 1.0 : eps / (bound > 1.0 ? bound : 1.0);
        } else if (i < OFF_V3) {
            val = i - OFF_B2 < MLP_HALF ? 0.0 : -1.0;
        } else if (i < OFF_B3) {
            val = i - OFF_V3 < MLP_HALF ? eps : 1.0 / 8.0;
        } else {
            val = 1.0;
        }
        p[i] = init ? init[i] : (float)val;
        best[i] = p[i];
        m[i] = 0.0f;
        v[i] = 0.0f;
        // optimiser step scale: 1 / (bound of the input activation on [0, 1])
        // for layer-2 weights, 1 elsewhere
        double sc = 1.0;
        if (i >= OFF_V2 && i < OFF_B2) {
            const int c = (i - OFF_V2) % MLP_H;
            const double bound = fabs(v1[c]) + fabs(b1[c]);
            sc = 1.0 / (bound > 1.0 ? bound : 1.0);
        }
        scale[i] = (float)sc;
    }
    if (tid == 0) {
        *done = 0;
        *best_loss = INFINITY;
    }
}

// ---------------------------------------------------------------------------
// One full-batch training step.
//
// Optimiser: Adam (Kingma & Ba 2015) on q = p / scale, with scale = 1 except
// for layer-2 weights, where it is 1 / max(1, |V1_k| + |b1_k|) of their input
// unit k at the start point -- the bound of that unit's activation on
// t in [0, 1].  Adam moves every q by about lr per step whatever the size of
// its gradient; the scale keeps a layer-2 weight that multiplies a steep
// first-layer ramp from moving its pre-activation by more than about lr.
//
// Each workgroup takes a contiguous chunk of the samples, 256 at a time: a
// thread runs forward and backward for one sample and leaves the per-sample
// factors in LDS, field-major (rec[f][sample]).  The gradient is then a set
// of small products over the samples:
//   V2[i][k] = sum dz2_i * h1_k (16 x 16)   V1[k] = sum dz1_k * t   b1[k] = sum dz1_k
//   b2[i] = sum dz2_i   V3[k] = sum dout * h2_k   b3 = sum dout   loss = sum e * e
// (gradients with respect to the effective weights; dout = 2 e / S).  Thread
// (tile, group) keeps a 4 x 4 tile of V2 -- and tiles 0..12 one of the
// vectors above -- in registers for the 16 samples of its group in each
// batch, reading four samples of a field per 16-byte LDS load; the sixteen
// groups' sums are added in group order once, at the end of the chunk.  The
// workgroup partials go to global memory; the last workgroup to finish adds
// them in workgroup order (so the result does not depend on scheduling),
// applies d|V|/dV = sign(V) and, if asked, the Adam update.
// ---------------------------------------------------------------------------
constexpr int MLP_T = 256;
constexpr int NREC = 68;  // record fields
enum : int { R_H1 = 0, R_DZ2 = 16, R_DZ1 = 32, R_H2 = 48, R_DOUT = 64, R_T = 65, R_E = 66 };
constexpr int MLP_GROUP = 16;  // samples of one thread group per batch

__global__ __launch_bounds__(MLP_T) void k_mlp_step(MlpStep A) {
    if (A.gate && A.gate[0] == 0) return;
    __shared__ float w[MLP_NP];
    __shared__ __align__(16) float rec[NREC * MLP_T];
    __shared__ int last;
    const int tid = threadIdx.x;
    for (int i = tid; i < MLP_NP; i += MLP_T) w[i] = mlp_is_weight(i) ? fabsf(A.p[i]) : A.p[i];
    __syncthreads();
    const float inv_s = 1.0f / (float)A.S;
    const uint64_t chunk = (A.S + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = (uint64_t)blockIdx.x * chunk, hi = min(A.S, lo + chunk);
    // accumulation role: tile of V2 rows i0.., columns k0..; group of samples
    const int tile = tid & 15, grp = tid >> 4;
    const int i0 = (tile >> 2) * 4, k0 = (tile & 3) * 4;
    float a2[4][4], ax[8];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) a2[x][y] = 0.0f;
#pragma unroll
    for (int x = 0; x < 8; x++) ax[x] = 0.0f;
    auto rd4 = [&](int f, int s0) { return *(const float4*)&rec[f * MLP_T + s0]; };
    for (uint64_t base = lo; base < hi; base += MLP_T) {
        lds_reload_fence();
        const uint64_t s = base + tid;
        float r[NREC];
        if (s < hi) {
            // forward; a hidden unit is active (derivative 1) exactly when its
            // output is non-zero, so the activations double as the masks
            const float tt = A.t[s];
            float h1[MLP_H];
#pragma unroll
            for (int k = 0; k < MLP_H; k++) {
                const float z = __builtin_fmaf(w[OFF_V1 + k], tt, w[OFF_B1 + k]);
                h1[k] = k < MLP_HALF ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
                r[R_H1 + k] = h1[k];
            }
            float out = w[OFF_B3];
#pragma unroll
            for (int half = 0; half < 2; half++) {
#pragma unroll 1
                for (int i = half * MLP_HALF; i < (half + 1) * MLP_HALF; i++) {
                    float z = w[OFF_B2 + i];
#pragma unroll
                    for (int k = 0; k < MLP_H; k++) z = __builtin_fmaf(w[OFF_V2 + MLP_H * i + k], h1[k], z);
                    const float h = half == 0 ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
                    rec[(R_H2 + i) * MLP_T + tid] = h;
                    out = __builtin_fmaf(w[OFF_V3 + i], h, out);
                }
            }
            // backward
            const float e = out - A.y[s];
            const float dout = 2.0f * e * inv_s;
            float dh1[MLP_H];
#pragma unroll
            for (int k = 0; k < MLP_H; k++) dh1[k] = 0.0f;
#pragma unroll 1
            for (int i = 0; i < MLP_H; i++) {
                const float dz2 = rec[(R_H2 + i) * MLP_T + tid] != 0.0f ? dout * w[OFF_V3 + i] : 0.0f;
                r[R_DZ2 + i] = dz2;
#pragma unroll
                for (int k = 0; k < MLP_H; k++) dh1[k] = __builtin_fmaf(dz2, w[OFF_V2 + MLP_H * i + k], dh1[k]);
            }
#pragma unroll
            for (int k = 0; k < MLP_H; k++) r[R_DZ1 + k] = h1[k] != 0.0f ? dh1[k] : 0.0f;
            r[R_DOUT] = dout;
            r[R_T] = tt;
            r[R_E] = e;
        } else {
#pragma unroll
            for (int f = 0; f < NREC; f++) r[f] = 0.0f;
#pragma unroll
            for (int i = 0; i < MLP_H; i++) rec[(R_H2 + i) * MLP_T + tid] = 0.0f;
        }
#pragma unroll
        for (int f = 0; f < NREC; f++)
            if (f < R_H2 || f >= R_H2 + MLP_H) rec[f * MLP_T + tid] = r[f];
        __syncthreads();
        // this group's 16 samples of the batch, four at a time
#pragma unroll 1
        for (int c = 0; c < MLP_GROUP; c += 4) {
            const int s0 = grp * MLP_GROUP + c;
            float4 dz[4], hh[4];
#pragma unroll
            for (int x = 0; x < 4; x++) { dz[x] = rd4(R_DZ2 + i0 + x, s0); hh[x] = rd4(R_H1 + k0 + x, s0); }
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++) {
                    a2[x][y] = __builtin_fmaf(dz[x].x, hh[y].x, a2[x][y]);
                    a2[x][y] = __builtin_fmaf(dz[x].y, hh[y].y, a2[x][y]);
                    a2[x][y] = __builtin_fmaf(dz[x].z, hh[y].z, a2[x][y]);
                    a2[x][y] = __builtin_fmaf(dz[x].w, hh[y].w, a2[x][y]);
                }
            if (tile < 4) {  // V1[k0..], b1[k0..]
                const float4 t4 = rd4(R_T, s0);
#pragma unroll
                for (int y = 0; y < 4; y++) {
                    const float4 d = rd4(R_DZ1 + k0 + y, s0);
                    ax[y] = __builtin_fmaf(d.x, t4.x, ax[y]); ax[y] = __builtin_fmaf(d.y, t4.y, ax[y]);
                    ax[y] = __builtin_fmaf(d.z, t4.z, ax[y]); ax[y] = __builtin_fmaf(d.w, t4.w, ax[y]);
                    ax[4 + y] += d.x; ax[4 + y] += d.y; ax[4 + y] += d.z; ax[4 + y] += d.w;
                }
            } else if (tile < 8) {  // V3[k0..]
                const float4 o4 = rd4(R_DOUT, s0);
#pragma unroll
                for (int y = 0; y < 4; y++) {
                    const float4 hv = rd4(R_H2 + k0 + y, s0);
                    ax[y] = __builtin_fmaf(o4.x, hv.x, ax[y]); ax[y] = __builtin_fmaf(o4.y, hv.y, ax[y]);
                    ax[y] = __builtin_fmaf(o4.z, hv.z, ax[y]); ax[y] = __builtin_fmaf(o4.w, hv.w, ax[y]);
                }
            } else if (tile < 12) {  // b2[k0..]
#pragma unroll
                for (int y = 0; y < 4; y++) {
                    const float4 d = rd4(R_DZ2 + k0 + y, s0);
                    ax[y] += d.x; ax[y] += d.y; ax[y] += d.z; ax[y] += d.w;
                }
            } else if (tile == 12) {  // b3, squared error
                const float4 o4 = rd4(R_DOUT, s0), e4 = rd4(R_E, s0);
                ax[0] += o4.x; ax[0] += o4.y; ax[0] += o4.z; ax[0] += o4.w;
                ax[1] = __builtin_fmaf(e4.x, e4.x, ax[1]); ax[1] = __builtin_fmaf(e4.y, e4.y, ax[1]);
                ax[1] = __builtin_fmaf(e4.z, e4.z, ax[1]); ax[1] = __builtin_fmaf(e4.w, e4.w, ax[1]);
            }
        }
        __syncthreads();
    }
    // the groups' sums in group order: red[group][entry] in the record area
    float* red = rec;
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) red[grp * MLP_ACC + OFF_V2 + MLP_H * (i0 + x) + k0 + y] = a2[x][y];
    if (tile < 4) {
#pragma unroll
        for (int y = 0; y < 4; y++) {
            red[grp * MLP_ACC + OFF_V1 + k0 + y] = ax[y];
            red[grp * MLP_ACC + OFF_B1 + k0 + y] = ax[4 + y];
        }
    } else if (tile < 8) {
#pragma unroll
        for (int y = 0; y < 4; y++) red[grp * MLP_ACC + OFF_V3 + k0 + y] = ax[y];
    } else if (tile < 12) {
#pragma unroll
        for (int y = 0; y < 4; y++) red[grp * MLP_ACC + OFF_B2 + k0 + y] = ax[y];
    } else if (tile == 12) {
        red[grp * MLP_ACC + OFF_B3] = ax[0];
        red[grp * MLP_ACC + MLP_NP] = ax[1];
    }
    __syncthreads();
    const bool two = tid + MLP_T < MLP_ACC;
    float acc0 = 0.0f, acc1 = 0.0f;
    for (int g = 0; g < MLP_T / MLP_GROUP; g++) {
        acc0 += red[g * MLP_ACC + tid];
        if (two) acc1 += red[g * MLP_ACC + tid + MLP_T];
    }
    float* part = A.partial + (uint64_t)blockIdx.x * MLP_ACC;
    part[tid] = acc0;
    if (two) part[tid + MLP_T] = acc1;
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(A.done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    // totals in workgroup order: entries tid and tid + 256
    __shared__ float sh_loss;
    float gt[2] = {0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int i = tid + q * MLP_T;
        if (i >= MLP_ACC) continue;
        float g = 0.0f;
        // 64 loads in flight, added in workgroup order
        uint32_t b = 0;
        for (; b + 64 <= gridDim.x; b += 64) {
            float v[64];
#pragma unroll
            for (int u = 0; u < 64; u++)
                v[u] = __hip_atomic_load(&A.partial[(uint64_t)(b + u) * MLP_ACC + i], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int u = 0; u < 64; u++) g += v[u];
        }
        for (; b < gridDim.x; b++)
            g += __hip_atomic_load(&A.partial[(uint64_t)b * MLP_ACC + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        gt[q] = g;
        if (i == MLP_NP) sh_loss = g * inv_s;
    }
    __syncthreads();
    const float loss = sh_loss;
    // keep the parameters with the lowest loss seen so far (those the loss was
    // just computed at, before this step's update)
    const bool better = A.best && loss < *A.best_loss;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int i = tid + q * MLP_T;
        if (i >= MLP_NP) continue;
        float g = gt[q];
        const float pv = A.p[i];
        if (better) A.best[i] = pv;
        if (mlp_is_weight(i)) g *= pv > 0.0f ? 1.0f : (pv < 0.0f ? -1.0f : 0.0f);  // d|V|/dV
        if (A.grad_out) A.grad_out[i] = g;
        if (A.update) {
            // Adam on q = p / scale: its gradient is scale * g and p moves by scale * (q's step)
            const float sc = A.scale ? A.scale[i] : 1.0f;
            const float gs = sc * g;
            const float mm = A.b1 * A.m[i] + (1.0f - A.b1) * gs;
            const float vv = A.b2 * A.v[i] + (1.0f - A.b2) * gs * gs;
            A.m[i] = mm;
            A.v[i] = vv;
            A.p[i] = pv - sc * (A.lr * (mm / A.c1) / (sqrtf(vv / A.c2) + A.eps));
        }
    }
    if (tid == 0) {
        if (better) *A.best_loss = loss;
        if (A.loss_out) *A.loss_out = loss;
        if (A.losses) A.losses[A.step - 1] = loss;
        if (A.loss_pair) {
            if (A.step == 1) A.loss_pair[0] = loss;
            A.loss_pair[1] = A.best ? fminf(*A.best_loss, loss) : loss;
        }
    }
    if (tid == 0) *A.done = 0;
}

// ---------------------------------------------------------------------------
// Full-batch training by activation regions.
//
// Every hidden pre-activation is a non-decreasing function of the input t
// (effective weights |V| >= 0, and each operation of the forward pass --
// fma with a non-negative weight, max, min -- is monotone, in fp32 too), and
// the training set is sorted by t.  So each hidden unit switches once along
// the training set: a max unit is active from the first index where its
// pre-activation is > 0, a min unit up to the first index where it is >= 0.
// The 32 switch indices, found by binary search of the pre-activations,
// cut the training set into at most 33 contiguous regions, each with one
// activation pattern (the switches are decided in fp64, like the algebra
// below).  On a region the network is affine in t:
//   h1 = a1 t + c1,  z2 = a2 t + c2,  out = alpha t + gamma,
// so every term of the full-batch gradient of the mean squared error is a
// combination of the region's sums n, sum t, sum t^2, sum y, sum t y, sum y^2.
// Around the region's first input t_r (D = t - t_r, o_r = alpha t_r + gamma,
// the output there) with dout = 2 e / S, e = alpha D + o_r - y:
//   E0 = sum e = alpha SD + n o_r - Sy,   E1 = sum e t = t_r E0 + alpha SDD + o_r SD - SDy
//   dV1_k = m1_k s_k E1,  db1_k = m1_k s_k E0   (s_k = sum_i V2_ik u_i, u_i = m2_i V3_i)
//   dV2_ik = u_i (a1_k E1 + c1_k E0),  db2_i = u_i E0
//   dV3_i = m2_i (a2_i E1 + c2_i E0),  db3 = E0      (all times 2 / S)
//   loss = (alpha^2 SDD + 2 alpha (o_r SD - SDy) + n o_r^2 - 2 o_r Sy + Syy) / S
// Steep ramps give alpha up to ~1e6, so the region sums must be accurate far
// beyond fp64 rounding of a prefix sum of 1e6 terms: the prefix sums are
// double-double (Knuth's two-sum / Dekker's two-product; every sum in a fixed
// order), and the centred sums SD, SDD, SDy are formed in double-double too.
// The region algebra then runs in fp64 on the fp32 parameters: the result is
// the per-sample gradient summed over every sample, in another order.
// ---------------------------------------------------------------------------
constexpr int MOM_T = 256, MOM_E = MOM_BLOCK / MOM_T;

struct dd2 {  // double-double: hi + lo, |lo| <= ulp(hi) / 2
    double hi, lo;
};
__device__ __forceinline__ dd2 dd_add(dd2 a, dd2 b) {
    const double s = a.hi + b.hi, bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    e += a.lo + b.lo;
    const double h = s + e;
    return {h, e - (h - s)};
}
__device__ __forceinline__ dd2 dd_neg(dd2 a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd2 dd_mul(dd2 a, double b) {
    const double p = a.hi * b;
    double e = __builtin_fma(a.hi, b, -p);
    e += a.lo * b;
    const double h = p + e;
    return {h, e - (h - p)};
}
__device__ __forceinline__ dd2 dd_of(double a) { return {a, 0.0}; }

__device__ __forceinline__ void mom_of(float tf, float yf, double q[MOM_W]) {
    const double t = tf, y = yf;  // the products of fp32 values are exact in fp64
    q[0] = t; q[1] = t * t; q[2] = y; q[3] = t * y; q[4] = y * y;
}

// Per-block moment totals (fixed order: each thread's samples in order, lanes
// by a fixed butterfly, waves in order).  bsum: blocks x MOM_W x 2 doubles.
__global__ __launch_bounds__(MOM_T) void k_mlp_mom_blocks(const float* t, const float* y, uint64_t S, double* bsum,
                                                          const uint32_t* gate) {
    if (gate && gate[0] == 0) return;
    __shared__ dd2 red[MOM_T / 64][MOM_W];
    const uint64_t b0 = (uint64_t)blockIdx.x * MOM_BLOCK + (uint64_t)threadIdx.x * MOM_E;
    dd2 acc[MOM_W];
#pragma unroll
    for (int c = 0; c < MOM_W; c++) acc[c] = dd_of(0.0);
    for (int e = 0; e < MOM_E; e++) {
        const uint64_t i = b0 + e;
        if (i < S) {
            double q[MOM_W];
            mom_of(t[i], y[i], q);
#pragma unroll
            for (int c = 0; c < MOM_W; c++) acc[c] = dd_add(acc[c], dd_of(q[c]));
        }
    }
#pragma unroll
    for (int c = 0; c < MOM_W; c++) {
        dd2 v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v = dd_add(v, dd2{__shfl_xor(v.hi, o), __shfl_xor(v.lo, o)});
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < MOM_W) {
        dd2 v = dd_of(0.0);
        for (int w = 0; w < MOM_T / 64; w++) v = dd_add(v, red[w][threadIdx.x]);
        bsum[((uint64_t)blockIdx.x * MOM_W + threadIdx.x) * 2] = v.hi;
        bsum[((uint64_t)blockIdx.x * MOM_W + threadIdx.x) * 2 + 1] = v.lo;
    }
}

// mom[i] = sums over samples < i (double-double, MOM_W x 2 doubles per i):
// the totals of earlier blocks (in block order), of earlier threads of this
// block (lane-ordered scan, then waves in order) and of the thread's earlier
// samples; no subtraction anywhere.
__global__ __launch_bounds__(MOM_T) void k_mlp_mom_scan(const float* t, const float* y, uint64_t S, const double* bsum,
                                                        double* mom, const uint32_t* gate) {
    if (gate && gate[0] == 0) return;
    __shared__ dd2 base[MOM_W];
    __shared__ dd2 wsum[MOM_T / 64][MOM_W];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < MOM_W) {
        dd2 v = dd_of(0.0);
        for (uint32_t b = 0; b < blockIdx.x; b++)
            v = dd_add(v, dd2{bsum[((uint64_t)b * MOM_W + tid) * 2], bsum[((uint64_t)b * MOM_W + tid) * 2 + 1]});
        base[tid] = v;
    }
    const uint64_t b0 = (uint64_t)blockIdx.x * MOM_BLOCK + (uint64_t)tid * MOM_E;
    dd2 own[MOM_W];
#pragma unroll
    for (int c = 0; c < MOM_W; c++) own[c] = dd_of(0.0);
    for (int e = 0; e < MOM_E; e++) {
        const uint64_t i = b0 + e;
        if (i < S) {
            double q[MOM_W];
            mom_of(t[i], y[i], q);
#pragma unroll
            for (int c = 0; c < MOM_W; c++) own[c] = dd_add(own[c], dd_of(q[c]));
        }
    }
    dd2 excl[MOM_W];
#pragma unroll
    for (int c = 0; c < MOM_W; c++) {
        dd2 x = own[c];
        for (int o = 1; o < 64; o <<= 1) {
            const dd2 u{__shfl_up(x.hi, o), __shfl_up(x.lo, o)};
            if (lane >= o) x = dd_add(u, x);
        }
        const dd2 ex{__shfl_up(x.hi, 1), __shfl_up(x.lo, 1)};
        excl[c] = lane ? ex : dd_of(0.0);
        if (lane == 63) wsum[w][c] = x;
    }
    __syncthreads();
    dd2 run[MOM_W];
#pragma unroll
    for (int c = 0; c < MOM_W; c++) {
        dd2 before = base[c];
        for (int q = 0; q < w; q++) before = dd_add(before, wsum[q][c]);
        run[c] = dd_add(before, excl[c]);
    }
    for (int e = 0; e < MOM_E; e++) {
        const uint64_t i = b0 + e;
        if (i > S) break;
#pragma unroll
        for (int c = 0; c < MOM_W; c++) {
            mom[(i * MOM_W + c) * 2] = run[c].hi;
            mom[(i * MOM_W + c) * 2 + 1] = run[c].lo;
        }
        if (i == S) break;
        double q[MOM_W];
        mom_of(t[i], y[i], q);
#pragma unroll
        for (int c = 0; c < MOM_W; c++) run[c] = dd_add(run[c], dd_of(q[c]));
        if (i + 1 == S) {
#pragma unroll
            for (int c = 0; c < MOM_W; c++) {
                mom[(S * MOM_W + c) * 2] = run[c].hi;
                mom[(S * MOM_W + c) * 2 + 1] = run[c].lo;
            }
        }
    }
}

constexpr int RG_T = 1024;            // one workgroup: 16 waves
constexpr int RG_UNITS = 2 * MLP_H;   // hidden units (switch indices)
constexpr int RG_MAXR = RG_UNITS + 1; // regions
constexpr int RG_CN = 24576;          // coarse copy of t in LDS (every sp-th sample)
enum : int { RG_A1 = 0, RG_C1 = 16, RG_A2 = 32, RG_C2 = 48, RG_U = 64, RG_Q = 80, RG_E0 = 96, RG_E1 = 97, RG_L = 98,
             RG_REC = 100 };

// Pre-activation of hidden unit u (0..15 layer 1, 16..31 layer 2) at input tt,
// in fp64 from the fp32 parameters -- the arithmetic of the region algebra
// below, so a unit's switch and the affine piece it selects agree -- and
// whether it is past its switch: > 0 for a max unit, >= 0 for a min unit
// (non-decreasing along t: every operation is monotone).
__device__ __forceinline__ bool rg_past(const float* w, int u, float tt) {
    const double t = tt;
    if (u < MLP_H) {
        const double z = (double)w[OFF_V1 + u] * t + (double)w[OFF_B1 + u];
        return u < MLP_HALF ? z > 0.0 : z >= 0.0;
    }
    const int i = u - MLP_H;
    double z = (double)w[OFF_B2 + i];
#pragma unroll
    for (int k = 0; k < MLP_H; k++) {
        const double z1 = (double)w[OFF_V1 + k] * t + (double)w[OFF_B1 + k];
        const double h1 = k < MLP_HALF ? fmax(z1, 0.0) : fmin(z1, 0.0);
        z += (double)w[OFF_V2 + MLP_H * i + k] * h1;
    }
    return i < MLP_HALF ? z > 0.0 : z >= 0.0;
}

// First index in [lo, hi) at which unit u is past its switch (hi if none),
// by 32-ary search of one half-wavefront (lanes 0..31 or 32..63), so that a
// wavefront searches two units at once; at(i) gives the input of index i.
template <typename At>
__device__ __forceinline__ uint64_t rg_search_half(const float* w, int u, uint64_t lo, uint64_t hi, At at) {
    const int lane = threadIdx.x & 63, hl = lane & 31, hb = lane & 32;
    while (lo < hi) {
        // probes lo + l * step, l = 0..31: the last one is at or past hi
        // (taken as true), so some lane's predicate holds
        const uint64_t step = (hi - lo + 30) / 31;
        const uint64_t idx = lo + (uint64_t)hl * step;
        const bool pred = idx >= hi || rg_past(w, u, at(idx));
        const uint32_t mask = (uint32_t)(__ballot(pred) >> hb);
        const int f = __ffs(mask) - 1;
        if (f == 0) break;
        lo = lo + (uint64_t)(f - 1) * step + 1;
        hi = min<uint64_t>(lo - 1 + step, hi);
    }
    return lo;
}

__global__ __launch_bounds__(RG_T) void k_mlp_regions(MlpRegion A) {
    if (A.gate && A.gate[0] == 0) return;
    __shared__ float ct[RG_CN];
    __shared__ float w[MLP_NP + 3];
    __shared__ uint64_t thr[RG_UNITS];
    __shared__ uint64_t bnd[RG_MAXR + 1];
    __shared__ double rec[RG_MAXR][RG_REC];
    __shared__ double sh_loss;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t S = A.S;
    const uint64_t sp = (S + RG_CN - 1) / RG_CN > 0 ? (S + RG_CN - 1) / RG_CN : 1;
    const uint64_t nc = (S + sp - 1) / sp;
    for (uint64_t j = tid; j < nc; j += RG_T) ct[j] = A.t[j * sp];
    const double inv_s = 1.0 / (double)S;
    double pb1 = 1.0, pb2 = 1.0;
    const uint32_t nstep = A.steps ? A.steps : 1;
    // parameter tid's value, Adam moments and step scale live in thread
    // tid's registers for the whole training (written back at the end)
    static_assert(MLP_NP <= RG_T, "one thread per parameter");
    float pv = 0.0f, mv = 0.0f, vv = 0.0f, sc = 1.0f;
    if (tid < MLP_NP) {
        pv = A.p[tid];
        if (A.steps) {
            mv = A.m[tid];
            vv = A.v[tid];
            sc = A.scale ? A.scale[tid] : 1.0f;
        }
    }
    float best_loss = A.best ? *A.best_loss : 0.0f;
    for (uint32_t k = 1; k <= nstep; k++) {
        if (tid < MLP_NP) w[tid] = mlp_is_weight(tid) ? fabsf(pv) : pv;
        __syncthreads();
        // switch indices: the two halves of wave wv search units wv and wv + 16
        static_assert(RG_UNITS == 2 * (RG_T / 64), "two units per wavefront");
        {
            const int u = wv + (lane >= 32 ? RG_UNITS / 2 : 0);
            const uint64_t jc = rg_search_half(w, u, 0, nc, [&](uint64_t j) { return ct[j]; });
            uint64_t T;
            if (jc == 0) {
                T = 0;
            } else {
                const uint64_t lo = (jc - 1) * sp + 1, hi = min<uint64_t>(jc * sp, S);
                T = rg_search_half(w, u, lo, hi, [&](uint64_t i) { return A.t[i]; });
            }
            if ((lane & 31) == 0) thr[u] = T;
        }
        __syncthreads();
        if (tid < RG_UNITS) {  // region boundaries: the switch indices in order
            const uint64_t mine = thr[tid];
            uint32_t r = 0;
            for (int q = 0; q < RG_UNITS; q++) r += (thr[q] < mine || (thr[q] == mine && q < tid)) ? 1u : 0u;
            bnd[r + 1] = mine;
        }
        if (tid == 0) { bnd[0] = 0; bnd[RG_MAXR] = S; }
        __syncthreads();
        // one group of 16 lanes per region (four per wavefront, every region
        // in one round): its affine pieces, moments and the per-region
        // factors of the gradient
        static_assert(RG_MAXR <= RG_T / 16, "a lane group for every region");
        for (int r = tid >> 4; r < RG_MAXR; r += RG_T / 16) {
            const uint64_t b = bnd[r], e = bnd[r + 1];
            double* R = rec[r];
            const int kk = lane & 15, g0 = lane & 48;  // unit, the group's first lane
            if (b >= e) {
                for (int x = kk; x < RG_REC; x += 16) R[x] = 0.0;
                continue;
            }
            // unit masks at the region's first index
            const bool on1 = kk < MLP_HALF ? b >= thr[kk] : b < thr[kk];
            const bool on2 = kk < MLP_HALF ? b >= thr[MLP_H + kk] : b < thr[MLP_H + kk];
            const double a1 = on1 ? (double)w[OFF_V1 + kk] : 0.0, c1 = on1 ? (double)w[OFF_B1 + kk] : 0.0;
            double a2 = 0.0, c2 = (double)w[OFF_B2 + kk];
            for (int q = 0; q < MLP_H; q++) {
                const double wq = (double)w[OFF_V2 + MLP_H * kk + q];
                a2 += wq * __shfl(a1, g0 + q);
                c2 += wq * __shfl(c1, g0 + q);
            }
            const double u = on2 ? (double)w[OFF_V3 + kk] : 0.0;
            double s = 0.0;
            for (int q = 0; q < MLP_H; q++) s += (double)w[OFF_V2 + MLP_H * q + kk] * __shfl(u, g0 + q);
            double al = u * a2, ga = u * c2;
            for (int o = 8; o > 0; o >>= 1) { al += __shfl_xor(al, o); ga += __shfl_xor(ga, o); }
            al = __shfl(al, g0);
            ga = __shfl(ga, g0) + (double)w[OFF_B3];
            // region sums (double-double differences of the prefix sums),
            // centred at the region's first input t_r
            const double tr = (double)A.t[b];
            auto rsum = [&](int c) {
                const double* p0 = A.mom + (b * MOM_W + c) * 2;
                const double* p1 = A.mom + (e * MOM_W + c) * 2;
                return dd_add(dd2{p1[0], p1[1]}, dd_neg(dd2{p0[0], p0[1]}));
            };
            const double n = (double)(e - b);
            const dd2 St = rsum(0), Stt = rsum(1), Sy = rsum(2), Sty = rsum(3), Syy = rsum(4);
            const dd2 ntr = dd_mul(dd_of(n), tr);
            const double SD = dd_add(St, dd_neg(ntr)).hi;                                   // sum (t - t_r)
            const double SDD = dd_add(dd_add(Stt, dd_neg(dd_mul(St, 2.0 * tr))), dd_mul(ntr, tr)).hi;
            const double SDy = dd_add(Sty, dd_neg(dd_mul(Sy, tr))).hi;
            const double sy = Sy.hi;
            const double orr = al * tr + ga;  // output at t_r
            const double E0 = al * SD + n * orr - sy;
            const double E1 = tr * E0 + al * SDD + orr * SD - SDy;
            R[RG_A1 + kk] = a1; R[RG_C1 + kk] = c1;
            R[RG_A2 + kk] = on2 ? a2 : 0.0; R[RG_C2 + kk] = on2 ? c2 : 0.0;
            R[RG_U + kk] = u; R[RG_Q + kk] = on1 ? s : 0.0;
            if (kk == 0) {
                R[RG_E0] = E0; R[RG_E1] = E1;
                const double Soo = dd_add(dd_add(dd_mul(dd_of(n * orr), orr), dd_neg(dd_mul(Sy, 2.0 * orr))), Syy).hi;
                R[RG_L] = al * al * SDD + 2.0 * al * (orr * SD - SDy) + Soo;
            }
        }
        __syncthreads();
        // gradient entries, each summed over the regions in order
        double g = 0.0;
        if (tid < MLP_NP) {
            for (int r = 0; r < RG_MAXR; r++) {
                const double* R = rec[r];
                const double E0 = R[RG_E0], E1 = R[RG_E1];
                double c;
                if (tid < OFF_B1) c = R[RG_Q + tid] * E1;
                else if (tid < OFF_V2) c = R[RG_Q + tid - OFF_B1] * E0;
                else if (tid < OFF_B2) {
                    const int i = (tid - OFF_V2) / MLP_H, q = (tid - OFF_V2) % MLP_H;
                    c = R[RG_U + i] * (R[RG_A1 + q] * E1 + R[RG_C1 + q] * E0);
                } else if (tid < OFF_V3) c = R[RG_U + tid - OFF_B2] * E0;
                else if (tid < OFF_B3) c = R[RG_A2 + tid - OFF_V3] * E1 + R[RG_C2 + tid - OFF_V3] * E0;
                else c = E0;
                g += c;
            }
            g *= 2.0 * inv_s;
        } else if (tid == MLP_NP) {
            double l = 0.0;
            for (int r = 0; r < RG_MAXR; r++) l += rec[r][RG_L];
            sh_loss = l * inv_s;
        }
        __syncthreads();
        const float loss = (float)sh_loss;
        const bool better = A.best && loss < best_loss;
        pb1 *= (double)A.b1;
        pb2 *= (double)A.b2;
        if (tid < MLP_NP) {
            if (better) A.best[tid] = pv;
            float gf = (float)g;
            if (mlp_is_weight(tid)) gf *= pv > 0.0f ? 1.0f : (pv < 0.0f ? -1.0f : 0.0f);  // d|V|/dV
            if (k == 1 && A.grad_out) A.grad_out[tid] = gf;
            if (A.steps) {
                const float gs = sc * gf;
                mv = A.b1 * mv + (1.0f - A.b1) * gs;
                vv = A.b2 * vv + (1.0f - A.b2) * gs * gs;
                const float c1 = (float)(1.0 - pb1), c2 = (float)(1.0 - pb2);
                pv = pv - sc * (A.lr * (mv / c1) / (sqrtf(vv / c2) + A.eps));
            }
        }
        if (better) best_loss = loss;
        if (tid == 0) {
            if (better) *A.best_loss = loss;
            if (k == 1 && A.loss_out) *A.loss_out = loss;
            if (A.losses && A.steps) A.losses[k - 1] = loss;
            if (A.loss_pair) {
                if (k == 1) A.loss_pair[0] = loss;
                A.loss_pair[1] = A.best ? fminf(best_loss, loss) : loss;
            }
        }
        __syncthreads();  // the next step rewrites w and rec
    }
    if (tid < MLP_NP && A.steps) {
        A.p[tid] = pv;
        A.m[tid] = mv;
        A.v[tid] = vv;
    }
}

hipError_t launch_mlp_moments(const float* t, const float* y, uint64_t S, double* block_sums, double* mom,
                              const uint32_t* gate, hipStream_t st) {
    const uint32_t nb = (uint32_t)((S + MOM_BLOCK - 1) / MOM_BLOCK);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_mom_blocks, dim3(nb), dim3(MOM_T), 0, st, t, y, S, block_sums, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_mom_scan, dim3(nb), dim3(MOM_T), 0, st, t, y, S, block_sums, mom, gate);
    return hipGetLastError();
}

hipError_t launch_mlp_regions(const MlpRegion& A, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_regions, dim3(1), dim3(RG_T), 0, st, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Model record of the MLP-rooted model: header, effective weights and
// (optionally) the caller's pre-scaled leaves.
// ---------------------------------------------------------------------------
__global__ void k_mlp_install(const float* p, const double* lo_inv, uint32_t L, uint32_t B1, uint32_t log2B2, double R,
                              const double* leaves, const uint32_t* gate, uint32_t* set, uint64_t* dst) {
    if (gate && gate[0] == 0) return;
    float* w = (float*)(dst + MLP_W_WORD);
    for (int i = threadIdx.x; i < MLP_NP + 1; i += blockDim.x)
        w[i] = i == MLP_NP ? 0.0f : (mlp_is_weight(i) ? fabsf(p[i]) : p[i]);
    if (leaves)
        for (uint32_t i = threadIdx.x; i < 4 * L; i += blockDim.x) ((double*)dst)[MLP_LEAF_WORD + i] = leaves[i];
    if (threadIdx.x == 0) {
        MlpModel* h = (MlpModel*)dst;
        h->L = L; h->B1 = B1; h->log2B2 = log2B2; h->pad = 0;
        h->lo = lo_inv[0]; h->inv = lo_inv[1]; h->R = R; h->pad2 = 0;
        if (set) set[0] = 1;
    }
}

// Model record -> LDS (weights and leaves) for the per-key kernels.
__device__ __forceinline__ void load_mlp_model(const uint64_t* mdl, float* w, double* leaves, int tid, int nt) {
    const MlpModel* h = (const MlpModel*)mdl;
    const float* ws = (const float*)(mdl + MLP_W_WORD);
    for (int i = tid; i < MLP_NP; i += nt) w[i] = ws[i];
    for (uint32_t i = tid; i < 4 * h->L; i += nt) leaves[i] = ((const double*)mdl)[MLP_LEAF_WORD + i];
}

// Bucket ids of every key of the level's MLP-rooted segments, stored at the
// key's absolute position so that the histogram and scatter passes read
// them instead of evaluating the network twice.  K_MLP: level bucket
// g >> log2(B2); K_MLP_FINE: g - win inside the parent's fine window.
constexpr int IDS_T = 256;
constexpr int IDS_K = 4;  // keys per thread per network pass

__global__ __launch_bounds__(IDS_T) void k_mlp_ids(Params P) {
    __shared__ float w[MLP_NP];
    __shared__ double leaves[4 * L_MAX];
    const int tid = threadIdx.x;
    const int lvl = P.level;
    const uint32_t nunit = level_units(P, lvl);
    const uint32_t nseg = min(P.ctl->nseg[lvl], (uint32_t)P.seg_cap);
    const uint64_t* src = P.keys[lvl & 1];
    uint64_t cur = 0;
    for (uint32_t t = blockIdx.x; t < nunit; t += gridDim.x) {
        const Tile td = P.tiles[lvl & 1][t];
        if (td.seg >= nseg) continue;
        const Seg sg = P.segs[lvl & 1][td.seg];
        if ((sg.kind != K_MLP && sg.kind != K_MLP_FINE) || (sg.flags & SEG_FAILED)) continue;
        const uint64_t* mdl = (const uint64_t*)sg.model;
        if (sg.model != cur) {
            __syncthreads();
            load_mlp_model(mdl, w, leaves, tid, IDS_T);
            __syncthreads();
            cur = sg.model;
        }
        const MlpModel* h = (const MlpModel*)mdl;
        const double lo = h->lo, inv = h->inv, Rm1 = h->R - 1.0;
        const float Lf = (float)h->L;
        const uint32_t shift = sg.kind == K_MLP ? h->log2B2 : 0u;
        const uint32_t win = sg.kind == K_MLP ? 0u : sg.win;
        const uint32_t U = seg_unit(sg.flags);
        const uint64_t base = sg.off + (uint64_t)td.idx * U;
        const uint32_t un = (uint32_t)min<uint64_t>(U, sg.n - (uint64_t)td.idx * U);
        for (uint32_t i0 = 0; i0 < un; i0 += IDS_T * IDS_K) {
            lds_reload_fence();
            uint64_t raw[IDS_K];
            uint32_t g[IDS_K];
#pragma unroll
            for (int k = 0; k < IDS_K; k++) {
                const uint32_t i = i0 + k * IDS_T + tid;
                raw[k] = i < un ? src[base + i] : 0;
            }
            mlp_root_buckets<IDS_K>(w, leaves, lo, inv, Lf, Rm1, raw, P.u64, g);
#pragma unroll
            for (int k = 0; k < IDS_K; k++) {
                const uint32_t i = i0 + k * IDS_T + tid;
                if (i < un) P.ids[base + i] = (uint16_t)((g[k] >> shift) - win);
            }
        }
    }
}

// Bucket ids at total resolution under an MLP-rooted model record.
__global__ __launch_bounds__(IDS_T) void k_mlp_rmi_buckets(const uint64_t* mdl, const uint64_t* keys, uint64_t n,
                                                           int u64, uint32_t* out) {
    __shared__ float w[MLP_NP];
    __shared__ double leaves[4 * L_MAX];
    load_mlp_model(mdl, w, leaves, threadIdx.x, IDS_T);
    __syncthreads();
    const MlpModel* h = (const MlpModel*)mdl;
    const double lo = h->lo, inv = h->inv, Rm1 = h->R - 1.0;
    const float Lf = (float)h->L;
    const uint64_t step = (uint64_t)gridDim.x * IDS_T * IDS_K;
    for (uint64_t i0 = (uint64_t)blockIdx.x * IDS_T * IDS_K; i0 < n; i0 += step) {
        lds_reload_fence();
        uint64_t raw[IDS_K];
        uint32_t g[IDS_K];
#pragma unroll
        for (int k = 0; k < IDS_K; k++) {
            const uint64_t i = i0 + k * IDS_T + threadIdx.x;
            raw[k] = i < n ? keys[i] : 0;
        }
        mlp_root_buckets<IDS_K>(w, leaves, lo, inv, Lf, Rm1, raw, u64, g);
#pragma unroll
        for (int k = 0; k < IDS_K; k++) {
            const uint64_t i = i0 + k * IDS_T + threadIdx.x;
            if (i < n) out[i] = g[k];
        }
    }
}

// The network alone as a CDF: g = min(floor(F * R), R - 1) in fp32.
__global__ __launch_bounds__(IDS_T) void k_mlp_buckets(const float* p, const double* lo_inv, uint32_t R,
                                                       const uint64_t* keys, uint64_t n, int u64, uint32_t* out) {
    __shared__ float w[MLP_NP];
    for (int i = threadIdx.x; i < MLP_NP; i += IDS_T) w[i] = mlp_is_weight(i) ? fabsf(p[i]) : p[i];
    __syncthreads();
    const double lo = lo_inv[0], inv = lo_inv[1];
    const uint64_t step = (uint64_t)gridDim.x * IDS_T * IDS_K;
    for (uint64_t i0 = (uint64_t)blockIdx.x * IDS_T * IDS_K; i0 < n; i0 += step) {
        lds_reload_fence();
        uint64_t raw[IDS_K];
        uint32_t g[IDS_K];
#pragma unroll
        for (int k = 0; k < IDS_K; k++) {
            const uint64_t i = i0 + k * IDS_T + threadIdx.x;
            raw[k] = i < n ? keys[i] : 0;
        }
        mlp_buckets_multi<IDS_K>(w, lo, inv, (float)R, raw, u64, g);
#pragma unroll
        for (int k = 0; k < IDS_K; k++) {
            const uint64_t i = i0 + k * IDS_T + threadIdx.x;
            if (i < n) out[i] = g[k];
        }
    }
}

// ---------------------------------------------------------------------------
#define LAUNCH(kernel, grid, block, stream, ...)                                     \
    do {                                                                             \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

static uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t cap) {
    const uint64_t g = std::min<uint64_t>((n + threads - 1) / threads, cap);
    return g ? (uint32_t)g : 1u;
}

hipError_t launch_mlp_prep(const uint64_t* s, uint64_t S, uint64_t stride, int u64, float* t, float* y, double* lo_inv,
                           const uint32_t* gate, hipStream_t st) {
    LAUNCH(k_mlp_prep, grid_for((S + stride - 1) / stride, 256, 2048), 256, st, s, S, stride, u64, t, y, lo_inv, gate);
}
hipError_t launch_mlp_setup(const float* t, uint64_t S, const float* init, double eps, float* p, float* m, float* v,
                            float* best, float* scale, float* best_loss, unsigned int* done, const uint32_t* gate,
                            hipStream_t st) {
    LAUNCH(k_mlp_setup, 1, MLP_SETUP_T, st, t, S, init, eps, p, m, v, best, scale, best_loss, done, gate);
}
uint32_t mlp_step_grid(uint64_t S) { return grid_for(S, MLP_T, MLP_G); }
hipError_t launch_mlp_step(const MlpStep& A, hipStream_t st) { LAUNCH(k_mlp_step, mlp_step_grid(A.S), MLP_T, st, A); }
hipError_t launch_mlp_install(const float* p, const double* lo_inv, uint32_t L, uint32_t B1, uint32_t log2B2, double R,
                              const double* leaves, const uint32_t* gate, uint32_t* set, uint64_t* dst,
                              hipStream_t st) {
    LAUNCH(k_mlp_install, 1, 512, st, p, lo_inv, L, B1, log2B2, R, leaves, gate, set, dst);
}
hipError_t launch_mlp_ids(const Params& P, uint32_t grid, hipStream_t st) { LAUNCH(k_mlp_ids, grid, IDS_T, st, P); }
hipError_t launch_mlp_rmi_buckets(const uint64_t* mdl, const uint64_t* keys, uint64_t n, int u64, uint32_t* out,
                                  hipStream_t st) {
    LAUNCH(k_mlp_rmi_buckets, grid_for(n, IDS_T * IDS_K, 2048), IDS_T, st, mdl, keys, n, u64, out);
}
hipError_t launch_mlp_buckets(const float* p, const double* lo_inv, uint32_t R, const uint64_t* keys, uint64_t n,
                              int u64, uint32_t* out, hipStream_t st) {
    LAUNCH(k_mlp_buckets, grid_for(n, IDS_T * IDS_K, 2048), IDS_T, st, p, lo_inv, R, keys, n, u64, out);
}

}  // namespace ls
