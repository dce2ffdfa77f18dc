// lsort_kernels.hpp -- host-side launch wrappers of the liblsort kernels.
#pragma once
#include "lsort_internal.hpp"

namespace ls {

constexpr int FIT_T = 256;   // threads of the sample least-squares passes
constexpr int FIT_G = 256;   // workgroups of the sample least-squares passes

// Arguments of the model fit over a large sorted sample in global memory.
struct FitArgs {
    const uint64_t* s;   // sorted sample (raw keys)
    uint64_t S;          // sample size
    uint64_t n;          // keys the model will partition (policy input)
    int u64;
    int mode;            // 0 Alg. 5 policy, 1 force RMI, 2 force splitter tree
    int mlp;             // learned kind is the MLP (tree still possible)
    uint32_t L, B1, log2B2, Bt, G;
    double R;            // total resolution B1 << log2B2 of the scaled leaves
    double* part;        // G * 8 partial sums
    double* leaf;        // L_MAX * 8 leaf lines
    uint64_t* model;     // model destination (device)
    uint32_t* flag;      // [0] = 1 when the learned model was chosen
    Seg* seg;            // descriptor of the prebuilt first level (nullable)
};

// level kernels (lsort_kernels.hip)
hipError_t launch_reset(const Params& P, uint64_t* persist, hipStream_t st);
hipError_t launch_seed(const Params& P, const uint64_t* offsets, uint64_t m, uint64_t n_single, uint32_t prebuilt,
                       const uint64_t* persist, uint32_t grid, hipStream_t st);
hipError_t launch_model(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_hist(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_scan(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_scatter(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_base_small(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_base_big(const Params& P, uint32_t grid, hipStream_t st);

// sample fit and single steps (lsort_fit.hip)
hipError_t launch_gather(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t S, uint64_t* out, hipStream_t st);
hipError_t launch_fit1(const FitArgs& A, hipStream_t st);
hipError_t launch_fit2(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_root(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_leaves(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_finish(const FitArgs& A, hipStream_t st);
hipError_t launch_model_buckets(const uint64_t* model, uint32_t words, uint32_t kind, uint32_t nb, uint32_t win,
                                const uint64_t* keys, uint64_t n, int u64, uint32_t* out, hipStream_t st);
hipError_t launch_install_rmi(const double* params, uint32_t L, double R, uint32_t B1, uint32_t log2B2, uint64_t* dst,
                              hipStream_t st);
hipError_t launch_install_tree(const uint64_t* u, const uint8_t* eq, uint32_t m, uint64_t* dst, hipStream_t st);
hipError_t launch_splitters(const uint64_t* s, uint64_t S, int u64, uint32_t B, uint64_t* scratch, uint64_t* u_out,
                            uint8_t* eq_out, uint32_t* m_out, hipStream_t st);
hipError_t launch_copy_words(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t st);

}  // namespace ls
