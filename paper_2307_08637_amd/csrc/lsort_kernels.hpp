// lsort_kernels.hpp -- host-side launch wrappers of the liblsort kernels.
#pragma once
#include <vector>

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
    uint32_t* first_mlp; // set to 1 when the MLP-rooted model was chosen (nullable)
    uint64_t* bstart;    // [B1 + 1]: first sample index of each first-level bucket (nullable)
    double ratio;        // oversized bucket: more than ratio x expected keys
    double balance;      // share of the sample in oversized buckets above which the tree replaces the RMI
    double* lpart;       // leaf least squares: 4 sums per piece of a leaf (set by the launchers)
    uint64_t piece;      // sample points per piece
};
constexpr uint64_t FIT_PIECE = 8192;    // sample points per workgroup of a leaf's least-squares passes
constexpr uint64_t FIT_PIECES = 1024;   // pieces beyond one per leaf (the piece grows for larger samples)

// MLP training (lsort_mlp.hip)
constexpr int MLP_G = 512;           // workgroups of a training step (gradient partials; two per CU)
constexpr int MLP_ACC = MLP_NP + 1;  // gradient entries + the squared error per partial

struct MlpStep {
    const float* t;       // model inputs of the training set
    const float* y;       // targets (rank fractions)
    uint64_t S;
    float* p;             // parameters V / biases
    float* m;             // Adam first moment
    float* v;             // Adam second moment
    float* partial;       // MLP_G * MLP_ACC workgroup partials
    unsigned int* done;   // workgroups finished in this step; zero between steps
    float* grad_out;      // nullable: gradient w.r.t. p
    float* loss_out;      // nullable: loss (mean squared error) at p
    float* losses;        // nullable: loss of step `step` at losses[step - 1]
    double* loss_pair;    // nullable: [0] loss at step 1, [1] lowest loss so far
    float* best;          // nullable: parameters with the lowest loss seen (set up by k_mlp_setup)
    const float* scale;   // nullable: per-parameter optimiser step scale (set up by k_mlp_setup)
    float* best_loss;     // that loss (with best)
    const uint32_t* gate; // nullable: do nothing when gate[0] == 0
    uint32_t step;        // 1-based Adam step number
    uint32_t update;      // 1: apply Adam; 0: gradient only
    float lr, b1, b2, eps;
    float c1, c2;         // bias corrections 1 - b1^step, 1 - b2^step
};

// Full-batch training by activation regions (lsort_mlp.hip): the training
// set's prefix moments, then every Adam step in one workgroup.
constexpr int MOM_BLOCK = 4096;      // samples per block of the moment scan
constexpr int MOM_W = 5;             // moments per sample: t, t^2, y, t y, y^2
struct MlpRegion {
    const float* t;       // model inputs of the training set (non-decreasing)
    const double* mom;    // (S + 1) x MOM_W prefix moments, double-double (hi, lo): sums over samples < i
    uint64_t S;
    float* p;             // parameters V / biases
    float* m;             // Adam first moment
    float* v;             // Adam second moment
    const float* scale;   // nullable: per-parameter optimiser step scale
    float* best;          // nullable: parameters with the lowest loss seen
    float* best_loss;     // that loss (with best)
    float* grad_out;      // nullable: gradient of the first evaluation w.r.t. p
    float* loss_out;      // nullable: loss of the first evaluation
    float* losses;        // nullable: loss of step k at losses[k - 1]
    double* loss_pair;    // nullable: [0] loss at step 1, [1] lowest loss
    const uint32_t* gate; // nullable: do nothing when gate[0] == 0
    uint32_t steps;       // Adam steps; 0: one gradient evaluation, no update
    float lr, b1, b2, eps;
};
hipError_t launch_mlp_moments(const float* t, const float* y, uint64_t S, double* block_sums, double* mom,
                              const uint32_t* gate, hipStream_t st);
hipError_t launch_mlp_regions(const MlpRegion& A, hipStream_t st);

// level kernels (lsort_kernels.hip)
hipError_t launch_reset(const Params& P, uint64_t* persist, hipStream_t st);
hipError_t launch_seed(const Params& P, const uint64_t* offsets, uint64_t m, uint64_t n_single, uint32_t prebuilt,
                       const uint64_t* persist, uint32_t grid, hipStream_t st);
hipError_t launch_model(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_fit_block(const uint64_t* s, uint32_t S, int u64, uint32_t L, uint32_t B1, double* dst,
                            hipStream_t st);
hipError_t launch_hist(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_scan(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_scatter(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_base_small(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_base_big(const Params& P, uint32_t grid, hipStream_t st);
// classes: bit 0 items of up to 2048 keys, bit 1 of 2049..4096, bit 2 of
// 4097..8192 (a launch per class present); bit 3: one launch for all
hipError_t launch_base_merge(const Params& P, uint32_t cus, uint32_t classes, hipStream_t st);
hipError_t launch_base_model(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_resident(const Params& P, uint32_t grid, hipStream_t st);

// sample fit and single steps (lsort_fit.hip)
hipError_t launch_gather(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t S, uint64_t* out, hipStream_t st);
hipError_t launch_fit1(const FitArgs& A, hipStream_t st);
hipError_t launch_fit2(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_root(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_leaves(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_finish(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_bstart(const FitArgs& A, hipStream_t st);
hipError_t launch_fit_balance(const FitArgs& A, hipStream_t st);
hipError_t launch_model_buckets(const uint64_t* model, uint32_t words, uint32_t kind, uint32_t nb, uint32_t win,
                                const uint64_t* keys, uint64_t n, int u64, uint32_t* out, hipStream_t st);
hipError_t launch_install_rmi(const double* params, uint32_t L, double R, uint32_t B1, uint32_t log2B2, uint64_t* dst,
                              hipStream_t st);
hipError_t launch_install_tree(const uint64_t* u, const uint8_t* eq, uint32_t m, uint64_t* dst, hipStream_t st);
hipError_t launch_splitters(const uint64_t* s, uint64_t S, int u64, uint32_t B, uint64_t* scratch, uint64_t* u_out,
                            uint8_t* eq_out, uint32_t* m_out, hipStream_t st);
hipError_t launch_copy_words(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t st);

// MLP CDF (lsort_mlp.hip)
hipError_t launch_mlp_prep(const uint64_t* s, uint64_t S, uint64_t stride, int u64, float* t, float* y, double* lo_inv,
                           const uint32_t* gate, hipStream_t st);
hipError_t launch_mlp_setup(const float* t, uint64_t S, const float* init, double eps, float* p, float* m, float* v,
                            float* best, float* scale, float* best_loss, unsigned int* done, const uint32_t* gate,
                            hipStream_t st);
uint32_t mlp_step_grid(uint64_t S);
hipError_t launch_mlp_step(const MlpStep& A, hipStream_t st);
hipError_t launch_mlp_install(const float* p, const double* lo_inv, uint32_t L, uint32_t B1, uint32_t log2B2, double R,
                              const double* leaves, const uint32_t* gate, uint32_t* set, uint64_t* dst,
                              hipStream_t st);
hipError_t launch_mlp_ids(const Params& P, uint32_t grid, hipStream_t st);
hipError_t launch_mlp_rmi_buckets(const uint64_t* mdl, const uint64_t* keys, uint64_t n, int u64, uint32_t* out,
                                  hipStream_t st);
hipError_t launch_mlp_buckets(const float* p, const double* lo_inv, uint32_t R, const uint64_t* keys, uint64_t n,
                              int u64, uint32_t* out, hipStream_t st);

// tuning table (lsort_api.hip) and the synthetic inputs of the autotuner (lsort_tune.hip)
struct TuneEntry {
    int cls;                                // floor(log10(n / m))
    uint32_t buckets, cutoff, tree_buckets; // fastest options measured for the class
    double ms, default_ms;                  // their time and the defaults' time (informational)
    uint32_t tile;                          // first-level work-unit keys (ls_options.tile)
};
void tuning_install(const std::vector<TuneEntry>& t);
int report_error(int status, const char* msg);  // sets ls_last_error(), returns status
hipError_t launch_tune_fill(double* keys, const uint64_t* offsets, uint64_t m, uint64_t seed, hipStream_t st);

// key types and payload widths mapped onto the engine's (lsort_types.hip)
hipError_t launch_flip_sign(uint64_t* k, uint64_t n, uint32_t cus, hipStream_t st);
hipError_t launch_widen(const uint32_t* src, uint64_t* dst, uint64_t n, uint32_t cus, hipStream_t st);
hipError_t launch_narrow(const uint64_t* src, uint32_t* dst, uint64_t n, uint32_t cus, hipStream_t st);
hipError_t launch_index_save(const uint64_t* pay, uint64_t* save, uint32_t* idx, uint64_t n, uint32_t cus,
                             hipStream_t st);
hipError_t launch_gather64(const uint64_t* save, const uint32_t* idx, uint64_t* pay, uint64_t n, uint32_t cus,
                           hipStream_t st);

// reference streams (lsort_stream.hip): copy of n words; wrapping sum of n words into *sum
hipError_t launch_stream_copy(const uint64_t* src, uint64_t* dst, uint64_t n, uint32_t cus, hipStream_t st);
hipError_t launch_stream_read(const uint64_t* src, uint64_t n, uint64_t* sum, uint32_t cus, hipStream_t st);

}  // namespace ls
