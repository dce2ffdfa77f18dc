// lsort_tune.hip -- the autotuner of the batched and single-array sort: for
// each size class (decimal order of magnitude of the average array size) it
// times every candidate (bucket count, base-case cutoff, splitter fan-out)
// on synthetic arrays generated on the device, keeps the fastest, and writes
// a JSON table keyed by the device's architecture and compute-unit count.
// ls_load_tuning installs such a table; calls with LS_FLAG_TUNED (or no
// options at all) then take the table's values for the fields they leave 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "lsort.h"
#include "lsort_dev.hpp"
#include "lsort_kernels.hpp"

namespace ls {

// Keys of array s: law (hash of s) mod 3 -- U[0, 1), N(0, 1) by Box-Muller,
// LogNormal(0, 1) -- from SplitMix64 streams.  One workgroup per array.
__global__ void k_tune_fill(double* keys, const uint64_t* offsets, uint64_t m, uint64_t seed) {
    for (uint64_t s = blockIdx.x; s < m; s += gridDim.x) {
        const uint64_t lo = offsets[s], hi = offsets[s + 1];
        const uint64_t h = splitmix64_at(seed, s);
        const uint32_t law = (uint32_t)(h % 3);
        for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double u1 = ((double)(splitmix64_at(h, 2 * i) >> 11) + 0.5) * 0x1p-53;
            const double u2 = ((double)(splitmix64_at(h, 2 * i + 1) >> 11) + 0.5) * 0x1p-53;
            const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            keys[i] = law == 0 ? u1 : (law == 1 ? z : exp(z));
        }
    }
}

hipError_t launch_tune_fill(double* keys, const uint64_t* offsets, uint64_t m, uint64_t seed, hipStream_t st) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(m, 1), 4096);
    hipLaunchKernelGGL(k_tune_fill, dim3(grid), dim3(256), 0, st, keys, offsets, m, seed);
    return hipGetLastError();
}

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

#define TUNE_HIP(expr)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return (ls_status)report_error(LS_EHIP, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

struct Candidate {
    uint32_t buckets, cutoff, tree_buckets, tile;
};

// Device identity the table is keyed by.
ls_status device_id(std::string& arch, int& cus) {
    int dev = 0;
    TUNE_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    TUNE_HIP(hipGetDeviceProperties(&prop, dev));
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    cus = prop.multiProcessorCount;
    return LS_OK;
}

// Mean time of `reps` sorts of the pristine keys (restored before each).
ls_status time_sort(double* keys, const double* pristine, uint64_t n, const uint64_t* offsets, uint64_t m,
                    const ls_options& o, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, double& ms) {
    double total = 0;
    for (int r = -1; r < reps; r++) {  // r = -1: warm-up (workspace growth)
        TUNE_HIP(hipMemcpyAsync(keys, pristine, n * 8, hipMemcpyDeviceToDevice, st));
        TUNE_HIP(hipEventRecord(e0, st));
        ls_status s = m == 1 ? ls_sort(keys, n, LS_F64, nullptr, &o, st)
                             : ls_sort_segmented(keys, offsets, m, n, LS_F64, nullptr, &o, st);
        if (s) return s;
        TUNE_HIP(hipEventRecord(e1, st));
        TUNE_HIP(hipEventSynchronize(e1));
        float t = 0;
        TUNE_HIP(hipEventElapsedTime(&t, e0, e1));
        if (r >= 0) total += t;
    }
    ms = total / reps;
    return LS_OK;
}

// Extract the number after "key": inside [b, e); false if absent.
bool json_number(const std::string& txt, size_t b, size_t e, const char* key, double& v) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = txt.find(k, b);
    if (p == std::string::npos || p >= e) return false;
    p = txt.find(':', p + k.size());
    if (p == std::string::npos || p >= e) return false;
    char* end = nullptr;
    v = std::strtod(txt.c_str() + p + 1, &end);
    return end != txt.c_str() + p + 1;
}

bool json_string(const std::string& txt, const char* key, std::string& v) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = txt.find(k);
    if (p == std::string::npos) return false;
    p = txt.find('"', txt.find(':', p + k.size()));
    if (p == std::string::npos) return false;
    const size_t q = txt.find('"', p + 1);
    if (q == std::string::npos) return false;
    v = txt.substr(p + 1, q - p - 1);
    return true;
}

}  // namespace
}  // namespace ls

using namespace ls;

extern "C" {

ls_status ls_autotune(const char* table_path) {
    if (!table_path) return (ls_status)report_error(LS_EINVAL, "table_path is NULL");
    std::string arch;
    int cus = 0;
    ls_status s = device_id(arch, cus);
    if (s) return s;
    // (buckets, cutoff, tree fan-out) for every class; the first-level work
    // unit (tile) only matters for arrays of many units: searched from 1e6 keys
    const Candidate cands[] = {{256, 256, 128, 0}, {256, 512, 256, 0}, {512, 256, 128, 0}, {512, 512, 256, 0},
                               {1000, 256, 128, 0}, {1000, 512, 256, 0}, {1000, 512, 128, 0}, {1000, 256, 256, 0},
                               {512, 512, 128, 0}, {256, 512, 128, 0}, {1024, 512, 256, 0}, {1024, 256, 256, 0},
                               {1000, 1024, 256, 0}, {1000, 512, 256, 65536}, {1000, 512, 256, 131072},
                               {1000, 1024, 256, 131072}};
    const Candidate defaults = {1000, 512, 256, 0};
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TUNE_HIP(hipStreamCreate(&st));
    TUNE_HIP(hipEventCreate(&e0));
    TUNE_HIP(hipEventCreate(&e1));
    std::vector<TuneEntry> table;
    std::mt19937_64 rng(0x7A11E);
    for (int cls = 3; cls <= 8; cls++) {
        // batched classes: ~2e7 keys in arrays of about 10^cls keys (log-uniform
        // over [10^cls / 4, 4 x 10^cls)); single arrays of 10^cls keys above that
        const double avg = std::pow(10.0, cls);
        std::vector<uint64_t> off{0};
        if (cls <= 6) {
            std::uniform_real_distribution<double> u(std::log(avg / 4), std::log(avg * 4));
            while (off.back() < 20000000ull) off.push_back(off.back() + (uint64_t)std::floor(std::exp(u(rng))));
        } else {
            off.push_back((uint64_t)avg);
        }
        const uint64_t m = off.size() - 1, n = off.back();
        DevBuf keys, pristine, doff;
        TUNE_HIP(hipMalloc(&keys.p, n * 8));
        TUNE_HIP(hipMalloc(&pristine.p, n * 8));
        TUNE_HIP(hipMalloc(&doff.p, (m + 1) * 8));
        TUNE_HIP(hipMemcpy(doff.p, off.data(), (m + 1) * 8, hipMemcpyHostToDevice));
        TUNE_HIP(launch_tune_fill((double*)pristine.p, (const uint64_t*)doff.p, m, 0x5EED0000ull + cls, st));
        TuneEntry best{cls, 0, 0, 0, 1e30, 0, 32768};
        for (const Candidate& c : cands) {
            if (c.tile && cls < 6) continue;
            ls_options o;
            std::memset(&o, 0, sizeof(o));
            o.struct_size = sizeof(o);
            o.buckets = c.buckets; o.cutoff = c.cutoff; o.tree_buckets = c.tree_buckets; o.tile = c.tile;
            o.flags = LS_FLAG_SYNC_LEVELS;
            double ms = 0;
            s = time_sort((double*)keys.p, (const double*)pristine.p, n, (const uint64_t*)doff.p, m, o, st, e0, e1, 3,
                          ms);
            if (s) return s;
            if (c.buckets == defaults.buckets && c.cutoff == defaults.cutoff && c.tree_buckets == defaults.tree_buckets)
                best.default_ms = ms;
            if (ms < best.ms) {
                best.ms = ms; best.buckets = c.buckets; best.cutoff = c.cutoff; best.tree_buckets = c.tree_buckets;
                best.tile = c.tile ? c.tile : 32768;
            }
        }
        table.push_back(best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    FILE* f = std::fopen(table_path, "w");
    if (!f) return (ls_status)report_error(LS_EINVAL, (std::string("cannot write ") + table_path).c_str());
    std::fprintf(f, "{\n  \"format\": \"lsort-tuning-1\",\n  \"device\": \"%s\",\n  \"cus\": %d,\n  \"classes\": [\n",
                 arch.c_str(), cus);
    for (size_t i = 0; i < table.size(); i++) {
        const TuneEntry& e = table[i];
        std::fprintf(f,
                     "    {\"log10_avg_size\": %d, \"buckets\": %u, \"cutoff\": %u, \"tree_buckets\": %u, "
                     "\"tile\": %u, \"ms\": %.4f, \"default_ms\": %.4f}%s\n",
                     e.cls, e.buckets, e.cutoff, e.tree_buckets, e.tile, e.ms, e.default_ms,
                     i + 1 < table.size() ? "," : "");
    }
    std::fprintf(f, "  ]\n}\n");
    std::fclose(f);
    tuning_install(table);
    return LS_OK;
}

ls_status ls_load_tuning(const char* table_path) {
    if (!table_path) {
        tuning_install({});
        return LS_OK;
    }
    FILE* f = std::fopen(table_path, "r");
    if (!f) return (ls_status)report_error(LS_EINVAL, (std::string("cannot read ") + table_path).c_str());
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, k);
    std::fclose(f);
    std::string fmt, arch;
    double cus = 0;
    if (!json_string(txt, "format", fmt) || fmt != "lsort-tuning-1" || !json_string(txt, "device", arch) ||
        !json_number(txt, 0, txt.size(), "cus", cus))
        return (ls_status)report_error(LS_EINVAL, "not an lsort tuning table (format lsort-tuning-1)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        std::string here;
        int here_cus = 0;
        if (device_id(here, here_cus) == LS_OK && (here != arch || here_cus != (int)cus))
            return (ls_status)report_error(
                LS_EINVAL, ("tuning table was made on " + arch + " with " + std::to_string((int)cus) +
                            " compute units, not on this " + here + " with " + std::to_string(here_cus)).c_str());
    } else {
        (void)hipGetLastError();
    }
    std::vector<TuneEntry> table;
    size_t p = txt.find("\"classes\"");
    if (p == std::string::npos) return (ls_status)report_error(LS_EINVAL, "tuning table has no classes");
    while ((p = txt.find('{', p + 1)) != std::string::npos) {
        const size_t e = txt.find('}', p);
        if (e == std::string::npos) break;
        double cls, b, c, t, ms = 0, dms = 0, tile = 32768;
        if (!json_number(txt, p, e, "log10_avg_size", cls) || !json_number(txt, p, e, "buckets", b) ||
            !json_number(txt, p, e, "cutoff", c) || !json_number(txt, p, e, "tree_buckets", t))
            return (ls_status)report_error(LS_EINVAL, "tuning table entry lacks a field");
        json_number(txt, p, e, "ms", ms);
        json_number(txt, p, e, "default_ms", dms);
        json_number(txt, p, e, "tile", tile);  // optional: default work unit
        const uint32_t tb = (uint32_t)t;
        bool tile_ok = false;
        for (uint32_t s = 0; s <= USHIFT_MAX; s++) tile_ok |= tile == (double)((uint32_t)UNIT << s);
        if (b < 2 || b > B_MAX || c < 1 || c > C_MAX || tb < 2 || tb > 512 || (tb & (tb - 1)) || !tile_ok)
            return (ls_status)report_error(LS_EINVAL, "tuning table entry out of range");
        table.push_back(TuneEntry{(int)cls, (uint32_t)b, (uint32_t)c, tb, ms, dms, (uint32_t)tile});
        p = e;
    }
    if (table.empty()) return (ls_status)report_error(LS_EINVAL, "tuning table has no classes");
    tuning_install(table);
    return LS_OK;
}

}  // extern "C"
