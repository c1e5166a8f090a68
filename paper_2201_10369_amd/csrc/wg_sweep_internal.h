// Internal state of a sweep object (see wg_sweep_* in wg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wg {

struct SweepTune {
    int block;          // threads per block of the evaluation kernel
    int chunk;          // pool samples per work item
    int blocks_per_cu;  // persistent blocks per compute unit
};

// One scoring call: either family parameters (c1, c2) or explicit point
// lists (pts: n_cand x (alpha-1), c1 = c2 = null).
struct SweepArgs {
    const double* c1;
    const double* c2;
    const int* counts;
    int n_cand;
    double* out;
    const double* pts;
    bool operator==(const SweepArgs& o) const {
        return c1 == o.c1 && c2 == o.c2 && counts == o.counts && n_cand == o.n_cand && out == o.out &&
               pts == o.pts;
    }
};

struct Sweep {
    int m = 0, r = 0, dims = 0, alpha = 0, n_pool = 0, max_cand = 0, n_cu = 0;
    const float* d_pool = nullptr;
    const float* g_pool = nullptr;
    float* d_soa = nullptr;      // pool tiles, element-major: [alpha(^2)][n_pool]
    float* g_soa = nullptr;      // pool filters, element-major: [r(^2)][n_pool]
    double* yref = nullptr;      // float64 reference outputs, element-major: [outs][n_pool]
    double* ref_abs = nullptr;   // sum |yref| per sample
    double* prefix = nullptr;    // prefix sums of ref_abs (n_pool + 1)
    float* mats = nullptr;       // per candidate float32 A^T | G | B^T
    double* mats64 = nullptr;    // the same in float64 (mixed precision only)
    int mixed = 0;               // 1: float64 transforms, float32 Hadamard product
    int* flags = nullptr;        // per candidate: 1 = invalid or singular, 4 = built exactly
    int exact_all = 0;           // 1: every candidate built by the exact integer kernel
    uint8_t* row_status = nullptr;   // per candidate and row: 0 built, 1 flags, 2 pending
    double* partial = nullptr;   // per work item error sums
    SweepTune tune{128, 2048, 4};
    bool tuned = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SweepArgs captured{};
};

}  // namespace wg
