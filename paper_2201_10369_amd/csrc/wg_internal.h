// Internal declarations shared by the host code and the kernel launchers of
// the Winograd library.  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/wg.h"

namespace wg {

constexpr int kMaxAlpha = 16;

// Per-thread error state behind wg_last_error().
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

struct Plan {
    wg_layout L;
    // float32 matrices, row-major with their true sizes
    float AT[kMaxAlpha * kMaxAlpha];   // m x alpha
    float G[kMaxAlpha * kMaxAlpha];    // alpha x r
    float BT[kMaxAlpha * kMaxAlpha];   // alpha x alpha
    // the same rounded to float64 (the float64 transforms of WG_F64_TRANSFORMS)
    double AT64[kMaxAlpha * kMaxAlpha];
    double G64[kMaxAlpha * kMaxAlpha];
    double BT64[kMaxAlpha * kMaxAlpha];
    bool f64t;                         // float64 transforms, float32 Hadamard stage
    // binary exponents of the float64 row L1 norms of B^T and G
    int eB[kMaxAlpha];
    int eG[kMaxAlpha];
    int dB[kMaxAlpha];                 // eB - eG
    // GEMM tiling chosen at plan creation
    int gemm_bm, gemm_bn, gemm_bk;
    int gemm_tpb;                 // GEMM tiles per block (consecutive, pipelined)
};

// Exact construction (exact_construct.cpp): entries rounded to nearest float64.
bool construct_exact(int m, int r, const double* pts, int nf, bool modified, double* AT, double* G,
                     double* BT);

// HIP status -> WG_EHIP with message; returns WG_OK when hip_ok is true.
int hip_check(int hip_err, const char* what);

// Launchers implemented in the .hip translation units.  They assume the
// arguments were validated by the ABI layer.
int launch_filter_transform(const Plan& p, const float* w, const float* x_absmax, void* U,
                            void* stream);
int launch_input_transform(const Plan& p, const float* x, const void* U, void* ws,
                           void* stream);
int launch_filter_maxima(const Plan& p, const float* w, void* U, void* stream);
// per-batch 16-bit scaling: t[c] and the scale table from max |x_c| and
// max |w_c| in one launch (16-bit plans; else nothing)
int launch_layer_maxima(const Plan& p, const float* w, const float* x, void* U, void* stream);
// t_from_table: the transforms read t[c] from U's table (written by
// launch_layer_maxima), else derive it from x_absmax (or 1 when null) and the
// partial maxima of |w|
int launch_filter_input(const Plan& p, const float* w, const float* x_absmax, const float* x, void* U, void* ws,
                        void* stream, bool t_from_table = false);
int launch_hadamard_gemm(const Plan& p, const void* U, void* ws, void* stream);
// Times each candidate tiles-per-block value on the caller's operands and
// keeps the fastest in the plan (synchronous on `stream`).
int autotune_hadamard_gemm(Plan& p, const void* U, void* ws, int reps, int* chosen, void* stream);
int launch_output_transform(const Plan& p, const void* ws, float* y, void* stream);
int launch_channel_absmax(const float* x, int N, int C, int HW, float* out, void* stream);
int launch_direct_f64(const float* x, const float* w, double* y, int N, int C, int K, int H,
                      int W, int r, int pad, int Hout, int Wout, void* stream);
int launch_score(const float* y, const double* yref, size_t count, double* out2, void* ws,
                 void* stream);
size_t score_partials(size_t count);
// the same with the partial sums in the library's static device scratch
int launch_score_noalloc(const float* y, const double* yref, size_t count, double* out2, void* stream);

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Library scratch in the U buffer of a 16-bit plan (after the table t[c]):
// partial maxima of |w| per chunk of kKChunkW filters, [wchunks][C_pad].
constexpr int kKChunkW = 8;
inline int w_chunks(const wg_layout& L) { return (L.K + kKChunkW - 1) / kKChunkW; }
inline size_t wpart_offset(const wg_layout& L) { return L.chan_offset + round_up((size_t)L.C_pad * 4, 256); }

}  // namespace wg
