// Block body of the filter transform U = G g G^T (arXiv:2201.10369,
// Section 4, eq. conv_2d), shared by the filter-transform kernel and the
// combined filter-and-input launch.
//
// Each two-sided product P X P^T is evaluated as (P X) first and then
// (P X) P^T, every inner product accumulated in ascending index order with one
// fused multiply-add per term (acc <- fma(p, x, acc) from acc = 0).
//
// Layout: U'[e][k][c], e = tile element, c contiguous.
#pragma once

#include "wg_layer_common.h"

#pragma clang fp contract(off)

namespace wg {

// ---------------------------------------------------------------------------
// Filter transform U = G g G^T.  A block covers 128 channels (64 lanes, two
// adjacent channels each) of one filter k; wave wv takes the rows i of U
// with i mod 4 = wv.  Each thread transforms its two filter channels
// g = w[k][c], w[k][c+1] into those rows and stores each entry pair with one
// store, so every store of U'[e][k][.] is a contiguous run of 128 channels.
//
// For the 16-bit stage the block first finishes the per-channel exponent
// part t[c] = E(max |x_c|) - E(max_k |w[k][c]|) from the partial maxima of
// all filter chunks (every block of a channel group repeats this small
// reduction, so no second launch is needed), or reads the finished t[c]
// when the per-batch scaling launch has computed it, scales entry (i, j) by 2^s with
// s = floor((dB[i] + dB[j] + t[c]) / 2) before rounding, and the blocks of
// filter 0 also write t and the table s[e][c].
// ---------------------------------------------------------------------------
struct FilterArgs {
    const float* w;            // K x C x r x r
    void* U;                   // U'[e][k][c]
    const float* part;         // partial maxima of |w| per filter chunk (16-bit stage)
    const float* x_absmax;     // per-channel max |x| or null (bound 1)
    int32_t* s_tab;            // s[e][c] (written by the blocks of filter 0)
    int32_t* t_tab;            // t[c] (likewise)
    const int32_t* t_in;       // or: t[c] already final (then nothing is reduced
                               // or written to the tables)
    int kchunks;               // filter chunks of the partial maxima of |w|
};

// Host side (filter_transform.hip): the arguments for a plan and buffers,
// the channel groups of the grid, and the 16-bit partial-maxima launch
// (nothing to do for WG_F32).
FilterArgs filter_args(const Plan& p, const float* w, const float* x_absmax, void* U);
// the same with t[c] read from the table in U (written by the per-batch
// scaling launch)
FilterArgs filter_args_table(const Plan& p, const float* w, void* U);
inline int filter_groups(const wg_layout& L) { return (L.C_pad + 127) / 128; }
int launch_filter_absmax(const Plan& p, const FilterArgs& fa, hipStream_t s);

// LDS words the block body needs (its `sm` argument)
constexpr int kFilterLdsWords = 2 * 64 + 2 * 128;

// The block of channel group bx (128 channels) and filter k; sm: LDS
// scratch of kFilterLdsWords words.  CT: float, or double for the float64
// transforms (then DT is kF32 and each entry is rounded to float32).
template <int M, int R, int DT, typename CT = float>
__device__ __forceinline__ void filter_block(const FilterArgs& fa, const Mats<M, R, CT>& mt, const RowExps& ex,
                                             const Geo& g, int bx, int k, int* sm) {
    constexpr int A = M + R - 1;
    const float* __restrict__ w = fa.w;
    const float* __restrict__ part = fa.part;
    const float* __restrict__ x_absmax = fa.x_absmax;
    int32_t* __restrict__ s_tab = fa.s_tab;
    int32_t* __restrict__ t_tab = fa.t_tab;
    const int kchunks = fa.kchunks;
    using T = typename Elem<DT>::T;
    int (*stc)[64] = reinterpret_cast<int (*)[64]>(sm);                    // [2][64]
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = bx * 128 + 2 * lane;                    // channels c, c + 1
    // the filter taps first, so their loads overlap the exponent reduction
    CT g0[R][R], g1[R][R];
    const bool live0 = k < g.K && c < g.C, live1 = k < g.K && c + 1 < g.C;
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v) {
            g0[u][v] = (CT)(live0 ? w[(((size_t)k * g.C + c) * R + u) * R + v] : 0.0f);
            g1[u][v] = (CT)(live1 ? w[(((size_t)k * g.C + c + 1) * R + u) * R + v] : 0.0f);
        }
    int tc0 = 0, tc1 = 0;
    if (DT != kF32 && fa.t_in != nullptr) {
        tc0 = c < g.C ? fa.t_in[c] : 0;
        tc1 = c + 1 < g.C ? fa.t_in[c + 1] : 0;
    } else if (DT != kF32) {
        // t[c] from the partial maxima of every filter chunk: the two halves
        // of the block (one thread per channel of the block's 128) take the
        // even and the odd chunks
        float (*sred)[128] = reinterpret_cast<float (*)[128]>(sm + 2 * 64);  // [2][128]
        const int cl = (threadIdx.x & 127), half = threadIdx.x >> 7;
        const int cc = bx * 128 + cl;
        float aw = 0.0f;
        if (cc < g.C) {
#pragma unroll 8
            for (int q = half; q < kchunks; q += 2) aw = fmaxf(aw, part[(size_t)q * g.C_pad + cc]);
        }
        sred[half][cl] = aw;
        __syncthreads();
        // both halves derive t for channel cl; they split the table rows
        const float mw = fmaxf(sred[0][cl], sred[1][cl]);
        const int tc = cc < g.C ? bin_exp(x_absmax != nullptr ? x_absmax[cc] : 1.0f) - bin_exp(mw) : 0;
        if (half == 0) stc[cl & 1][cl >> 1] = tc;
        if (k == 0 && cc < g.C_pad) {
            if (half == 0) t_tab[cc] = tc;
#pragma unroll
            for (int e1 = 0; e1 < A; ++e1)
                if ((e1 & 1) == half) {
#pragma unroll
                    for (int e2 = 0; e2 < A; ++e2)
                        s_tab[(size_t)(e1 * A + e2) * g.C_pad + cc] = floor_half(ex.dB[e1] + ex.dB[e2] + tc);
                }
        }
        __syncthreads();
        tc0 = stc[0][lane];
        tc1 = stc[1][lane];
    }
    if (c >= g.C_pad) return;
    T* U = reinterpret_cast<T*>(fa.U);
    const size_t plane = in_vgpr((size_t)g.K_pad * g.C_pad);
    T* const U0 = U + ((size_t)k * g.C_pad + c);
#pragma unroll
    for (int i = 0; i < A; ++i) {
        if ((i & 3) != wv) continue;                  // uniform over the wave
        T* Up = U0 + (size_t)(i * A) * plane;          // plane e = i*A + j, one plane per entry
        // row i of P1 = G g for both channels
        CT p0[R], p1[R];
#pragma unroll
        for (int v = 0; v < R; ++v) p0[v] = p1[v] = CT(0);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const CT b = mt.G[i][u];
#pragma unroll
            for (int v = 0; v < R; ++v) {
                p0[v] = madd(b, g0[u][v], p0[v]);
                p1[v] = madd(b, g1[u][v], p1[v]);
            }
        }
        const int si0 = tc0 + ex.dB[i], si1 = tc1 + ex.dB[i];
#pragma unroll
        for (int j = 0; j < A; ++j) {
            CT q0 = CT(0), q1 = CT(0);
#pragma unroll
            for (int v = 0; v < R; ++v) {
                q0 = madd(mt.G[j][v], p0[v], q0);
                q1 = madd(mt.G[j][v], p1[v], q1);
            }
            float a0 = (float)q0, a1 = (float)q1;
            if (DT != kF32) {                       // padded channels hold zeros
                a0 = ldexpf(a0, floor_half(si0 + ex.dB[j]));
                a1 = ldexpf(a1, floor_half(si1 + ex.dB[j]));
            }
            Elem<DT>::store2(Up, a0, a1);
            Up += plane;
        }
    }
}

}  // namespace wg
