// Filter transform U = G g G^T of the Winograd layer on gfx950
// (arXiv:2201.10369, Section 4, eq. conv_2d), with the per-channel exponent
// part of the 16-bit scaling, and the per-channel max |x| helper.
//
// Each two-sided product P X P^T is evaluated as (P X) first and then
// (P X) P^T, every inner product accumulated in ascending index order with one
// fused multiply-add per term (acc <- fma(p, x, acc) from acc = 0).  The
// float32 error of this evaluation is what gets scored against the float64
// direct convolution (arXiv:2201.10369, Section 6).
//
// Layout: U'[e][k][c], e = tile element, c contiguous.
#include <hip/hip_runtime.h>

#include "wg_layer_common.h"

#pragma clang fp contract(off)

namespace wg {

// ---------------------------------------------------------------------------
// 16-bit Hadamard stage: partial maxima of |w| over chunks of kKChunk
// filters for 64 channels per block (coalesced: a wave reads 64 consecutive
// channels' r*r taps).  part[kc][c] for filter chunk kc.
// ---------------------------------------------------------------------------
constexpr int kKChunk = 8;

template <int RR>
__global__ __launch_bounds__(256) void filter_absmax_kernel(const float* __restrict__ w,
                                                            float* __restrict__ part, int K, int C,
                                                            int C_pad) {
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, kq = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    const int kc = blockIdx.y;
    float mx = 0.0f;
    if (c < C) {
        float v[kKChunk / 4][RR];
#pragma unroll
        for (int i = 0; i < kKChunk / 4; ++i) {
            const int k = kc * kKChunk + kq + 4 * i;
#pragma unroll
            for (int t = 0; t < RR; ++t) v[i][t] = k < K ? w[((size_t)k * C + c) * RR + t] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < kKChunk / 4; ++i)
#pragma unroll
            for (int t = 0; t < RR; ++t) mx = fmaxf(mx, fabsf(v[i][t]));
    }
    red[kq][cl] = mx;
    __syncthreads();
    if (kq == 0 && c < C_pad)
        part[(size_t)kc * C_pad + c] = fmaxf(fmaxf(red[0][cl], red[1][cl]), fmaxf(red[2][cl], red[3][cl]));
}

// ---------------------------------------------------------------------------
// Filter transform U = G g G^T.  A block covers 128 channels (64 lanes, two
// adjacent channels each) of one filter k; wave wv takes the rows i of U
// with i mod 4 = wv.  Each thread transforms its two filter channels
// g = w[k][c], w[k][c+1] into those rows and stores each entry pair with one
// store, so every store of U'[e][k][.] is a contiguous run of 128 channels.
//
// For the 16-bit stage the block first finishes the per-channel exponent
// part t[c] = E(x_absmax[c]) - E(max_k |w[k][c]|) from the partial maxima of
// all filter chunks (every block of a channel group repeats this small
// reduction, so no second launch is needed), scales entry (i, j) by 2^s with
// s = floor((dB[i] + dB[j] + t[c]) / 2) before rounding, and the blocks of
// filter 0 also write t and the table s[e][c].
// ---------------------------------------------------------------------------
template <int M, int R, int DT>
__global__ __launch_bounds__(256) void filter_transform_kernel(const float* __restrict__ w,
                                                               void* __restrict__ Uout,
                                                               const float* __restrict__ part,
                                                               const float* __restrict__ x_absmax,
                                                               int32_t* __restrict__ s_tab,
                                                               int32_t* __restrict__ t_tab, int kchunks,
                                                               Mats<M, R> mt, RowExps ex, Geo g) {
    constexpr int A = M + R - 1;
    using T = typename Elem<DT>::T;
    __shared__ int stc[2][64];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = blockIdx.x * 128 + 2 * lane;            // channels c, c + 1
    const int k = blockIdx.y;
    // the filter taps first, so their loads overlap the exponent reduction
    float g0[R][R], g1[R][R];
    const bool live0 = k < g.K && c < g.C, live1 = k < g.K && c + 1 < g.C;
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v) {
            g0[u][v] = live0 ? w[(((size_t)k * g.C + c) * R + u) * R + v] : 0.0f;
            g1[u][v] = live1 ? w[(((size_t)k * g.C + c + 1) * R + u) * R + v] : 0.0f;
        }
    int tc0 = 0, tc1 = 0;
    if (DT != kF32) {
        // t[c] from the partial maxima of every filter chunk: the two halves
        // of the block (one thread per channel of the block's 128) take the
        // even and the odd chunks
        __shared__ float sred[2][128];
        const int cl = (threadIdx.x & 127), half = threadIdx.x >> 7;
        const int cc = blockIdx.x * 128 + cl;
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
        if (blockIdx.y == 0 && cc < g.C_pad) {
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
    T* U = reinterpret_cast<T*>(Uout);
    const size_t plane = in_vgpr((size_t)g.K_pad * g.C_pad);
    T* const U0 = U + ((size_t)k * g.C_pad + c);
#pragma unroll
    for (int i = 0; i < A; ++i) {
        if ((i & 3) != wv) continue;                  // uniform over the wave
        T* Up = U0 + (size_t)(i * A) * plane;          // plane e = i*A + j, one plane per entry
        // row i of P1 = G g for both channels
        float p0[R], p1[R];
#pragma unroll
        for (int v = 0; v < R; ++v) p0[v] = p1[v] = 0.0f;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const float b = mt.G[i][u];
#pragma unroll
            for (int v = 0; v < R; ++v) {
                p0[v] = __builtin_fmaf(b, g0[u][v], p0[v]);
                p1[v] = __builtin_fmaf(b, g1[u][v], p1[v]);
            }
        }
        const int si0 = tc0 + ex.dB[i], si1 = tc1 + ex.dB[i];
#pragma unroll
        for (int j = 0; j < A; ++j) {
            float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
            for (int v = 0; v < R; ++v) {
                a0 = __builtin_fmaf(mt.G[j][v], p0[v], a0);
                a1 = __builtin_fmaf(mt.G[j][v], p1[v], a1);
            }
            if (DT != kF32) {                       // padded channels hold zeros
                a0 = ldexpf(a0, floor_half(si0 + ex.dB[j]));
                a1 = ldexpf(a1, floor_half(si1 + ex.dB[j]));
            }
            Elem<DT>::store2(Up, a0, a1);
            Up += plane;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-channel max |x|
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void channel_absmax_kernel(const float* __restrict__ x, int N, int C,
                                                             int HW, float* __restrict__ out) {
    __shared__ float red[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    float mx = 0.0f;
    for (int n = 0; n < N; ++n) {
        const float* src = x + ((size_t)n * C + c) * HW;
        for (int q = tid; q < HW; q += 256) mx = fmaxf(mx, fabsf(src[q]));
    }
    red[tid] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) out[c] = red[0];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int M, int R>
static int filter_impl(const Plan& p, const float* w, const float* x_absmax, void* U, hipStream_t s) {
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    RowExps ex{};
    for (int i = 0; i < L.alpha; ++i) ex.dB[i] = p.dB[i];
    char* Ub = static_cast<char*>(U);
    int32_t* s_tab = reinterpret_cast<int32_t*>(Ub + L.scale_offset);
    int32_t* t_tab = reinterpret_cast<int32_t*>(Ub + L.chan_offset);
    float* part = reinterpret_cast<float*>(Ub + L.chan_offset + round_up((size_t)L.C_pad * 4, 256));
    const int kchunks = (L.K + kKChunk - 1) / kKChunk;
    if (L.dtype != WG_F32) {
        hipLaunchKernelGGL((filter_absmax_kernel<R * R>), dim3((unsigned)((L.C_pad + 63) / 64), (unsigned)kchunks),
                           dim3(256), 0, s, w, part, L.K, L.C, L.C_pad);
        const int st = last_launch("filter_absmax_kernel");
        if (st != WG_OK) return st;
    }
    const dim3 grid((unsigned)((L.C_pad + 127) / 128), (unsigned)L.K_pad);
    switch (L.dtype) {
        case WG_F32:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF32>), grid, dim3(256), 0, s, w, U, part, x_absmax,
                               s_tab, t_tab, kchunks, mt, ex, g);
            break;
        case WG_F16:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF16>), grid, dim3(256), 0, s, w, U, part, x_absmax,
                               s_tab, t_tab, kchunks, mt, ex, g);
            break;
        default:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kBF16>), grid, dim3(256), 0, s, w, U, part, x_absmax,
                               s_tab, t_tab, kchunks, mt, ex, g);
            break;
    }
    return last_launch("filter_transform_kernel");
}

int launch_filter_transform(const Plan& p, const float* w, const float* x_absmax, void* U, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_filter(MM, RR) case MM * 16 + RR: return filter_impl<MM, RR>(p, w, x_absmax, U, s);
    WG_DISPATCH(filter)
#undef WG_CASE_filter
}

int launch_channel_absmax(const float* x, int N, int C, int HW, float* out, void* stream) {
    hipLaunchKernelGGL(channel_absmax_kernel, dim3(C), dim3(256), 0, static_cast<hipStream_t>(stream),
                       x, N, C, HW, out);
    return last_launch("channel_absmax_kernel");
}

int hip_check(int hip_err, const char* what) {
    if (hip_err == (int)hipSuccess) return WG_OK;
    return fail(WG_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)hip_err));
}

}  // namespace wg
