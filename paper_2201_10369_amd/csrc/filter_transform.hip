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

#include "wg_filter_block.h"

#pragma clang fp contract(off)

namespace wg {

// ---------------------------------------------------------------------------
// 16-bit Hadamard stage: partial maxima of |w| over chunks of kKChunkW
// filters for 64 channels per block (coalesced: a wave reads 64 consecutive
// channels' r*r taps).  part[kc][c] for filter chunk kc.
// ---------------------------------------------------------------------------
template <int RR>
__device__ __forceinline__ void w_absmax_block(const float* __restrict__ w, float* __restrict__ part, int K, int C,
                                               int C_pad, int bx, int kc) {
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, kq = threadIdx.x >> 6;
    const int c = bx * 64 + cl;
    float mx = 0.0f;
    if (c < C) {
        float v[kKChunkW / 4][RR];
#pragma unroll
        for (int i = 0; i < kKChunkW / 4; ++i) {
            const int k = kc * kKChunkW + kq + 4 * i;
#pragma unroll
            for (int t = 0; t < RR; ++t) v[i][t] = k < K ? w[((size_t)k * C + c) * RR + t] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < kKChunkW / 4; ++i)
#pragma unroll
            for (int t = 0; t < RR; ++t) mx = fmaxf(mx, fabsf(v[i][t]));
    }
    red[kq][cl] = mx;
    __syncthreads();
    if (kq == 0 && c < C_pad)
        part[(size_t)kc * C_pad + c] = fmaxf(fmaxf(red[0][cl], red[1][cl]), fmaxf(red[2][cl], red[3][cl]));
}

template <int RR>
__global__ __launch_bounds__(256) void filter_absmax_kernel(const float* __restrict__ w,
                                                            float* __restrict__ part, int K, int C,
                                                            int C_pad) {
    w_absmax_block<RR>(w, part, K, C, C_pad, (int)blockIdx.x, (int)blockIdx.y);
}

// Per-batch 16-bit scaling in one launch: block c takes channel c, reduces
// max |x[., c, ., .]| over every image and max |w[., c, ., .]| over every
// filter, and writes t[c] = E(max |x_c|) - E(max |w_c|) and the column
// s[e][c] = floor((dB[e1] + dB[e2] + t[c]) / 2) of the scale table (blocks
// of padding channels write t = 0 and its column).  vec: every plane of x is
// a whole number of 16-byte vectors at a 16-byte aligned address; then the
// block walks (image, vector) pairs as one flat index with sixteen vector
// loads in flight per thread (one round for a channel of up to 16K vectors,
// 64 images of 28 x 28 among them; a maximum does not depend on the order).
constexpr int kScaleThreads = 1024;
constexpr int kScaleLoads = 16;

__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    float m = red[0];
    for (int i = 1; i < kScaleThreads / 64; ++i) m = fmaxf(m, red[i]);
    return m;
}

template <int RR>
__global__ __launch_bounds__(kScaleThreads) void layer_scale_kernel(const float* __restrict__ x,
                                                                    const float* __restrict__ w, int N, int C,
                                                                    int K, int HW, int C_pad, int vec, int alpha,
                                                                    RowExps ex, int32_t* __restrict__ s_tab,
                                                                    int32_t* __restrict__ t_tab) {
    __shared__ float red[2][kScaleThreads / 64];
    // consecutive channels on one XCD: their filter taps share cache lines
    // (a channel's taps are 4 * RR bytes at a stride of C * 4 * RR), which
    // one L2 then fetches once
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int c = nb % kXcdCount == 0 ? (b % kXcdCount) * (nb / kXcdCount) + b / kXcdCount : b;
    const int tid = (int)threadIdx.x;
    int tc = 0;
    if (c < C) {
        // the filter taps first (their loads overlap the walk over x)
        float mw = 0.0f;
        for (int q = tid; q < K * RR; q += kScaleThreads) {
            const int k = q / RR, t = q - k * RR;
            mw = fmaxf(mw, fabsf(w[((size_t)k * C + c) * RR + t]));
        }
        float mx = 0.0f;
        if (vec) {
            const int hw4 = HW / 4;
            const long long total = (long long)N * hw4;
            for (long long i0 = tid; i0 < total; i0 += kScaleThreads * kScaleLoads) {
                float4 v[kScaleLoads];
#pragma unroll
                for (int u = 0; u < kScaleLoads; ++u) {
                    const long long i = i0 + kScaleThreads * u;
                    v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (i < total) {
                        const long long n = i / hw4;
                        v[u] = reinterpret_cast<const float4*>(x + ((size_t)n * C + c) * HW)[i - n * hw4];
                    }
                }
#pragma unroll
                for (int u = 0; u < kScaleLoads; ++u)
                    mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)), fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
            }
        } else {
            for (int n = 0; n < N; ++n) {
                const float* src = x + ((size_t)n * C + c) * HW;
                for (int i = tid; i < HW; i += kScaleThreads) mx = fmaxf(mx, fabsf(src[i]));
            }
        }
        mx = block_max(mx, red[0]);
        mw = block_max(mw, red[1]);
        tc = bin_exp(mx) - bin_exp(mw);
    }
    if (tid == 0) t_tab[c] = tc;
    for (int e = tid; e < alpha * alpha; e += kScaleThreads)
        s_tab[(size_t)e * C_pad + c] = floor_half(ex.dB[e / alpha] + ex.dB[e % alpha] + tc);
}

// ---------------------------------------------------------------------------
// Filter transform kernel: grid (channel groups of 128, K_pad filters).
// ---------------------------------------------------------------------------
template <int M, int R, int DT, typename CT>
__global__ __launch_bounds__(256) void filter_transform_kernel(FilterArgs fa, Mats<M, R, CT> mt, RowExps ex,
                                                               Geo g) {
    __shared__ int sm[kFilterLdsWords];
    filter_block<M, R, DT, CT>(fa, mt, ex, g, (int)blockIdx.x, (int)blockIdx.y, sm);
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
FilterArgs filter_args(const Plan& p, const float* w, const float* x_absmax, void* U) {
    const wg_layout& L = p.L;
    char* Ub = static_cast<char*>(U);
    int32_t* s_tab = reinterpret_cast<int32_t*>(Ub + L.scale_offset);
    int32_t* t_tab = reinterpret_cast<int32_t*>(Ub + L.chan_offset);
    float* part = reinterpret_cast<float*>(Ub + wpart_offset(L));
    return FilterArgs{w, U, part, x_absmax, s_tab, t_tab, nullptr, w_chunks(L)};
}

FilterArgs filter_args_table(const Plan& p, const float* w, void* U) {
    FilterArgs fa = filter_args(p, w, nullptr, U);
    fa.t_in = fa.t_tab;
    return fa;
}

int launch_filter_absmax(const Plan& p, const FilterArgs& fa, hipStream_t s) {
    const wg_layout& L = p.L;
    if (L.dtype == WG_F32) return WG_OK;
    const dim3 grid((unsigned)((L.C_pad + 63) / 64), (unsigned)fa.kchunks);
    float* part = const_cast<float*>(fa.part);
    switch (L.r) {
        case 3: hipLaunchKernelGGL((filter_absmax_kernel<9>), grid, dim3(256), 0, s, fa.w, part, L.K, L.C, L.C_pad); break;
        case 5: hipLaunchKernelGGL((filter_absmax_kernel<25>), grid, dim3(256), 0, s, fa.w, part, L.K, L.C, L.C_pad); break;
        default: return fail(WG_EUNSUPPORTED, "filter transform: r not compiled");
    }
    return last_launch("filter_absmax_kernel");
}

template <int M, int R>
static int filter_impl(const Plan& p, const float* w, const float* x_absmax, void* U, hipStream_t s) {
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    const Mats<M, R, double> mt64 = pack_mats<M, R, double>(p);
    RowExps ex{};
    for (int i = 0; i < L.alpha; ++i) ex.dB[i] = p.dB[i];
    const FilterArgs fa = filter_args(p, w, x_absmax, U);
    const int st = launch_filter_absmax(p, fa, s);
    if (st != WG_OK) return st;
    const dim3 grid((unsigned)filter_groups(L), (unsigned)L.K_pad);
    if (p.f64t) {
        hipLaunchKernelGGL((filter_transform_kernel<M, R, kF32, double>), grid, dim3(256), 0, s, fa, mt64, ex, g);
        return last_launch("filter_transform_kernel");
    }
    switch (L.dtype) {
        case WG_F32:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF32, float>), grid, dim3(256), 0, s, fa, mt, ex, g);
            break;
        case WG_F16:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF16, float>), grid, dim3(256), 0, s, fa, mt, ex, g);
            break;
        default:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kBF16, float>), grid, dim3(256), 0, s, fa, mt, ex, g);
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

int launch_filter_maxima(const Plan& p, const float* w, void* U, void* stream) {
    return launch_filter_absmax(p, filter_args(p, w, nullptr, U), static_cast<hipStream_t>(stream));
}

int launch_layer_maxima(const Plan& p, const float* w, const float* x, void* U, void* stream) {
    const wg_layout& L = p.L;
    if (L.dtype == WG_F32) return WG_OK;
    const FilterArgs fa = filter_args(p, w, nullptr, U);
    RowExps ex{};
    for (int i = 0; i < L.alpha; ++i) ex.dB[i] = p.dB[i];
    const int HW = L.H * L.W;
    const int vec = (HW % 4 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0) ? 1 : 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)L.C_pad);
    switch (L.r) {
        case 3:
            hipLaunchKernelGGL((layer_scale_kernel<9>), grid, dim3(kScaleThreads), 0, s, x, w, L.N, L.C, L.K, HW,
                               L.C_pad, vec, L.alpha, ex, fa.s_tab, fa.t_tab);
            break;
        case 5:
            hipLaunchKernelGGL((layer_scale_kernel<25>), grid, dim3(kScaleThreads), 0, s, x, w, L.N, L.C, L.K, HW,
                               L.C_pad, vec, L.alpha, ex, fa.s_tab, fa.t_tab);
            break;
        default: return fail(WG_EUNSUPPORTED, "layer maxima: r not compiled");
    }
    return last_launch("layer_scale_kernel");
}

// The same maximum when every plane is a whole number of 16-byte vectors:
// the block walks (image, vector) pairs as one flat index and keeps eight
// vector loads in flight per thread (a maximum does not depend on order).
__global__ __launch_bounds__(256) void channel_absmax4_kernel(const float* __restrict__ x, int N, int C,
                                                              int HW, float* __restrict__ out) {
    __shared__ float red[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int hw4 = HW / 4;
    const long long total = (long long)N * hw4;
    float mx = 0.0f;
    for (long long i0 = tid; i0 < total; i0 += 256 * 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long long i = i0 + 256 * u;
            v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (i < total) {
                const long long n = i / hw4;
                const float4* plane = reinterpret_cast<const float4*>(x + ((size_t)n * C + c) * HW);
                v[u] = plane[i - n * hw4];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)), fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
    }
    red[tid] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) out[c] = red[0];
}

int launch_channel_absmax(const float* x, int N, int C, int HW, float* out, void* stream) {
    if (HW % 4 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0) {
        hipLaunchKernelGGL(channel_absmax4_kernel, dim3(C), dim3(256), 0, static_cast<hipStream_t>(stream),
                           x, N, C, HW, out);
        return last_launch("channel_absmax4_kernel");
    }
    hipLaunchKernelGGL(channel_absmax_kernel, dim3(C), dim3(256), 0, static_cast<hipStream_t>(stream),
                       x, N, C, HW, out);
    return last_launch("channel_absmax_kernel");
}

int hip_check(int hip_err, const char* what) {
    if (hip_err == (int)hipSuccess) return WG_OK;
    return fail(WG_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)hip_err));
}

}  // namespace wg
