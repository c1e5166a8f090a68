// Scoring kernels: float64 direct convolution (the reference of Section 6 of
// arXiv:2201.10369, eq. conv as a zero-padded cross-correlation) and the L1
// error sums against it, with a fixed reduction tree.
#include <hip/hip_runtime.h>

#include "wg_internal.h"

namespace wg {

// ---------------------------------------------------------------------------
// float64 direct convolution.  A block computes a 32 x 32 output patch of 16
// output channels of one image; each thread owns 2 x 2 pixels x 16 channels.
// Per input channel the (32+r-1)^2 input patch and the 16 x r x r filter taps
// are staged in LDS as float64.
// ---------------------------------------------------------------------------
constexpr int kDTile = 32;
constexpr int kDK = 16;

template <int R>
__global__ __launch_bounds__(256) void direct_f64_kernel(const float* __restrict__ x,
                                                         const float* __restrict__ w,
                                                         double* __restrict__ y, int C, int K, int H,
                                                         int W, int pad, int Hout, int Wout,
                                                         int tiles_x) {
    constexpr int XP = kDTile + R - 1;
    __shared__ double xs[XP * XP];
    __shared__ double ws[kDK * R * R];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int ty0 = (blockIdx.x / tiles_x) * kDTile, tx0 = (blockIdx.x % tiles_x) * kDTile;
    const int k0 = blockIdx.y * kDK;
    const int n = blockIdx.z;

    double acc[kDK][2][2];
#pragma unroll
    for (int k = 0; k < kDK; ++k)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[k][a][b] = 0.0;

    for (int c = 0; c < C; ++c) {
        const float* xc = x + ((size_t)n * C + c) * H * W;
        for (int q = tid; q < XP * XP; q += 256) {
            const int i = q / XP, j = q - i * XP;
            const int gi = ty0 + i - pad, gj = tx0 + j - pad;
            xs[q] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? (double)xc[(size_t)gi * W + gj] : 0.0;
        }
        for (int q = tid; q < kDK * R * R; q += 256) {
            const int k = q / (R * R), uv = q - k * (R * R);
            ws[q] = (k0 + k < K) ? (double)w[((size_t)(k0 + k) * C + c) * R * R + uv] : 0.0;
        }
        __syncthreads();
        double xv[R + 1][R + 1];
#pragma unroll
        for (int i = 0; i < R + 1; ++i)
#pragma unroll
            for (int j = 0; j < R + 1; ++j) xv[i][j] = xs[(2 * ty + i) * XP + 2 * tx + j];
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
            for (int v = 0; v < R; ++v)
#pragma unroll
                for (int k = 0; k < kDK; ++k) {
                    const double wv = ws[k * R * R + u * R + v];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b) acc[k][a][b] = fma(xv[u + a][v + b], wv, acc[k][a][b]);
                }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kDK; ++k) {
        if (k0 + k >= K) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int oy = ty0 + 2 * ty + a;
            if (oy >= Hout) continue;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int ox = tx0 + 2 * tx + b;
                if (ox < Wout) y[(((size_t)n * K + k0 + k) * Hout + oy) * Wout + ox] = acc[k][a][b];
            }
        }
    }
}

int launch_direct_f64(const float* x, const float* w, double* y, int N, int C, int K, int H, int W,
                      int r, int pad, int Hout, int Wout, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int tiles_y = (Hout + kDTile - 1) / kDTile, tiles_x = (Wout + kDTile - 1) / kDTile;
    const dim3 grid((unsigned)(tiles_y * tiles_x), (unsigned)((K + kDK - 1) / kDK), (unsigned)N);
    switch (r) {
#define WG_DIRECT_CASE(RR)                                                                            \
    case RR:                                                                                          \
        hipLaunchKernelGGL((direct_f64_kernel<RR>), grid, dim3(256), 0, s, x, w, y, C, K, H, W, pad, \
                           Hout, Wout, tiles_x);                                                       \
        break;
        WG_DIRECT_CASE(1) WG_DIRECT_CASE(2) WG_DIRECT_CASE(3) WG_DIRECT_CASE(4) WG_DIRECT_CASE(5)
        WG_DIRECT_CASE(6) WG_DIRECT_CASE(7)
#undef WG_DIRECT_CASE
        default: return fail(WG_EINVAL, "direct conv: r out of range");
    }
    return hip_check((int)hipGetLastError(), "direct_f64_kernel");
}

// ---------------------------------------------------------------------------
// L1 error sums: partial sums per block (grid-stride), then one block adds
// the partials in index order; both trees are fixed, so the result depends
// only on the inputs and the count.
// ---------------------------------------------------------------------------
size_t score_partials(size_t count) {
    size_t nb = (count + 4095) / 4096;
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return nb;
}

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sa, double* sb) {
    const int tid = threadIdx.x;
    sa[tid] = a;
    sb[tid] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sa[tid] += sa[tid + s];
            sb[tid] += sb[tid + s];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
}

__global__ __launch_bounds__(256) void score_partial_kernel(const float* __restrict__ y,
                                                            const double* __restrict__ yref, size_t count,
                                                            double* __restrict__ part) {
    __shared__ double sa[256], sb[256];
    double e = 0.0, r = 0.0;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
        const double ref = yref[i];
        e += fabs((double)y[i] - ref);
        r += fabs(ref);
    }
    block_sum2(e, r, sa, sb);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = e;
        part[2 * blockIdx.x + 1] = r;
    }
}

__global__ __launch_bounds__(256) void score_final_kernel(const double* __restrict__ part, int nb,
                                                          double* __restrict__ out2) {
    __shared__ double sa[256], sb[256];
    double e = 0.0, r = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        e += part[2 * i];
        r += part[2 * i + 1];
    }
    block_sum2(e, r, sa, sb);
    if (threadIdx.x == 0) {
        out2[0] = e;
        out2[1] = r;
    }
}

int launch_score(const float* y, const double* yref, size_t count, double* out2, void* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = (int)score_partials(count);
    double* part = static_cast<double*>(ws);
    hipLaunchKernelGGL(score_partial_kernel, dim3(nb), dim3(256), 0, s, y, yref, count, part);
    int st = hip_check((int)hipGetLastError(), "score_partial_kernel");
    if (st != WG_OK) return st;
    hipLaunchKernelGGL(score_final_kernel, dim3(1), dim3(256), 0, s, part, nb, out2);
    return hip_check((int)hipGetLastError(), "score_final_kernel");
}

}  // namespace wg
