// Filter, input and output transforms of the Winograd layer on gfx950.
//
// The 2D algorithm is Y = A^T [ (G g G^T) (.) (B^T d B) ] A (arXiv:2201.10369,
// Section 4, eq. conv_2d), applied to every m x m output tile of the layer.
// Each two-sided product P X P^T is evaluated as (P X) first and then
// (P X) P^T, every inner product in ascending index order with the product
// and the sum rounded separately (no fused multiply-add).  Terms whose matrix
// entry is exactly zero are skipped, which changes no finite result.  This is
// the evaluation order whose float32 error the paper scores (Section 6).
//
// Memory layout (see wg.h, wg_layout):
//   U'[e][k][c]  transformed filters, e = tile element, c contiguous
//   V'[e][p][c]  transformed input tiles, c contiguous (the GEMM contraction)
//   M [e][k][p]  Hadamard/channel sums, p (tile index) contiguous
#include <hip/hip_runtime.h>

#include <cmath>

#include "wg_device.h"
#include "wg_internal.h"

#pragma clang fp contract(off)

namespace wg {

struct Geo {
    int N, C, K, H, W, pad, Hout, Wout, Th, Tw, P, P_pad, K_pad, C_pad;
};

static Geo make_geo(const wg_layout& L) {
    return Geo{L.N, L.C, L.K, L.H, L.W, L.pad, L.Hout, L.Wout, L.Th, L.Tw, L.P, L.P_pad, L.K_pad, L.C_pad};
}

struct RowExps {
    int eB[kMaxAlpha];
    int eG[kMaxAlpha];
};

// ---------------------------------------------------------------------------
// Power-of-two scale exponents of the 16-bit Hadamard stage, one block per
// input channel c:  s[e][c] = floor((E_V - E_U) / 2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bin_exp(float v) {
    int e = 0;
    if (v != 0.0f) frexpf(v, &e);
    return e;
}

__global__ __launch_bounds__(256) void filter_scales_kernel(const float* __restrict__ w,
                                                            const float* __restrict__ x_absmax,
                                                            int32_t* __restrict__ scales, RowExps ex,
                                                            int alpha, int K, int C, int C_pad, int rr) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    float mx = 0.0f;
    if (c < C) {
        const int per = K * rr;
        for (int q = tid; q < per; q += 256) {
            const int k = q / rr, uv = q - k * rr;
            mx = fmaxf(mx, fabsf(w[((size_t)k * C + c) * rr + uv]));
        }
    }
    red[tid] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    const float aw = red[0];
    const float ax = (x_absmax != nullptr && c < C) ? x_absmax[c] : 1.0f;
    const int E = alpha * alpha;
    for (int e = tid; e < E; e += 256) {
        const int e1 = e / alpha, e2 = e - e1 * alpha;
        int s = 0;
        if (c < C) {
            const int ev = ex.eB[e1] + ex.eB[e2] + bin_exp(ax);
            const int eu = ex.eG[e1] + ex.eG[e2] + bin_exp(aw);
            const int d = ev - eu;
            s = d >= 0 ? d / 2 : -((1 - d) / 2);      // floor(d / 2)
        }
        scales[(size_t)e * C_pad + c] = s;
    }
}

// ---------------------------------------------------------------------------
// Filter transform U = G g G^T, one thread per (k, c) of the padded K x C.
// ---------------------------------------------------------------------------
template <int M, int R, int DT>
__global__ __launch_bounds__(256) void filter_transform_kernel(const float* __restrict__ w,
                                                               void* __restrict__ Uout,
                                                               const int32_t* __restrict__ scales,
                                                               Mats<M, R> mt, Geo g) {
    constexpr int A = M + R - 1;
    using T = typename Elem<DT>::T;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const long total = (long)g.K_pad * g.C_pad;
    if (idx >= total) return;
    const int k = (int)(idx / g.C_pad);
    const int c = (int)(idx - (long)k * g.C_pad);
    float gg[R][R];
    const bool live = k < g.K && c < g.C;
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v)
            gg[u][v] = live ? w[(((size_t)k * g.C + c) * R + u) * R + v] : 0.0f;
    // P1 = G g  (A x R)
    float p1[A][R];
#pragma unroll
    for (int i = 0; i < A; ++i)
#pragma unroll
        for (int v = 0; v < R; ++v) p1[i][v] = 0.0f;
#pragma unroll
    for (int i = 0; i < A; ++i)
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const float b = mt.G[i][u];
            if (b != 0.0f) {
#pragma unroll
                for (int v = 0; v < R; ++v) p1[i][v] = p1[i][v] + b * gg[u][v];
            }
        }
    T* U = reinterpret_cast<T*>(Uout);
#pragma unroll
    for (int i = 0; i < A; ++i)
#pragma unroll
        for (int j = 0; j < A; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int v = 0; v < R; ++v) {
                const float b = mt.G[j][v];
                if (b != 0.0f) acc = acc + b * p1[i][v];
            }
            const int e = i * A + j;
            if (DT != kF32) acc = ldexpf(acc, scales[(size_t)e * g.C_pad + c]);
            U[((size_t)e * g.K_pad + k) * g.C_pad + c] = Elem<DT>::from_f32(acc);
        }
}

// ---------------------------------------------------------------------------
// Input transform V = B^T d B.  A block covers one image n, one tile row th,
// up to `twb` consecutive tiles of that row and 64 input channels: it stages
// the alpha input rows of those channels in LDS with coalesced reads (zeros
// outside the image), then each thread transforms one (channel, tile) pair;
// a wave holds one tile and 64 consecutive channels, so every V' store is a
// contiguous run of channels.
// ---------------------------------------------------------------------------
constexpr int kInCh = 64;

template <int M, int R, int DT>
__global__ __launch_bounds__(256) void input_transform_kernel(const float* __restrict__ x,
                                                              void* __restrict__ Vout,
                                                              const int32_t* __restrict__ scales,
                                                              Mats<M, R> mt, Geo g, int twb, int n_twb,
                                                              int row_w, int ch_stride) {
    constexpr int A = M + R - 1;
    using T = typename Elem<DT>::T;
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    int bx = blockIdx.x;
    const int tb = bx % n_twb;
    bx /= n_twb;
    const int th = bx % g.Th;
    const int n = bx / g.Th;
    const int c0 = blockIdx.y * kInCh;
    const int tw0 = tb * twb;
    const int ntw = min(twb, g.Tw - tw0);
    const int wl = ntw * M + R - 1;               // columns actually needed
    const int row0 = th * M - g.pad, col0 = tw0 * M - g.pad;

    // stage: rows (c, a), columns 0..wl-1; groups of wl lanes read one row
    {
        const int per = 256 / wl;                  // rows loaded per pass
        const int lane_row = tid / wl, col = tid - lane_row * wl;
        if (lane_row < per) {
            const int gj = col0 + col;
            const bool colok = gj >= 0 && gj < g.W;
            for (int cr = lane_row; cr < kInCh * A; cr += per) {
                const int c = cr / A, a = cr - c * A;
                const int gc = c0 + c, gi = row0 + a;
                float v = 0.0f;
                if (colok && gc < g.C && gi >= 0 && gi < g.H)
                    v = x[(((size_t)n * g.C + gc) * g.H + gi) * g.W + gj];
                lds[c * ch_stride + a * row_w + col] = v;
            }
        }
    }
    __syncthreads();

    T* V = reinterpret_cast<T*>(Vout);
    const int items = kInCh * ntw;
    for (int it = tid; it < items; it += 256) {
        const int c = it % kInCh, t = it / kInCh;
        const int gc = c0 + c;
        if (gc >= g.C_pad) continue;
        const float* src = lds + c * ch_stride + t * M;
        float d[A][A];
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
            for (int b = 0; b < A; ++b) d[a][b] = src[a * row_w + b];
        // T1 = B^T d
        float t1[A][A];
#pragma unroll
        for (int i = 0; i < A; ++i)
#pragma unroll
            for (int b = 0; b < A; ++b) t1[i][b] = 0.0f;
#pragma unroll
        for (int i = 0; i < A; ++i)
#pragma unroll
            for (int l = 0; l < A; ++l) {
                const float bv = mt.BT[i][l];
                if (bv != 0.0f) {
#pragma unroll
                    for (int b = 0; b < A; ++b) t1[i][b] = t1[i][b] + bv * d[l][b];
                }
            }
        const size_t p = ((size_t)n * g.Th + th) * g.Tw + tw0 + t;
        // V = T1 B, written element by element
#pragma unroll
        for (int i = 0; i < A; ++i)
#pragma unroll
            for (int j = 0; j < A; ++j) {
                float acc = 0.0f;
#pragma unroll
                for (int l = 0; l < A; ++l) {
                    const float bv = mt.BT[j][l];
                    if (bv != 0.0f) acc = acc + bv * t1[i][l];
                }
                const int e = i * A + j;
                if (DT != kF32) acc = ldexpf(acc, -scales[(size_t)e * g.C_pad + gc]);
                V[((size_t)e * g.P_pad + p) * g.C_pad + gc] = Elem<DT>::from_f32(acc);
            }
    }
}

// ---------------------------------------------------------------------------
// Output transform Y = A^T M A.  A block covers one output channel k and
// `nb` consecutive tile rows ("bands", band = n*Th + th).  Each thread
// transforms one tile into LDS; the block then writes every band, which is a
// contiguous run of up to m*Wout floats of y, with consecutive threads.
// ---------------------------------------------------------------------------
template <int M, int R>
__global__ __launch_bounds__(256) void output_transform_kernel(const float* __restrict__ Mbuf,
                                                               float* __restrict__ y, Mats<M, R> mt,
                                                               Geo g, int nb) {
    constexpr int A = M + R - 1;
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int k = blockIdx.y;
    const int band0 = blockIdx.x * nb;
    const int nbands = g.N * g.Th;
    const int nbl = min(nb, nbands - band0);
    const int row_w = g.Tw * M;
    const int items = nbl * g.Tw;
    const size_t E = (size_t)A * A;
    for (int it = tid; it < items; it += 256) {
        const int bl = it / g.Tw, tw = it - bl * g.Tw;
        const size_t p = (size_t)(band0 + bl) * g.Tw + tw;
        float mm[A][A];
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
            for (int b = 0; b < A; ++b)
                mm[a][b] = Mbuf[((size_t)(a * A + b) * g.K_pad + k) * g.P_pad + p];
        (void)E;
        // Z = A^T M  (M x A)
        float z[M][A];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int b = 0; b < A; ++b) z[i][b] = 0.0f;
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int l = 0; l < A; ++l) {
                const float av = mt.AT[i][l];
                if (av != 0.0f) {
#pragma unroll
                    for (int b = 0; b < A; ++b) z[i][b] = z[i][b] + av * mm[l][b];
                }
            }
        float* dst = lds + (bl * M) * row_w + tw * M;
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                float acc = 0.0f;
#pragma unroll
                for (int l = 0; l < A; ++l) {
                    const float av = mt.AT[j][l];
                    if (av != 0.0f) acc = acc + av * z[i][l];
                }
                dst[i * row_w + j] = acc;
            }
    }
    __syncthreads();
    // write the bands: band (n, th) is rows th*M .. th*M+M-1 of plane (n, k)
    const int per_band = M * g.Wout;
    const int total = nbl * per_band;
    for (int q = tid; q < total; q += 256) {
        const int bl = q / per_band;
        const int rem = q - bl * per_band;
        const int i = rem / g.Wout, j = rem - i * g.Wout;
        const int band = band0 + bl;
        const int n = band / g.Th, th = band - n * g.Th;
        const int oi = th * M + i;
        if (oi < g.Hout)
            y[(((size_t)n * g.K + k) * g.Hout + oi) * g.Wout + j] = lds[(bl * M + i) * row_w + j];
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
static Mats<M, R> pack_mats(const Plan& p) {
    constexpr int A = M + R - 1;
    Mats<M, R> mt;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < A; ++j) mt.AT[i][j] = p.AT[i * A + j];
    for (int i = 0; i < A; ++i)
        for (int j = 0; j < R; ++j) mt.G[i][j] = p.G[i * R + j];
    for (int i = 0; i < A; ++i)
        for (int j = 0; j < A; ++j) mt.BT[i][j] = p.BT[i * A + j];
    return mt;
}

static int last_launch(const char* what) {
    return hip_check((int)hipGetLastError(), what);
}

template <int M, int R>
static int filter_impl(const Plan& p, const float* w, const float* x_absmax, void* U, hipStream_t s) {
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    int32_t* scales = reinterpret_cast<int32_t*>(static_cast<char*>(U) + L.scale_offset);
    if (L.dtype != WG_F32) {
        RowExps ex{};
        for (int i = 0; i < L.alpha; ++i) {
            ex.eB[i] = p.eB[i];
            ex.eG[i] = p.eG[i];
        }
        hipLaunchKernelGGL(filter_scales_kernel, dim3(L.C_pad), dim3(256), 0, s, w, x_absmax, scales,
                           ex, L.alpha, L.K, L.C, L.C_pad, L.r * L.r);
        int st = last_launch("filter_scales_kernel");
        if (st != WG_OK) return st;
    }
    const long total = (long)L.K_pad * L.C_pad;
    const dim3 grid((unsigned)((total + 255) / 256));
    switch (L.dtype) {
        case WG_F32:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF32>), grid, dim3(256), 0, s, w, U, scales, mt, g);
            break;
        case WG_F16:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF16>), grid, dim3(256), 0, s, w, U, scales, mt, g);
            break;
        default:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kBF16>), grid, dim3(256), 0, s, w, U, scales, mt, g);
            break;
    }
    return last_launch("filter_transform_kernel");
}

template <int M, int R>
static int input_impl(const Plan& p, const float* x, const void* U, void* ws, hipStream_t s) {
    constexpr int A = M + R - 1;
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    // tiles per block: as many of the tile row as fit 64 KB of LDS
    const int max_w = (16384 / (kInCh * A)) - 1;            // floats per staged row
    int twb = (max_w - (R - 1)) / M;
    if (twb < 1) twb = 1;
    if (twb > L.Tw) twb = L.Tw;
    const int row_w = twb * M + R - 1;
    int ch_stride = A * row_w;
    if ((ch_stride & 1) == 0) ch_stride += 1;                // odd stride: no LDS bank conflicts
    const size_t lds_bytes = (size_t)kInCh * ch_stride * sizeof(float);
    const int n_twb = (L.Tw + twb - 1) / twb;
    const dim3 grid((unsigned)((long)L.N * L.Th * n_twb), (unsigned)((L.C_pad + kInCh - 1) / kInCh));
    const int32_t* scales =
        reinterpret_cast<const int32_t*>(static_cast<const char*>(U) + L.scale_offset);
    void* V = static_cast<char*>(ws) + L.v_offset;
    switch (L.dtype) {
        case WG_F32:
            hipLaunchKernelGGL((input_transform_kernel<M, R, kF32>), grid, dim3(256), lds_bytes, s, x, V, scales, mt, g, twb, n_twb, row_w, ch_stride);
            break;
        case WG_F16:
            hipLaunchKernelGGL((input_transform_kernel<M, R, kF16>), grid, dim3(256), lds_bytes, s, x, V, scales, mt, g, twb, n_twb, row_w, ch_stride);
            break;
        default:
            hipLaunchKernelGGL((input_transform_kernel<M, R, kBF16>), grid, dim3(256), lds_bytes, s, x, V, scales, mt, g, twb, n_twb, row_w, ch_stride);
            break;
    }
    return last_launch("input_transform_kernel");
}

template <int M, int R>
static int output_impl(const Plan& p, const void* ws, float* y, hipStream_t s) {
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    int nb = 256 / L.Tw;
    if (nb < 1) nb = 1;
    const size_t row_w = (size_t)L.Tw * M;
    while (nb > 1 && (size_t)nb * M * row_w * sizeof(float) > 65536) --nb;
    const size_t lds_bytes = (size_t)nb * M * row_w * sizeof(float);
    if (lds_bytes > 65536) return fail(WG_EUNSUPPORTED, "output transform: output rows too wide");
    const int nbands = L.N * L.Th;
    const dim3 grid((unsigned)((nbands + nb - 1) / nb), (unsigned)L.K);
    const float* Mbuf = reinterpret_cast<const float*>(static_cast<const char*>(ws) + L.m_offset);
    hipLaunchKernelGGL((output_transform_kernel<M, R>), grid, dim3(256), lds_bytes, s, Mbuf, y, mt, g, nb);
    return last_launch("output_transform_kernel");
}

#define WG_DISPATCH(FN, ...)                                              \
    switch (p.L.m * 16 + p.L.r) {                                         \
        WG_FOR_EACH_SIZE(WG_CASE_##FN)                                    \
        default: return fail(WG_EUNSUPPORTED, "tile size not compiled");   \
    }

int launch_filter_transform(const Plan& p, const float* w, const float* x_absmax, void* U, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_filter(MM, RR) case MM * 16 + RR: return filter_impl<MM, RR>(p, w, x_absmax, U, s);
    WG_DISPATCH(filter)
#undef WG_CASE_filter
}

int launch_input_transform(const Plan& p, const float* x, const void* U, void* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_input(MM, RR) case MM * 16 + RR: return input_impl<MM, RR>(p, x, U, ws, s);
    WG_DISPATCH(input)
#undef WG_CASE_input
}

int launch_output_transform(const Plan& p, const void* ws, float* y, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_output(MM, RR) case MM * 16 + RR: return output_impl<MM, RR>(p, ws, y, s);
    WG_DISPATCH(output)
#undef WG_CASE_output
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
