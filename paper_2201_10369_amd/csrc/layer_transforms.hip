// Filter, input and output transforms of the Winograd layer on gfx950.
//
// The 2D algorithm is Y = A^T [ (G g G^T) (.) (B^T d B) ] A (arXiv:2201.10369,
// Section 4, eq. conv_2d), applied to every m x m output tile of the layer.
// Each two-sided product P X P^T is evaluated as (P X) first and then
// (P X) P^T, every inner product accumulated in ascending index order with one
// fused multiply-add per term (acc <- fma(p, x, acc) from acc = 0).  Terms
// whose matrix entry is exactly zero are skipped, which changes no finite
// result.  The float32 error of this evaluation is what gets scored against
// the float64 direct convolution (Section 6).
//
// Memory layout (see wg.h, wg_layout):
//   U'[e][k][c]  transformed filters, e = tile element, c contiguous
//   V'[e][p][c]  transformed input tiles, c contiguous (the GEMM contraction)
//   M [e][k][p]  Hadamard/channel sums, p (tile index) contiguous
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <set>
#include <utility>

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
    int dB[kMaxAlpha];     // E(|B^T row i|_1) - E(|G row i|_1)
};

__device__ __forceinline__ int bin_exp(float v) {
    int e = 0;
    if (v != 0.0f) frexpf(v, &e);
    return e;
}

// floor(d / 2): arithmetic right shift of a two's-complement int
__device__ __forceinline__ int floor_half(int d) { return d >> 1; }

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
// Filter transform U = G g G^T.  A block covers 64 channels (the lanes of a
// wave) and four filters (one per wave); each thread transforms one filter
// channel g = w[k][c] into all alpha x alpha entries, so every store of
// U'[e][k][.] is a contiguous run of 64 channels.
//
// For the 16-bit stage the block first finishes the per-channel exponent
// part t[c] = E(x_absmax[c]) - E(max_k |w[k][c]|) from the partial maxima of
// all filter chunks (every block of a channel group repeats this small
// reduction, so no second launch is needed), scales entry (i, j) by 2^s with
// s = floor((dB[i] + dB[j] + t[c]) / 2) before rounding, and the blocks of
// the first filter group also write t and the table s[e][c].
// ---------------------------------------------------------------------------
template <int M, int R, int DT>
__global__ __launch_bounds__(256) void filter_transform_kernel(const float* __restrict__ w,
                                                               void* __restrict__ Uout,
                                                               const float* __restrict__ part,
                                                               const float* __restrict__ x_absmax,
                                                               int32_t* __restrict__ s_tab,
                                                               int32_t* __restrict__ t_tab, int kchunks,
                                                               Mats<M, R> mt, NzMasks nzm, RowExps ex, Geo g) {
    constexpr int A = M + R - 1;
    using T = typename Elem<DT>::T;
    __shared__ float sG[A][R];
    __shared__ float sred[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    const int k = blockIdx.y * 4 + wv;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
            for (int u = 0; u < R; ++u) sG[a][u] = mt.G[a][u];
    }
    int tc = 0;
    if (DT != kF32) {
        float aw = 0.0f;
        if (c < g.C) {
#pragma unroll 8
            for (int q = wv; q < kchunks; q += 4) aw = fmaxf(aw, part[(size_t)q * g.C_pad + c]);
        }
        sred[wv][lane] = aw;
    }
    __syncthreads();
    if (DT != kF32 && c < g.C) {
        const float mw = fmaxf(fmaxf(sred[0][lane], sred[1][lane]), fmaxf(sred[2][lane], sred[3][lane]));
        tc = bin_exp(x_absmax != nullptr ? x_absmax[c] : 1.0f) - bin_exp(mw);
    }
    if (DT != kF32 && blockIdx.y == 0 && c < g.C_pad) {
        if (wv == 0) t_tab[c] = tc;
#pragma unroll
        for (int e1 = 0; e1 < A; ++e1)
            if ((e1 & 3) == wv) {
#pragma unroll
                for (int e2 = 0; e2 < A; ++e2)
                    s_tab[(size_t)(e1 * A + e2) * g.C_pad + c] = c < g.C ? floor_half(ex.dB[e1] + ex.dB[e2] + tc) : 0;
            }
    }
    if (c >= g.C_pad) return;
    const bool live = k < g.K && c < g.C;
    float gg[R][R];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v) gg[u][v] = live ? w[(((size_t)k * g.C + c) * R + u) * R + v] : 0.0f;
    T* U = reinterpret_cast<T*>(Uout);
    const unsigned off = (unsigned)k * g.C_pad + c;
    const size_t plane = in_vgpr((size_t)g.K_pad * g.C_pad);
#pragma unroll
    for (int i = 0; i < A; ++i) {
        // row i of P1 = G g
        float p1[R];
#pragma unroll
        for (int v = 0; v < R; ++v) p1[v] = 0.0f;
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (nz(nzm.g, i * R + u)) {
                const float b = sG[i][u];
#pragma unroll
                for (int v = 0; v < R; ++v) p1[v] = __builtin_fmaf(b, gg[u][v], p1[v]);
            }
        const int si = tc + ex.dB[i];
#pragma unroll
        for (int j = 0; j < A; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int v = 0; v < R; ++v)
                if (nz(nzm.g, j * R + v)) acc = __builtin_fmaf(sG[j][v], p1[v], acc);
            if (DT != kF32) acc = ldexpf(acc, c < g.C ? floor_half(si + ex.dB[j]) : 0);
            T* Ue = U + (size_t)(i * A + j) * plane;
            Ue[off] = Elem<DT>::from_f32(acc);
        }
    }
}

// ---------------------------------------------------------------------------
// Input transform V = B^T d B.  A block covers one image n, one tile row th,
// `twb` consecutive tiles of that row and kInCh input channels.  It stages the
// alpha input rows of those channels in LDS (threads own fixed positions of
// the band and walk the channels, so consecutive threads read contiguous row
// segments; zeros outside the image), then transforms in two passes over LDS:
//   pass 1: every staged column b of every channel, T1[:, b] = B^T d[:, b],
//           written back in place (columns shared by neighbouring tiles are
//           transformed once);
//   pass 2: every (channel, tile, row i), V[i][j] = sum_l T1[i][l] B^T[j][l],
//           scaled and rounded to the GEMM type and stored; consecutive lanes
//           hold consecutive channels, so every V' store is a contiguous run.
// Zero entries of B^T are not skipped: fma(0, x, acc) == acc for finite x,
// and a per-term branch costs more than the multiply-add.  Block indices are
// mapped so
// that each XCD runs a contiguous range of bands, keeping the channel blocks
// of one tile row (which write the halves of the same V' lines) and
// neighbouring tile rows (which share R-1 input rows) in one L2.
// ---------------------------------------------------------------------------
constexpr int kInCh = 32;
constexpr int kInThreads = 256;
constexpr int kXcdCount = 8;

template <int A, bool kFull>
__device__ __forceinline__ void stage_band(const float* __restrict__ x, float* lds, const Geo& g, int n, int c0,
                                           int nch, int row0, int col0, int wl, int row_w, int ch_stride) {
    constexpr int kBatch = 16;
    const size_t hw = in_vgpr((size_t)g.H * g.W);
    const int cstride = in_vgpr(ch_stride);
    const int last = in_vgpr(max(nch - 1, 0));
    for (int ac = threadIdx.x; ac < A * wl; ac += kInThreads) {
        const int a = ac / wl, col = ac - a * wl;
        const int gi = row0 + a, gj = col0 + col;
        const bool inside = gi >= 0 && gi < g.H && gj >= 0 && gj < g.W && nch > 0;
        // loads are unconditional (from a valid address) and masked after,
        // so a whole batch is in flight at once
        const float* src = inside ? x + (((size_t)n * g.C + c0) * g.H + gi) * g.W + gj : x;
        float* dst = lds + a * row_w + col;
#pragma unroll
        for (int cb = 0; cb < kInCh; cb += kBatch) {
            float v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                v[u] = *src;                        // channel min(cb + u, last)
                if (kFull || cb + u < last) src += hw;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) v[u] = (inside && (kFull || cb + u <= last)) ? v[u] : 0.0f;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                *dst = v[u];
                dst += cstride;
            }
        }
    }
}

template <int M, int R, int DT>
__global__ __launch_bounds__(kInThreads) void input_transform_kernel(const float* __restrict__ x,
                                                                     void* __restrict__ Vout,
                                                                     const int32_t* __restrict__ t_tab,
                                                                     Mats<M, R> mt, NzMasks nzm, RowExps ex,
                                                                     Geo g, int twb, int n_twb, int row_w,
                                                                     int ch_stride, int n_blocks) {
    constexpr int A = M + R - 1;
    using T = typename Elem<DT>::T;
    extern __shared__ float lds[];
    __shared__ float sBT[A][A];
    __shared__ int sdB[A];
    __shared__ int stc[kInCh];
    const int tid = threadIdx.x;
    const int per_xcd = (int)(gridDim.x / kXcdCount);
    const int w = (int)(blockIdx.x % kXcdCount) * per_xcd + (int)(blockIdx.x / kXcdCount);
    if (w >= n_blocks) return;                      // whole block: before any barrier
    const int n_cb = g.C_pad / kInCh;
    int bx = w;
    const int c0 = (bx % n_cb) * kInCh;
    bx /= n_cb;
    const int tb = bx % n_twb;
    bx /= n_twb;
    const int th = bx % g.Th;
    const int n = bx / g.Th;
    const int tw0 = tb * twb;
    const int ntw = min(twb, g.Tw - tw0);
    const int wl = ntw * M + R - 1;               // columns actually needed
    const int row0 = th * M - g.pad, col0 = tw0 * M - g.pad;
    if (tid == 0) {
#pragma unroll
        for (int a = 0; a < A; ++a) {
#pragma unroll
            for (int b = 0; b < A; ++b) sBT[a][b] = mt.BT[a][b];
            sdB[a] = ex.dB[a];
        }
    }
    if (DT != kF32 && tid < kInCh) stc[tid] = c0 + tid < g.C ? t_tab[c0 + tid] : 0;

    // stage the band (channel tail handled apart so that the full case
    // carries no per-channel conditions)
    const int nch = min(kInCh, g.C - c0);          // channels present (may be <= 0)
    if (nch == kInCh)
        stage_band<A, true>(x, lds, g, n, c0, nch, row0, col0, wl, row_w, ch_stride);
    else
        stage_band<A, false>(x, lds, g, n, c0, nch, row0, col0, wl, row_w, ch_stride);
    __syncthreads();

    // pass 1: T1 = B^T d, column by column, in place
    for (int q = tid; q < kInCh * wl; q += kInThreads) {
        const int ch = q / wl, col = q - ch * wl;
        float* colp = lds + ch * ch_stride + col;
        float d[A];
#pragma unroll
        for (int l = 0; l < A; ++l) d[l] = colp[l * row_w];
        float t1[A];
#pragma unroll
        for (int i = 0; i < A; ++i) {
            float acc = 0.0f;
#pragma unroll
            for (int l = 0; l < A; ++l) acc = __builtin_fmaf(sBT[i][l], d[l], acc);
            t1[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < A; ++i) colp[i * row_w] = t1[i];
    }
    __syncthreads();

    // pass 2: V = T1 B, row by row; scaling, rounding, stores
    T* V = reinterpret_cast<T*>(Vout);
    const size_t plane = in_vgpr((size_t)g.P_pad * g.C_pad);
    for (int q = tid; q < kInCh * ntw * A; q += kInThreads) {
        const int ch = q % kInCh, rest = q / kInCh;
        const int t = rest / A, i = rest - t * A;
        const int gc = c0 + ch;
        const float* rowp = lds + ch * ch_stride + i * row_w + t * M;
        float r[A];
#pragma unroll
        for (int l = 0; l < A; ++l) r[l] = rowp[l];
        const int sv = (DT != kF32 && gc < g.C) ? sdB[i] + stc[ch] : 0;
        const unsigned p = ((unsigned)n * g.Th + th) * g.Tw + tw0 + t;
        T* Vp = V + (size_t)(i * A) * plane + ((size_t)p * g.C_pad + gc);
#pragma unroll
        for (int j = 0; j < A; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int l = 0; l < A; ++l) acc = __builtin_fmaf(sBT[j][l], r[l], acc);
            if (DT != kF32) acc = ldexpf(acc, gc < g.C ? -floor_half(sv + ex.dB[j]) : 0);
            *Vp = Elem<DT>::from_f32(acc);
            Vp += plane;
        }
    }
}

// ---------------------------------------------------------------------------
// Output transform Y = A^T M A.  A block covers one output channel k and
// `nb` consecutive tile rows ("bands", band = n*Th + th).  Each thread
// transforms one tile (reading it one row of M at a time, consecutive
// threads at consecutive tiles of each plane) and leaves its in-range
// outputs in LDS laid out exactly like the image rows (pitch Wout); the rows
// of consecutive bands of one image are contiguous in y, so the block then
// copies each image's run with consecutive threads.  Zero entries of A^T are
// not skipped (fma(0, x, acc) == acc for finite x).
// ---------------------------------------------------------------------------
template <int M, int R>
__global__ __launch_bounds__(256) void output_transform_kernel(const float* __restrict__ Mbuf,
                                                               float* __restrict__ y, Mats<M, R> mt,
                                                               NzMasks nzm, Geo g, int nb,
                                                               unsigned plane_stride) {
    constexpr int A = M + R - 1;
    extern __shared__ float lds[];
    __shared__ float sAT[M][A];
    const int tid = threadIdx.x;
    if (tid == 0) {
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int b = 0; b < A; ++b) sAT[a][b] = mt.AT[a][b];
    }
    __syncthreads();
    const int k = blockIdx.y;
    const int band0 = blockIdx.x * nb;
    const int nbands = g.N * g.Th;
    const int nbl = min(nb, nbands - band0);
    const int items = nbl * g.Tw;
    for (int it = tid; it < items; it += 256) {
        const int bl = it / g.Tw, tw = it - bl * g.Tw;
        // offset inside one plane of M; the alpha^2 planes are plane_stride apart
        const unsigned off = (unsigned)k * g.P_pad + (unsigned)(band0 + bl) * g.Tw + tw;
        // Z = A^T M, streaming the rows of M (plane a*A + b holds M[a][b])
        const size_t pstride = in_vgpr((size_t)plane_stride);
        const float* mp = Mbuf + off;
        float z[M][A];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int b = 0; b < A; ++b) z[i][b] = 0.0f;
#pragma unroll
        for (int a = 0; a < A; ++a) {
            float row[A];
#pragma unroll
            for (int b = 0; b < A; ++b) {
                row[b] = *mp;
                mp += pstride;
            }
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const float av = sAT[i][a];
#pragma unroll
                for (int b = 0; b < A; ++b) z[i][b] = __builtin_fmaf(av, row[b], z[i][b]);
            }
        }
        const int th = (band0 + bl) % g.Th;
        const int rows = min(M, g.Hout - th * M);
        const int cols = min(M, g.Wout - tw * M);
        float* dst = lds + (bl * M) * g.Wout + tw * M;
        // Y = Z A one column j at a time: Y[i][j] = sum_l Z[i][l] A^T[j][l]
#pragma unroll
        for (int j = 0; j < M; ++j) {
            float arow[A];
#pragma unroll
            for (int l = 0; l < A; ++l) arow[l] = sAT[j][l];
            float col[M];
#pragma unroll
            for (int i = 0; i < M; ++i) col[i] = 0.0f;
#pragma unroll
            for (int l = 0; l < A; ++l)
#pragma unroll
                for (int i = 0; i < M; ++i) col[i] = __builtin_fmaf(arow[l], z[i][l], col[i]);
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (i < rows && j < cols) dst[i * g.Wout + j] = col[i];
        }
    }
    __syncthreads();
    // copy runs: the bands of one image are consecutive rows of plane (n, k)
    int bl = 0;
    while (bl < nbl) {
        const int band = band0 + bl;
        const int n = band / g.Th, th = band - n * g.Th;
        const int last = min(nbl, bl + (g.Th - th));          // bands of image n in this block
        const int row_first = th * M;
        const int row_end = min(g.Hout, (th + (last - bl)) * M);
        const int len = (row_end - row_first) * g.Wout;
        const float* src = lds + bl * M * g.Wout;
        float* dst = y + (((size_t)n * g.K + k) * g.Hout + row_first) * g.Wout;
        for (int q = tid; q < len; q += 256) dst[q] = src[q];
        bl = last;
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
static NzMasks pack_masks(const Plan& p) {
    NzMasks z{};
    const int A = p.L.alpha, m = p.L.m, r = p.L.r;
    for (int q = 0; q < m * A; ++q)
        if (p.AT[q] != 0.0f) z.at[q >> 6] |= 1ull << (q & 63);
    for (int q = 0; q < A * r; ++q)
        if (p.G[q] != 0.0f) z.g[q >> 6] |= 1ull << (q & 63);
    for (int q = 0; q < A * A; ++q)
        if (p.BT[q] != 0.0f) z.bt[q >> 6] |= 1ull << (q & 63);
    return z;
}

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
    const NzMasks nzm = pack_masks(p);
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
    const dim3 grid((unsigned)((L.C_pad + 63) / 64), (unsigned)(L.K_pad / 4));
    switch (L.dtype) {
        case WG_F32:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF32>), grid, dim3(256), 0, s, w, U, part, x_absmax,
                               s_tab, t_tab, kchunks, mt, nzm, ex, g);
            break;
        case WG_F16:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kF16>), grid, dim3(256), 0, s, w, U, part, x_absmax,
                               s_tab, t_tab, kchunks, mt, nzm, ex, g);
            break;
        default:
            hipLaunchKernelGGL((filter_transform_kernel<M, R, kBF16>), grid, dim3(256), 0, s, w, U, part, x_absmax,
                               s_tab, t_tab, kchunks, mt, nzm, ex, g);
            break;
    }
    return last_launch("filter_transform_kernel");
}

// Raise a kernel's dynamic LDS limit above 64 KB (gfx950 has 160 KB per CU);
// done once per kernel and size.
template <typename F>
static void allow_lds(F kernel, size_t bytes) {
    static std::mutex mu;
    static std::set<std::pair<const void*, size_t>> done;
    if (bytes <= 65536) return;
    const void* key = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    if (done.insert({key, bytes}).second)
        (void)hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int M, int R>
static int input_impl(const Plan& p, const float* x, const void* U, void* ws, hipStream_t s) {
    constexpr int A = M + R - 1;
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    const NzMasks nzm = pack_masks(p);
    RowExps ex{};
    for (int i = 0; i < L.alpha; ++i) ex.dB[i] = p.dB[i];
    // as many tiles of a tile row per block as fit in 40 KB of staged rows,
    // split evenly; the channel stride is 33 mod 64 words, so neither the
    // column pass (lanes along columns) nor the row pass (lanes along
    // channels) has LDS bank conflicts
    int nsplit = 1, twb = 0, row_w = 0, ch_stride = 0;
    size_t lds_bytes = 0;
    for (;; ++nsplit) {
        twb = (L.Tw + nsplit - 1) / nsplit;
        row_w = twb * M + R - 1;
        ch_stride = A * row_w;
        ch_stride += (33 - ch_stride % 64 + 64) % 64;
        lds_bytes = (size_t)kInCh * ch_stride * sizeof(float);
        if (lds_bytes <= 40 * 1024 || twb == 1) break;
    }
    if (lds_bytes > 128 * 1024) return fail(WG_EUNSUPPORTED, "input transform: tile too large for LDS");
    if (L.C_pad % kInCh != 0) return fail(WG_EUNSUPPORTED, "input transform: channel padding");
    const int n_twb = (L.Tw + twb - 1) / twb;
    const long n_blocks = (long)L.N * L.Th * n_twb * (L.C_pad / kInCh);
    if (n_blocks > (1L << 30)) return fail(WG_EUNSUPPORTED, "input transform: grid too large");
    const dim3 grid((unsigned)((n_blocks + kXcdCount - 1) / kXcdCount * kXcdCount));
    const dim3 block(kInThreads);
    const int32_t* t_tab = reinterpret_cast<const int32_t*>(static_cast<const char*>(U) + L.chan_offset);
    void* V = static_cast<char*>(ws) + L.v_offset;
    const int nb = (int)n_blocks;
    switch (L.dtype) {
        case WG_F32:
            allow_lds(input_transform_kernel<M, R, kF32>, lds_bytes);
            hipLaunchKernelGGL((input_transform_kernel<M, R, kF32>), grid, block, lds_bytes, s, x, V, t_tab, mt, nzm, ex, g, twb, n_twb, row_w, ch_stride, nb);
            break;
        case WG_F16:
            allow_lds(input_transform_kernel<M, R, kF16>, lds_bytes);
            hipLaunchKernelGGL((input_transform_kernel<M, R, kF16>), grid, block, lds_bytes, s, x, V, t_tab, mt, nzm, ex, g, twb, n_twb, row_w, ch_stride, nb);
            break;
        default:
            allow_lds(input_transform_kernel<M, R, kBF16>, lds_bytes);
            hipLaunchKernelGGL((input_transform_kernel<M, R, kBF16>), grid, block, lds_bytes, s, x, V, t_tab, mt, nzm, ex, g, twb, n_twb, row_w, ch_stride, nb);
            break;
    }
    return last_launch("input_transform_kernel");
}

template <int M, int R>
static int output_impl(const Plan& p, const void* ws, float* y, hipStream_t s) {
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R> mt = pack_mats<M, R>(p);
    const NzMasks nzm = pack_masks(p);
    int nb = 256 / L.Tw;
    if (nb < 1) nb = 1;
    while (nb > 1 && (size_t)nb * M * L.Wout * sizeof(float) > 65536) --nb;
    const size_t lds_bytes = (size_t)nb * M * L.Wout * sizeof(float);
    if (lds_bytes > 65536) return fail(WG_EUNSUPPORTED, "output transform: output rows too wide");
    const int nbands = L.N * L.Th;
    const dim3 grid((unsigned)((nbands + nb - 1) / nb), (unsigned)L.K);
    const float* Mbuf = reinterpret_cast<const float*>(static_cast<const char*>(ws) + L.m_offset);
    hipLaunchKernelGGL((output_transform_kernel<M, R>), grid, dim3(256), lds_bytes, s, Mbuf, y, mt, nzm, g, nb, (unsigned)((size_t)L.K_pad * L.P_pad));
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
