// Input transform V = B^T d B of the Winograd layer on gfx950
// (arXiv:2201.10369, Section 4, eq. conv_2d), applied to every input tile.
//
// Each two-sided product P X P^T is evaluated as (P X) first and then
// (P X) P^T, every inner product accumulated in ascending index order with one
// fused multiply-add per term (acc <- fma(p, x, acc) from acc = 0).  The
// float32 error of this evaluation is what gets scored against the float64
// direct convolution (arXiv:2201.10369, Section 6).
//
// Layout: V'[e][p][c], c contiguous (the GEMM contraction), p = tile index.
#include <hip/hip_runtime.h>

#include "wg_layer_common.h"

#pragma clang fp contract(off)

namespace wg {

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

// S: B^T has the zero structure of sets with 0 and infinity (rows arrive in
// the order of RowPerm: point 0 first, infinity last), so column 0 is used
// only by the first row and column alpha-1 only by the last.
template <int A, bool S>
struct BtTerms {
    __device__ static constexpr int lo(int q) { return (S && q > 0) ? 1 : 0; }
    __device__ static constexpr int hi(int q) { return (S && q < A - 1) ? A - 2 : A - 1; }
};

template <int M, int R, int DT, bool S>
__global__ __launch_bounds__(kInThreads) void input_transform_kernel(const float* __restrict__ x,
                                                                     void* __restrict__ Vout,
                                                                     const int32_t* __restrict__ t_tab,
                                                                     Mats<M, R> mt, RowPerm rp, RowExps ex,
                                                                     Geo g, int twb, int n_twb, int row_w,
                                                                     int ch_stride, int n_blocks) {
    constexpr int A = M + R - 1;
    using T = typename Elem<DT>::T;
    using Terms = BtTerms<A, S>;
    extern __shared__ float lds[];
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
        for (int a = 0; a < A; ++a) sdB[a] = ex.dB[a];
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

    // pass 1: T1 = B^T d, column by column, in place (task indices advance
    // by constant steps instead of being divided out each time)
    {
        const int dch = kInThreads / wl, dcol = kInThreads - dch * wl;
        int ch = tid / wl, col = tid - ch * wl;
        for (int q = tid; q < kInCh * wl; q += kInThreads) {
            float* colp = lds + ch * ch_stride + col;
            float d[A];
#pragma unroll
            for (int l = 0; l < A; ++l) d[l] = colp[l * row_w];
            float t1[A];
#pragma unroll
            for (int k = 0; k < A; ++k) {
                float acc = 0.0f;
#pragma unroll
                for (int l = Terms::lo(k); l <= Terms::hi(k); ++l) acc = __builtin_fmaf(mt.BT[k][l], d[l], acc);
                t1[k] = acc;
            }
#pragma unroll
            for (int k = 0; k < A; ++k) colp[rp.row[k] * row_w] = t1[k];
            col += dcol;
            ch += dch;
            if (col >= wl) {
                col -= wl;
                ++ch;
            }
        }
    }
    __syncthreads();

    // pass 2: V = T1 B, row by row for pairs of adjacent channels; scaling,
    // rounding, and one store per pair.  The 16-bit exponent
    // -floor((dB[i] + dB[j] + t[c]) / 2) is taken as
    // (1 - dB[i] - t[c] - dB[j]) >> 1 (padded channels hold zeros).
    T* V = reinterpret_cast<T*>(Vout);
    const size_t plane = (size_t)g.P_pad * g.C_pad;
    constexpr int kPairs = kInCh / 2;
    for (int q = tid; q < kPairs * ntw * A; q += kInThreads) {
        const int pc = q % kPairs, rest = q / kPairs;
        const int t = rest / A, i = rest - t * A;
        const int ch = 2 * pc;
        const int gc = c0 + ch;
        const float* rowp = lds + ch * ch_stride + i * row_w + t * M;
        float r0[A], r1[A];
#pragma unroll
        for (int l = 0; l < A; ++l) {
            r0[l] = rowp[l];
            r1[l] = rowp[ch_stride + l];
        }
        int nb0 = 0, nb1 = 0;
        if (DT != kF32) {
            nb0 = 1 - sdB[i] - stc[ch];
            nb1 = 1 - sdB[i] - stc[ch + 1];
        }
        const unsigned p = ((unsigned)n * g.Th + th) * g.Tw + tw0 + t;
        T* Vi = V + (size_t)(i * A) * plane + ((size_t)p * g.C_pad + gc);
#pragma unroll
        for (int k = 0; k < A; ++k) {
            float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
            for (int l = Terms::lo(k); l <= Terms::hi(k); ++l) {
                a0 = __builtin_fmaf(mt.BT[k][l], r0[l], a0);
                a1 = __builtin_fmaf(mt.BT[k][l], r1[l], a1);
            }
            if (DT != kF32) {
                a0 = ldexpf(a0, (nb0 - rp.dB[k]) >> 1);
                a1 = ldexpf(a1, (nb1 - rp.dB[k]) >> 1);
            }
            Elem<DT>::store2(Vi + rp.plane_off[k], a0, a1);
        }
    }
}

template <int M, int R, int DT, bool S>
static void input_launch(dim3 grid, size_t lds_bytes, hipStream_t s, const float* x, void* V,
                         const int32_t* t_tab, const Mats<M, R>& mt, const RowPerm& rp, const RowExps& ex,
                         const Geo& g, int twb, int n_twb, int row_w, int ch_stride, int nb) {
    allow_lds(input_transform_kernel<M, R, DT, S>, lds_bytes);
    hipLaunchKernelGGL((input_transform_kernel<M, R, DT, S>), grid, dim3(kInThreads), lds_bytes, s, x, V, t_tab, mt,
                       rp, ex, g, twb, n_twb, row_w, ch_stride, nb);
}

template <int M, int R>
static int input_impl(const Plan& p, const float* x, const void* U, void* ws, hipStream_t s) {
    constexpr int A = M + R - 1;
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const bool structured = zero_shape(p).bt;
    const RowPerm rp = bt_row_perm(p, structured, (size_t)L.P_pad * L.C_pad);
    // B^T rows in RowPerm order
    Mats<M, R> mt = pack_mats<M, R>(p);
    for (int k = 0; k < A; ++k)
        for (int l = 0; l < A; ++l) mt.BT[k][l] = p.BT[rp.row[k] * A + l];
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
    const int32_t* t_tab = reinterpret_cast<const int32_t*>(static_cast<const char*>(U) + L.chan_offset);
    void* V = static_cast<char*>(ws) + L.v_offset;
    const int nb = (int)n_blocks;
#define WG_IN(DT)                                                                                              \
    (structured ? input_launch<M, R, DT, true>(grid, lds_bytes, s, x, V, t_tab, mt, rp, ex, g, twb, n_twb, row_w, \
                                               ch_stride, nb)                                                  \
                : input_launch<M, R, DT, false>(grid, lds_bytes, s, x, V, t_tab, mt, rp, ex, g, twb, n_twb,       \
                                                row_w, ch_stride, nb))
    switch (L.dtype) {
        case WG_F32: WG_IN(kF32); break;
        case WG_F16: WG_IN(kF16); break;
        default: WG_IN(kBF16); break;
    }
#undef WG_IN
    return last_launch("input_transform_kernel");
}

int launch_input_transform(const Plan& p, const float* x, const void* U, void* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_input(MM, RR) case MM * 16 + RR: return input_impl<MM, RR>(p, x, U, ws, s);
    WG_DISPATCH(input)
#undef WG_CASE_input
}

}  // namespace wg
