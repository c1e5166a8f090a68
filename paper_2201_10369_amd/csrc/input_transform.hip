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

#include <algorithm>

#include "wg_filter_block.h"
#include "wg_layer_common.h"

#pragma clang fp contract(off)

namespace wg {

// ---------------------------------------------------------------------------
// Input transform V = B^T d B.  A block covers one image n, one tile row th,
// `twb` consecutive tiles of that row and kInCh input channels, handled as
// channel pairs throughout:
//   load + pass 1: a thread takes one column of the alpha-row band for two
//           adjacent channels (coalesced: lanes along columns), transforms
//           it at once, T1[:, b] = B^T d[:, b] (columns shared by
//           neighbouring tiles are transformed once), and writes it to LDS;
//   pass 2: a thread takes one row of T1 of one tile for a channel pair,
//           V[i][j] = sum_l T1[i][l] B^T[j][l], scales and rounds both
//           channels and stores them with one store (consecutive lanes hold
//           consecutive pairs, so every V' store is a contiguous run).
// Input reads go through a buffer resource on image n: columns outside the
// image and channels past C get an out-of-range offset and read as zero;
// rows outside the image are block-uniform and skipped.
// With the B^T structure of sets with 0 and infinity (S), rows are taken in
// RowPerm order and the structurally zero terms are left out.  Block indices
// are mapped so that each XCD runs a contiguous range of bands, keeping the
// channel blocks of one tile row (which write the halves of the same V'
// lines) and neighbouring tile rows (which share R-1 input rows) in one L2.
//
// LDS: T1 of the band, lds[pc * pair_stride + col * CS + k * 2 + (c & 1)]
// for pair pc, column col, T1 row slot k (RowPerm order); CS = 2 (alpha | 1)
// words (an odd number of word pairs: lanes along columns hit distinct
// banks), pair_stride = 8 mod 64 words (lanes along pairs likewise).
// ---------------------------------------------------------------------------
constexpr int kInCh = 32;
constexpr int kInPairs = kInCh / 2;
constexpr int kInThreads = 256;

// S: B^T has the zero structure of sets with 0 and infinity (rows arrive in
// the order of RowPerm: point 0 first, infinity last), so column 0 is used
// only by the first row and column alpha-1 only by the last.
template <int A, bool S>
struct BtTerms {
    __device__ static constexpr int lo(int q) { return (S && q > 0) ? 1 : 0; }
    __device__ static constexpr int hi(int q) { return (S && q < A - 1) ? A - 2 : A - 1; }
};

struct InputArgs {
    const float* x;            // N x C x H x W
    void* V;                   // V'[e][p][c]
    const int32_t* t_tab;      // t[c] from the filter transform (16-bit stage)
    const float* part;         // or: partial maxima of |w| per filter chunk ...
    const float* x_absmax;     // ... with the per-channel max |x| (null: bound 1)
    int kchunks;
    int twb, n_twb, pair_stride, n_blocks;
};

// Pair of adjacent channels' values in LDS
template <typename CT>
struct PairOf;
template <>
struct PairOf<float> {
    using type = wg_f32x2;
};
template <>
struct PairOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

// The block of work item w (image, tile row, tile group, channel group).
// TP: the 16-bit exponent part t[c] is derived here from the partial maxima
// (as the filter transform derives it) instead of read from t_tab.
// CT: float, or double for the float64 transforms (then DT is kF32, T1 is
// kept in LDS as float64 and each V entry is rounded to float32).
template <int M, int R, int DT, bool S, bool TP, typename CT = float>
__device__ __forceinline__ void input_block(const InputArgs& ia, const Mats<M, R, CT>& mt, const RowPerm& rp,
                                            const Geo& g, int w) {
    constexpr int A = M + R - 1;
    constexpr int CS = 2 * (A | 1);               // LDS elements (CT) per column
    using T = typename Elem<DT>::T;
    using P2 = typename PairOf<CT>::type;
    using Terms = BtTerms<A, S>;
    // B^T per lane (vector registers) for alpha <= 7, and for alpha = 8 with
    // the zero structure: the combined launch otherwise runs out of scalar
    // registers and reloads spilled coefficients in its first pass (36.0 ->
    // 33.5 us for the fp16 F(6x6,3x3) launch; the opaque zero keeps the
    // compiler from folding the copy back into scalar registers; larger
    // alpha would cost occupancy)
    constexpr bool kBtVgpr = sizeof(CT) == 4 && (A <= 7 || (A == 8 && S));
    unsigned vz = 0;
    if constexpr (kBtVgpr) asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
    CT btv[A][A];
#pragma unroll
    for (int k = 0; k < A; ++k)
#pragma unroll
        for (int l = 0; l < A; ++l) {
            if constexpr (kBtVgpr) btv[k][l] = __uint_as_float(__float_as_uint((float)mt.BT[k][l]) | vz);
            else btv[k][l] = mt.BT[k][l];
        }
    const float* __restrict__ x = ia.x;
    const int twb = ia.twb, n_twb = ia.n_twb, pair_stride = ia.pair_stride;
    extern __shared__ __align__(16) float lds_raw[];
    CT* lds = reinterpret_cast<CT*>(lds_raw);
    __shared__ int sdB[A];                        // dB of T1 row slot k (RowPerm order)
    __shared__ int srow[A];                       // T1 row index of slot k
    __shared__ int stc[kInCh];
    const int tid = threadIdx.x;
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
        for (int k = 0; k < A; ++k) {
            srow[k] = rp.row[k];
            sdB[k] = rp.dB[k];
        }
    }
    if (DT != kF32 && !TP && tid < kInCh) stc[tid] = c0 + tid < g.C ? ia.t_tab[c0 + tid] : 0;
    // 16-bit exponent part t[c] from the partial maxima (TP): eight threads
    // per channel, each every eighth filter chunk; the first loads are issued
    // here and reduced after pass 1, so they overlap the input loads
    constexpr int kPartStep = kInThreads / kInCh, kPartRegs = 4;
    __shared__ float spart[kPartStep][kInCh];
    float pv[kPartRegs];
    const int pcc = c0 + (tid & (kInCh - 1));
#pragma unroll
    for (int j = 0; j < kPartRegs; ++j) {
        const int q = tid / kInCh + j * kPartStep;
        pv[j] = (DT != kF32 && TP && pcc < g.C && q < ia.kchunks) ? ia.part[(size_t)q * g.C_pad + pcc] : 0.0f;
    }
    // load + pass 1
    {
        const size_t img = (size_t)g.C * g.H * g.W;
        const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(x) + (size_t)n * img, 0, (int)(img * sizeof(float)), kBufferWord3);
        const int hw4 = g.H * g.W * 4;
        const int dpc = kInThreads / wl, dcol = kInThreads - dpc * wl;
        int pc = tid / wl, col = tid - pc * wl;
        for (int q = tid; q < kInPairs * wl; q += kInThreads) {
            // per-lane byte offsets of (channel, row 0, column) for both
            // channels, or an out-of-range marker (reads as zero) for columns
            // outside the image and channels past C; the row goes in the
            // scalar offset
            const int gj = col0 + col;
            const int cch = c0 + 2 * pc;
            const bool cok = gj >= 0 && gj < g.W;
            const unsigned base = (unsigned)(cch * hw4 + gj * 4);
            const unsigned voff0 = (cok && cch < g.C) ? base : 0x80000000u;
            const unsigned voff1 = (cok && cch + 1 < g.C) ? base + (unsigned)hw4 : 0x80000000u;
            CT d0[A], d1[A];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const int gi = row0 + a;                      // uniform over the block
                if (gi >= 0 && gi < g.H) {
                    d0[a] = (CT)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, (int)voff0, gi * g.W * 4, 0));
                    d1[a] = (CT)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, (int)voff1, gi * g.W * 4, 0));
                } else {
                    d0[a] = CT(0);
                    d1[a] = CT(0);
                }
            }
            CT* dst = lds + pc * pair_stride + col * CS;
#pragma unroll
            for (int k = 0; k < A; ++k) {
                CT t0 = CT(0), t1 = CT(0);
#pragma unroll
                for (int l = Terms::lo(k); l <= Terms::hi(k); ++l) {
                    t0 = madd(btv[k][l], d0[l], t0);
                    t1 = madd(btv[k][l], d1[l], t1);
                }
                *reinterpret_cast<P2*>(dst + 2 * k) = P2{t0, t1};
            }
            col += dcol;
            pc += dpc;
            if (col >= wl) {
                col -= wl;
                ++pc;
            }
        }
    }
    if (DT != kF32 && TP) {
        float aw = fmaxf(fmaxf(pv[0], pv[1]), fmaxf(pv[2], pv[3]));
        if (pcc < g.C)
            for (int q = tid / kInCh + kPartRegs * kPartStep; q < ia.kchunks; q += kPartStep)
                aw = fmaxf(aw, ia.part[(size_t)q * g.C_pad + pcc]);
        spart[tid / kInCh][tid & (kInCh - 1)] = aw;
    }
    __syncthreads();
    if (DT != kF32 && TP) {
        if (tid < kInCh) {
            float mw = spart[0][tid];
#pragma unroll
            for (int q = 1; q < kInThreads / kInCh; ++q) mw = fmaxf(mw, spart[q][tid]);
            stc[tid] = c0 + tid < g.C
                           ? bin_exp(ia.x_absmax != nullptr ? ia.x_absmax[c0 + tid] : 1.0f) - bin_exp(mw)
                           : 0;
        }
        __syncthreads();
    }

    // pass 2: V = T1 B, row by row for pairs of adjacent channels; scaling,
    // rounding, and one store per pair.  The 16-bit exponent
    // -floor((dB[i] + dB[j] + t[c]) / 2) is taken as
    // (1 - dB[i] - t[c] - dB[j]) >> 1 (padded channels hold zeros).
    T* V = reinterpret_cast<T*>(ia.V);
    const size_t plane = (size_t)g.P_pad * g.C_pad;
    for (int q = tid; q < kInPairs * ntw * A; q += kInThreads) {
        const int pc = q % kInPairs, rest = q / kInPairs;
        const int t = rest / A, k = rest - t * A;
        const int i = srow[k];
        const int gc = c0 + 2 * pc;
        const CT* rowp = lds + pc * pair_stride + (t * M) * CS + 2 * k;
        CT r0[A], r1[A];
#pragma unroll
        for (int l = 0; l < A; ++l) {
            const P2 v = *reinterpret_cast<const P2*>(rowp + l * CS);
            r0[l] = v.x;
            r1[l] = v.y;
        }
        int nb0 = 0, nb1 = 0;
        if (DT != kF32) {
            nb0 = 1 - sdB[k] - stc[2 * pc];
            nb1 = 1 - sdB[k] - stc[2 * pc + 1];
        }
        const unsigned p = ((unsigned)n * g.Th + th) * g.Tw + tw0 + t;
        T* Vi = V + (size_t)(i * A) * plane + ((size_t)p * g.C_pad + gc);
#pragma unroll
        for (int kk = 0; kk < A; ++kk) {
            CT q0 = CT(0), q1 = CT(0);
#pragma unroll
            for (int l = Terms::lo(kk); l <= Terms::hi(kk); ++l) {
                q0 = madd(btv[kk][l], r0[l], q0);
                q1 = madd(btv[kk][l], r1[l], q1);
            }
            float a0 = (float)q0, a1 = (float)q1;
            if (DT != kF32) {
                a0 = ldexpf(a0, (nb0 - rp.dB[kk]) >> 1);
                a1 = ldexpf(a1, (nb1 - rp.dB[kk]) >> 1);
            }
            Elem<DT>::store2(Vi + rp.plane_off[kk], a0, a1);
        }
    }
}

// Block b of a grid of n_grid blocks (a multiple of kXcdCount) -> work item:
// each XCD runs a contiguous range of items.
__device__ __forceinline__ int xcd_item(int b, int n_grid) {
    const int per_xcd = n_grid / kXcdCount;
    return (b % kXcdCount) * per_xcd + b / kXcdCount;
}

template <int M, int R, int DT, bool S, typename CT>
__global__ __launch_bounds__(kInThreads) void input_transform_kernel(InputArgs ia, Mats<M, R, CT> mt, RowPerm rp,
                                                                     Geo g) {
    const int w = xcd_item((int)blockIdx.x, (int)gridDim.x);
    if (w >= ia.n_blocks) return;                   // whole block: before any barrier
    input_block<M, R, DT, S, false, CT>(ia, mt, rp, g, w);
}

// Filter and input transforms in one launch: the first gridDim.x - n_in_grid
// blocks are filter-transform blocks (channel group, filter), dispatched
// first, the last n_in_grid input-transform blocks (t[c] from the partial
// maxima), which take over the compute units as the short filter blocks
// finish; no launch boundary separates the two stages.
template <int M, int R, int DT, bool S, bool TP, typename CT>
__global__ __launch_bounds__(kInThreads) void filter_input_kernel(InputArgs ia, FilterArgs fa, Mats<M, R, CT> mt,
                                                                  RowPerm rp, RowExps ex, Geo g, int n_in_grid,
                                                                  int f_groups) {
    const int nf = (int)gridDim.x - n_in_grid;
    const int b = (int)blockIdx.x - nf;
    if (b >= 0) {
        const int w = xcd_item(b, n_in_grid);
        if (w >= ia.n_blocks) return;
        input_block<M, R, DT, S, TP, CT>(ia, mt, rp, g, w);
    } else {
        extern __shared__ __align__(16) float lds_f[];
        const int f = (int)blockIdx.x;
        filter_block<M, R, DT, CT>(fa, mt, ex, g, f % f_groups, f / f_groups, reinterpret_cast<int*>(lds_f));
    }
}

template <int M, int R, int DT, bool S, typename CT>
static void input_launch(dim3 grid, size_t lds_bytes, hipStream_t s, const InputArgs& ia,
                         const Mats<M, R, CT>& mt, const RowPerm& rp, const Geo& g) {
    allow_lds(input_transform_kernel<M, R, DT, S, CT>, lds_bytes);
    hipLaunchKernelGGL((input_transform_kernel<M, R, DT, S, CT>), grid, dim3(kInThreads), lds_bytes, s, ia, mt, rp,
                       g);
}

template <int M, int R, int DT, bool S, bool TP, typename CT>
static void filter_input_launch(unsigned n_in_grid, unsigned n_f_blocks, int f_groups, size_t lds_bytes,
                                hipStream_t s, const InputArgs& ia, const FilterArgs& fa, const Mats<M, R, CT>& mt,
                                const RowPerm& rp, const RowExps& ex, const Geo& g) {
    allow_lds(filter_input_kernel<M, R, DT, S, TP, CT>, lds_bytes);
    hipLaunchKernelGGL((filter_input_kernel<M, R, DT, S, TP, CT>), dim3(n_in_grid + n_f_blocks), dim3(kInThreads),
                       lds_bytes, s, ia, fa, mt, rp, ex, g, (int)n_in_grid, f_groups);
}

// fused: w non-null -> the filter transform of w runs in the same launch
// (the 16-bit partial maxima of |w| must already be in U), t[c] derived in
// the input blocks.  CT: the transforms' arithmetic (double: float64
// transforms, dtype WG_F32 only).
template <int M, int R, typename CT>
static int input_impl(const Plan& p, const float* x, const void* U, void* ws, hipStream_t s, const float* w,
                      const float* x_absmax, bool t_from_table) {
    constexpr int A = M + R - 1;
    constexpr int CS = 2 * (A | 1);
    constexpr bool f64 = sizeof(CT) == 8;
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const bool structured = zero_shape(p).bt;
    // the offsets of the alpha planes of a V' row block are 32-bit element counts
    if ((size_t)(A - 1) * L.P_pad * L.C_pad >= (1ull << 32))
        return fail(WG_EUNSUPPORTED, "input transform: V' planes too large for 32-bit offsets");
    const RowPerm rp = bt_row_perm(p, structured, (size_t)L.P_pad * L.C_pad);
    // B^T rows in RowPerm order
    Mats<M, R, CT> mt = pack_mats<M, R, CT>(p);
    for (int k = 0; k < A; ++k)
        for (int l = 0; l < A; ++l) mt.BT[k][l] = f64 ? (CT)p.BT64[rp.row[k] * A + l] : (CT)p.BT[rp.row[k] * A + l];
    RowExps ex{};
    for (int i = 0; i < L.alpha; ++i) ex.dB[i] = p.dB[i];
    // one image's input is addressed with 32-bit byte offsets (channels up to
    // C_pad, and an out-of-range marker at 2^31)
    if ((size_t)L.C_pad * L.H * L.W * sizeof(float) >= (1ull << 31))
        return fail(WG_EUNSUPPORTED, "input transform: one image of the input exceeds 2 GB");
    // as many tiles of a tile row per block as fit in 40 KB of LDS, split
    // evenly; pair_stride in elements of CT (even, 8 mod 64 words for float)
    int nsplit = 1, twb = 0, pair_stride = 0;
    size_t lds_bytes = 0;
    for (;; ++nsplit) {
        twb = (L.Tw + nsplit - 1) / nsplit;
        const int wl = twb * M + R - 1;
        pair_stride = wl * CS;
        pair_stride += (8 - pair_stride % 64 + 64) % 64;
        lds_bytes = (size_t)kInPairs * pair_stride * sizeof(CT);
        if (lds_bytes <= 40 * 1024 || twb == 1) break;
    }
    if (lds_bytes > 128 * 1024) return fail(WG_EUNSUPPORTED, "input transform: tile too large for LDS");
    if (L.C_pad % kInCh != 0) return fail(WG_EUNSUPPORTED, "input transform: channel padding");
    const int n_twb = (L.Tw + twb - 1) / twb;
    const long n_blocks = (long)L.N * L.Th * n_twb * (L.C_pad / kInCh);
    if (n_blocks > (1L << 30)) return fail(WG_EUNSUPPORTED, "input transform: grid too large");
    const unsigned n_in_grid = (unsigned)((n_blocks + kXcdCount - 1) / kXcdCount * kXcdCount);
    const dim3 grid(n_in_grid);
    const int32_t* t_tab = reinterpret_cast<const int32_t*>(static_cast<const char*>(U) + L.chan_offset);
    void* V = static_cast<char*>(ws) + L.v_offset;
    if (w == nullptr) {
        const InputArgs ia{x, V, t_tab, nullptr, nullptr, 0, twb, n_twb, pair_stride, (int)n_blocks};
#define WG_IN(DT)                                                                                 \
    (structured ? input_launch<M, R, DT, true, CT>(grid, lds_bytes, s, ia, mt, rp, g)             \
                : input_launch<M, R, DT, false, CT>(grid, lds_bytes, s, ia, mt, rp, g))
        if constexpr (f64) {
            WG_IN(kF32);
        } else {
            switch (L.dtype) {
                case WG_F32: WG_IN(kF32); break;
                case WG_F16: WG_IN(kF16); break;
                default: WG_IN(kBF16); break;
            }
        }
#undef WG_IN
        return last_launch("input_transform_kernel");
    }
    // the partial maxima of |w| (16-bit stage) are already in U (wg_filter_maxima)
    const FilterArgs fa = t_from_table ? filter_args_table(p, w, const_cast<void*>(U))
                                       : filter_args(p, w, x_absmax, const_cast<void*>(U));
    const InputArgs ia{x, V, t_tab, fa.part, fa.x_absmax, fa.kchunks, twb, n_twb, pair_stride, (int)n_blocks};
    const int fg = filter_groups(L);
    const unsigned n_f = (unsigned)fg * (unsigned)L.K_pad;
    if ((size_t)n_in_grid + n_f > (1u << 31)) return fail(WG_EUNSUPPORTED, "filter and input transform: grid too large");
    const size_t lds = std::max(lds_bytes, sizeof(int) * (size_t)kFilterLdsWords);
#define WG_FI(DT, TP)                                                                                             \
    (structured ? filter_input_launch<M, R, DT, true, TP, CT>(n_in_grid, n_f, fg, lds, s, ia, fa, mt, rp, ex, g)   \
                : filter_input_launch<M, R, DT, false, TP, CT>(n_in_grid, n_f, fg, lds, s, ia, fa, mt, rp, ex, g))
    // float32 stages have no exponent part: one instantiation
    if constexpr (f64) {
        WG_FI(kF32, false);
    } else {
        switch (L.dtype) {
            case WG_F32: WG_FI(kF32, false); break;
            case WG_F16:
                if (t_from_table) WG_FI(kF16, false);
                else WG_FI(kF16, true);
                break;
            default:
                if (t_from_table) WG_FI(kBF16, false);
                else WG_FI(kBF16, true);
                break;
        }
    }
#undef WG_FI
    return last_launch("filter_input_kernel");
}

template <int M, int R>
static int input_dispatch(const Plan& p, const float* x, const void* U, void* ws, hipStream_t s, const float* w,
                          const float* x_absmax, bool t_from_table) {
    return p.f64t ? input_impl<M, R, double>(p, x, U, ws, s, w, x_absmax, t_from_table)
                  : input_impl<M, R, float>(p, x, U, ws, s, w, x_absmax, t_from_table);
}

int launch_input_transform(const Plan& p, const float* x, const void* U, void* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_input(MM, RR) \
    case MM * 16 + RR: return input_dispatch<MM, RR>(p, x, U, ws, s, nullptr, nullptr, false);
    WG_DISPATCH(input)
#undef WG_CASE_input
}

int launch_filter_input(const Plan& p, const float* w, const float* x_absmax, const float* x, void* U, void* ws,
                        void* stream, bool t_from_table) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_fi(MM, RR) \
    case MM * 16 + RR: return input_dispatch<MM, RR>(p, x, U, ws, s, w, x_absmax, t_from_table);
    WG_DISPATCH(fi)
#undef WG_CASE_fi
}

}  // namespace wg
