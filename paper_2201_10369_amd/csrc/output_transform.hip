// Output transform Y = A^T M A of the Winograd layer on gfx950
// (arXiv:2201.10369, Section 4, eq. conv_2d), applied to every output tile.
//
// Each two-sided product P X P^T is evaluated as (P X) first and then
// (P X) P^T, every inner product accumulated in ascending index order with one
// fused multiply-add per term (acc <- fma(p, x, acc) from acc = 0).  The
// float32 error of this evaluation is what gets scored against the float64
// direct convolution (arXiv:2201.10369, Section 6).
//
// Layout: M[e][k][p], p (tile index) contiguous; y is N x K x Hout x Wout.
#include <hip/hip_runtime.h>

#include "wg_layer_common.h"

#pragma clang fp contract(off)

namespace wg {

// ---------------------------------------------------------------------------
// Output transform Y = A^T M A.  A block covers one output channel k and
// `nb` consecutive tile rows ("bands", band = n*Th + th).  Each thread
// transforms one tile (reading it one row of M at a time, consecutive
// threads at consecutive tiles of each plane) and leaves its in-range
// outputs in LDS laid out exactly like the image rows (pitch Wout); the rows
// of consecutive bands of one image are contiguous in y, so the block then
// copies each image's run with consecutive threads (16-byte copies when the
// run and its ends are aligned).  Zero entries of A^T are
// not skipped (fma(0, x, acc) == acc for finite x).
// ---------------------------------------------------------------------------
constexpr int kOutThreads = 128;

// CT: float, or double for the float64 transform (Y rounded to float32).
template <int M, int R, typename CT>
__global__ __launch_bounds__(256) void output_transform_kernel(const float* __restrict__ Mbuf,
                                                               float* __restrict__ y, Mats<M, R, CT> mt,
                                                               Geo g, int nb, unsigned plane_stride,
                                                               unsigned plane_bytes) {
    constexpr int A = M + R - 1;
    extern __shared__ __align__(16) float lds[];
    const int tid = threadIdx.x;
    // XCD-aware mapping: each XCD runs a contiguous range of (band group, k)
    // work items, so the partial 128-byte lines of M that neighbouring band
    // groups share are fetched into one L2
    const int per_xcd = (int)(gridDim.x / kXcdCount);
    const int w = (int)(blockIdx.x % kXcdCount) * per_xcd + (int)(blockIdx.x / kXcdCount);
    const int nbg = (g.N * g.Th + nb - 1) / nb;
    if (w >= nbg * g.K) return;
    const int k = w / nbg;
    const int band0 = (w - k * nbg) * nb;
    const int nbands = g.N * g.Th;
    const int nbl = min(nb, nbands - band0);
    const int items = nbl * g.Tw;
    const int nthr = blockDim.x;
    for (int it = tid; it < items; it += nthr) {
        const int bl = it / g.Tw, tw = it - bl * g.Tw;
        // Z = A^T M, streaming the rows of M: row a of the tile is planes
        // a*A .. a*A+A-1, read through a buffer resource on plane a*A with
        // the plane step as scalar offset and the tile's offset in a VGPR
        const unsigned voff = ((unsigned)k * g.P_pad + (unsigned)(band0 + bl) * g.Tw + tw) * 4u;
        CT z[M][A];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int b = 0; b < A; ++b) z[i][b] = CT(0);
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(Mbuf) + (size_t)(a * A) * plane_stride, 0, (int)(A * plane_bytes), kBufferWord3);
            CT row[A];
#pragma unroll
            for (int b = 0; b < A; ++b)
                row[b] = (CT)__uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)(b * plane_bytes), 0));
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const CT av = mt.AT[i][a];
#pragma unroll
                for (int b = 0; b < A; ++b) z[i][b] = madd(av, row[b], z[i][b]);
            }
        }
        const int th = (band0 + bl) % g.Th;
        const int rows = min(M, g.Hout - th * M);
        const int cols = min(M, g.Wout - tw * M);
        float* dst = lds + (bl * M) * g.Wout + tw * M;
        // Y = Z A one column j at a time: Y[i][j] = sum_l Z[i][l] A^T[j][l]
#pragma unroll
        for (int j = 0; j < M; ++j) {
            CT arow[A];
#pragma unroll
            for (int l = 0; l < A; ++l) arow[l] = mt.AT[j][l];
            CT col[M];
#pragma unroll
            for (int i = 0; i < M; ++i) col[i] = CT(0);
#pragma unroll
            for (int l = 0; l < A; ++l)
#pragma unroll
                for (int i = 0; i < M; ++i) col[i] = madd(arow[l], z[i][l], col[i]);
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (i < rows && j < cols) dst[i * g.Wout + j] = (float)col[i];
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
        const int src_off = bl * M * g.Wout;
        const float* src = lds + src_off;
        float* dst = y + (((size_t)n * g.K + k) * g.Hout + row_first) * g.Wout;
        if ((reinterpret_cast<uintptr_t>(dst) & 15u) == 0 && (src_off & 3) == 0 && (len & 3) == 0) {
            // 16-byte copies where the run and both ends allow them
            for (int q = tid; q < (len >> 2); q += nthr)
                reinterpret_cast<float4*>(dst)[q] = reinterpret_cast<const float4*>(src)[q];
        } else {
            for (int q = tid; q < len; q += nthr) dst[q] = src[q];
        }
        bl = last;
    }
}

template <int M, int R, typename CT>
static int output_impl(const Plan& p, const void* ws, float* y, hipStream_t s) {
    const wg_layout& L = p.L;
    const Geo g = make_geo(L);
    const Mats<M, R, CT> mt = pack_mats<M, R, CT>(p);
    const int nthr = kOutThreads;
    int nb = nthr / L.Tw;
    if (nb < 1) nb = 1;
    while (nb > 1 && (size_t)nb * M * L.Wout * sizeof(float) > 65536) --nb;
    const size_t lds_bytes = (size_t)nb * M * L.Wout * sizeof(float);
    if (lds_bytes > 65536) return fail(WG_EUNSUPPORTED, "output transform: output rows too wide");
    // one row of alpha planes is addressed with 32-bit byte offsets
    const size_t plane_elems = (size_t)L.K_pad * L.P_pad;
    if ((size_t)L.alpha * plane_elems * sizeof(float) >= (1ull << 31))
        return fail(WG_EUNSUPPORTED, "output transform: planes of M too large");
    const int nbands = L.N * L.Th;
    const long items = (long)((nbands + nb - 1) / nb) * L.K;
    if (items > (1L << 30)) return fail(WG_EUNSUPPORTED, "output transform: grid too large");
    const dim3 grid((unsigned)((items + kXcdCount - 1) / kXcdCount * kXcdCount));
    const float* Mbuf = reinterpret_cast<const float*>(static_cast<const char*>(ws) + L.m_offset);
    hipLaunchKernelGGL((output_transform_kernel<M, R, CT>), grid, dim3(nthr), lds_bytes, s, Mbuf, y, mt, g, nb,
                       (unsigned)plane_elems, (unsigned)(plane_elems * sizeof(float)));
    return last_launch("output_transform_kernel");
}

int launch_output_transform(const Plan& p, const void* ws, float* y, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
#define WG_CASE_output(MM, RR)                                                                  \
    case MM * 16 + RR:                                                                          \
        return p.f64t ? output_impl<MM, RR, double>(p, ws, y, s) : output_impl<MM, RR, float>(p, ws, y, s);
    WG_DISPATCH(output)
#undef WG_CASE_output
}

}  // namespace wg
