// Scoring kernels: float64 direct convolution (the reference of Section 6 of
// arXiv:2201.10369, eq. conv as a zero-padded cross-correlation) and the L1
// error sums against it, with a fixed reduction tree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "wg_device.h"
#include "wg_internal.h"

namespace wg {

// ---------------------------------------------------------------------------
// float64 direct convolution on the vector units, for images whose output
// rows are too wide for the matrix-core form below.  A block computes a
// 32 x 32 output patch of 16 output channels of one image; each thread owns 2 x 2 pixels x 16 channels.
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

// ---------------------------------------------------------------------------
// float64 direct convolution as an implicit GEMM on the float64 matrix cores:
// Y[k][p] = sum_q Wt[k][q] X[q][p] with q = (c, u, v) flattened (w's own row
// layout) and p an output pixel, X[q][p] the zero-padded input under tap
// (u, v) of channel c.  A block owns 16 output channels and TH whole output
// rows of one image; each wave holds up to kDfTiles 16 x 16 accumulator
// tiles (16 channels x 16 consecutive pixels of the block's rows) and issues
// v_mfma_f64_16x16x4 over four reduction terms at a time.  The reduction runs
// in stages of kDfCh channels: the stage's input patch ((TH + R - 1) rows x
// (Wout + R - 1) columns per channel, zeros outside the image) and its
// 16 x kDfCh R^2 weights sit in LDS as float64, and the next stage's floats
// are loaded into registers while the current stage computes.  Every product
// of two floats is exact in float64; only the order of the sums differs from
// the plain loop.
// ---------------------------------------------------------------------------
constexpr int kDfWaves = 4;
constexpr int kDfTiles = 13;                 // 16-pixel tiles per wave (832 pixels per block)
constexpr int kDfCh = 4;                     // channels per stage (4 R^2 terms: whole MFMA steps)
constexpr int kDfPatch = 1024;               // max patch elements per channel
constexpr int kDfThreads = 64 * kDfWaves;
constexpr int kDfXPerThread = kDfCh * kDfPatch / kDfThreads;

using f64x4 = double __attribute__((ext_vector_type(4)));

struct DirectGeo {
    int C, K, H, W, pad, Hout, Wout;
    int TH, NRB, NKB, n_items;               // rows per block, row blocks, channel blocks, blocks
    int PH, PW;                              // patch rows and columns
};

template <int R>
__global__ __launch_bounds__(kDfThreads, 2) void direct_f64_mfma_kernel(const float* __restrict__ x,
                                                                         const float* __restrict__ w,
                                                                         double* __restrict__ y, DirectGeo g) {
    constexpr int RR = R * R;
    constexpr int KK = kDfCh * RR;           // reduction terms per stage
    static_assert(KK % 4 == 0, "a stage must hold whole matrix-instruction steps");
    constexpr int WS = KK + 1;               // LDS row stride of the stage's weights
    constexpr int WPT = (16 * KK + kDfThreads - 1) / kDfThreads;
    __shared__ double xs[kDfCh * kDfPatch];
    __shared__ double wsh[16 * WS];

    // consecutive items (the channel blocks of one image's rows, which read
    // the same input patch) go to one XCD and share its L2
    const int item = (int)(blockIdx.x % kXcdCount) * (int)(gridDim.x / kXcdCount) + (int)(blockIdx.x / kXcdCount);
    if (item >= g.n_items) return;           // whole block, before any barrier
    const int kb = item % g.NKB;
    const int rb = (item / g.NKB) % g.NRB;
    const int n = item / (g.NKB * g.NRB);
    const int k0 = kb * 16, oy0 = rb * g.TH;
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int col = lane & 15, grp = lane >> 4;
    // rotate which wave takes the block's extra tile over the SIMDs
    const int wv = (__builtin_amdgcn_readfirstlane(tid >> 6) + item) % kDfWaves;
    const int PHPW = g.PH * g.PW;
    const int stage_elems = kDfCh * PHPW;
    const int HW = g.H * g.W;
    const int CRR = g.C * RR;

    // input offset of each staged element relative to the stage's first
    // channel (-1: zero padding), the same for every stage; kept in LDS (each
    // thread reads back only its own entries) to leave registers for the
    // operands of two steps
    __shared__ int goffs[kDfCh * kDfPatch];
#pragma unroll
    for (int j = 0; j < kDfXPerThread; ++j) {
        const int e = tid + kDfThreads * j;
        int o = -1;
        if (e < stage_elems) {
            const int cl = e / PHPW, rem = e - cl * PHPW;
            const int i = rem / g.PW, jj = rem - i * g.PW;
            const int gi = oy0 - g.pad + i, gj = jj - g.pad;
            if (gi >= 0 && gi < g.H && gj >= 0 && gj < g.W) o = cl * HW + gi * g.W + gj;
        }
        goffs[tid + kDfThreads * j] = o;
    }
    // patch offset of each owned pixel (0 for the padding lanes of the last tile)
    const int npx = min(g.TH, g.Hout - oy0) * g.Wout;
    const int ntiles = (npx + 15) / 16;
    const int nt_w = (ntiles - wv + kDfWaves - 1) / kDfWaves;   // this wave's tiles (wave-uniform)
    int pix[kDfTiles];
#pragma unroll
    for (int t = 0; t < kDfTiles; ++t) {
        const int q = min((wv + kDfWaves * t) * 16 + col, npx - 1);
        const int oy = q / g.Wout;
        pix[t] = oy * g.PW + (q - oy * g.Wout);
    }

    float xr[kDfXPerThread], wr[WPT];
    auto load_stage = [&](int c0) {
        const float* xb = x + ((size_t)n * g.C + c0) * HW;
        const int lim = (g.C - c0) * PHPW;   // elements of channels below C
#pragma unroll
        for (int j = 0; j < kDfXPerThread; ++j)
        {
            const int o = goffs[tid + kDfThreads * j];
            xr[j] = (o >= 0 && tid + kDfThreads * j < lim) ? xb[o] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            const int f = tid + kDfThreads * j;
            const int r = f / KK, kl = f - r * KK;
            const int q = c0 * RR + kl;
            wr[j] = (f < 16 * KK && k0 + r < g.K && q < CRR) ? w[(size_t)(k0 + r) * CRR + q] : 0.f;
        }
    };

    f64x4 acc[kDfTiles];
#pragma unroll
    for (int t = 0; t < kDfTiles; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int n_stages = (g.C + kDfCh - 1) / kDfCh;
    load_stage(0);
    for (int s = 0; s < n_stages; ++s) {
        __syncthreads();                     // the previous stage's reads are done
#pragma unroll
        for (int j = 0; j < kDfXPerThread; ++j)
            if (tid + kDfThreads * j < stage_elems) xs[tid + kDfThreads * j] = (double)xr[j];
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            const int f = tid + kDfThreads * j;
            if (f < 16 * KK) {
                const int r = f / KK, kl = f - r * KK;
                wsh[r * WS + kl] = (double)wr[j];
            }
        }
        __syncthreads();
        if (s + 1 < n_stages) load_stage((s + 1) * kDfCh);
        // For step st, lane (col, grp) supplies A[col][grp] = weight of channel
        // k0 + col at term 4 st + grp and B[grp][col] = the input under that
        // term at pixel col.  The operands of step st + 1 are read while the
        // products of step st issue.
        double bn[kDfTiles], an;
        {
            const int kl = grp;
            const int cl = kl / RR, uv = kl - cl * RR, u = uv / R, v = uv - u * R;
            const int koff = cl * PHPW + u * g.PW + v;
            an = wsh[col * WS + kl];
#pragma unroll
            for (int t = 0; t < kDfTiles; ++t) bn[t] = xs[koff + pix[t]];
        }
#pragma unroll 1
        for (int st = 0; st < KK / 4; ++st) {
            double b[kDfTiles];
#pragma unroll
            for (int t = 0; t < kDfTiles; ++t) b[t] = bn[t];
            const double a = an;
            {
                // operands of the next step (the last step re-reads its own)
                const int kl = 4 * min(st + 1, KK / 4 - 1) + grp;
                const int cl = kl / RR, uv = kl - cl * RR, u = uv / R, v = uv - u * R;
                const int koff = cl * PHPW + u * g.PW + v;
                an = wsh[col * WS + kl];
#pragma unroll
                for (int t = 0; t < kDfTiles; ++t) bn[t] = xs[koff + pix[t]];
            }
            // every wave issues all kDfTiles products: a wave with fewer tiles
            // accumulates its clamped padding pixels and drops them at the
            // store, which keeps the step free of branches
#pragma unroll
            for (int t = 0; t < kDfTiles; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[t], acc[t], 0, 0, 0);
            // scheduling: alternate one LDS read (mask 0x100) and one matrix
            // instruction (mask 0x008)
#pragma unroll
            for (int t = 0; t < kDfTiles; ++t) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
        }
    }
    // accumulator element i of lane (col, grp) is row grp + 4 i of the 16 x 16
    // tile (channel k0 + grp + 4 i) at column col (pixel col): the float64
    // matrix instruction interleaves its rows over the lane groups
#pragma unroll
    for (int t = 0; t < kDfTiles; ++t) {
        const int q = (wv + kDfWaves * t) * 16 + col;
        if (t >= nt_w || q >= npx) continue;
        const int oyl = q / g.Wout, ox = q - oyl * g.Wout;
        double* yp = y + ((size_t)n * g.K * g.Hout + oy0 + oyl) * g.Wout + ox;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + grp + 4 * i;
            if (k < g.K) yp[(size_t)k * g.Hout * g.Wout] = acc[t][i];
        }
    }
}

// Rows per block for the MFMA form: as many whole output rows as fit in
// kDfWaves * kDfTiles tiles and a kDfPatch-element patch, balanced over the
// row blocks; 0 when not even one row fits.
int direct_rows_per_block(int r, int Hout, int Wout) {
    const int PW = Wout + r - 1;
    int th = std::min(Hout, kDfWaves * kDfTiles * 16 / Wout);
    while (th >= 1 && (th + r - 1) * PW > kDfPatch) --th;
    if (th < 1) return 0;
    const int nrb = (Hout + th - 1) / th;
    return (Hout + nrb - 1) / nrb;
}

int launch_direct_f64(const float* x, const float* w, double* y, int N, int C, int K, int H, int W,
                      int r, int pad, int Hout, int Wout, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (r < 1 || r > 7) return fail(WG_EINVAL, "direct conv: r out of range");
    // the matrix-core form keeps input offsets within a stage in 32 bits
    const bool small_planes = (long long)kDfCh * H * W <= 0x7fffffffLL;
    const int th = small_planes ? direct_rows_per_block(r, Hout, Wout) : 0;
    if (th >= 1) {
        DirectGeo g{C, K, H, W, pad, Hout, Wout, th, (Hout + th - 1) / th, (K + 15) / 16, 0, th + r - 1,
                    Wout + r - 1};
        const long long items = (long long)N * g.NRB * g.NKB;
        const long long grid = (items + kXcdCount - 1) / kXcdCount * kXcdCount;
        if (grid > 0x7fffffffLL) return fail(WG_EINVAL, "direct conv: too many blocks");
        g.n_items = (int)items;
        switch (r) {
#define WG_DIRECT_MFMA_CASE(RR)                                                                    \
    case RR:                                                                                       \
        hipLaunchKernelGGL((direct_f64_mfma_kernel<RR>), dim3((unsigned)grid), dim3(kDfThreads), 0, s, x, \
                           w, y, g);                                                               \
        break;
            WG_DIRECT_MFMA_CASE(1) WG_DIRECT_MFMA_CASE(2) WG_DIRECT_MFMA_CASE(3) WG_DIRECT_MFMA_CASE(4)
            WG_DIRECT_MFMA_CASE(5) WG_DIRECT_MFMA_CASE(6) WG_DIRECT_MFMA_CASE(7)
#undef WG_DIRECT_MFMA_CASE
        }
        return hip_check((int)hipGetLastError(), "direct_f64_mfma_kernel");
    }
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

// ---------------------------------------------------------------------------
// Allocation-free scoring: the same two kernels with their partial sums in a
// file-scope device array (one copy per GPU, kept until the process ends)
// instead of a caller workspace.  The partial-sum grid never exceeds
// kScorePartials blocks, so the array holds the partials of every count.
// Host code never passes the array's name to a kernel: its device address is
// looked up once per device (with that device current) and kept.
// ---------------------------------------------------------------------------
constexpr int kScorePartials = 1024;
static __device__ __align__(256) double scratch[2 * kScorePartials];

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_ptr;      // per device; null until looked up

static int scratch_for_current_device(double** out) {
    int dev = 0;
    int st = hip_check((int)hipGetDevice(&dev), "wg_score_error_noalloc: hipGetDevice");
    if (st != WG_OK) return st;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        st = hip_check((int)hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                       "wg_score_error_noalloc: hipGetSymbolAddress");
        if (st != WG_OK) return st;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return WG_OK;
}

int launch_score_noalloc(const float* y, const double* yref, size_t count, double* out2, void* stream) {
    if (score_partials(count) > (size_t)kScorePartials)
        return fail(WG_EUNSUPPORTED, "wg_score_error_noalloc: more partial sums than the static scratch holds");
    double* part = nullptr;
    const int st = scratch_for_current_device(&part);
    if (st != WG_OK) return st;
    return launch_score(y, yref, count, out2, part, stream);
}

}  // namespace wg
