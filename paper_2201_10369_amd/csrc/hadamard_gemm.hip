// Hadamard product + channel sum of the Winograd layer as alpha^2 independent
// matrix products on the gfx950 matrix cores (MFMA):
//
//     M[e] (K x P) = U'[e] (K x C) . V'[e]^T        for every tile element e
//
// The paper points out that this stage dominates the run time of a Winograd
// layer and is a matrix multiplication independent of the points
// (arXiv:2201.10369, Sections 4.1 and 5.2).  Both operands are stored with
// the contraction index c contiguous (U'[e][k][c], V'[e][p][c]), which is the
// register layout the MFMA instructions want for both A and B; M[e][k][p]
// keeps p contiguous for the output transform.
//
// Tiling: a 256-thread block computes a BM x BN tile of M[e] with four waves
// in a 2 x 2 arrangement, each wave a (BM/2) x (BN/2) sub-tile made of 32 x 32
// MFMA blocks.  The contraction runs in steps of BK elements (128 bytes of
// each operand row) through double-buffered LDS, with the next step's global
// loads in flight while the current one is multiplied; a block may take
// several tiles, and the pipeline then runs on across the tile boundaries.
// Block ids are mapped so that the blocks running together on one XCD work on
// neighbouring tiles (same e) and share its L2.
//
// Element types: float32 (v_mfma_f32_32x32x2_f32), float16 and bfloat16 with
// float32 accumulation (v_mfma_f32_32x32x16_{f16,bf16}).
#include <hip/hip_runtime.h>

#include "wg_device.h"
#include "wg_internal.h"

namespace wg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;
// Word 3 of a raw buffer resource on gfx9-family chips (dword data format,
// no swizzle); out-of-range stores are dropped by the hardware.
constexpr int kBufferWord3 = 0x00020000;

// Bytes per operand row per contraction step, and LDS row pitch (16 bytes of
// padding keep the 16-byte LDS reads of 8 consecutive rows on distinct banks).
constexpr int kStepBytes = 128;
constexpr int kPitchBytes = kStepBytes + 16;

template <int DT>
struct MfmaOp;

template <>
struct MfmaOp<kF32> {
    static constexpr int kElem = 4;
    // per 128-byte step (32 floats): each half-wave holds 16 consecutive k of
    // one row; instruction q multiplies element q of both operands.
    __device__ static __forceinline__ void step(const char* a_row, const char* b_row, int half,
                                                f32x16& acc) {
        const f32x4* pa = reinterpret_cast<const f32x4*>(a_row + half * 64);
        const f32x4* pb = reinterpret_cast<const f32x4*>(b_row + half * 64);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const f32x4 a = pa[v];
            const f32x4 b = pb[v];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b[3], acc, 0, 0, 0);
        }
    }
};

template <>
struct MfmaOp<kF16> {
    static constexpr int kElem = 2;
    // per 128-byte step (64 halves): 4 instructions of k = 16, each half-wave
    // holding 8 consecutive k of its row.
    __device__ static __forceinline__ void step(const char* a_row, const char* b_row, int half,
                                                f32x16& acc) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const u32x4 a = *reinterpret_cast<const u32x4*>(a_row + s * 32 + half * 16);
            const u32x4 b = *reinterpret_cast<const u32x4*>(b_row + s * 32 + half * 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                         __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
        }
    }
};

template <>
struct MfmaOp<kBF16> {
    static constexpr int kElem = 2;
    __device__ static __forceinline__ void step(const char* a_row, const char* b_row, int half,
                                                f32x16& acc) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const u32x4 a = *reinterpret_cast<const u32x4*>(a_row + s * 32 + half * 16);
            const u32x4 b = *reinterpret_cast<const u32x4*>(b_row + s * 32 + half * 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                          __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
        }
    }
};

template <int BM, int BN, int DT>
__global__ __launch_bounds__(256) void hadamard_gemm_kernel(const char* __restrict__ U,
                                                            const char* __restrict__ V,
                                                            float* __restrict__ Mout, int K, int K_pad, int P,
                                                            int P_pad, int C_pad, int nKb, int nPb,
                                                            int total, int tiles_per_xcd, int blocks_per_xcd) {
    constexpr int WM = BM / 2, WN = BN / 2;          // wave sub-tile
    constexpr int FM = WM / 32, FN = WN / 32;         // 32 x 32 blocks per wave
    constexpr int ELEM = MfmaOp<DT>::kElem;
    constexpr int A_CHUNKS = BM * kStepBytes / 16;    // 16-byte chunks per A tile
    constexpr int B_CHUNKS = BN * kStepBytes / 16;
    constexpr int A_PER_T = A_CHUNKS / 256, B_PER_T = B_CHUNKS / 256;
    static_assert(A_CHUNKS % 256 == 0 && B_CHUNKS % 256 == 0, "tile too small");
    constexpr int kStagePitch = BN + 4;               // floats per staged row of M
    static_assert((BM / 2) * kStagePitch * 4 <= (BM + BN) * kPitchBytes, "epilogue stage exceeds one buffer");

    __shared__ __attribute__((aligned(16))) char smem[2 * (BM + BN) * kPitchBytes];

    // XCD-aware work mapping: XCD x (blocks b = x mod 8) owns the contiguous
    // tile range [x * tiles_per_xcd, (x+1) * tiles_per_xcd); its block in
    // slot s takes tiles s, s + blocks_per_xcd, s + 2 blocks_per_xcd, ... of
    // that range, so the blocks running together on one XCD always work on
    // neighbouring tiles (same e, shared operand rows in its L2)
    const int b = blockIdx.x;
    const int xcd = b % kXcds, slot = b / kXcds;
    const int lo = xcd * tiles_per_xcd, hi = min(total, lo + tiles_per_xcd);
    const int t0 = lo + slot;
    if (t0 >= hi) return;
    const int nt = (hi - t0 + blocks_per_xcd - 1) / blocks_per_xcd;
    const int tstride = blocks_per_xcd;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;   // wave index is uniform
    const int wm = wave >> 1, wn = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;

    const size_t row_bytes = (size_t)C_pad * ELEM;
    // tile t -> (e, pb, kb) with kb fastest
    // operand tiles are read through buffer resources that end at the last
    // real row (k < K for U', p < P for V'): padding rows read as zero without
    // touching memory
    u32x4 ra[A_PER_T], rb[B_PER_T];
    auto tile_rsrc = [&](const char* base, int rows_left, int rows) {
        const int n = rows_left < rows ? (rows_left > 0 ? rows_left : 0) : rows;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), 0, (int)(n * row_bytes), kBufferWord3);
    };
    auto a_tile = [&](int t) {
        const int kb = t % nKb, e = t / (nKb * nPb);
        return tile_rsrc(U + ((size_t)e * K_pad + (size_t)kb * BM) * row_bytes, K - kb * BM, BM);
    };
    auto b_tile = [&](int t) {
        const int pb = (t / nKb) % nPb, e = t / (nKb * nPb);
        return tile_rsrc(V + ((size_t)e * P_pad + (size_t)pb * BN) * row_bytes, P - pb * BN, BN);
    };

    auto gload = [&](const __amdgpu_buffer_rsrc_t& Ar, const __amdgpu_buffer_rsrc_t& Br, int step) {
        const int koff = step * kStepBytes;
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int q = tid + i * 256;
            const int row = q >> 3, ch = q & 7;
            ra[i] = __builtin_amdgcn_raw_buffer_load_b128(Ar, (int)(row * row_bytes) + koff + ch * 16, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < B_PER_T; ++i) {
            const int q = tid + i * 256;
            const int row = q >> 3, ch = q & 7;
            rb[i] = __builtin_amdgcn_raw_buffer_load_b128(Br, (int)(row * row_bytes) + koff + ch * 16, 0, 0);
        }
    };
    auto sstore = [&](int buf) {
        char* As = smem + buf * (BM + BN) * kPitchBytes;
        char* Bs = As + BM * kPitchBytes;
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int q = tid + i * 256;
            const int row = q >> 3, ch = q & 7;
            *reinterpret_cast<u32x4*>(As + row * kPitchBytes + ch * 16) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < B_PER_T; ++i) {
            const int q = tid + i * 256;
            const int row = q >> 3, ch = q & 7;
            *reinterpret_cast<u32x4*>(Bs + row * kPitchBytes + ch * 16) = rb[i];
        }
    };


    // one pipeline over all (tile, step) pairs of the block: the next pair's
    // global loads are in flight while the current pair is multiplied, also
    // across tile boundaries, where the finished tile is written out
    const int nsteps = (int)(row_bytes / kStepBytes);
    const int niter = nt * nsteps;
    __amdgpu_buffer_rsrc_t nA = a_tile(t0);
    __amdgpu_buffer_rsrc_t nB = b_tile(t0);
    gload(nA, nB, 0);
    sstore(0);
    __syncthreads();
    int it = 0;
    for (int t = 0; t < nt; ++t) {
        f32x16 acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
        for (int st = 0; st < nsteps; ++st, ++it) {
            const int buf = it & 1;
            const bool more = it + 1 < niter;
            if (more) {
                if (st + 1 == nsteps) {
                    nA = a_tile(t0 + (t + 1) * tstride);
                    nB = b_tile(t0 + (t + 1) * tstride);
                }
                gload(nA, nB, st + 1 == nsteps ? 0 : st + 1);
            }
            const char* As = smem + buf * (BM + BN) * kPitchBytes;
            const char* Bs = As + BM * kPitchBytes;
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const char* arow = As + (wm * WM + i * 32 + l32) * kPitchBytes;
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const char* brow = Bs + (wn * WN + j * 32 + l32) * kPitchBytes;
                    MfmaOp<DT>::step(arow, brow, half, acc[i][j]);
                }
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
        }
        // Epilogue through LDS: the buffer the last step consumed is free (the
        // other one may already hold the next tile's first step), and holds
        // half a tile.  In round h the waves of row group wm == h write their
        // accumulators there (32 x 32 layout: lane holds column lane % 32
        // and, in register r, row 8*(r/4) + 4*(lane/32) + r%4); then every
        // thread writes 16 bytes of a full tile row, so each store
        // instruction covers two whole 512-byte rows of M.  Stores go through
        // a buffer resource on the tile (lane offset in a VGPR, no 64-bit
        // address per store).
        const int ct = t0 + t * tstride;
        const int kb = ct % nKb, pb = (ct / nKb) % nPb, e = ct / (nKb * nPb);
        float* Mg = Mout + ((size_t)e * K_pad + (size_t)kb * BM) * P_pad + (size_t)pb * BN;
        // rows k >= K fall outside the resource (dropped); 16-byte column
        // groups starting at p >= P are not written
        const int krows = min(BM, K - kb * BM);
        const int pcols = P - pb * BN;
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(Mg, 0, krows * P_pad * 4, kBufferWord3);
        float* stage = reinterpret_cast<float*>(smem + ((it & 1) ^ 1) * (BM + BN) * kPitchBytes);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (wm == h) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int row = i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                            stage[row * kStagePitch + wn * WN + j * 32 + l32] = acc[i][j][r];
                        }
            }
            __syncthreads();
#pragma unroll
            for (int q = tid; q < WM * (BN / 4); q += 256) {
                const int row = q / (BN / 4), c4 = q - row * (BN / 4);
                const u32x4 v = *reinterpret_cast<const u32x4*>(stage + row * kStagePitch + 4 * c4);
                if (4 * c4 < pcols)
                    __builtin_amdgcn_raw_buffer_store_b128(v, rsrc, ((h * WM + row) * P_pad + 4 * c4) * 4, 0, 0);
            }
            __syncthreads();
        }
    }
}

template <int BM, int BN, int DT>
static int gemm_launch(const Plan& p, const void* U, void* ws, hipStream_t s) {
    const wg_layout& L = p.L;
    const int nKb = L.K_pad / BM, nPb = L.P_pad / BN;
    const long total = (long)L.alpha * L.alpha * nKb * nPb;
    if (total > (1L << 30)) return fail(WG_EUNSUPPORTED, "hadamard gemm: too many tiles");
    // the epilogue addresses one tile with 32-bit byte offsets
    if ((long)BM * L.P_pad * 4 >= (1L << 31) || (long)BN * L.C_pad * 4 >= (1L << 31))
        return fail(WG_EUNSUPPORTED, "hadamard gemm: tile rows too long");
    const int tpb = p.gemm_tpb > 0 ? p.gemm_tpb : 1;
    const int tiles_per_xcd = (int)((total + kXcds - 1) / kXcds);
    const int blocks_per_xcd = (tiles_per_xcd + tpb - 1) / tpb;
    const char* V = static_cast<const char*>(ws) + L.v_offset;
    float* Mb = reinterpret_cast<float*>(static_cast<char*>(ws) + L.m_offset);
    hipLaunchKernelGGL((hadamard_gemm_kernel<BM, BN, DT>), dim3((unsigned)(blocks_per_xcd * kXcds)), dim3(256), 0, s,
                       static_cast<const char*>(U), V, Mb, L.K, L.K_pad, L.P, L.P_pad, L.C_pad, nKb, nPb, (int)total,
                       tiles_per_xcd, blocks_per_xcd);
    return hip_check((int)hipGetLastError(), "hadamard_gemm_kernel");
}

template <int DT>
static int gemm_dtype(const Plan& p, const void* U, void* ws, hipStream_t s) {
    if (p.gemm_bm == 128 && p.gemm_bn == 128) return gemm_launch<128, 128, DT>(p, U, ws, s);
    if (p.gemm_bm == 64 && p.gemm_bn == 64) return gemm_launch<64, 64, DT>(p, U, ws, s);
    return fail(WG_EUNSUPPORTED, "hadamard gemm: tile shape not compiled");
}

int launch_hadamard_gemm(const Plan& p, const void* U, void* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((size_t)p.L.C_pad * p.L.elem_bytes % kStepBytes != 0)
        return fail(WG_EINVAL, "hadamard gemm: padded channel count not a multiple of the step");
    switch (p.L.dtype) {
        case WG_F32: return gemm_dtype<kF32>(p, U, ws, s);
        case WG_F16: return gemm_dtype<kF16>(p, U, ws, s);
        default: return gemm_dtype<kBF16>(p, U, ws, s);
    }
}

int autotune_hadamard_gemm(Plan& p, const void* U, void* ws, int reps, int* chosen, void* stream) {
    static const int kCand[] = {1, 2, 3, 4, 6, 8};
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    int st = hip_check((int)hipEventCreate(&e0), "hipEventCreate");
    if (st != WG_OK) return st;
    st = hip_check((int)hipEventCreate(&e1), "hipEventCreate");
    if (st != WG_OK) {
        (void)hipEventDestroy(e0);
        return st;
    }
    const int keep = p.gemm_tpb;
    int best = keep;
    float best_ms = -1.0f;
    for (int t : kCand) {
        p.gemm_tpb = t;
        st = launch_hadamard_gemm(p, U, ws, stream);                 // warm-up
        if (st == WG_OK) st = hip_check((int)hipEventRecord(e0, s), "hipEventRecord");
        for (int i = 0; i < reps && st == WG_OK; ++i) st = launch_hadamard_gemm(p, U, ws, stream);
        if (st == WG_OK) st = hip_check((int)hipEventRecord(e1, s), "hipEventRecord");
        if (st == WG_OK) st = hip_check((int)hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.0f;
        if (st == WG_OK) st = hip_check((int)hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (st != WG_OK) break;
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p.gemm_tpb = st == WG_OK ? best : keep;
    if (st == WG_OK && chosen) *chosen = best;
    return st;
}

}  // namespace wg
