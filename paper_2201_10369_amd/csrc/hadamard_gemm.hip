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
// MFMA blocks.  The contraction runs in steps of 64 bytes of each operand row
// through a ring of kStages LDS stages filled by direct global-to-LDS buffer
// loads (no staging registers): the loads of kStages-1 steps are in flight
// while one is multiplied.  Within a stage an operand row is 64 bytes; its
// four 16-byte chunks are stored XOR-swizzled by bits 2-3 of the row index,
// so the 32 rows an MFMA operand read touches spread over all banks.  The
// operand buffer resources end at the last real row, so padding rows are not
// fetched (they read as zero).  The finished tile goes out through LDS as
// whole 512-byte rows of M.  Block ids are mapped so that the blocks running
// together on one XCD work on neighbouring tiles (same e) and share its L2.
//
// Element types: float32 (v_mfma_f32_32x32x2_f32), float16 and bfloat16 with
// float32 accumulation (v_mfma_f32_32x32x16_{f16,bf16}).
#include <hip/hip_runtime.h>

#include "wg_device.h"
#include "wg_internal.h"

namespace wg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;


constexpr int kStepBytes = 64;        // bytes of each operand row per pipeline step
constexpr int kStages = 3;            // LDS ring depth (48 KB: three blocks per CU)

// byte offset of 16-byte chunk c of row r inside a stage region
__device__ __forceinline__ int chunk_at(int r, int c) { return r * kStepBytes + ((c ^ ((r >> 2) & 3)) << 4); }

template <int DT>
struct MfmaOp;

template <>
struct MfmaOp<kF32> {
    static constexpr int kElem = 4;
    // per 64-byte step (16 floats): half-wave h holds k = 8h .. 8h+7 of its
    // row (chunks 2h, 2h+1); instruction q multiplies element q of both.
    __device__ static __forceinline__ void step(const char* A, const char* B, int ra, int rb, int half,
                                                f32x16& acc) {
        const u32x4 a0 = *reinterpret_cast<const u32x4*>(A + chunk_at(ra, 2 * half));
        const u32x4 a1 = *reinterpret_cast<const u32x4*>(A + chunk_at(ra, 2 * half + 1));
        const u32x4 b0 = *reinterpret_cast<const u32x4*>(B + chunk_at(rb, 2 * half));
        const u32x4 b1 = *reinterpret_cast<const u32x4*>(B + chunk_at(rb, 2 * half + 1));
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a0[q]), __uint_as_float(b0[q]), acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a1[q]), __uint_as_float(b1[q]), acc, 0, 0, 0);
    }
};

template <>
struct MfmaOp<kF16> {
    static constexpr int kElem = 2;
    // per 64-byte step (32 halves): two instructions of k = 16, half-wave h
    // holding 8 consecutive k (chunk 2s + h of slice s).
    __device__ static __forceinline__ void step(const char* A, const char* B, int ra, int rb, int half,
                                                f32x16& acc) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const u32x4 a = *reinterpret_cast<const u32x4*>(A + chunk_at(ra, 2 * s + half));
            const u32x4 b = *reinterpret_cast<const u32x4*>(B + chunk_at(rb, 2 * s + half));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                         __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
        }
    }
};

template <>
struct MfmaOp<kBF16> {
    static constexpr int kElem = 2;
    __device__ static __forceinline__ void step(const char* A, const char* B, int ra, int rb, int half,
                                                f32x16& acc) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const u32x4 a = *reinterpret_cast<const u32x4*>(A + chunk_at(ra, 2 * s + half));
            const u32x4 b = *reinterpret_cast<const u32x4*>(B + chunk_at(rb, 2 * s + half));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                          __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
        }
    }
};

// s_waitcnt vmcnt(n) for the few counts the ring needs (expcnt and lgkmcnt
// left at their maxima)
__device__ __forceinline__ void wait_vmcnt(int n) {
    switch (n) {
        case 0: __builtin_amdgcn_s_waitcnt(0x0F70); break;
        case 2: __builtin_amdgcn_s_waitcnt(0x0F72); break;
        case 4: __builtin_amdgcn_s_waitcnt(0x0F74); break;
        case 6: __builtin_amdgcn_s_waitcnt(0x0F76); break;
        case 8: __builtin_amdgcn_s_waitcnt(0x0F78); break;
        default: __builtin_amdgcn_s_waitcnt(0x0F70); break;
    }
}

// barrier without a memory fence (the waits are explicit), and no compiler
// motion of memory accesses across it
__device__ __forceinline__ void block_barrier() {
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int BM, int BN, int DT>
__global__ __launch_bounds__(256) void hadamard_gemm_kernel(const char* __restrict__ U,
                                                            const char* __restrict__ V,
                                                            float* __restrict__ Mout, int K, int K_pad, int P,
                                                            int P_pad, int C_pad, int nKb, int nPb,
                                                            int total, int tiles_per_xcd, int blocks_per_xcd) {
    constexpr int WM = BM / 2, WN = BN / 2;          // wave sub-tile
    constexpr int FM = WM / 32, FN = WN / 32;         // 32 x 32 blocks per wave
    constexpr int ELEM = MfmaOp<DT>::kElem;
    constexpr int ROWS = BM + BN;                     // operand rows per stage (A then B)
    constexpr int STAGE_BYTES = ROWS * kStepBytes;
    constexpr int LOADS = ROWS / 64;                  // 16-row DMA loads per wave per step
    static_assert(ROWS % 64 == 0 && BM % 16 == 0, "tile shape");
    constexpr int kStagePitch = BN + 4;               // floats per staged row of M
    static_assert((BM / 2) * kStagePitch * 4 <= kStages * STAGE_BYTES, "epilogue stage exceeds the ring");
    static_assert(kStages - 2 <= 2 && LOADS <= 4, "vmcnt table");

    __shared__ __attribute__((aligned(16))) char smem[kStages * STAGE_BYTES];

    // XCD-aware work mapping: XCD x (blocks b = x mod 8) owns the contiguous
    // tile range [x * tiles_per_xcd, (x+1) * tiles_per_xcd); its block in
    // slot s takes tiles s, s + blocks_per_xcd, s + 2 blocks_per_xcd, ... of
    // that range, so the blocks running together on one XCD always work on
    // neighbouring tiles (same e, shared operand rows in its L2)
    const int b = blockIdx.x;
    const int xcd = b % kXcdCount, slot = b / kXcdCount;
    const int lo = xcd * tiles_per_xcd, hi = min(total, lo + tiles_per_xcd);
    const int t0 = lo + slot;
    if (t0 >= hi) return;
    const int nt = (hi - t0 + blocks_per_xcd - 1) / blocks_per_xcd;
    const int tstride = blocks_per_xcd;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;   // wave index is uniform
    const int wm = wave >> 1, wn = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;
    const int row_bytes = C_pad * ELEM;
    const int nsteps = row_bytes / kStepBytes;

    for (int t = 0; t < nt; ++t) {
        const int ct = t0 + t * tstride;
        const int kb = ct % nKb, pb = (ct / nKb) % nPb, e = ct / (nKb * nPb);
        // operand resources end at the last real row (k < K, p < P)
        const int arows = min(BM, K - kb * BM), brows = min(BN, P - pb * BN);
        const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(U) + ((size_t)e * K_pad + (size_t)kb * BM) * row_bytes, 0, arows * row_bytes,
            kBufferWord3);
        const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(V) + ((size_t)e * P_pad + (size_t)pb * BN) * row_bytes, 0, brows * row_bytes,
            kBufferWord3);
        // DMA of step st into its stage: wave w moves combined rows
        // (w*LOADS + j)*16 .. +16; lane L takes row +L/4, stored chunk L%4,
        // which holds global chunk (L%4) ^ swizzle(row)
        auto issue = [&](int st) {
            char* stage = smem + (st % kStages) * STAGE_BYTES;
#pragma unroll
            for (int j = 0; j < LOADS; ++j) {
                const int R0 = (wave * LOADS + j) * 16;                   // uniform
                const bool isA = R0 < BM;
                const int lr = (isA ? R0 : R0 - BM) + (lane >> 2);
                const int c = (lane & 3) ^ ((lr >> 2) & 3);
                const int voff = lr * row_bytes + st * kStepBytes + c * 16;
                lds_void* dst = (lds_void*)(stage + R0 * kStepBytes);
                if (isA)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsA, dst, 16, voff, 0, 0, 0);
                else
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsB, dst, 16, voff, 0, 0, 0);
            }
        };
#pragma unroll
        for (int s = 0; s < kStages - 1; ++s)
            if (s < nsteps) issue(s);

        f32x16 acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
        for (int st = 0; st < nsteps; ++st) {
            // step st has landed once at most the later steps' loads remain
            wait_vmcnt(min(kStages - 2, nsteps - 1 - st) * LOADS);
            block_barrier();                         // ... in every wave; stage st-1 is free
            if (st + kStages - 1 < nsteps) issue(st + kStages - 1);
            const char* As = smem + (st % kStages) * STAGE_BYTES;
            const char* Bs = As + BM * kStepBytes;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    MfmaOp<DT>::step(As, Bs, wm * WM + i * 32 + l32, wn * WN + j * 32 + l32, half, acc[i][j]);
        }
        __syncthreads();                             // every wave done with the ring

        // Epilogue through LDS, in two halves: the waves of row group wm == h
        // write their accumulators (32 x 32 layout: lane holds column
        // lane % 32 and, in register r, row 8*(r/4) + 4*(lane/32) + r%4),
        // then every thread writes 16 bytes of a full tile row.  Rows k >= K
        // fall outside the store resource (dropped); 16-byte column groups
        // starting at p >= P are not written.
        float* Mg = Mout + ((size_t)e * K_pad + (size_t)kb * BM) * P_pad + (size_t)pb * BN;
        const int pcols = P - pb * BN;
        const __amdgpu_buffer_rsrc_t rsM = __builtin_amdgcn_make_buffer_rsrc(Mg, 0, arows * P_pad * 4, kBufferWord3);
        float* stage = reinterpret_cast<float*>(smem);
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
                    __builtin_amdgcn_raw_buffer_store_b128(v, rsM, ((h * WM + row) * P_pad + 4 * c4) * 4, 0, 0);
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
    // one tile of each operand and of M is addressed with 32-bit byte offsets
    if ((long)BM * L.P_pad * 4 >= (1L << 31) || (long)BN * L.C_pad * 4 >= (1L << 31) ||
        (long)BM * L.C_pad * 4 >= (1L << 31))
        return fail(WG_EUNSUPPORTED, "hadamard gemm: tile rows too long");
    const int tpb = p.gemm_tpb > 0 ? p.gemm_tpb : 1;
    const int tiles_per_xcd = (int)((total + kXcdCount - 1) / kXcdCount);
    const int blocks_per_xcd = (tiles_per_xcd + tpb - 1) / tpb;
    const char* V = static_cast<const char*>(ws) + L.v_offset;
    float* Mb = reinterpret_cast<float*>(static_cast<char*>(ws) + L.m_offset);
    hipLaunchKernelGGL((hadamard_gemm_kernel<BM, BN, DT>), dim3((unsigned)(blocks_per_xcd * kXcdCount)), dim3(256), 0, s,
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
