// Error surrogate: a small fully connected network (4 -> 128 -> 128 -> 128
// -> 1, GELU) trained on sweep errors and used to propose point-family
// parameters.  The paper observes that the error curve over c is smooth
// enough to localise good values (arXiv:2201.10369, Sections 1, 5 and 6.1);
// the network interpolates that curve across parameters and tile sizes so
// that only its best proposals need an exact sweep evaluation.
//
// Kernels (float32, deterministic reduction orders):
//   fwd_bwd : a block takes 16 samples, runs the forward pass with all
//             activations in LDS and, for training, the backward pass, and
//             writes its partial gradient (one full parameter vector); the
//             128 x 128 products of the hidden layers and their gradients
//             run on the float32 matrix cores
//   reduce  : per parameter, four thread groups add interleaved block
//             partials, the group sums are added in order, then Adam (or
//             the gradient is written)
//   predict : forward pass only
//   topk    : the k smallest values of a vector (ties -> smaller index)
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "wg_internal.h"

namespace wg {

constexpr int kIn = 4, kH = 128;
constexpr int kS = 16;            // samples per block, in kHalves row tiles of kHalf
constexpr int kHalf = 16;         // samples per matrix-core row tile
constexpr int kHalves = kS / kHalf;
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
// each row tile of the block (8 waves) runs one 16-column tile of a
// 128-wide layer per wave for its kHalf samples (a block of 32 samples in
// two row tiles of 1024 threads measured slower: 43.5 against 35.8 us per
// gradient step, half the compute units idle)
static_assert(kH / 16 * kHalves == kWaves, "tile per wave");
constexpr size_t kMlpLds = sizeof(float) * (kS * kIn + 6 * kS * kH);
// parameter layout (row-major W[out][in]):
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH, kParams = ob4 + 1;
static_assert(kParams == 33793, "parameter count");
// partial gradients of the blocks are kPartStride floats apart (16-byte aligned)
constexpr int kPartStride = (kParams + 3) / 4 * 4;

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = expf(-0.5f * z * z) * 0.39894228040143268f;
    return cdf + z * pdf;
}

// Input encoding: (ln c1 / ln 20, ln c2 / ln 20, (m - 5) / 3, r - 4).
__device__ __forceinline__ void encode(const double* c1, const double* c2, const int* m, const int* r, int q,
                                       float* f) {
    const double ln20 = 2.995732273553991;
    f[0] = (float)(log(c1[q]) / ln20);
    f[1] = c2 != nullptr ? (float)(log(c2[q]) / ln20) : 0.0f;
    f[2] = (float)((m[q] - 5) / 3.0);
    f[3] = (float)(r[q] - 4);
}

struct MlpData {
    const double* c1;
    const double* c2;
    const int* m;
    const int* r;
    const float* target;   // training only
    const int* idx;        // sample indices of this batch (NULL: 0..n-1)
    int n;                 // samples in this launch
    float inv_batch2;      // 2 / batch
};

// The 128-wide products of a block's samples run on the float32
// matrix cores (v_mfma_f32_16x16x4_f32: a 16 x 16 tile of D += A (16 x 4)
// B (4 x 16) per instruction).  Operand layout of one instruction: lane l
// gives A[row l % 16][k-slot l / 16] and B[k-slot l / 16][col l % 16]; the
// result tile has lane l holding rows 4 (l / 16) + r, r = 0..3, of column
// l % 16.  Instruction t of a 128-long contraction gives k-slot q the index
// k = 32 q + t, so that every lane reads 32 consecutive values of its row.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// The weight operands a lane needs for its tile, loaded at the start of the
// kernel so that their latency overlaps the layers before them:
//   rows: W[j0 + l % 16][32 q .. 32 q + 31] (Z = A W^T), q = l / 16
//   cols: W[32 q .. 32 q + 31][i0 + l % 16] (dH = D W)
struct WRows {
    float4 v[8];
};
struct WCols {
    float v[32];
};
__device__ __forceinline__ WRows load_rows(const float* __restrict__ W, int j0) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const float4* wr = reinterpret_cast<const float4*>(W + (size_t)(j0 + c) * kH + 32 * q);
    WRows r;
#pragma unroll
    for (int u = 0; u < 8; ++u) r.v[u] = wr[u];
    return r;
}
__device__ __forceinline__ WCols load_cols(const float* __restrict__ W, int i0) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const float* wc = W + (size_t)(32 * q) * kH + i0 + c;
    WCols r;
#pragma unroll
    for (int t = 0; t < 32; ++t) r.v[t] = wc[(size_t)t * kH];
    return r;
}

// Z[s][j] = sum_k A[s][k] W[j][k] for the lane's 16-column tile (A in LDS,
// the W operand preloaded).  Returns the lane's four entries (rows
// 4 (l / 16) + r of column j0 + l % 16).
__device__ __forceinline__ f32x4 mm_rows_w(const float (*A)[kH], const WRows& w) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const float4* ar = reinterpret_cast<const float4*>(&A[c][32 * q]);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float4 av = ar[u];
        acc = mfma16(av.x, w.v[u].x, acc);
        acc = mfma16(av.y, w.v[u].y, acc);
        acc = mfma16(av.z, w.v[u].z, acc);
        acc = mfma16(av.w, w.v[u].w, acc);
    }
    return acc;
}

// dH[s][i] = sum_j D[s][j] W[j][i] for the lane's 16-column tile (the
// columns of W preloaded).
__device__ __forceinline__ f32x4 mm_rows_wt(const float (*D)[kH], const WCols& w) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const float4* dr = reinterpret_cast<const float4*>(&D[c][32 * q]);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float4 dv = dr[u];
        acc = mfma16(dv.x, w.v[4 * u + 0], acc);
        acc = mfma16(dv.y, w.v[4 * u + 1], acc);
        acc = mfma16(dv.z, w.v[4 * u + 2], acc);
        acc = mfma16(dv.w, w.v[4 * u + 3], acc);
    }
    return acc;
}

// dW[j][i] = sum_s D[s][j] H[s][i] over the block's kS samples for the
// tile j0 .. j0+15 x i0 .. i0+15 (kS / 4 instructions, k-slot q of
// instruction t holds sample 4 t + q), written to the partial gradient gW
// (row-major [j][i], pitch kH).
__device__ __forceinline__ void mm_dw(const float (*D)[kH], const float (*H)[kH], int j0, int i0,
                                      float* __restrict__ gW) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < kS / 4; ++t) acc = mfma16(D[4 * t + q][j0 + c], H[4 * t + q][i0 + c], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) gW[(size_t)(j0 + 4 * q + r) * kH + i0 + c] = acc[r];
}

// One hidden layer forward: Z = A W^T + b on the matrix cores (in each half
// of the block, for its kHalf samples, wave w of the half takes the column
// tile w; bj: the bias of the lane's column), then H = gelu(Z) and
// G = gelu'(Z) to LDS.
__device__ __forceinline__ void dense_layer(const float (*A)[kH], const WRows& W, float bj, float (*H)[kH],
                                            float (*G)[kH]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int half = wave / (kH / 16), r0 = half * kHalf;     // this half's sample rows
    A += r0;
    H += r0;
    G += r0;
    {
        const int j0 = (wave % (kH / 16)) * 16;
        const f32x4 z = mm_rows_w(A, W);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float zz = z[r] + bj;
            H[4 * q + r][j0 + c] = gelu_f(zz);
            G[4 * q + r][j0 + c] = gelu_grad_f(zz);
        }
    }
}

// One hidden layer backward: from D = dL/dZ of the layer's output (LDS),
// writes dW = D^T Hin and db = sum_s D to the partial gradient, and replaces
// Gin (gelu'(Zin)) by dL/dZin = (D W) * gelu'(Zin).
__device__ __forceinline__ void backprop_hidden(const float (*D)[kH], const float (*Hin)[kH], float (*Gin)[kH],
                                                const WCols& W, float* __restrict__ gW, float* __restrict__ gb) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
    const int half = wave / (kH / 16), w8 = wave % (kH / 16);
    // dW over all kS samples: wave w of row tile h takes the row tile w of
    // dW and its share of the column tiles
    constexpr int kColTiles = kH / 16 / kHalves;
#pragma unroll
    for (int it = 0; it < kColTiles; ++it) mm_dw(D, Hin, w8 * 16, (half * kColTiles + it) * 16, gW);
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kS; ++s) a += D[s][tid];
        gb[tid] = a;
    }
    // dL/dZin = (D W) * gelu'(Zin) for this half's samples, in place over
    // Gin (read only by this lane)
    {
        const int i0 = w8 * 16, r0 = half * kHalf;
        const f32x4 dh = mm_rows_wt(D + r0, W);
#pragma unroll
        for (int r = 0; r < 4; ++r) Gin[r0 + 4 * q + r][i0 + c] *= dh[r];
    }
    __syncthreads();
}

// A block takes kS samples: forward pass with all activations in LDS (H_l
// and gelu'(Z_l) per layer) and, for training, the backward pass, writing
// its partial gradient (one full parameter vector) and its loss sum.
__global__ __launch_bounds__(kThreads) void mlp_fwd_bwd_kernel(const float* __restrict__ P, MlpData d, int train,
                                                               float* __restrict__ part,
                                                               float* __restrict__ part_loss,
                                                               float* __restrict__ pred) {
    extern __shared__ __attribute__((aligned(16))) float mlp_lds[];
    float (*X)[kIn] = reinterpret_cast<float (*)[kIn]>(mlp_lds);
    float (*H1)[kH] = reinterpret_cast<float (*)[kH]>(mlp_lds + kS * kIn);
    float (*H2)[kH] = H1 + kS;
    float (*H3)[kH] = H2 + kS;
    float (*G1)[kH] = H3 + kS;
    float (*G2)[kH] = G1 + kS;
    float (*G3)[kH] = G2 + kS;
    __shared__ float OUT[kS], DOUT[kS], TGT[kS], W4s[kH];
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * kS;
    const int ns = min(kS, d.n - s0);
    // every weight operand of this wave's tiles and every small parameter,
    // loaded up front so that their latency overlaps the layers before them
    const int tile0 = ((tid >> 6) % (kH / 16)) * 16, lc = tid & 15;
    const WRows w2r = load_rows(P + oW2, tile0), w3r = load_rows(P + oW3, tile0);
    WCols w3c, w2c;
    if (train) {
        w3c = load_cols(P + oW3, tile0);
        w2c = load_cols(P + oW2, tile0);
    }
    const int j1 = tid & (kH - 1);
    const float4 w1v = *reinterpret_cast<const float4*>(P + oW1 + j1 * kIn);
    const float b1v = P[ob1 + j1], b2v = P[ob2 + tile0 + lc], b3v = P[ob3 + tile0 + lc], b4v = P[ob4];
    if (tid < kH) W4s[tid] = P[oW4 + tid];
    if (tid < kS) {
        float f[kIn] = {0.0f, 0.0f, 0.0f, 0.0f};
        float tg = 0.0f;
        if (tid < ns) {
            const int q = d.idx ? d.idx[s0 + tid] : s0 + tid;
            if (train) tg = d.target[q];
            encode(d.c1, d.c2, d.m, d.r, q, f);
        }
        TGT[tid] = tg;
#pragma unroll
        for (int k = 0; k < kIn; ++k) X[tid][k] = f[k];
    }
    __syncthreads();
    // layer 1 (4 -> 128) on the vector units
    {
        const int j = j1, part0 = tid / kH;
        const float w0 = w1v.x, w1 = w1v.y, w2 = w1v.z, w3 = w1v.w, bj = b1v;
        for (int s = part0; s < kS; s += kThreads / kH) {
            float a = fmaf(w0, X[s][0], 0.0f);
            a = fmaf(w1, X[s][1], a);
            a = fmaf(w2, X[s][2], a);
            a = fmaf(w3, X[s][3], a);
            a += bj;
            H1[s][j] = gelu_f(a);
            G1[s][j] = gelu_grad_f(a);
        }
    }
    __syncthreads();
    dense_layer(H1, w2r, b2v, H2, G2);
    __syncthreads();
    dense_layer(H2, w3r, b3v, H3, G3);
    __syncthreads();
    if (tid < kS) {
        float a = 0.0f;
        for (int i = 0; i < kH; ++i) a = fmaf(W4s[i], H3[tid][i], a);
        a += b4v;
        OUT[tid] = a;
        if (tid < ns) {
            if (pred) pred[s0 + tid] = a;
            if (train) DOUT[tid] = d.inv_batch2 * (a - TGT[tid]);
        } else {
            DOUT[tid] = 0.0f;
        }
    }
    __syncthreads();
    if (!train) return;
    float* g = part + (size_t)blockIdx.x * kPartStride;
    if (tid == 0) {
        float l = 0.0f, db = 0.0f;
        for (int s = 0; s < ns; ++s) {
            const float e = OUT[s] - TGT[s];
            l = fmaf(e, e, l);
            db += DOUT[s];
        }
        part_loss[blockIdx.x] = l;
        g[ob4] = db;
    }
    // output layer: dW4; then dL/dZ3 = DOUT W4 gelu'(Z3) in place over G3
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kS; ++s) a = fmaf(DOUT[s], H3[s][tid], a);
        g[oW4 + tid] = a;
    }
    for (int q = tid; q < kS * kH; q += kThreads) {
        const int s = q / kH, i = q % kH;
        G3[s][i] = DOUT[s] * W4s[i] * G3[s][i];
    }
    __syncthreads();
    // hidden layers 3 and 2: dW = dZ^T H_in, db = sum dZ, dZ_in = (dZ W) gelu'(Z_in)
    backprop_hidden(G3, H2, G2, w3c, g + oW3, g + ob3);
    backprop_hidden(G2, H1, G1, w2c, g + oW2, g + ob2);
    // first layer: dW1[j][k] = sum_s dZ1[s][j] X[s][k], db1
    if (tid < kH) {
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, b = 0.0f;
        for (int s = 0; s < kS; ++s) {
            const float dz = G1[s][tid];
            a0 = fmaf(dz, X[s][0], a0);
            a1 = fmaf(dz, X[s][1], a1);
            a2 = fmaf(dz, X[s][2], a2);
            a3 = fmaf(dz, X[s][3], a3);
            b += dz;
        }
        g[oW1 + tid * kIn + 0] = a0;
        g[oW1 + tid * kIn + 1] = a1;
        g[oW1 + tid * kIn + 2] = a2;
        g[oW1 + tid * kIn + 3] = a3;
        g[ob1 + tid] = b;
    }
}

// Sum of the block partials -> Adam update or plain gradient.  A block takes
// kRedParams parameters; its thread (group g, quad u) adds parameters
// 4u .. 4u+3 of every kRedGroups-th partial (g, g + kRedGroups, ...) with
// 16-byte loads, eight in flight, and the group sums are added in group
// order, so the result is fixed for a given number of partials.
constexpr int kRedParams = 64;
constexpr int kRedGroups = 256 / (kRedParams / 4);

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part, int nblk,
                                                         float* __restrict__ P, float* __restrict__ adam,
                                                         float* __restrict__ grad_out, float lr, float b1, float b2,
                                                         float eps, float bc1, float bc2,
                                                         const float* __restrict__ part_loss, float inv_batch,
                                                         float* __restrict__ loss_out) {
    __shared__ float gs[kRedGroups][kRedParams];
    const int quad = threadIdx.x % (kRedParams / 4), grp = threadIdx.x / (kRedParams / 4);
    const int p4 = blockIdx.x * kRedParams + 4 * quad;        // first of the thread's four parameters
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss_out) {
        float l = 0.0f;
        int b = 0;
        for (; b + 8 <= nblk; b += 8) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = part_loss[b + i];
#pragma unroll
            for (int i = 0; i < 8; ++i) l += v[i];
        }
        for (; b < nblk; ++b) l += part_loss[b];
        *loss_out = l * inv_batch;
    }
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (p4 < kParams) {
        int b = grp;
        for (; b + 7 * kRedGroups < nblk; b += 8 * kRedGroups) {
            float4 v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                v[i] = *reinterpret_cast<const float4*>(part + (size_t)(b + i * kRedGroups) * kPartStride + p4);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                acc.x += v[i].x;
                acc.y += v[i].y;
                acc.z += v[i].z;
                acc.w += v[i].w;
            }
        }
        for (; b < nblk; b += kRedGroups) {
            const float4 v = *reinterpret_cast<const float4*>(part + (size_t)b * kPartStride + p4);
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    gs[grp][4 * quad + 0] = acc.x;
    gs[grp][4 * quad + 1] = acc.y;
    gs[grp][4 * quad + 2] = acc.z;
    gs[grp][4 * quad + 3] = acc.w;
    __syncthreads();
    const int pl = threadIdx.x, p = blockIdx.x * kRedParams + pl;
    if (pl >= kRedParams || p >= kParams) return;
    float gsum = gs[0][pl];
#pragma unroll
    for (int g = 1; g < kRedGroups; ++g) gsum += gs[g][pl];
    if (grad_out) {
        grad_out[p] = gsum;
        return;
    }
    float m = adam[p], v = adam[kParams + p];
    m = b1 * m + (1.0f - b1) * gsum;
    v = b2 * v + (1.0f - b2) * gsum * gsum;
    adam[p] = m;
    adam[kParams + p] = v;
    const float mh = m / bc1, vh = v / bc2;
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// k smallest entries of v (k <= 64), ascending, ties to the smaller index;
// NaN entries are never chosen and missing ranks are -1.  The winners come
// out in increasing (value, index) order, so each round takes the smallest
// (value, index) pair after the previous round's winner.
__global__ __launch_bounds__(1024) void topk_min_kernel(const float* __restrict__ v, int n, int k,
                                                        int* __restrict__ idx_out) {
    __shared__ float sv[1024];
    __shared__ int si[1024];
    const int tid = threadIdx.x;
    float pv = -INFINITY;                  // previous winner
    int pi = -1;
    for (int round = 0; round < k; ++round) {
        float best = INFINITY;
        int bi = 0x7fffffff;
        for (int q = tid; q < n; q += 1024) {
            const float x = v[q];
            const bool after = x > pv || (x == pv && q > pi);
            if (!(x != x) && after && (x < best || (x == best && q < bi))) {
                best = x;
                bi = q;
            }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int st = 512; st > 0; st >>= 1) {
            if (tid < st) {
                const float o = sv[tid + st];
                const int oi = si[tid + st];
                if (o < sv[tid] || (o == sv[tid] && oi < si[tid])) {
                    sv[tid] = o;
                    si[tid] = oi;
                }
            }
            __syncthreads();
        }
        pv = sv[0];
        pi = si[0];
        if (tid == 0) idx_out[round] = pi == 0x7fffffff ? -1 : pi;
        __syncthreads();                   // sv, si are rewritten next round
    }
}

struct Mlp {
    int max_batch = 0;
    float* part = nullptr;
    float* part_loss = nullptr;
};

// The forward/backward kernel takes more than 64 KB of LDS: raise its limit
// once (gfx950 has 160 KB per compute unit).
static int fwd_bwd_lds_once() {
    static const int st = hip_check((int)hipFuncSetAttribute(reinterpret_cast<const void*>(mlp_fwd_bwd_kernel),
                                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                                             (int)kMlpLds),
                                    "hipFuncSetAttribute");
    return st;
}

static int launch_fwd_bwd(const float* P, const MlpData& d, int train, float* part, float* part_loss, float* pred,
                          hipStream_t s) {
    const int st = fwd_bwd_lds_once();
    if (st != WG_OK) return st;
    const int nblk = (d.n + kS - 1) / kS;
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(nblk), dim3(kThreads), kMlpLds, s, P, d, train, part, part_loss,
                       pred);
    return hip_check((int)hipGetLastError(), "mlp_fwd_bwd_kernel");
}

static int launch_step(Mlp& M, const float* P, const MlpData& d, int train, float* pred, hipStream_t s) {
    return launch_fwd_bwd(P, d, train, M.part, M.part_loss, pred, s);
}

}  // namespace wg

using namespace wg;

extern "C" {

int wg_mlp_param_count(void) { return kParams; }

int wg_mlp_create(wg_mlp** out, int max_batch) {
    if (!out || max_batch <= 0) return fail(WG_EINVAL, "wg_mlp_create: bad arguments");
    Mlp* M = new (std::nothrow) Mlp();
    if (!M) return fail(WG_ENOMEM, "wg_mlp_create: out of host memory");
    M->max_batch = max_batch;
    const size_t nblk = (size_t)(max_batch + kS - 1) / kS;
    if (hipMalloc((void**)&M->part, sizeof(float) * nblk * kPartStride) != hipSuccess ||
        hipMalloc((void**)&M->part_loss, sizeof(float) * nblk) != hipSuccess) {
        if (M->part) (void)hipFree(M->part);
        delete M;
        return fail(WG_ENOMEM, "wg_mlp_create: device allocation failed");
    }
    *out = reinterpret_cast<wg_mlp*>(M);
    return WG_OK;
}

int wg_mlp_destroy(wg_mlp* mlp) {
    Mlp* M = reinterpret_cast<Mlp*>(mlp);
    if (!M) return WG_OK;
    if (M->part) (void)hipFree(M->part);
    if (M->part_loss) (void)hipFree(M->part_loss);
    delete M;
    return WG_OK;
}

static int check_data(const double* c1, const int* m, const int* r, int n) {
    if (!c1 || !m || !r) return fail(WG_EINVAL, "mlp: null data pointer");
    if (n <= 0) return fail(WG_EINVAL, "mlp: n must be positive");
    return WG_OK;
}

int wg_mlp_gradient(wg_mlp* mlp, const float* params, const double* c1, const double* c2, const int* m,
                    const int* r, const float* target, int n, float* grad_out, float* loss_out,
                    wg_stream_t stream) {
    if (!mlp || !params || !target || !grad_out) return fail(WG_EINVAL, "wg_mlp_gradient: null pointer");
    Mlp& M = *reinterpret_cast<Mlp*>(mlp);
    int st = check_data(c1, m, r, n);
    if (st != WG_OK) return st;
    if (n > M.max_batch) return fail(WG_EINVAL, "wg_mlp_gradient: n exceeds max_batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MlpData d{c1, c2, m, r, target, nullptr, n, 2.0f / n};
    st = launch_step(M, params, d, 1, nullptr, s);
    if (st != WG_OK) return st;
    const int nblk = (n + kS - 1) / kS;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + kRedParams - 1) / kRedParams), dim3(256), 0, s, M.part,
                       nblk, nullptr,
                       nullptr, grad_out, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f, M.part_loss, 1.0f / n, loss_out);
    return hip_check((int)hipGetLastError(), "mlp_reduce_kernel");
}

int wg_mlp_train(wg_mlp* mlp, float* params, float* adam_state, int step0, float lr, const double* c1,
                 const double* c2, const int* m, const int* r, const float* target, int n, const int* perm,
                 int epochs, int batch, float* losses, wg_stream_t stream) {
    if (!mlp || !params || !adam_state || !target || !perm || !losses)
        return fail(WG_EINVAL, "wg_mlp_train: null pointer");
    Mlp& M = *reinterpret_cast<Mlp*>(mlp);
    int st = check_data(c1, m, r, n);
    if (st != WG_OK) return st;
    if (batch <= 0 || batch > M.max_batch || batch > n || epochs <= 0 || step0 < 1 || !(lr > 0.0f))
        return fail(WG_EINVAL, "wg_mlp_train: bad batch, epochs, step0 or lr");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int steps = n / batch;                      // the tail of each permutation is dropped
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int t = step0;
    for (int e = 0; e < epochs; ++e) {
        for (int b = 0; b < steps; ++b, ++t) {
            const MlpData d{c1, c2, m, r, target, perm + (size_t)e * n + (size_t)b * batch, batch, 2.0f / batch};
            st = launch_step(M, params, d, 1, nullptr, s);
            if (st != WG_OK) return st;
            const float bc1 = 1.0f - powf(b1, (float)t), bc2 = 1.0f - powf(b2, (float)t);
            hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + kRedParams - 1) / kRedParams), dim3(256), 0, s,
                               M.part,
                               (batch + kS - 1) / kS, params, adam_state, nullptr, lr, b1, b2, eps, bc1, bc2,
                               M.part_loss, 1.0f / batch, losses + (size_t)e * steps + b);
            st = hip_check((int)hipGetLastError(), "mlp_reduce_kernel");
            if (st != WG_OK) return st;
        }
    }
    return WG_OK;
}

int wg_mlp_predict(const float* params, const double* c1, const double* c2, const int* m, const int* r, int n,
                   float* out, wg_stream_t stream) {
    if (!params || !out) return fail(WG_EINVAL, "wg_mlp_predict: null pointer");
    int st = check_data(c1, m, r, n);
    if (st != WG_OK) return st;
    const MlpData d{c1, c2, m, r, nullptr, nullptr, n, 0.0f};
    return launch_fwd_bwd(params, d, 0, nullptr, nullptr, out, static_cast<hipStream_t>(stream));
}

int wg_topk_min(const float* v, int n, int k, int* idx_out, wg_stream_t stream) {
    if (!v || !idx_out || n <= 0 || k <= 0 || k > 64) return fail(WG_EINVAL, "wg_topk_min: bad arguments");
    hipLaunchKernelGGL(topk_min_kernel, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), v, n, k, idx_out);
    return hip_check((int)hipGetLastError(), "topk_min_kernel");
}

}  // extern "C"
