// Error surrogate: a small fully connected network (4 -> 128 -> 128 -> 128
// -> 1, GELU) trained on sweep errors and used to propose point-family
// parameters.  The paper observes that the error curve over c is smooth
// enough to localise good values (arXiv:2201.10369, Sections 1, 5 and 6.1);
// the network interpolates that curve across parameters and tile sizes so
// that only its best proposals need an exact sweep evaluation.
//
// Kernels (float32, fixed reduction orders):
//   encode  : once per pass over the data, the input features and targets
//             of the samples in minibatch order, so that a training step
//             reads its samples with one contiguous load
//   fwd_bwd : a block takes 16 samples: forward pass with all activations
//             in LDS, the output layer and, for training, the backward pass
//             down to dL/dZ1 (the 128 x 128 products on the float32 matrix
//             cores).  It writes H1, H2, dL/dZ2 and dL/dZ3 of its samples
//             (the operands of the two 128 x 128 weight gradients) and its
//             partial sums of the small gradients (W1, b1, b2, b3, W4, b4)
//             and of the loss
//   wgrad   : the weight gradients dW = dZ^T H of the two 128 x 128 layers
//             on the matrix cores, a block per 32 x 32 parameter tile and
//             slice of the batch; the small gradients summed over the
//             fwd_bwd blocks in a fixed order and their parameters updated
//   wadam   : the slice sums of dW2 and dW3 added in order, then Adam (or
//             the plain gradient) on those parameters
//   predict : the forward part of fwd_bwd
//   topk    : the k smallest values of a vector (ties -> smaller index)
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "wg_device.h"
#include "wg_internal.h"

namespace wg {

constexpr int kIn = 4, kH = 128;
constexpr int kS = 16;            // samples per fwd_bwd block: one matrix-core row tile
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
// wave w takes the 16-column tile w of each 128-wide layer (a block of 32
// samples in two row tiles of 1024 threads measured slower: with 4096
// samples only half the compute units get a block)
static_assert(kH / 16 == kWaves, "one column tile per wave");
// LDS row pitch of the activations: rows 4 floats apart in the bank map, so
// that the 16 rows a matrix-core operand load reads do not collide
constexpr int kP = kH + 4;
constexpr size_t kMlpLds = sizeof(float) * (kS * kIn + 6 * kS * kP);
// parameter layout (row-major W[out][in]):
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH, kParams = ob4 + 1;
static_assert(kParams == 33793, "parameter count");
// Per fwd_bwd block, the partial sums of the small gradients and of the
// loss, kSmallStride floats apart (16-byte aligned):
constexpr int sW1 = 0, sb1 = sW1 + kH * kIn, sb2 = sb1 + kH, sb3 = sb2 + kH, sW4 = sb3 + kH, sb4 = sW4 + kH,
              sLoss = sb4 + 1, kSmall = sLoss + 1;
constexpr int kSmallStride = (kSmall + 3) / 4 * 4;
__device__ __forceinline__ int small_param(int k) {
    return k < sb1 ? oW1 + k
         : k < sb2 ? ob1 + (k - sb1)
         : k < sb3 ? ob2 + (k - sb2)
         : k < sW4 ? ob3 + (k - sb3)
         : k < sb4 ? oW4 + (k - sW4)
                   : ob4;
}
// Weight gradients of W2 and W3: 32 x 32 tiles, the batch cut into at most
// kMaxSlices slices of consecutive fwd_bwd blocks, a block per (tile,
// slice); the slice sums go to a [slice][kBig] buffer and a last launch adds
// them in slice order.
constexpr int kTile = 32, kTilesPerMat = (kH / kTile) * (kH / kTile), kTiles = 2 * kTilesPerMat;
constexpr int kMaxSlices = kXcdCount;
constexpr int kBig = 2 * kH * kH;            // W2 then W3
constexpr int kUpdThreads = 512;
constexpr int kUpdWaves = kUpdThreads / 64;
constexpr int kUpdDepth = 4;       // fwd_bwd blocks whose operands a wave keeps in flight
constexpr int kSmallPerBlock = 64;
constexpr int kSmallBlocks = (kSmall + kSmallPerBlock - 1) / kSmallPerBlock;
constexpr int kRedGroups = kUpdThreads / (kSmallPerBlock / 4);
constexpr int kAdamThreads = 256;

// GELU h = z Phi(z) and its derivative g = Phi(z) + z phi(z), from one
// exponential e = exp(-z^2 / 2).  The normal tail 1 - Phi(|z|) =
// erfc(|z| / sqrt 2) / 2 uses the rational approximation of Abramowitz and
// Stegun (Handbook of Mathematical Functions, 7.1.26: erfc(x) ~
// (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x), x >= 0, absolute error
// at most 1.5e-7), which shares that exponential and has no cancellation for
// z < 0.
__device__ __forceinline__ void gelu_parts(float z, float& h, float& g, bool grad) {
    const float p = 0.3275911f, a1 = 0.254829592f, a2 = -0.284496736f, a3 = 1.421413741f, a4 = -1.453152027f,
                a5 = 1.061405429f;
    const float e = __expf(-0.5f * z * z);
    const float t = __builtin_amdgcn_rcpf(fmaf(p * 0.70710678118654752f, fabsf(z), 1.0f));
    const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, a5, a4), a3), a2), a1);
    const float tail = 0.5f * poly * e;                      // 1 - Phi(|z|)
    const float cdf = z >= 0.0f ? 1.0f - tail : tail;
    h = z * cdf;
    if (grad) g = fmaf(z * e, 0.39894228040143268f, cdf);
}
__device__ __forceinline__ float gelu_f(float z) {
    float h, g;
    gelu_parts(z, h, g, false);
    return h;
}
__device__ __forceinline__ void gelu_and_grad(float z, float& h, float& g) { gelu_parts(z, h, g, true); }

// Input encoding: (ln c1 / ln 20, ln c2 / ln 20, (m - 5) / 3, r - 4).
__device__ __forceinline__ float4 encode(const double* c1, const double* c2, const int* m, const int* r, int q) {
    const double ln20 = 2.995732273553991;
    return make_float4((float)(log(c1[q]) / ln20), c2 != nullptr ? (float)(log(c2[q]) / ln20) : 0.0f,
                       (float)((m[q] - 5) / 3.0), (float)(r[q] - 4));
}

struct MlpData {
    const double* c1;
    const double* c2;
    const int* m;
    const int* r;
    const float* target;   // training with inline features only
    const float4* xe;      // encoded features of this launch's samples (NULL: encode from c1 .. r)
    const float* te;       // and their targets
    int n;                 // samples in this launch
    float inv_batch2;      // 2 / batch
};

// The per-sample operands of the two 128 x 128 weight gradients, written by
// fwd_bwd: per array, per fwd_bwd block b, a [kH][kS] slab (unit-major, the
// block's 16 samples contiguous) at offset b * kH * kS.
struct Acts {
    float* h1;   // H1 (input of layer 2)
    float* h2;   // H2 (input of layer 3)
    float* d2;   // dL/dZ2
    float* d3;   // dL/dZ3
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

// A float4 to a slab read by the next launch: a streaming store, so that the
// end of the launch has little left to write back from L2 (measured: the
// fwd_bwd launch about 4 us shorter than with ordinary stores).
__device__ __forceinline__ void slab_store(float* p, float4 v) {
    const f32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(p));
}

// Block barrier for LDS traffic: waits for this wave's LDS operations only,
// not for its global loads and stores, so that the weight operands stay in
// flight across the forward layers (the waves of a fwd_bwd block exchange
// data through LDS only; __syncthreads would wait for every outstanding
// global access).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// The weight operands a lane needs for its tile, loaded once per block:
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
// the W operand preloaded), in two accumulators (the instructions alternate
// between them in groups of four) added at the end.  Returns the lane's four
// entries (rows 4 (l / 16) + r of column j0 + l % 16).
__device__ __forceinline__ f32x4 mm_rows_w(const float (*A)[kP], const WRows& w) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const float4* ar = reinterpret_cast<const float4*>(&A[c][32 * q]);
    f32x4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float4 av = ar[u];
        acc[u & 1] = mfma16(av.x, w.v[u].x, acc[u & 1]);
        acc[u & 1] = mfma16(av.y, w.v[u].y, acc[u & 1]);
        acc[u & 1] = mfma16(av.z, w.v[u].z, acc[u & 1]);
        acc[u & 1] = mfma16(av.w, w.v[u].w, acc[u & 1]);
    }
    return acc[0] + acc[1];
}

// dH[s][i] = sum_j D[s][j] W[j][i] for the lane's 16-column tile (the
// columns of W preloaded), in two accumulators as above.
__device__ __forceinline__ f32x4 mm_rows_wt(const float (*D)[kP], const WCols& w) {
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const float4* dr = reinterpret_cast<const float4*>(&D[c][32 * q]);
    f32x4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float4 dv = dr[u];
        acc[u & 1] = mfma16(dv.x, w.v[4 * u + 0], acc[u & 1]);
        acc[u & 1] = mfma16(dv.y, w.v[4 * u + 1], acc[u & 1]);
        acc[u & 1] = mfma16(dv.z, w.v[4 * u + 2], acc[u & 1]);
        acc[u & 1] = mfma16(dv.w, w.v[4 * u + 3], acc[u & 1]);
    }
    return acc[0] + acc[1];
}

// One hidden layer forward: Z = A W^T + b on the matrix cores (wave w takes
// the column tile w for all kS samples; bj: the bias of the lane's column),
// then H = gelu(Z) and, for training, G = gelu'(Z) to LDS and H to the
// block's slab hg (when not NULL).
__device__ __forceinline__ void dense_layer(const float (*A)[kP], const WRows& W, float bj, float (*H)[kP],
                                            float (*G)[kP], int train, float* __restrict__ hg) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int j0 = wave * 16;
    const f32x4 z = mm_rows_w(A, W);
    float h[4];
    if (train) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float g;
            gelu_and_grad(z[r] + bj, h[r], g);
            H[4 * q + r][j0 + c] = h[r];
            G[4 * q + r][j0 + c] = g;
        }
        if (hg) slab_store(hg + (size_t)(j0 + c) * kS + 4 * q, make_float4(h[0], h[1], h[2], h[3]));
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) H[4 * q + r][j0 + c] = gelu_f(z[r] + bj);
    }
}

// One hidden layer backward: from D = dL/dZ of the layer's output (LDS),
// writes db = sum_s D to the block's small partials and replaces Gin
// (gelu'(Zin)) by dL/dZin = (D W) * gelu'(Zin), also to the block's slab dg
// (when not NULL).
__device__ __forceinline__ void backprop_hidden(const float (*D)[kP], float (*Gin)[kP], const WCols& W,
                                                float* __restrict__ gb, float* __restrict__ dg) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kS; ++s) a += D[s][tid];
        gb[tid] = a;
    }
    const int i0 = wave * 16;
    const f32x4 dh = mm_rows_wt(D, W);
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v[r] = Gin[4 * q + r][i0 + c] * dh[r];
        Gin[4 * q + r][i0 + c] = v[r];
    }
    if (dg) slab_store(dg + (size_t)(i0 + c) * kS + 4 * q, make_float4(v[0], v[1], v[2], v[3]));
    lds_barrier();
}

// A block takes kS samples: forward pass with all activations in LDS (H_l
// and, for training, gelu'(Z_l) per layer) and, for training, the backward
// pass (see the file comment for what it writes).
__global__ __launch_bounds__(kThreads) void mlp_fwd_bwd_kernel(const float* __restrict__ P, MlpData d, int train,
                                                               Acts act, float* __restrict__ small,
                                                               float* __restrict__ pred) {
    extern __shared__ __attribute__((aligned(16))) float mlp_lds[];
    float (*X)[kIn] = reinterpret_cast<float (*)[kIn]>(mlp_lds);
    float (*H1)[kP] = reinterpret_cast<float (*)[kP]>(mlp_lds + kS * kIn);
    float (*H2)[kP] = H1 + kS;
    float (*H3)[kP] = H2 + kS;
    float (*G1)[kP] = H3 + kS;
    float (*G2)[kP] = G1 + kS;
    float (*G3)[kP] = G2 + kS;
    __shared__ float OUT[kS], DOUT[kS], TGT[kS], W4s[kH];
    const int tid = threadIdx.x, wave = tid >> 6;
    const int blk = blockIdx.x, s0 = blk * kS;
    const int ns = min(kS, d.n - s0);
    // layer 1: thread (unit j1, samples 4 p1 .. 4 p1 + 3)
    const int j1 = tid & (kH - 1), p1 = tid / kH;
    const float4 w1v = *reinterpret_cast<const float4*>(P + oW1 + j1 * kIn);
    const float b1v = P[ob1 + j1];
    // the small parameters and the samples, all in flight together before
    // the first barrier (the weight operands follow it)
    const int t0 = wave * 16, lc = tid & 15;
    const float b2v = P[ob2 + t0 + lc], b3v = P[ob3 + t0 + lc], b4v = P[ob4];
    const float w4v = P[oW4 + j1];
    float4 f = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float tg = 0.0f;
    if (tid < ns) {
        if (d.xe) {
            f = d.xe[s0 + tid];
            if (train) tg = d.te[s0 + tid];
        } else {
            f = encode(d.c1, d.c2, d.m, d.r, s0 + tid);
            if (train) tg = d.target[s0 + tid];
        }
    }
    if (tid < kS) {
        TGT[tid] = tg;
        X[tid][0] = f.x;
        X[tid][1] = f.y;
        X[tid][2] = f.z;
        X[tid][3] = f.w;
    }
    if (tid < kH) W4s[tid] = w4v;
    lds_barrier();
    // the weight operands of this wave's tiles, each issued one layer
    // before its use (loads complete in issue order, and a wave keeps at most
    // 63 in flight)
    const WRows w2r = load_rows(P + oW2, t0);
    const size_t slab = (size_t)blk * kH * kS;
    // layer 1 (4 -> 128) on the vector units
    {
        float h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int s = 4 * p1 + k;
            float a = fmaf(w1v.x, X[s][0], 0.0f);
            a = fmaf(w1v.y, X[s][1], a);
            a = fmaf(w1v.z, X[s][2], a);
            a = fmaf(w1v.w, X[s][3], a);
            a += b1v;
            if (train) {
                float g;
                gelu_and_grad(a, h[k], g);
                G1[s][j1] = g;
            } else {
                h[k] = gelu_f(a);
            }
            H1[s][j1] = h[k];
        }
        if (train)
            slab_store(act.h1 + slab + (size_t)j1 * kS + 4 * p1, make_float4(h[0], h[1], h[2], h[3]));
    }
    lds_barrier();
    const WRows w3r = load_rows(P + oW3, t0);
    dense_layer(H1, w2r, b2v, H2, G2, train, train ? act.h2 + slab : nullptr);
    lds_barrier();
    WCols w3c, w2c;
    if (train) w3c = load_cols(P + oW3, t0);
    dense_layer(H2, w3r, b3v, H3, G3, train, nullptr);
    lds_barrier();
    if (train) w2c = load_cols(P + oW2, t0);
    // output layer: 32 threads per sample, a butterfly sum over them
    {
        const int s = tid >> 5, l = tid & 31;
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < kH / 32; ++k) a = fmaf(W4s[l + 32 * k], H3[s][l + 32 * k], a);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) a += __shfl_xor(a, off, 32);
        if (l == 0) {
            a += b4v;
            OUT[s] = a;
            if (s < ns) {
                if (pred) pred[s0 + s] = a;
                DOUT[s] = train ? d.inv_batch2 * (a - TGT[s]) : 0.0f;
            } else {
                DOUT[s] = 0.0f;
            }
        }
    }
    lds_barrier();
    if (!train) return;
    float* sp = small + (size_t)blk * kSmallStride;
    if (tid == 0) {
        float l = 0.0f, db = 0.0f;
        for (int s = 0; s < ns; ++s) {
            const float e = OUT[s] - TGT[s];
            l = fmaf(e, e, l);
            db += DOUT[s];
        }
        sp[sLoss] = l;
        sp[sb4] = db;
        for (int k = kSmall; k < kSmallStride; ++k) sp[k] = 0.0f;
    }
    // output layer: dW4; dL/dZ3 = DOUT W4 gelu'(Z3) in place over G3 and to
    // the block's slab
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kS; ++s) a = fmaf(DOUT[s], H3[s][tid], a);
        sp[sW4 + tid] = a;
    }
    {
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int s = 4 * p1 + k;
            v[k] = DOUT[s] * W4s[j1] * G3[s][j1];
            G3[s][j1] = v[k];
        }
        slab_store(act.d3 + slab + (size_t)j1 * kS + 4 * p1, make_float4(v[0], v[1], v[2], v[3]));
    }
    lds_barrier();
    // hidden layers 3 and 2: db = sum dZ, dZ_in = (dZ W) gelu'(Z_in)
    backprop_hidden(G3, G2, w3c, sp + sb3, act.d2 + slab);
    backprop_hidden(G2, G1, w2c, sp + sb2, nullptr);
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
        sp[sW1 + tid * kIn + 0] = a0;
        sp[sW1 + tid * kIn + 1] = a1;
        sp[sW1 + tid * kIn + 2] = a2;
        sp[sW1 + tid * kIn + 3] = a3;
        sp[sb1 + tid] = b;
    }
}

// Features and targets of `count` samples in the order `order` (entries
// outside [0, n) give NaN features and targets rather than a load).
__global__ __launch_bounds__(256) void mlp_encode_kernel(const double* __restrict__ c1, const double* __restrict__ c2,
                                                         const int* __restrict__ m, const int* __restrict__ r,
                                                         const float* __restrict__ target,
                                                         const int* __restrict__ order, int n, int count,
                                                         float4* __restrict__ xe, float* __restrict__ te) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const int q = order[k];
    if (q < 0 || q >= n) {
        xe[k] = make_float4(NAN, NAN, NAN, NAN);
        te[k] = NAN;
        return;
    }
    xe[k] = encode(c1, c2, m, r, q);
    te[k] = target[q];
}

struct AdamArgs {
    float lr, b1, b2, eps, bc1, bc2;
};

// Adam on parameter p with gradient g (or, with grad_out, the gradient).
__device__ __forceinline__ void apply_grad(int p, float g, float* __restrict__ P, float* __restrict__ adam,
                                           float* __restrict__ grad_out, const AdamArgs& h) {
    if (grad_out) {
        grad_out[p] = g;
        return;
    }
    float m = adam[p], v = adam[kParams + p];
    m = h.b1 * m + (1.0f - h.b1) * g;
    v = h.b2 * v + (1.0f - h.b2) * g * g;
    adam[p] = m;
    adam[kParams + p] = v;
    const float mh = m / h.bc1, vh = v / h.bc2;
    P[p] -= h.lr * mh / (sqrtf(vh) + h.eps);
}

// Gradient sums.  Blocks [0, kTiles * nslice) take a (tile, slice) pair,
// tile = block / nslice, slice = block % nslice (with 8 slices, slice k runs
// on XCD k, whose L2 then holds only that slice's operands): the 32 x 32
// tile of dW2 = dZ2^T H1 or dW3 = dZ3^T H2 over the slice's fwd_bwd blocks
// on the matrix cores, wave w of 8 adding the slice's blocks w, w + 8, ...
// in four 16 x 16 accumulators, the 8 wave sums added in order, to
// slice_part[slice].  Blocks [kTiles * nslice, + kSmallBlocks) take
// kSmallPerBlock entries of the small partials each: thread (group g, quad
// u) adds entries 4u .. 4u+3 of every kRedGroups-th block partial (g,
// g + kRedGroups, ...) with 16-byte loads, eight in flight, the group sums
// are added in group order, and the parameter is updated (or the gradient
// written).  No block reads what another block of the launch writes.
__global__ __launch_bounds__(kUpdThreads) void mlp_wgrad_kernel(Acts act, const float* __restrict__ small, int nblk,
                                                                int nslice, float* __restrict__ slice_part,
                                                                float* __restrict__ P, float* __restrict__ adam,
                                                                float* __restrict__ grad_out, AdamArgs h,
                                                                float inv_batch, float* __restrict__ loss_out) {
    const int tid = threadIdx.x;
    if (blockIdx.x >= kTiles * nslice) {
        __shared__ float gs[kRedGroups][kSmallPerBlock];
        const int sb = blockIdx.x - kTiles * nslice;
        const int quad = tid % (kSmallPerBlock / 4), grp = tid / (kSmallPerBlock / 4);
        const int k4 = sb * kSmallPerBlock + 4 * quad;
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (k4 < kSmallStride) {
            int b = grp;
            for (; b + 7 * kRedGroups < nblk; b += 8 * kRedGroups) {
                float4 v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v[i] = *reinterpret_cast<const float4*>(small + (size_t)(b + i * kRedGroups) * kSmallStride + k4);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    acc.x += v[i].x;
                    acc.y += v[i].y;
                    acc.z += v[i].z;
                    acc.w += v[i].w;
                }
            }
            for (; b < nblk; b += kRedGroups) {
                const float4 v = *reinterpret_cast<const float4*>(small + (size_t)b * kSmallStride + k4);
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
        const int k = sb * kSmallPerBlock + tid;
        if (tid >= kSmallPerBlock || k >= kSmall) return;
        float g = gs[0][tid];
#pragma unroll
        for (int i = 1; i < kRedGroups; ++i) g += gs[i][tid];
        if (k == sLoss) {
            if (loss_out) *loss_out = g * inv_batch;
            return;
        }
        apply_grad(small_param(k), g, P, adam, grad_out, h);
        return;
    }
    __shared__ float red[kUpdWaves][kTile * kTile];
    const int tile = blockIdx.x / nslice, slice = blockIdx.x % nslice;
    const int mat = tile / kTilesPerMat, tj = (tile % kTilesPerMat) / (kH / kTile), ti = tile % (kH / kTile);
    const int j0 = tj * kTile, i0 = ti * kTile;
    const float* __restrict__ D = mat == 0 ? act.d2 : act.d3;
    const float* __restrict__ Hs = mat == 0 ? act.h1 : act.h2;
    const int blo = slice * nblk / nslice, bhi = (slice + 1) * nblk / nslice;
    const int wave = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
    // lane (q, c): the k-slot q of instruction t is sample 4 q + t of the
    // fwd_bwd block; rows j0 + c, j0 + 16 + c of dZ^T, columns i0 + c,
    // i0 + 16 + c of H
    const size_t dro = (size_t)(j0 + c) * kS + 4 * q, hco = (size_t)(i0 + c) * kS + 4 * q;
    constexpr size_t k16 = (size_t)16 * kS;
    f32x4 a00 = {0.0f, 0.0f, 0.0f, 0.0f}, a01 = a00, a10 = a00, a11 = a00;
    // the operands of the wave's next kUpdDepth blocks in flight: each
    // block's loads are issued when the block kUpdDepth before it has been
    // consumed
    float4 da[kUpdDepth], db[kUpdDepth], ha[kUpdDepth], hb[kUpdDepth];
#pragma unroll
    for (int u = 0; u < kUpdDepth; ++u) {
        const int b = blo + wave + u * kUpdWaves;
        if (b < bhi) {
            const float* Db = D + (size_t)b * kH * kS + dro;
            const float* Hb = Hs + (size_t)b * kH * kS + hco;
            da[u] = *reinterpret_cast<const float4*>(Db);
            db[u] = *reinterpret_cast<const float4*>(Db + k16);
            ha[u] = *reinterpret_cast<const float4*>(Hb);
            hb[u] = *reinterpret_cast<const float4*>(Hb + k16);
        }
    }
    for (int i0b = 0; blo + wave + i0b * kUpdWaves < bhi; i0b += kUpdDepth) {
#pragma unroll
        for (int u = 0; u < kUpdDepth; ++u) {
            const int b = blo + wave + (i0b + u) * kUpdWaves;
            if (b < bhi) {
                a00 = mfma16(da[u].x, ha[u].x, a00);
                a01 = mfma16(da[u].x, hb[u].x, a01);
                a10 = mfma16(db[u].x, ha[u].x, a10);
                a11 = mfma16(db[u].x, hb[u].x, a11);
                a00 = mfma16(da[u].y, ha[u].y, a00);
                a01 = mfma16(da[u].y, hb[u].y, a01);
                a10 = mfma16(db[u].y, ha[u].y, a10);
                a11 = mfma16(db[u].y, hb[u].y, a11);
                a00 = mfma16(da[u].z, ha[u].z, a00);
                a01 = mfma16(da[u].z, hb[u].z, a01);
                a10 = mfma16(db[u].z, ha[u].z, a10);
                a11 = mfma16(db[u].z, hb[u].z, a11);
                a00 = mfma16(da[u].w, ha[u].w, a00);
                a01 = mfma16(da[u].w, hb[u].w, a01);
                a10 = mfma16(db[u].w, ha[u].w, a10);
                a11 = mfma16(db[u].w, hb[u].w, a11);
                const int bn = b + kUpdDepth * kUpdWaves;
                if (bn < bhi) {
                    const float* Db = D + (size_t)bn * kH * kS + dro;
                    const float* Hb = Hs + (size_t)bn * kH * kS + hco;
                    da[u] = *reinterpret_cast<const float4*>(Db);
                    db[u] = *reinterpret_cast<const float4*>(Db + k16);
                    ha[u] = *reinterpret_cast<const float4*>(Hb);
                    hb[u] = *reinterpret_cast<const float4*>(Hb + k16);
                }
            }
        }
    }
    // tile entry e = (j - j0) * kTile + (i - i0)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        red[wave][(4 * q + r) * kTile + c] = a00[r];
        red[wave][(4 * q + r) * kTile + 16 + c] = a01[r];
        red[wave][(16 + 4 * q + r) * kTile + c] = a10[r];
        red[wave][(16 + 4 * q + r) * kTile + 16 + c] = a11[r];
    }
    __syncthreads();
    float* out = slice_part + (size_t)slice * kBig + (size_t)mat * kH * kH;
#pragma unroll
    for (int u = 0; u < kTile * kTile / kUpdThreads; ++u) {
        const int e = tid + u * kUpdThreads;
        float g = red[0][e];
#pragma unroll
        for (int w = 1; w < kUpdWaves; ++w) g += red[w][e];
        out[(j0 + e / kTile) * kH + i0 + e % kTile] = g;
    }
}

// W2 and W3: the slice sums added in slice order, then the update (or the
// gradient).
__global__ __launch_bounds__(kAdamThreads) void mlp_wadam_kernel(const float* __restrict__ slice_part, int nslice,
                                                                 float* __restrict__ P, float* __restrict__ adam,
                                                                 float* __restrict__ grad_out, AdamArgs h) {
    const int k = blockIdx.x * kAdamThreads + threadIdx.x;
    if (k >= kBig) return;
    float g = slice_part[k];
    for (int sl = 1; sl < nslice; ++sl) g += slice_part[(size_t)sl * kBig + k];
    apply_grad(k < kH * kH ? oW2 + k : oW3 + (k - kH * kH), g, P, adam, grad_out, h);
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
    int nblk_cap = 0;
    float* acts = nullptr;         // 4 arrays of nblk_cap [kH][kS] slabs
    float* small = nullptr;        // nblk_cap x kSmallStride
    float* slice_part = nullptr;   // kMaxSlices x kBig
    float4* xe = nullptr;          // encoded samples of a pass (training)
    float* te = nullptr;
    size_t enc_cap = 0;
    Acts act() const {
        const size_t a = (size_t)nblk_cap * kH * kS;
        return Acts{acts, acts + a, acts + 2 * a, acts + 3 * a};
    }
};

// The forward/backward kernel's dynamic LDS (kMlpLds, 50 KB with the padded
// rows) is declared to the runtime once, so that a larger kS or pitch (up to
// the 160 KB of a gfx950 compute unit) needs no other change.
static int fwd_bwd_lds_once() {
    static const int st = hip_check((int)hipFuncSetAttribute(reinterpret_cast<const void*>(mlp_fwd_bwd_kernel),
                                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                                             (int)kMlpLds),
                                    "hipFuncSetAttribute");
    return st;
}

static int launch_fwd_bwd(const float* P, const MlpData& d, int train, const Acts& act, float* small, float* pred,
                          hipStream_t s) {
    const int st = fwd_bwd_lds_once();
    if (st != WG_OK) return st;
    const int nblk = (d.n + kS - 1) / kS;
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(nblk), dim3(kThreads), kMlpLds, s, P, d, train, act, small, pred);
    return hip_check((int)hipGetLastError(), "mlp_fwd_bwd_kernel");
}

// One gradient step over the n samples of d: fwd_bwd, the gradient sums and
// the update of the small parameters, then that of W2 and W3 (Adam with h,
// or the gradient to grad_out).
static int launch_step(Mlp& M, float* P, const MlpData& d, float* adam, float* grad_out, const AdamArgs& h,
                       float* loss_out, hipStream_t s) {
    const Acts act = M.act();
    int st = launch_fwd_bwd(P, d, 1, act, M.small, nullptr, s);
    if (st != WG_OK) return st;
    const int nblk = (d.n + kS - 1) / kS;
    const int nslice = nblk < kMaxSlices ? nblk : kMaxSlices;
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(kTiles * nslice + kSmallBlocks), dim3(kUpdThreads), 0, s, act, M.small,
                       nblk, nslice, M.slice_part, P, adam, grad_out, h, 1.0f / d.n, loss_out);
    st = hip_check((int)hipGetLastError(), "mlp_wgrad_kernel");
    if (st != WG_OK) return st;
    hipLaunchKernelGGL(mlp_wadam_kernel, dim3((kBig + kAdamThreads - 1) / kAdamThreads), dim3(kAdamThreads), 0, s,
                       M.slice_part, nslice, P, adam, grad_out, h);
    return hip_check((int)hipGetLastError(), "mlp_wadam_kernel");
}

static void free_mlp(Mlp* M) {
    if (M->acts) (void)hipFree(M->acts);
    if (M->small) (void)hipFree(M->small);
    if (M->slice_part) (void)hipFree(M->slice_part);
    if (M->xe) (void)hipFree(M->xe);
    if (M->te) (void)hipFree(M->te);
    delete M;
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
    M->nblk_cap = (max_batch + kS - 1) / kS;
    const size_t nb = (size_t)M->nblk_cap;
    if (hipMalloc((void**)&M->acts, sizeof(float) * 4 * nb * kH * kS) != hipSuccess ||
        hipMalloc((void**)&M->small, sizeof(float) * nb * kSmallStride) != hipSuccess ||
        hipMalloc((void**)&M->slice_part, sizeof(float) * kMaxSlices * kBig) != hipSuccess) {
        free_mlp(M);
        return fail(WG_ENOMEM, "wg_mlp_create: device allocation failed");
    }
    *out = reinterpret_cast<wg_mlp*>(M);
    return WG_OK;
}

int wg_mlp_destroy(wg_mlp* mlp) {
    Mlp* M = reinterpret_cast<Mlp*>(mlp);
    if (!M) return WG_OK;
    free_mlp(M);
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
    const MlpData d{c1, c2, m, r, target, nullptr, nullptr, n, 2.0f / n};
    const AdamArgs none{0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f};
    // params is read only: the update writes the gradient, not the parameters
    return launch_step(M, const_cast<float*>(params), d, nullptr, grad_out, none, loss_out,
                       static_cast<hipStream_t>(stream));
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
    const int used = steps * batch;
    if ((size_t)used > M.enc_cap) {
        // grow the per-pass sample buffers (hipFree waits for work that may
        // still read the old ones)
        if (M.xe) (void)hipFree(M.xe);
        if (M.te) (void)hipFree(M.te);
        M.xe = nullptr;
        M.te = nullptr;
        M.enc_cap = 0;
        if (hipMalloc((void**)&M.xe, sizeof(float4) * used) != hipSuccess ||
            hipMalloc((void**)&M.te, sizeof(float) * used) != hipSuccess) {
            if (M.xe) (void)hipFree(M.xe);
            M.xe = nullptr;
            return fail(WG_ENOMEM, "wg_mlp_train: device allocation failed");
        }
        M.enc_cap = (size_t)used;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int t = step0;
    for (int e = 0; e < epochs; ++e) {
        hipLaunchKernelGGL(mlp_encode_kernel, dim3((used + 255) / 256), dim3(256), 0, s, c1, c2, m, r, target,
                           perm + (size_t)e * n, n, used, M.xe, M.te);
        st = hip_check((int)hipGetLastError(), "mlp_encode_kernel");
        if (st != WG_OK) return st;
        for (int b = 0; b < steps; ++b, ++t) {
            const size_t o = (size_t)b * batch;
            const MlpData d{c1, c2, m, r, target, M.xe + o, M.te + o, batch, 2.0f / batch};
            const AdamArgs h{lr, b1, b2, eps, 1.0f - powf(b1, (float)t), 1.0f - powf(b2, (float)t)};
            st = launch_step(M, params, d, adam_state, nullptr, h, losses + (size_t)e * steps + b, s);
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
    const MlpData d{c1, c2, m, r, nullptr, nullptr, nullptr, n, 0.0f};
    return launch_fwd_bwd(params, d, 0, Acts{nullptr, nullptr, nullptr, nullptr}, nullptr, out,
                          static_cast<hipStream_t>(stream));
}

int wg_topk_min(const float* v, int n, int k, int* idx_out, wg_stream_t stream) {
    if (!v || !idx_out || n <= 0 || k <= 0 || k > 64) return fail(WG_EINVAL, "wg_topk_min: bad arguments");
    hipLaunchKernelGGL(topk_min_kernel, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), v, n, k, idx_out);
    return hip_check((int)hipGetLastError(), "topk_min_kernel");
}

}  // extern "C"
