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
//             writes its partial gradient (one full parameter vector)
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
constexpr int kS = 16;            // samples per block
constexpr int kThreads = 256;
// parameter layout (row-major W[out][in]):
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH, kParams = ob4 + 1;
static_assert(kParams == 33793, "parameter count");

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

// 128-wide dense layer for the block's kS samples held in LDS:
// out[s][j] = b[j] + sum_i W[j][i] in[s][i]   (thread: j = tid % 128, two sample halves)
__device__ __forceinline__ void dense128(const float* __restrict__ W, const float* __restrict__ b,
                                         const float (*in)[kH], float (*out)[kH], int ns) {
    const int j = threadIdx.x & (kH - 1), half = threadIdx.x >> 7;
    float acc[kS / 2];
#pragma unroll
    for (int q = 0; q < kS / 2; ++q) acc[q] = 0.0f;
    // weights are loaded eight float4 at a time ahead of their products;
    // each sum still runs over i in ascending order
    const float4* wr = reinterpret_cast<const float4*>(W + (size_t)j * kH);
    for (int i4 = 0; i4 < kH / 4; i4 += 8) {
        float4 w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = wr[i4 + u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < kS / 2; ++q) {
                const float4 h = *reinterpret_cast<const float4*>(&in[half + 2 * q][4 * (i4 + u)]);
                acc[q] = fmaf(w[u].x, h.x, acc[q]);
                acc[q] = fmaf(w[u].y, h.y, acc[q]);
                acc[q] = fmaf(w[u].z, h.z, acc[q]);
                acc[q] = fmaf(w[u].w, h.w, acc[q]);
            }
    }
    const float bj = b[j];
#pragma unroll
    for (int q = 0; q < kS / 2; ++q) {
        const int s = half + 2 * q;
        if (s < ns) out[s][j] = acc[q] + bj;
    }
}

// One hidden layer of the backward pass for the block's samples: from
// DZ = dL/dZ of the layer's output, writes dW[j][i] = sum_s DZ[s][j] Hin[s][i]
// and db[j] = sum_s DZ[s][j] to the partial gradient, and replaces DZ by
// dL/dZ of the layer's input, (DZ W) * gelu'(Zin).
__device__ __forceinline__ void backprop_hidden(float (*DZ)[kH], float (*DH)[kH], const float (*Hin)[kH],
                                                const float (*Zin)[kH], const float* __restrict__ W,
                                                float* __restrict__ gW, float* __restrict__ gb) {
    const int tid = threadIdx.x;
    {
        // thread: column i of dW for 64 rows j (consecutive lanes hold
        // consecutive i, so each row of dW is written with whole-wave stores)
        const int i = tid & (kH - 1), j0 = (tid >> 7) * 64;
        float acc[64];
#pragma unroll
        for (int u = 0; u < 64; ++u) acc[u] = 0.0f;
        for (int s = 0; s < kS; ++s) {
            const float h = Hin[s][i];
            const float4* dz4 = reinterpret_cast<const float4*>(&DZ[s][j0]);
#pragma unroll
            for (int u4 = 0; u4 < 16; ++u4) {
                const float4 dz = dz4[u4];
                acc[4 * u4 + 0] = fmaf(dz.x, h, acc[4 * u4 + 0]);
                acc[4 * u4 + 1] = fmaf(dz.y, h, acc[4 * u4 + 1]);
                acc[4 * u4 + 2] = fmaf(dz.z, h, acc[4 * u4 + 2]);
                acc[4 * u4 + 3] = fmaf(dz.w, h, acc[4 * u4 + 3]);
            }
        }
        float* gw = gW + (size_t)j0 * kH + i;
#pragma unroll
        for (int u = 0; u < 64; ++u) gw[(size_t)u * kH] = acc[u];
    }
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kS; ++s) a += DZ[s][tid];
        gb[tid] = a;
    }
    {
        const int i = tid & (kH - 1), half = tid >> 7;
        float acc[kS / 2];
#pragma unroll
        for (int q = 0; q < kS / 2; ++q) acc[q] = 0.0f;
        for (int jj = 0; jj < kH; jj += 8) {
            float w[8];                          // eight loads ahead, jj ascending
#pragma unroll
            for (int u = 0; u < 8; ++u) w[u] = W[(size_t)(jj + u) * kH + i];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int q = 0; q < kS / 2; ++q) acc[q] = fmaf(DZ[half + 2 * q][jj + u], w[u], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < kS / 2; ++q) DH[half + 2 * q][i] = acc[q];
    }
    __syncthreads();
    for (int q = tid; q < kS * kH; q += kThreads) {
        const int s = q / kH, i = q % kH;
        DZ[s][i] = DH[s][i] * gelu_grad_f(Zin[s][i]);
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void mlp_fwd_bwd_kernel(const float* __restrict__ P, MlpData d, int train,
                                                               float* __restrict__ part,
                                                               float* __restrict__ part_loss,
                                                               float* __restrict__ pred) {
    __shared__ __attribute__((aligned(16))) float X[kS][kIn];
    __shared__ __attribute__((aligned(16))) float Z1[kS][kH], H1[kS][kH], Z2[kS][kH], H2[kS][kH], Z3[kS][kH],
        H3[kS][kH];
    __shared__ __attribute__((aligned(16))) float DZ[kS][kH], DH[kS][kH];
    __shared__ float OUT[kS], DOUT[kS];
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * kS;
    const int ns = min(kS, d.n - s0);
    if (tid < kS) {
        float f[kIn] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (tid < ns) {
            const int q = d.idx ? d.idx[s0 + tid] : s0 + tid;
            encode(d.c1, d.c2, d.m, d.r, q, f);
        }
#pragma unroll
        for (int k = 0; k < kIn; ++k) X[tid][k] = f[k];
    }
    __syncthreads();
    // layer 1 (4 -> 128)
    {
        const int j = tid & (kH - 1), half = tid >> 7;
        const float w0 = P[oW1 + j * kIn + 0], w1 = P[oW1 + j * kIn + 1], w2 = P[oW1 + j * kIn + 2],
                    w3 = P[oW1 + j * kIn + 3], bj = P[ob1 + j];
        for (int s = half; s < kS; s += 2) {
            float a = fmaf(w0, X[s][0], 0.0f);
            a = fmaf(w1, X[s][1], a);
            a = fmaf(w2, X[s][2], a);
            a = fmaf(w3, X[s][3], a);
            a += bj;
            Z1[s][j] = a;
            H1[s][j] = gelu_f(a);
        }
    }
    __syncthreads();
    dense128(P + oW2, P + ob2, H1, Z2, kS);
    __syncthreads();
    for (int q = tid; q < kS * kH; q += kThreads) H2[q / kH][q % kH] = gelu_f(Z2[q / kH][q % kH]);
    __syncthreads();
    dense128(P + oW3, P + ob3, H2, Z3, kS);
    __syncthreads();
    for (int q = tid; q < kS * kH; q += kThreads) H3[q / kH][q % kH] = gelu_f(Z3[q / kH][q % kH]);
    __syncthreads();
    if (tid < kS) {
        float a = 0.0f;
        for (int i = 0; i < kH; ++i) a = fmaf(P[oW4 + i], H3[tid][i], a);
        a += P[ob4];
        OUT[tid] = a;
        if (tid < ns) {
            if (pred) pred[s0 + tid] = a;
            if (train) {
                const int q = d.idx ? d.idx[s0 + tid] : s0 + tid;
                DOUT[tid] = d.inv_batch2 * (a - d.target[q]);
            }
        } else {
            DOUT[tid] = 0.0f;
        }
    }
    __syncthreads();
    if (!train) return;
    float* g = part + (size_t)blockIdx.x * kParams;
    if (tid == 0) {
        float l = 0.0f, db = 0.0f;
        for (int s = 0; s < ns; ++s) {
            const int q = d.idx ? d.idx[s0 + s] : s0 + s;
            const float e = OUT[s] - d.target[q];
            l = fmaf(e, e, l);
            db += DOUT[s];
        }
        part_loss[blockIdx.x] = l;
        g[ob4] = db;
    }
    // output layer: dW4, dZ3
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kS; ++s) a = fmaf(DOUT[s], H3[s][tid], a);
        g[oW4 + tid] = a;
    }
    for (int q = tid; q < kS * kH; q += kThreads) {
        const int s = q / kH, i = q % kH;
        DZ[s][i] = DOUT[s] * P[oW4 + i] * gelu_grad_f(Z3[s][i]);
    }
    __syncthreads();
    // hidden layers 3 and 2: dW = dZ^T H_in, db = sum dZ, dH_in = dZ W
    backprop_hidden(DZ, DH, H2, Z2, P + oW3, g + oW3, g + ob3);
    backprop_hidden(DZ, DH, H1, Z1, P + oW2, g + oW2, g + ob2);
    // first layer: dW1[j][k] = sum_s dZ1[s][j] X[s][k], db1
    if (tid < kH) {
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, b = 0.0f;
        for (int s = 0; s < kS; ++s) {
            const float dz = DZ[s][tid];
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
// kRedParams parameters; its kRedGroups thread groups each add every
// kRedGroups-th partial (group g: partials g, g + kRedGroups, ...), and the
// group sums are added in group order, so the result is fixed for a given
// number of partials.
constexpr int kRedParams = 64;
constexpr int kRedGroups = 256 / kRedParams;

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part, int nblk,
                                                         float* __restrict__ P, float* __restrict__ adam,
                                                         float* __restrict__ grad_out, float lr, float b1, float b2,
                                                         float eps, float bc1, float bc2,
                                                         const float* __restrict__ part_loss, float inv_batch,
                                                         float* __restrict__ loss_out) {
    __shared__ float gs[kRedGroups][kRedParams];
    const int pl = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    // both sums issue their loads eight at a time and add them in the same
    // order as a plain loop
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
    float acc = 0.0f;
    if (p < kParams) {
        int b = grp;
        for (; b + 7 * kRedGroups < nblk; b += 8 * kRedGroups) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = part[(size_t)(b + i * kRedGroups) * kParams + p];
#pragma unroll
            for (int i = 0; i < 8; ++i) acc += v[i];
        }
        for (; b < nblk; b += kRedGroups) acc += part[(size_t)b * kParams + p];
    }
    gs[grp][pl] = acc;
    __syncthreads();
    if (grp != 0 || p >= kParams) return;
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

static int launch_step(Mlp& M, const float* P, const MlpData& d, int train, float* pred, hipStream_t s) {
    const int nblk = (d.n + kS - 1) / kS;
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(nblk), dim3(kThreads), 0, s, P, d, train, M.part, M.part_loss,
                       pred);
    return hip_check((int)hipGetLastError(), "mlp_fwd_bwd_kernel");
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
    if (hipMalloc((void**)&M->part, sizeof(float) * nblk * kParams) != hipSuccess ||
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
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3((n + kS - 1) / kS), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), params, d, 0, nullptr, nullptr, out);
    return hip_check((int)hipGetLastError(), "mlp_fwd_bwd_kernel");
}

int wg_topk_min(const float* v, int n, int k, int* idx_out, wg_stream_t stream) {
    if (!v || !idx_out || n <= 0 || k <= 0 || k > 64) return fail(WG_EINVAL, "wg_topk_min: bad arguments");
    hipLaunchKernelGGL(topk_min_kernel, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), v, n, k, idx_out);
    return hip_check((int)hipGetLastError(), "topk_min_kernel");
}

}  // extern "C"
