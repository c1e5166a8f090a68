// Batched error sweep over point-family parameters on gfx950.
//
// For thousands of candidate point sets (the families of Section 5 of
// arXiv:2201.10369, parameterised by c1 and c2) the sweep builds each set's
// transform matrices on the device (Sections 4.1, 4.2) as the float64
// roundings of their exact values, rounds those to float32, evaluates
// float32 Winograd tiles (1D eq. conv_1d or 2D
// eq. conv_2d) on the first n_i samples of a shared pool, and sums the L1
// error against the float64 direct correlation of each sample (Section 6;
// Section 6.1 sweeps c over a range, Section 6.3 scores many combinations).
//
// Launch structure (one hipGraph, replayed):
//   construct : one thread per (candidate, matrix row), float64 with a
//               running error bound -> the float32 matrices
//   rebuild   : the same threads for the candidates the first launch left
//               pending (others return at once): double words with an error
//               bound, exact integers for rows they cannot decide
//   evaluate  : persistent blocks stride over work items (candidate, or
//               in 1D a group of four candidates that share each loaded
//               sample; chunk of `chunk` samples); per item a fixed-order
//               block reduction writes one float64 partial sum per candidate
//   finalize  : one thread per candidate adds its partials in index order
// so the result is bitwise reproducible for a given tuning.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "wg_construct.h"
#include "wg_device.h"
#include "wg_internal.h"
#include "wg_sweep_internal.h"

#pragma clang fp contract(off)

namespace wg {

constexpr int kMatStride = 256;     // floats per candidate: A^T | G | B^T

// ---------------------------------------------------------------------------
// Family points (same definition as wg_family_points)
// ---------------------------------------------------------------------------
__device__ int family_points_dev(int alpha, double c1, double c2, double* p) {
    const double ic = 1.0 / c1;
    int n = 0;
    if (alpha == 4) {
        p[n++] = -c1; p[n++] = 0.0; p[n++] = c1;
        return n;
    }
    if (alpha == 5) {
        p[n++] = 0.0; p[n++] = -c1; p[n++] = c1; p[n++] = ic;
        return n;
    }
    p[n++] = -ic; p[n++] = -c1; p[n++] = 0.0; p[n++] = c1; p[n++] = ic;
    const double id = 1.0 / c2;
    if (alpha == 7) { p[n++] = c2; }
    if (alpha == 8) { p[n++] = -c2; p[n++] = c2; }
    if (alpha == 9) { p[n++] = -id; p[n++] = -c2; p[n++] = c2; }
    if (alpha == 10) { p[n++] = -id; p[n++] = -c2; p[n++] = c2; p[n++] = id; }
    return n;
}

// Candidate flags between the launches of a run: kFlagBad (not finite,
// zero parameter, coinciding points, |N_i| < 1e-300, an entry overflows
// float32, or integers beyond the exact construction's limbs), kFlagPending
// (left to sweep_rebuild_kernel) and kFlagExact (some row built from exact
// integers).
constexpr int kFlagBad = 1;
constexpr int kFlagPending = 2;
constexpr int kFlagExact = 4;

// Both construction kernels: one thread per (candidate, row), thread i <
// alpha-1 builds what point i owns (column i of A^T, row i of G, row i of
// B^T), thread alpha-1 the infinity row and column.  A wave holds row i of
// kConsCands consecutive candidates, so its lanes follow the same path
// through the root grouping (the rows of one candidate differ in it).  With
// explicit point lists (pts_in, n_cand x (alpha-1), infinity implied last)
// a non-finite point flags the candidate.  Row statuses pass from the first
// kernel to the second in row_status[cand][row] (kRowStride bytes per
// candidate): 0 built, 1 flags the candidate, 2 left to the second kernel.
constexpr int kConsCands = 64;
constexpr int kRowStride = 16;

template <int M, int R>
__device__ __forceinline__ void candidate_points(const double* __restrict__ c1, const double* __restrict__ c2,
                                                 const double* __restrict__ pts_in, int cand, double* pts,
                                                 int& flag) {
    constexpr int A = M + R - 1;
    constexpr int NF = A - 1;
    if (pts_in != nullptr) {
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            pts[j] = pts_in[(size_t)cand * NF + j];
            if (!isfinite(pts[j])) flag = 1;
        }
    } else {
        const double x1 = c1[cand], x2 = c2 != nullptr ? c2[cand] : 1.0;
        if (!isfinite(x1) || x1 == 0.0 || (A > 6 && (!isfinite(x2) || x2 == 0.0))) flag = 1;
        if (!flag) family_points_dev(A, x1, x2, pts);
    }
}

// Writes one row (RowOut layout) into the candidate's float32 matrices and,
// when given, its float64 ones; returns whether a float32 entry overflows.
template <int M, int R>
__device__ __forceinline__ int store_row(const cons::RowOut<M, R>& o, int i, float* out, double* out64) {
    constexpr int A = M + R - 1;
    int nonfinite = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        out[j * A + i] = o.v32[j];
        nonfinite |= !isfinite(o.v32[j]);
        if (out64) out64[j * A + i] = o.v64[j];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        out[M * A + i * R + k] = o.v32[M + k];
        nonfinite |= !isfinite(o.v32[M + k]);
        if (out64) out64[M * A + i * R + k] = o.v64[M + k];
    }
#pragma unroll
    for (int l = 0; l < A; ++l) {
        out[M * A + A * R + i * A + l] = o.v32[M + R + l];
        nonfinite |= !isfinite(o.v32[M + R + l]);
        if (out64) out64[M * A + A * R + i * A + l] = o.v64[M + R + l];
    }
    return nonfinite;
}

// First construction: float64 with a running error bound decides the
// float32 matrices (RN32 of RN64 of the exact entries) of nearly every
// candidate.  Grid (candidate groups, alpha), one wave per block: the whole
// chip takes part.  Rows it cannot decide, every valid row of a
// mixed-precision run (which needs the float64 matrices) and, with
// force_exact, every valid row are left to the second kernel.
template <int M, int R>
__global__ __launch_bounds__(kConsCands) void sweep_construct_kernel(const double* __restrict__ c1,
                                                                     const double* __restrict__ c2,
                                                                     const double* __restrict__ pts_in,
                                                                     int n_cand, int defer_all,
                                                                     float* __restrict__ mats,
                                                                     uint8_t* __restrict__ row_status) {
    constexpr int A = M + R - 1;
    constexpr int NF = A - 1;
    static_assert(A <= kRowStride, "rows per candidate");
    const int cand = blockIdx.x * kConsCands + threadIdx.x, i = blockIdx.y;
    if (cand >= n_cand) return;
    double pts[NF];
    int flag = 0;
    candidate_points<M, R>(c1, c2, pts_in, cand, pts, flag);
    int st = 1;
    if (!flag) {
        cons::RowOut<M, R> o;
        st = cons::row_cert<cons::ArithF64, M, R>(pts, i, o);
        if (st == 0 && defer_all) st = 2;
        if (st == 0 && store_row<M, R>(o, i, mats + (size_t)cand * kMatStride, nullptr)) st = 1;
    }
    row_status[(size_t)cand * kRowStride + i] = (uint8_t)st;
}

// Second construction: combines the row statuses of each candidate into
// its flag and rebuilds the candidates with an undecided row: double words
// with an error bound decide the float64 entries, rows they cannot decide
// (or every row, with force_exact) are built from exact integers.  Writes
// the float32 matrices and, when mats64 is given, the float64 ones; flagged
// candidates get zero matrices.  A block holds kConsCands candidates and
// alpha waves (wave i: row i).
template <int M, int R>
__global__ __launch_bounds__(kConsCands * 10) void sweep_rebuild_kernel(const double* __restrict__ c1,
                                                                        const double* __restrict__ c2,
                                                                        const double* __restrict__ pts_in,
                                                                        int n_cand, int force_exact,
                                                                        const uint8_t* __restrict__ row_status,
                                                                        float* __restrict__ mats,
                                                                        double* __restrict__ mats64,
                                                                        int* __restrict__ flags) {
    constexpr int NF = M + R - 2;
    static_assert(M + R - 1 <= 10, "rows per block");
    // per candidate: a row flags it, exact integers used, a row pending, the
    // rebuild failed or overflowed float32
    __shared__ int s_flag[kConsCands], s_exact[kConsCands], s_pend[kConsCands], s_fail[kConsCands];
    const int slot = threadIdx.x % kConsCands, i = threadIdx.x / kConsCands;
    const int cand = blockIdx.x * kConsCands + slot;
    const bool live = cand < n_cand;
    if (i == 0) s_flag[slot] = s_exact[slot] = s_pend[slot] = s_fail[slot] = 0;
    __syncthreads();
    const int st0 = live ? row_status[(size_t)cand * kRowStride + i] : 0;
    if (st0 == 1) s_flag[slot] = 1;
    if (st0 == 2) s_pend[slot] = 1;
    __syncthreads();
    const bool pending = live && !s_flag[slot] && s_pend[slot];
    cons::RowOut<M, R> o;
    if (pending) {
        double pts[NF];
        int flag = 0;
        candidate_points<M, R>(c1, c2, pts_in, cand, pts, flag);
        int st = force_exact ? 2 : cons::row_cert<cons::ArithDW, M, R>(pts, i, o);
        if (st == 2) {
            st = cons::exact_row<M, R>(pts, i, o);
            s_exact[slot] = 1;
        }
        if (flag || st != 0) s_fail[slot] = 1;
    }
    __syncthreads();
    const bool bad = live && (s_flag[slot] || s_fail[slot]);
    if (live && (bad || pending)) {
        if (bad) {
#pragma unroll
            for (int q = 0; q < cons::RowOut<M, R>::kN; ++q) {
                o.v32[q] = 0.0f;
                o.v64[q] = 0.0;
            }
        }
        float* out = mats + (size_t)cand * kMatStride;
        double* out64 = mats64 != nullptr ? mats64 + (size_t)cand * kMatStride : nullptr;
        if (store_row<M, R>(o, i, out, out64)) s_fail[slot] = 1;      // float32 overflow
    }
    __syncthreads();
    if (live && i == 0)
        flags[cand] = (s_flag[slot] || s_fail[slot]) ? kFlagBad : (s_exact[slot] ? kFlagExact : 0);
}

// ---------------------------------------------------------------------------
// float64 reference of the pool (once per sweep object)
// ---------------------------------------------------------------------------
// Also copies the pool into element-major arrays so that consecutive
// threads (consecutive samples) of the evaluation read consecutive addresses.
template <int M, int R, int DIMS>
__global__ __launch_bounds__(256) void sweep_reference_kernel(const float* __restrict__ d_pool,
                                                              const float* __restrict__ g_pool, int n_pool,
                                                              float* __restrict__ d_soa,
                                                              float* __restrict__ g_soa,
                                                              double* __restrict__ yref,
                                                              double* __restrict__ ref_abs) {
    constexpr int A = M + R - 1;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_pool) return;
    double tot = 0.0;
    if (DIMS == 1) {
        const float* d = d_pool + (size_t)s * A;
        const float* g = g_pool + (size_t)s * R;
        for (int q = 0; q < A; ++q) d_soa[(size_t)q * n_pool + s] = d[q];
        for (int q = 0; q < R; ++q) g_soa[(size_t)q * n_pool + s] = g[q];
        for (int j = 0; j < M; ++j) {
            double acc = 0.0;
            for (int k = 0; k < R; ++k) acc = fma((double)d[j + k], (double)g[k], acc);
            yref[(size_t)j * n_pool + s] = acc;
            tot += fabs(acc);
        }
    } else {
        const float* d = d_pool + (size_t)s * A * A;
        const float* g = g_pool + (size_t)s * R * R;
        for (int q = 0; q < A * A; ++q) d_soa[(size_t)q * n_pool + s] = d[q];
        for (int q = 0; q < R * R; ++q) g_soa[(size_t)q * n_pool + s] = g[q];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                double acc = 0.0;
                for (int u = 0; u < R; ++u)
                    for (int v = 0; v < R; ++v) acc = fma((double)d[(i + u) * A + j + v], (double)g[u * R + v], acc);
                yref[(size_t)(i * M + j) * n_pool + s] = acc;
                tot += fabs(acc);
            }
    }
    ref_abs[s] = tot;
}

__global__ void sweep_prefix_kernel(const double* __restrict__ ref_abs, int n_pool, double* __restrict__ prefix) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double acc = 0.0;
    prefix[0] = 0.0;
    for (int s = 0; s < n_pool; ++s) {
        acc += ref_abs[s];
        prefix[s + 1] = acc;
    }
}

// ---------------------------------------------------------------------------
// Evaluation.  Each thread evaluates whole tiles.  The block's current
// candidate is staged in LDS as columns of B^T, columns and rows of G and
// columns and rows of A^T (each padded to a multiple of 4 floats, read as
// broadcast 16-byte loads).  Every term is a fused multiply-add in ascending
// index order from zero; the exact zeros that every family set has are left
// out at compile time (FamilyZeros), other zero entries are not tested for,
// which changes nothing because fma(0, x, acc) == acc for the finite values
// involved (flagged candidates, the only ones that could hold non-finite
// entries, are never evaluated).
// ---------------------------------------------------------------------------
template <int M, int R>
struct EvalLds {
    static constexpr int A = M + R - 1;
    static constexpr int AP = (A + 3) & ~3, MP = (M + 3) & ~3, RP = (R + 3) & ~3;
    static constexpr int kBc = 0;                  // [A][AP]  B^T column l at l*AP
    static constexpr int kGc = kBc + A * AP;       // [R][AP]  G column v at v*AP
    static constexpr int kGr = kGc + R * AP;       // [A][RP]  G row i at i*RP
    static constexpr int kAc = kGr + A * RP;       // [A][MP]  A^T column i at i*MP
    static constexpr int kAr = kAc + A * MP;       // [M][AP]  A^T row q at q*AP
    static constexpr int kSize = kAr + M * AP;

    // value of LDS slot q from the candidate's row-major A^T | G | B^T
    template <typename T>
    __device__ static T slot(const T* __restrict__ m, int q) {
        const T* AT = m;
        const T* G = m + M * A;
        const T* BT = m + M * A + A * R;
        if (q < kGc) { const int l = q / AP, i = q % AP; return i < A ? BT[i * A + l] : T(0); }
        if (q < kGr) { q -= kGc; const int v = q / AP, j = q % AP; return j < A ? G[j * R + v] : T(0); }
        if (q < kAc) { q -= kGr; const int i = q / RP, u = q % RP; return u < R ? G[i * R + u] : T(0); }
        if (q < kAr) { q -= kAc; const int i = q / MP, k = q % MP; return k < M ? AT[k * A + i] : T(0); }
        q -= kAr;
        const int qq = q / AP, j = q % AP;
        return j < A ? AT[qq * A + j] : T(0);
    }
};

// Exact zeros that every family set has (it contains 0, at index z0, and
// ends with infinity): column 0 of B^T only in row z0 (every other row's
// polynomial has the factor x) and column alpha-1 only in the infinity row;
// row z0 of G only in column 0 (0^k) and the infinity row only in column
// r-1; column z0 of A^T only in row 0 and the infinity column only in row
// m-1.  Terms with these entries are left out (fma(0, x, acc) == acc for the
// finite values involved, so nothing changes).
template <int M, int R>
struct FamilyZeros {
    static constexpr int A = M + R - 1;
    static constexpr int Z0 = A == 4 ? 1 : (A == 5 ? 0 : 2);     // position of 0 in the family order
    __device__ static constexpr bool bt(int i, int l) {          // B^T[i][l] may be nonzero
        return !((l == 0 && i != Z0) || (l == A - 1 && i != A - 1));
    }
    __device__ static constexpr bool g(int j, int v) {           // G[j][v]
        return !((j == Z0 && v != 0) || (j == A - 1 && v != R - 1));
    }
    __device__ static constexpr bool at(int k, int i) {          // A^T[k][i]
        return !((i == Z0 && k != 0) || (i == A - 1 && k != M - 1));
    }
};

// Explicit point lists: no zero pattern is assumed, every term is taken.
template <int M, int R>
struct AllTerms {
    __device__ static constexpr bool bt(int, int) { return true; }
    __device__ static constexpr bool g(int, int) { return true; }
    __device__ static constexpr bool at(int, int) { return true; }
};

template <int N>
__device__ __forceinline__ void lds_vec(const float* p, float (&v)[N]) {
    static_assert(N % 4 == 0, "padded length");
#pragma unroll
    for (int q = 0; q < N; q += 4) {
        const float4 t = *reinterpret_cast<const float4*>(p + q);
        v[q] = t.x; v[q + 1] = t.y; v[q + 2] = t.z; v[q + 3] = t.w;
    }
}
template <int N>
__device__ __forceinline__ void lds_vec(const double* p, double (&v)[N]) {
    static_assert(N % 2 == 0, "padded length");
#pragma unroll
    for (int q = 0; q < N; q += 2) {
        const double2 t = *reinterpret_cast<const double2*>(p + q);
        v[q] = t.x; v[q + 1] = t.y;
    }
}


// One 2D tile: Y = A^T [(G g G^T) .* (B^T d B)] A against the float64
// reference; `lds` is the staged candidate.  T is the type of the
// transforms: float (every step in float32), or double (float64 transforms,
// U and V rounded to float32, their product in float32, Y rounded to
// float32 at the end: the mixed-precision evaluation).
template <int M, int R, typename Z, typename T>
__device__ __forceinline__ double tile_error_2d(const float* __restrict__ d_soa, const float* __restrict__ g_soa,
                                                const double* __restrict__ yref, int s, int np, const T* lds) {
    using L = EvalLds<M, R>;
    constexpr int A = L::A, AP = L::AP, MP = L::MP, RP = L::RP;
    T gg[R][R];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v) gg[u][v] = (T)g_soa[(size_t)(u * R + v) * np + s];
    // T1 = B^T d, one row of d at a time
    T t1[A][A];
#pragma unroll
    for (int i = 0; i < A; ++i)
#pragma unroll
        for (int b = 0; b < A; ++b) t1[i][b] = T(0);
#pragma unroll
    for (int l = 0; l < A; ++l) {
        T drow[A], bc[AP];
#pragma unroll
        for (int b = 0; b < A; ++b) drow[b] = (T)d_soa[(size_t)(l * A + b) * np + s];
        lds_vec(lds + L::kBc + l * AP, bc);
#pragma unroll
        for (int i = 0; i < A; ++i)
            if (Z::bt(i, l)) {
#pragma unroll
                for (int b = 0; b < A; ++b) t1[i][b] = madd(bc[i], drow[b], t1[i][b]);
            }
    }
    // V = T1 B, one column of B^T at a time (float); in float64 row i of V
    // is formed only when row i of the Hadamard stage needs it (same terms in
    // the same order), which keeps the double tile within the registers
    constexpr bool kRowV = sizeof(T) == 8;
    T vv[kRowV ? 1 : A][A];
    if constexpr (!kRowV) {
#pragma unroll
        for (int i = 0; i < A; ++i)
#pragma unroll
            for (int j = 0; j < A; ++j) vv[i][j] = T(0);
#pragma unroll
        for (int l = 0; l < A; ++l) {
            T bc[AP];
            lds_vec(lds + L::kBc + l * AP, bc);
#pragma unroll
            for (int i = 0; i < A; ++i)
#pragma unroll
                for (int j = 0; j < A; ++j)
                    if (Z::bt(j, l)) vv[i][j] = madd(t1[i][l], bc[j], vv[i][j]);
        }
    }
    // row i of U = G g G^T, Hadamard with row i of V (float32), accumulate
    // Z = A^T Mh
    T z[M][A];
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
        for (int j = 0; j < A; ++j) z[k][j] = T(0);
#pragma unroll
    for (int i = 0; i < A; ++i) {
        T gr[RP], p1[R], urow[A], ac[MP];
        T* vr = vv[kRowV ? 0 : i];
        if constexpr (kRowV) asm volatile("" ::: "memory");
        if constexpr (kRowV) {
#pragma unroll
            for (int j = 0; j < A; ++j) vr[j] = T(0);
#pragma unroll
            for (int l = 0; l < A; ++l) {
                asm volatile("" ::: "memory");
                T bc[AP];
                lds_vec(lds + L::kBc + l * AP, bc);
#pragma unroll
                for (int j = 0; j < A; ++j)
                    if (Z::bt(j, l)) vr[j] = madd(t1[i][l], bc[j], vr[j]);
            }
        }
        lds_vec(lds + L::kGr + i * RP, gr);
#pragma unroll
        for (int v = 0; v < R; ++v) p1[v] = T(0);
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (Z::g(i, u)) {
#pragma unroll
                for (int v = 0; v < R; ++v) p1[v] = madd(gr[u], gg[u][v], p1[v]);
            }
#pragma unroll
        for (int j = 0; j < A; ++j) urow[j] = T(0);
#pragma unroll
        for (int v = 0; v < R; ++v) {
            T gc[AP];
            lds_vec(lds + L::kGc + v * AP, gc);
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (Z::g(j, v)) urow[j] = madd(gc[j], p1[v], urow[j]);
        }
        lds_vec(lds + L::kAc + i * MP, ac);
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const float mh = (float)urow[j] * (float)vr[j];
#pragma unroll
            for (int k = 0; k < M; ++k)
                if (Z::at(k, i)) z[k][j] = madd(ac[k], (T)mh, z[k][j]);
        }
    }
    // Y = Z A, one row of A^T at a time
    double err = 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        T ar[AP];
        lds_vec(lds + L::kAr + q * AP, ar);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            T y = T(0);
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (Z::at(q, j)) y = madd(z[k][j], ar[j], y);
            err += fabs((double)(float)y - yref[(size_t)(k * M + q) * np + s]);
        }
    }
    return err;
}

// The data of NT 1D pool samples (s[t]): tile, filter and float64 reference.
template <int M, int R, int NT, typename T>
struct Samples1d {
    static constexpr int A = M + R - 1;
    T gv[NT][R], dv[NT][A];
    double yr[NT][M];
    __device__ __forceinline__ void load(const float* __restrict__ d_soa, const float* __restrict__ g_soa,
                                         const double* __restrict__ yref, const int (&s)[NT], int np) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int k = 0; k < R; ++k) gv[t][k] = (T)g_soa[(size_t)k * np + s[t]];
#pragma unroll
            for (int l = 0; l < A; ++l) dv[t][l] = (T)d_soa[(size_t)l * np + s[t]];
#pragma unroll
            for (int j = 0; j < M; ++j) yr[t][j] = yref[(size_t)j * np + s[t]];
        }
    }
};

// NT 1D tiles (loaded samples; the ones with ok[t] false are evaluated and
// not counted) of the candidate staged at `lds`, sharing each matrix value
// read.  T as for the 2D tile.
template <int M, int R, int NT, typename Z, typename T>
__device__ __forceinline__ double tile_error_1d(const Samples1d<M, R, NT, T>& sp, const bool (&ok)[NT],
                                                const T* lds) {
    using L = EvalLds<M, R>;
    constexpr int A = L::A, AP = L::AP, MP = L::MP;
    T u[NT][A], v[NT][A];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < A; ++i) u[t][i] = v[t][i] = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {                       // U = G g, column k of G
        T gc[AP];
        lds_vec(lds + L::kGc + k * AP, gc);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < A; ++i)
                if (Z::g(i, k)) u[t][i] = madd(gc[i], sp.gv[t][k], u[t][i]);
    }
#pragma unroll
    for (int l = 0; l < A; ++l) {                       // V = B^T d, column l of B^T
        T bc[AP];
        lds_vec(lds + L::kBc + l * AP, bc);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < A; ++i)
                if (Z::bt(i, l)) v[t][i] = madd(bc[i], sp.dv[t][l], v[t][i]);
    }
    T y[NT][M];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < M; ++j) y[t][j] = T(0);
#pragma unroll
    for (int i = 0; i < A; ++i) {                       // Y = A^T Mh, column i of A^T
        T ac[MP];
        lds_vec(lds + L::kAc + i * MP, ac);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float mh = (float)u[t][i] * (float)v[t][i];
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (Z::at(j, i)) y[t][j] = madd(ac[j], (T)mh, y[t][j]);
        }
    }
    double err = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double e = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) e += fabs((double)(float)y[t][j] - sp.yr[t][j]);
        err += ok[t] ? e : 0.0;
    }
    return err;
}

constexpr int kTiles1d = 4;
constexpr int kGroup1d = 4;          // candidates per 1D work item

// Waves per SIMD the compiler must leave room for.  The float64 2D tiles of
// F(6x6,3x3) need 281 registers per lane, one wave per SIMD; held to two
// waves they spill 25 (104 bytes per lane) and the 4096-candidate mixed
// sweep takes 1.34-1.40 ms instead of 2.02 ms, with identical sums.  Larger
// tiles would spill 316-940 bytes and keep one wave; the 1D float64 tiles
// (0.22 ms with the bound against 0.18 ms) and the float32 ones keep theirs.
template <int M, int R, int DIMS, typename T>
constexpr int eval_min_waves() {
    return DIMS == 2 && sizeof(T) == 8 && R == 3 && M + R - 1 <= 8 ? 2 : 1;
}

// FAM: candidates are family sets (FamilyZeros applies), else explicit lists.
// T: float (float32 evaluation) or double (mixed precision; mats holds the
// float64 matrices).
template <int M, int R, int DIMS, bool FAM, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(eval_min_waves<M, R, DIMS, T>())))
void sweep_eval_kernel(const float* __restrict__ d_soa,
                                                         const float* __restrict__ g_soa,
                                                         const double* __restrict__ yref,
                                                         const T* __restrict__ mats,
                                                         const int* __restrict__ flags,
                                                         const int* __restrict__ counts, int n_cand, int n_pool,
                                                         int ipc, int chunk, double* __restrict__ partial) {
    using L = EvalLds<M, R>;
    // (the float64 tiles take every term: skipping the exact zeros changes no
    // result and made the compiler spill them)
    using Z = typename std::conditional<FAM && sizeof(T) == 4, FamilyZeros<M, R>, AllTerms<M, R>>::type;
    // 1D items take kGroup1d candidates: each loaded sample serves all of them
    constexpr int G = DIMS == 1 ? kGroup1d : 1;
    __shared__ __align__(16) T sm[G][L::kSize];
    __shared__ double red[G][4];                       // one sum per wave and candidate
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n_grp = (n_cand + G - 1) / G;
    const long items = (long)n_grp * ipc;
    for (long item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = (int)(item / ipc), ch = (int)(item - (long)grp * ipc);
        const int start = ch * chunk;
        int nj[G];
        bool lj[G];
        bool any = false;
        int nmax = 0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int cand = grp * G + j;
            int n = cand < n_cand ? counts[cand] : 0;
            n = n < 0 ? 0 : (n > n_pool ? n_pool : n);
            nj[j] = n;
            lj[j] = cand < n_cand && !(flags[cand] & kFlagBad) && start < n;    // uniform over the block
            any |= lj[j];
            if (lj[j]) nmax = max(nmax, n);
        }
        if (!any) {
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (tid == j && grp * G + j < n_cand) partial[(size_t)(grp * G + j) * ipc + ch] = 0.0;
            continue;
        }
        __syncthreads();                                      // previous item done with sm
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (lj[j])
                for (int q = tid; q < L::kSize; q += nthr)
                    sm[j][q] = L::slot(mats + (size_t)(grp * G + j) * kMatStride, q);
        __syncthreads();
        const int stop = min(nmax, start + chunk);
        double err[G];
#pragma unroll
        for (int j = 0; j < G; ++j) err[j] = 0.0;
        if (DIMS == 1) {
            for (int s0 = start + tid; s0 < stop; s0 += kTiles1d * nthr) {
                int ss[kTiles1d];
#pragma unroll
                for (int t = 0; t < kTiles1d; ++t) {
                    const int si = s0 + t * nthr;
                    ss[t] = si < stop ? si : s0;
                }
                Samples1d<M, R, kTiles1d, T> sp;
                sp.load(d_soa, g_soa, yref, ss, n_pool);
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    if (!lj[j]) continue;
                    asm volatile("" ::: "memory");       // one candidate at a time
                    // an opaque zero offset keeps the matrix reads inside the loop
                    int z0 = 0;
                    asm volatile("" : "+v"(z0));
                    const int sj = min(nj[j], start + chunk);
                    bool ok[kTiles1d];
#pragma unroll
                    for (int t = 0; t < kTiles1d; ++t) ok[t] = s0 + t * nthr < sj;
                    err[j] += tile_error_1d<M, R, kTiles1d, Z, T>(sp, ok, &sm[j][0] + z0);
                }
            }
        } else {
            for (int s = start + tid; s < stop; s += nthr) {
                int z0 = 0;
                asm volatile("" : "+v"(z0));
                err[0] += tile_error_2d<M, R, Z, T>(d_soa, g_soa, yref, s, n_pool, &sm[0][0] + z0);
            }
        }
        // fixed-order reduction: a butterfly inside each wave, then the wave
        // sums in wave order
#pragma unroll
        for (int j = 0; j < G; ++j) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) err[j] += __shfl_xor(err[j], off, 64);
            if ((tid & 63) == 0) red[j][tid >> 6] = err[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (tid == j && grp * G + j < n_cand) {
                double tot = red[j][0];
                for (int wv = 1; wv < nthr / 64; ++wv) tot += red[j][wv];
                partial[(size_t)(grp * G + j) * ipc + ch] = lj[j] ? tot : 0.0;
            }
    }
}

__global__ __launch_bounds__(256) void sweep_finalize_kernel(const double* __restrict__ partial,
                                                             const double* __restrict__ prefix,
                                                             const int* __restrict__ flags,
                                                             const int* __restrict__ counts, int n_cand,
                                                             int n_pool, int ipc, int outs_per_sample,
                                                             double* __restrict__ out) {
    const int cand = blockIdx.x * 256 + threadIdx.x;
    if (cand >= n_cand) return;
    int n = counts[cand];
    n = n < 0 ? 0 : (n > n_pool ? n_pool : n);
    double e = 0.0;
    for (int q = 0; q < ipc; ++q) e += partial[(size_t)cand * ipc + q];
    const int fl = flags[cand] & kFlagBad;
    out[(size_t)cand * 4 + 0] = fl ? INFINITY : e;
    out[(size_t)cand * 4 + 1] = prefix[n];
    out[(size_t)cand * 4 + 2] = (double)n * outs_per_sample;
    out[(size_t)cand * 4 + 3] = (double)fl;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int hipc(hipError_t e, const char* what) { return hip_check((int)e, what); }

template <int M, int R, int DIMS>
struct SweepOps {
    template <bool FAM, typename T>
    static void eval(const Sweep& S, const SweepArgs& a, const SweepTune& t, hipStream_t st, long grid, int ipc,
                     const T* mats) {
        hipLaunchKernelGGL((sweep_eval_kernel<M, R, DIMS, FAM, T>), dim3((unsigned)grid), dim3(t.block), 0, st,
                           S.d_soa, S.g_soa, S.yref, mats, S.flags, a.counts, a.n_cand, S.n_pool, ipc, t.chunk,
                           S.partial);
    }
    static void reference(const Sweep& S, hipStream_t st) {
        hipLaunchKernelGGL((sweep_reference_kernel<M, R, DIMS>), dim3((S.n_pool + 255) / 256), dim3(256), 0, st,
                           S.d_pool, S.g_pool, S.n_pool, S.d_soa, S.g_soa, S.yref, S.ref_abs);
        hipLaunchKernelGGL(sweep_prefix_kernel, dim3(1), dim3(64), 0, st, S.ref_abs, S.n_pool, S.prefix);
    }
    static void run(const Sweep& S, const SweepArgs& a, const SweepTune& t, hipStream_t st) {
        const int ipc = (S.n_pool + t.chunk - 1) / t.chunk;
        double* m64 = S.mixed ? S.mats64 : nullptr;
        const unsigned cons_grid = (unsigned)((a.n_cand + kConsCands - 1) / kConsCands);
        hipLaunchKernelGGL((sweep_construct_kernel<M, R>), dim3(cons_grid, M + R - 1), dim3(kConsCands), 0, st,
                           a.c1, a.c2, a.pts, a.n_cand, (S.exact_all || S.mixed) ? 1 : 0, S.mats, S.row_status);
        hipLaunchKernelGGL((sweep_rebuild_kernel<M, R>), dim3(cons_grid), dim3(kConsCands * (M + R - 1)), 0, st,
                           a.c1, a.c2, a.pts, a.n_cand, S.exact_all, S.row_status, S.mats, m64, S.flags);
        const long items = (long)((a.n_cand + (DIMS == 1 ? kGroup1d : 1) - 1) / (DIMS == 1 ? kGroup1d : 1)) * ipc;
        long grid = (long)S.n_cu * t.blocks_per_cu;
        if (grid > items) grid = items;
        if (grid < 1) grid = 1;
        if (S.mixed) {
            if (a.pts == nullptr) eval<true>(S, a, t, st, grid, ipc, (const double*)S.mats64);
            else eval<false>(S, a, t, st, grid, ipc, (const double*)S.mats64);
        } else {
            if (a.pts == nullptr) eval<true>(S, a, t, st, grid, ipc, (const float*)S.mats);
            else eval<false>(S, a, t, st, grid, ipc, (const float*)S.mats);
        }
        hipLaunchKernelGGL(sweep_finalize_kernel, dim3((a.n_cand + 255) / 256), dim3(256), 0, st, S.partial,
                           S.prefix, S.flags, a.counts, a.n_cand, S.n_pool, ipc, DIMS == 1 ? M : M * M, a.out);
    }
};

#define WG_SWEEP_SIZES(X) \
    X(2, 3) X(3, 3) X(4, 3) X(5, 3) X(6, 3) X(7, 3) X(8, 3) X(2, 5) X(3, 5) X(4, 5) X(5, 5) X(6, 5)

static bool sweep_supported(int m, int r) {
    switch (m * 16 + r) {
#define WG_SW_CASE(MM, RR) case MM * 16 + RR: return true;
        WG_SWEEP_SIZES(WG_SW_CASE)
#undef WG_SW_CASE
        default: return false;
    }
}

static void dispatch_reference(const Sweep& S, hipStream_t st) {
    switch (S.m * 16 + S.r) {
#define WG_SW_CASE(MM, RR)                                                              \
    case MM * 16 + RR:                                                                  \
        if (S.dims == 1) SweepOps<MM, RR, 1>::reference(S, st);                         \
        else SweepOps<MM, RR, 2>::reference(S, st);                                      \
        return;
        WG_SWEEP_SIZES(WG_SW_CASE)
#undef WG_SW_CASE
        default: return;
    }
}

static void dispatch_run(const Sweep& S, const SweepArgs& a, const SweepTune& t, hipStream_t st) {
    switch (S.m * 16 + S.r) {
#define WG_SW_CASE(MM, RR)                                                              \
    case MM * 16 + RR:                                                                  \
        if (S.dims == 1) SweepOps<MM, RR, 1>::run(S, a, t, st);                         \
        else SweepOps<MM, RR, 2>::run(S, a, t, st);                                      \
        return;
        WG_SWEEP_SIZES(WG_SW_CASE)
#undef WG_SW_CASE
        default: return;
    }
}

static const SweepTune kCandidates[] = {
    {64, 64, 8}, {64, 128, 8}, {128, 128, 4}, {128, 256, 4}, {256, 256, 2},
    {256, 512, 2}, {128, 128, 8}, {256, 256, 4}, {64, 256, 8}, {128, 512, 4},
    {128, 1024, 4}, {256, 1024, 4}, {64, 512, 8}, {128, 2048, 4}, {64, 1024, 8}, {256, 2048, 2},
};

static void release(Sweep* S) {
    if (!S) return;
    if (S->exec) (void)hipGraphExecDestroy(S->exec);
    if (S->graph) (void)hipGraphDestroy(S->graph);
    if (S->cap_stream) (void)hipStreamDestroy(S->cap_stream);
    void* bufs[] = {S->d_soa, S->g_soa, S->yref, S->ref_abs, S->prefix, S->mats, S->mats64, S->flags, S->row_status,
                    S->partial};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete S;
}

}  // namespace wg

using namespace wg;

extern "C" {

int wg_sweep_create(wg_sweep** out, int m, int r, int dims, const float* d_pool, const float* g_pool,
                    int n_pool, int max_cand, wg_stream_t stream) {
    if (!out || !d_pool || !g_pool) return fail(WG_EINVAL, "wg_sweep_create: null pointer");
    if (dims != 1 && dims != 2) return fail(WG_EINVAL, "wg_sweep_create: dims must be 1 or 2");
    if (n_pool <= 0 || max_cand <= 0) return fail(WG_EINVAL, "wg_sweep_create: sizes must be positive");
    if (!sweep_supported(m, r))
        return fail(WG_EUNSUPPORTED, "wg_sweep_create: F(" + std::to_string(m) + "," + std::to_string(r) +
                                         ") has no point family here (alpha = m+r-1 must be 4..10, r 3 or 5)");
    Sweep* S = new (std::nothrow) Sweep();
    if (!S) return fail(WG_ENOMEM, "wg_sweep_create: out of host memory");
    S->m = m; S->r = r; S->dims = dims; S->alpha = m + r - 1;
    S->n_pool = n_pool; S->max_cand = max_cand;
    S->d_pool = d_pool; S->g_pool = g_pool;
    int dev = 0;
    int st = hipc(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    if (st == WG_OK) st = hipc(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (st != WG_OK) { release(S); return st; }
    S->n_cu = prop.multiProcessorCount;
    const int outs = dims == 1 ? m : m * m;
    const size_t max_ipc = (size_t)(n_pool + 63) / 64;
    const int a2 = dims == 1 ? S->alpha : S->alpha * S->alpha, r2 = dims == 1 ? r : r * r;
    struct { void** p; size_t bytes; } allocs[] = {
        {(void**)&S->d_soa, sizeof(float) * (size_t)n_pool * a2},
        {(void**)&S->g_soa, sizeof(float) * (size_t)n_pool * r2},
        {(void**)&S->yref, sizeof(double) * (size_t)n_pool * outs},
        {(void**)&S->ref_abs, sizeof(double) * (size_t)n_pool},
        {(void**)&S->prefix, sizeof(double) * (size_t)(n_pool + 1)},
        {(void**)&S->mats, sizeof(float) * (size_t)max_cand * kMatStride},
        {(void**)&S->flags, sizeof(int) * (size_t)max_cand},
        {(void**)&S->row_status, (size_t)kRowStride * max_cand},
        {(void**)&S->partial, sizeof(double) * (size_t)max_cand * max_ipc},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            release(S);
            return fail(WG_ENOMEM, "wg_sweep_create: device allocation failed");
        }
    }
    st = hipc(hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (st != WG_OK) { release(S); return st; }
    dispatch_reference(*S, static_cast<hipStream_t>(stream));
    st = hipc(hipGetLastError(), "sweep reference");
    if (st == WG_OK) st = hipc(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "sweep reference");
    if (st != WG_OK) { release(S); return st; }
    S->tune = SweepTune{128, 2048, 4};      // the shape the autotuner picks for F(6,3) on 2000 samples
    *out = reinterpret_cast<wg_sweep*>(S);
    return WG_OK;
}

int wg_sweep_destroy(wg_sweep* sweep) {
    release(reinterpret_cast<Sweep*>(sweep));
    return WG_OK;
}

static int check_args(const Sweep& S, const double* c1, const int* counts, int n_cand, double* out,
                      const char* who = "wg_sweep_run") {
    if (!c1 || !counts || !out) return fail(WG_EINVAL, std::string(who) + ": null pointer");
    if (n_cand <= 0 || n_cand > S.max_cand)
        return fail(WG_EINVAL, std::string(who) + ": n_cand must be 1.." + std::to_string(S.max_cand));
    return WG_OK;
}

int wg_sweep_autotune(wg_sweep* sweep, const double* c1, const double* c2, const int* counts, int n_cand,
                      double* out, wg_stream_t stream) {
    if (!sweep) return fail(WG_EINVAL, "wg_sweep_autotune: null sweep");
    Sweep& S = *reinterpret_cast<Sweep*>(sweep);
    int st = check_args(S, c1, counts, n_cand, out);
    if (st != WG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SweepArgs a{c1, c2, counts, n_cand, out, nullptr};
    hipEvent_t e0, e1;
    if ((st = hipc(hipEventCreate(&e0), "hipEventCreate")) != WG_OK) return st;
    if ((st = hipc(hipEventCreate(&e1), "hipEventCreate")) != WG_OK) { (void)hipEventDestroy(e0); return st; }
    float best = 1e30f;
    SweepTune best_t = S.tune;
    for (const SweepTune& t : kCandidates) {
        if ((size_t)((S.n_pool + t.chunk - 1) / t.chunk) > (size_t)(S.n_pool + 63) / 64) continue;
        dispatch_run(S, a, t, s);                         // warm
        (void)hipEventRecord(e0, s);
        dispatch_run(S, a, t, s);
        dispatch_run(S, a, t, s);
        (void)hipEventRecord(e1, s);
        if ((st = hipc(hipEventSynchronize(e1), "sweep autotune")) != WG_OK) break;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            best_t = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != WG_OK) return st;
    S.tune = best_t;
    S.tuned = true;
    if (S.exec) { (void)hipGraphExecDestroy(S.exec); S.exec = nullptr; }
    if (S.graph) { (void)hipGraphDestroy(S.graph); S.graph = nullptr; }
    return WG_OK;
}

int wg_sweep_tuning(const wg_sweep* sweep, int* block, int* chunk, int* blocks_per_cu) {
    if (!sweep) return fail(WG_EINVAL, "wg_sweep_tuning: null sweep");
    const Sweep& S = *reinterpret_cast<const Sweep*>(sweep);
    if (block) *block = S.tune.block;
    if (chunk) *chunk = S.tune.chunk;
    if (blocks_per_cu) *blocks_per_cu = S.tune.blocks_per_cu;
    return S.tuned ? 1 : 0;
}

// Replays the captured graph of this argument set, capturing it first when
// the arguments differ from the last capture.
static int run_graph(Sweep& S, const SweepArgs& a, wg_stream_t stream) {
    int st = WG_OK;
    if (!S.exec || !(a == S.captured)) {
        if (S.exec) { (void)hipGraphExecDestroy(S.exec); S.exec = nullptr; }
        if (S.graph) { (void)hipGraphDestroy(S.graph); S.graph = nullptr; }
        st = hipc(hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (st != WG_OK) return st;
        dispatch_run(S, a, S.tune, S.cap_stream);
        const int launch = hipc(hipGetLastError(), "sweep capture");
        st = hipc(hipStreamEndCapture(S.cap_stream, &S.graph), "hipStreamEndCapture");
        if (launch != WG_OK) return launch;
        if (st != WG_OK) return st;
        st = hipc(hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        if (st != WG_OK) return st;
        S.captured = a;
    }
    return hipc(hipGraphLaunch(S.exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

int wg_sweep_run(wg_sweep* sweep, const double* c1, const double* c2, const int* counts, int n_cand,
                 double* out, wg_stream_t stream) {
    if (!sweep) return fail(WG_EINVAL, "wg_sweep_run: null sweep");
    Sweep& S = *reinterpret_cast<Sweep*>(sweep);
    int st = check_args(S, c1, counts, n_cand, out);
    if (st != WG_OK) return st;
    return run_graph(S, SweepArgs{c1, c2, counts, n_cand, out, nullptr}, stream);
}

int wg_sweep_run_points(wg_sweep* sweep, const double* pts, const int* counts, int n_cand, double* out,
                        wg_stream_t stream) {
    if (!sweep) return fail(WG_EINVAL, "wg_sweep_run_points: null sweep");
    Sweep& S = *reinterpret_cast<Sweep*>(sweep);
    int st = check_args(S, pts, counts, n_cand, out, "wg_sweep_run_points");
    if (st != WG_OK) return st;
    return run_graph(S, SweepArgs{nullptr, nullptr, counts, n_cand, out, pts}, stream);
}

int wg_sweep_set_precision(wg_sweep* sweep, int mode) {
    if (!sweep) return fail(WG_EINVAL, "wg_sweep_set_precision: null sweep");
    if (mode != WG_SWEEP_F32 && mode != WG_SWEEP_MIXED)
        return fail(WG_EINVAL, "wg_sweep_set_precision: mode must be WG_SWEEP_F32 or WG_SWEEP_MIXED");
    Sweep& S = *reinterpret_cast<Sweep*>(sweep);
    if (mode == WG_SWEEP_MIXED && !S.mats64) {
        if (hipMalloc(&S.mats64, sizeof(double) * (size_t)S.max_cand * kMatStride) != hipSuccess) {
            S.mats64 = nullptr;
            return fail(WG_ENOMEM, "wg_sweep_set_precision: device allocation failed");
        }
    }
    if (S.mixed != (mode == WG_SWEEP_MIXED)) {
        S.mixed = mode == WG_SWEEP_MIXED;
        if (S.exec) { (void)hipGraphExecDestroy(S.exec); S.exec = nullptr; }
        if (S.graph) { (void)hipGraphDestroy(S.graph); S.graph = nullptr; }
    }
    return WG_OK;
}

int wg_sweep_set_exact(wg_sweep* sweep, int always) {
    if (!sweep) return fail(WG_EINVAL, "wg_sweep_set_exact: null sweep");
    if (always != 0 && always != 1) return fail(WG_EINVAL, "wg_sweep_set_exact: always must be 0 or 1");
    Sweep& S = *reinterpret_cast<Sweep*>(sweep);
    if (S.exact_all != always) {
        S.exact_all = always;
        if (S.exec) { (void)hipGraphExecDestroy(S.exec); S.exec = nullptr; }
        if (S.graph) { (void)hipGraphDestroy(S.graph); S.graph = nullptr; }
    }
    return WG_OK;
}

int wg_sweep_matrices_f64(const wg_sweep* sweep, int cand, double* AT, double* G, double* BT) {
    if (!sweep || !AT || !G || !BT) return fail(WG_EINVAL, "wg_sweep_matrices_f64: null pointer");
    const Sweep& S = *reinterpret_cast<const Sweep*>(sweep);
    if (cand < 0 || cand >= S.max_cand) return fail(WG_EINVAL, "wg_sweep_matrices_f64: candidate out of range");
    if (!S.mats64) return fail(WG_EINVAL, "wg_sweep_matrices_f64: the sweep has not run in mixed precision");
    const int m = S.m, r = S.r, A = S.alpha;
    double buf[kMatStride];
    int st = hipc(hipMemcpy(buf, S.mats64 + (size_t)cand * kMatStride, sizeof(buf), hipMemcpyDeviceToHost),
                  "hipMemcpy");
    if (st != WG_OK) return st;
    std::memcpy(AT, buf, sizeof(double) * m * A);
    std::memcpy(G, buf + m * A, sizeof(double) * A * r);
    std::memcpy(BT, buf + m * A + A * r, sizeof(double) * A * A);
    return WG_OK;
}

int wg_sweep_matrices(const wg_sweep* sweep, int cand, float* AT, float* G, float* BT, int* flag) {
    if (!sweep || !AT || !G || !BT || !flag) return fail(WG_EINVAL, "wg_sweep_matrices: null pointer");
    const Sweep& S = *reinterpret_cast<const Sweep*>(sweep);
    if (cand < 0 || cand >= S.max_cand) return fail(WG_EINVAL, "wg_sweep_matrices: candidate out of range");
    const int m = S.m, r = S.r, A = S.alpha;
    float buf[kMatStride];
    int st = hipc(hipMemcpy(buf, S.mats + (size_t)cand * kMatStride, sizeof(buf), hipMemcpyDeviceToHost),
                  "hipMemcpy");
    int raw = 0;
    if (st == WG_OK) st = hipc(hipMemcpy(&raw, S.flags + cand, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
    if (st != WG_OK) return st;
    *flag = (raw & kFlagBad) ? 1 : ((raw & kFlagExact) ? 2 : 0);
    std::memcpy(AT, buf, sizeof(float) * m * A);
    std::memcpy(G, buf + m * A, sizeof(float) * A * r);
    std::memcpy(BT, buf + m * A + A * r, sizeof(float) * A * A);
    return WG_OK;
}

}  // extern "C"
