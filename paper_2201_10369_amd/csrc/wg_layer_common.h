// Shared pieces of the layer transform kernels (filter, input, output):
// geometry passed to kernels, per-row exponent offsets for the 16-bit
// scaling, host-side packing of the transform matrices into kernel arguments
// and the launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <set>
#include <string>
#include <utility>

#include "wg_device.h"
#include "wg_internal.h"

namespace wg {

struct Geo {
    int N, C, K, H, W, pad, Hout, Wout, Th, Tw, P, P_pad, K_pad, C_pad;
};

inline Geo make_geo(const wg_layout& L) {
    return Geo{L.N, L.C, L.K, L.H, L.W, L.pad, L.Hout, L.Wout, L.Th, L.Tw, L.P, L.P_pad, L.K_pad, L.C_pad};
}

struct RowExps {
    int dB[kMaxAlpha];     // E(|B^T row i|_1) - E(|G row i|_1)
};

__device__ __forceinline__ int bin_exp(float v) {
    int e = 0;
    if (v != 0.0f) frexpf(v, &e);
    return e;
}

// floor(d / 2): arithmetic right shift of a two's-complement int
__device__ __forceinline__ int floor_half(int d) { return d >> 1; }

// ---------------------------------------------------------------------------
// Host-side packing and launch helpers
// ---------------------------------------------------------------------------
template <int M, int R, typename E = float>
inline Mats<M, R, E> pack_mats(const Plan& p) {
    constexpr int A = M + R - 1;
    constexpr bool d = sizeof(E) == 8;
    Mats<M, R, E> mt;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < A; ++j) mt.AT[i][j] = d ? (E)p.AT64[i * A + j] : (E)p.AT[i * A + j];
    for (int i = 0; i < A; ++i)
        for (int j = 0; j < R; ++j) mt.G[i][j] = d ? (E)p.G64[i * R + j] : (E)p.G[i * R + j];
    for (int i = 0; i < A; ++i)
        for (int j = 0; j < A; ++j) mt.BT[i][j] = d ? (E)p.BT64[i * A + j] : (E)p.BT[i * A + j];
    return mt;
}

inline int last_launch(const char* what) {
    return hip_check((int)hipGetLastError(), what);
}

// Raise a kernel's dynamic LDS limit above 64 KB (gfx950 has 160 KB per CU);
// done once per kernel and size.
template <typename F>
inline void allow_lds(F kernel, size_t bytes) {
    static std::mutex mu;
    static std::set<std::pair<const void*, size_t>> done;
    if (bytes <= 65536) return;
    const void* key = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    if (done.insert({key, bytes}).second)
        (void)hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------------------
// Zero structure of B^T shared by every point set that contains 0 and ends
// with infinity (the modified construction of Section 4.2, and all the
// families of Section 5): column 0 is nonzero only in the row of point 0
// (every other row's polynomial has the factor x), column alpha-1 only in the
// infinity row (the finite rows have degree alpha-2).  Kernels compiled for
// this structure leave those terms out; the host checks that the entries are
// exactly zero before choosing them, so the results are the same as with all
// terms (fma(0, x, acc) == acc for finite x).
// ---------------------------------------------------------------------------
struct ZeroShape {
    int z0;            // index of the point 0, or -1
    bool bt;           // the B^T pattern holds
};

inline ZeroShape zero_shape(const Plan& p) {
    const int A = p.L.alpha;
    ZeroShape z{-1, false};
    int found = 0;
    for (int i = 0; i < A - 1; ++i)
        if (p.BT[i * A] != 0.0f) {
            z.z0 = i;
            ++found;
        }
    if (found != 1 || p.BT[(A - 1) * A] != 0.0f) {
        z.z0 = -1;
        return z;
    }
    z.bt = true;
    for (int i = 0; i < A - 1; ++i)
        if (p.BT[i * A + (A - 1)] != 0.0f) z.bt = false;
    return z;
}

// B^T rows in processing order (with the structure: the row of point 0
// first, the infinity row last, the others ascending; else the identity),
// with each row's exponent offset and the element offset of its V' plane.
struct RowPerm {
    int row[kMaxAlpha];
    int dB[kMaxAlpha];
    unsigned plane_off[kMaxAlpha];           // elements; the launcher checks the range
};

inline RowPerm bt_row_perm(const Plan& p, bool structured, size_t plane_elems) {
    const int A = p.L.alpha;
    RowPerm rp{};
    int q = 0;
    if (structured) {
        const int z0 = zero_shape(p).z0;
        rp.row[q++] = z0;
        for (int i = 0; i < A - 1; ++i)
            if (i != z0) rp.row[q++] = i;
        rp.row[q++] = A - 1;
    } else {
        for (int i = 0; i < A; ++i) rp.row[q++] = i;
    }
    for (int k = 0; k < A; ++k) {
        rp.dB[k] = p.dB[rp.row[k]];
        rp.plane_off[k] = (unsigned)(rp.row[k] * plane_elems);
    }
    return rp;
}

// switch over the compiled (m, r) pairs; FN names a WG_CASE_FN(MM, RR) macro
#define WG_DISPATCH(FN, ...)                                              \
    switch (p.L.m * 16 + p.L.r) {                                         \
        WG_FOR_EACH_SIZE(WG_CASE_##FN)                                    \
        default: return fail(WG_EUNSUPPORTED, "tile size not compiled");   \
    }

}  // namespace wg
