// Device-side helpers shared by the Winograd HIP kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wg {

constexpr int kXcdCount = 8;     // XCDs of the chip, each with its own L2
// Word 3 of a raw buffer resource on gfx9-family chips (dword data format,
// no swizzle); accesses outside the resource's range are dropped (stores)
// or read as zero (loads).
constexpr int kBufferWord3 = 0x00020000;

// The matrices of one F(M x M, R x R) algorithm (float32, or float64 for
// the float64 transforms of the mixed-precision layer), passed by value as a
// kernel argument so that every entry is a wave-uniform scalar.
template <int M_, int R_, typename E = float>
struct Mats {
    static constexpr int M = M_;
    static constexpr int R = R_;
    static constexpr int A = M_ + R_ - 1;
    E AT[M_][A];
    E G[A][R_];
    E BT[A][A];
};

// One term of an ascending-order inner product.  float: one fused
// multiply-add.  double (float64 transforms): a rounded product, then a
// rounded sum.
__device__ __forceinline__ float madd(float a, float b, float acc) { return __builtin_fmaf(a, b, acc); }
__device__ __forceinline__ double madd(double a, double b, double acc) { return acc + a * b; }

// Returns v unchanged but held in a vector register the compiler cannot see
// through.  Used for the stride between the planes of a transformed tensor:
// otherwise every plane's base address is a separate uniform value, they are
// all hoisted into scalar registers and spilled.
__device__ __forceinline__ size_t in_vgpr(size_t v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ int in_vgpr(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Element types of the Hadamard stage.
enum : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

template <int DT>
struct Elem;
typedef float wg_f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 wg_f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 wg_bf16x2 __attribute__((ext_vector_type(2)));

// store2: two adjacent elements (a at the lower address) in one store,
// rounded to nearest even by the packed conversions (v_cvt_pk_f16_f32 /
// v_cvt_pk_bf16_f32 on gfx950).
template <>
struct Elem<kF32> {
    using T = float;
    __device__ static __forceinline__ void store2(float* p, float a, float b) {
        *reinterpret_cast<wg_f32x2*>(p) = wg_f32x2{a, b};
    }
};
template <>
struct Elem<kF16> {
    using T = uint16_t;
    __device__ static __forceinline__ void store2(uint16_t* p, float a, float b) {
        const wg_f16x2 h = __builtin_convertvector(wg_f32x2{a, b}, wg_f16x2);
        *reinterpret_cast<uint32_t*>(p) = __builtin_bit_cast(uint32_t, h);
    }
};
template <>
struct Elem<kBF16> {
    using T = uint16_t;
    __device__ static __forceinline__ void store2(uint16_t* p, float a, float b) {
        const wg_bf16x2 h = __builtin_convertvector(wg_f32x2{a, b}, wg_bf16x2);
        *reinterpret_cast<uint32_t*>(p) = __builtin_bit_cast(uint32_t, h);
    }
};

}  // namespace wg

// The (m, r) pairs with compiled kernels: r in {3, 5}, 1 <= m <= 8.
#define WG_FOR_EACH_SIZE(X) \
    X(1, 3) X(2, 3) X(3, 3) X(4, 3) X(5, 3) X(6, 3) X(7, 3) X(8, 3) \
    X(1, 5) X(2, 5) X(3, 5) X(4, 5) X(5, 5) X(6, 5) X(7, 5) X(8, 5)
