// Winograd transform matrices from float64 points, exactly rounded, on the
// device (and on the host: every function here is __host__ __device__).
//
// Sections 4.1 and 4.2 of arXiv:2201.10369 define, for finite points
// a_0..a_{n-1} and the point at infinity last (the modified form):
//   A^T[j][i] = a_i^j                        (infinity: 1 in the last row)
//   G[i][k]   = a_i^k / N_i,  N_i = prod_{j != i} (a_i - a_j)
//                                             (infinity: 1 in the last column)
//   B^T[i][:] = coefficients of prod_{j != i} (x - a_j)
//                                             (infinity: of prod_j (x - a_j))
// Every float64 point is a dyadic rational, so every entry has an exact
// rational value v.  The matrices used are RN64(v), the nearest float64 with
// ties to even, and RN32(RN64(v)) for the float32 evaluation, as in the exact
// host construction.  Three ways to get there, each used where the one
// before cannot decide:
//
//  1. float64 arithmetic with a running error bound (ArithF64): every
//     operation adds its own rounding error, computed exactly by an
//     error-free transformation, to the bound it inherits (so exactly
//     computed values carry none).  It decides RN32(RN64(v)) when no float32
//     rounding boundary (a float32 midpoint, within one float64 unit) lies
//     within the bound: float32 midpoints are 2^29 times further apart than
//     float64 ones, so this nearly always succeeds.
//  2. double words (ArithDW): hi + lo with hi = RN64(hi + lo) and a bound on
//     |v - (hi + lo)|; decides RN64(v) when no float64 rounding boundary
//     lies within the bound.  Products of two double words and quotients
//     use the published algorithms of Joldes, Muller and Popescu ("Tight and
//     rigorous error bounds for basic building blocks of double-word
//     arithmetic", ACM TOMS 44(2), 2017: DWTimesDW with fmas, relative error
//     < 5u^2; DWDivDW, < 15u^2 + 56u^3; u = 2^-53), each charged 2^-95 of
//     its result (over 2000 u^2).  Sums, and products by a float64, are
//     four-term cascades of error-free transformations (Knuth's TwoSum, the
//     fma product) whose two rounding errors are themselves computed, so
//     their bound is exact and exact results carry none: a sum of float64
//     roots lies on a float64 midpoint often, and only an exact bound decides
//     its rounding.
//  3. exact integers (exact_row): writing every point as a_j = I_j 2^-F with
//     integers I_j, each entry is an integer, or a ratio of integers, times a
//     power of two (the scheme of construct_exact in the host library),
//     evaluated with 32-bit limbs and rounded once.
//
// Both bounded forms group the roots of each B^T row first: zero roots (a
// shift), pairs {a, -a} (one factor x^2 - a^2, a^2 exact) and the rest two
// at a time, each root with the remaining one closest to its negative (one
// factor x^2 - s x + p, s = u + v and p = u v), a last one alone.  Coefficients that vanish by
// the +-a symmetry (the point families of Section 5 are built to make them
// vanish) are never computed, so they come out as exact zeros with a zero
// bound, and near-negatives (float64 Chebyshev nodes, a family's d next to
// its 1/c) do not cancel through their small sum.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace wg {
namespace cons {

// ---------------------------------------------------------------------------
// Error-free transformations
// ---------------------------------------------------------------------------
struct DW {
    double hi, lo;    // value hi + lo, hi = RN64(hi + lo)
    double err;       // |exact - (hi + lo)| <= err
};

constexpr double kOpRel = 0x1p-95;      // charged per double-word product or quotient
constexpr double kUp = 1.0 + 0x1p-40;   // covers the rounding of the bound arithmetic
constexpr double kBig = 0x1p600;        // bounded range of nonzero values
constexpr double kSmall = 0x1p-600;

__host__ __device__ inline DW two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e, 0.0};
}

__host__ __device__ inline DW fast_two_sum(double a, double b) {   // |a| >= |b| or a == 0
    const double s = a + b;
    const double e = b - (s - a);
    return {s, e, 0.0};
}

__host__ __device__ inline DW two_prod(double a, double b) {
    const double p = a * b;
    return {p, fma(a, b, -p), 0.0};
}

// two_prod whose error term may be inexact when the product of nonzero
// operands falls below 2^-960: err_extra then grows by 2^-1070
__host__ __device__ inline DW two_prod_b(double a, double b, double& err_extra) {
    const DW t = two_prod(a, b);
    if (a != 0.0 && b != 0.0 && fabs(t.hi) < 0x1p-960) err_extra += 0x1p-1070;
    return t;
}

__host__ __device__ inline bool in_range(double v) {
    const double a = fabs(v);
    return v == 0.0 || (a >= kSmall && a <= kBig);
}

// ---------------------------------------------------------------------------
// 1. float64 with a running error bound
// ---------------------------------------------------------------------------
struct FB {
    double v;      // computed value
    double err;    // |exact - v| <= err
};

struct ArithF64 {
    using T = FB;
    __host__ __device__ static T of(double a) { return {a, 0.0}; }
    __host__ __device__ static T neg(const T& x) { return {-x.v, x.err}; }
    // a + b and a * b of float64 inputs, their rounding errors computed
    __host__ __device__ static T sum2(double a, double b, bool& ok) {
        const DW s = two_sum(a, b);
        if (!in_range(s.hi)) ok = false;
        return {s.hi, fabs(s.lo)};
    }
    __host__ __device__ static T prod2(double a, double b, bool& ok) {
        double extra = 0.0;
        const DW p = two_prod_b(a, b, extra);
        if (!in_range(p.hi) || (p.hi == 0.0 && a != 0.0 && b != 0.0)) ok = false;
        return {p.hi, fabs(p.lo) + extra};
    }
    // every rounding error below is the exact one (TwoSum, the fma product
    // residual, the fma quotient residual x - z y, which is representable),
    // so results computed without rounding carry a zero bound
    __host__ __device__ static T add(const T& x, const T& y, bool& ok) {
        const DW s = two_sum(x.v, y.v);
        if (!in_range(s.hi)) ok = false;
        const double e = x.err + y.err + fabs(s.lo);
        return {s.hi, e == 0.0 ? 0.0 : e * kUp};
    }
    __host__ __device__ static T mul(const T& x, const T& y, bool& ok) {
        double extra = 0.0;
        const DW p = two_prod_b(x.v, y.v, extra);
        if (!in_range(p.hi) || (p.hi == 0.0 && x.v != 0.0 && y.v != 0.0)) ok = false;
        const double e = fabs(x.v) * y.err + fabs(y.v) * x.err + x.err * y.err + fabs(p.lo) + extra;
        return {p.hi, e == 0.0 ? 0.0 : e * kUp};
    }
    __host__ __device__ static T mul_d(const T& x, double y, bool& ok) {
        double extra = 0.0;
        const DW p = two_prod_b(x.v, y, extra);
        if (!in_range(p.hi) || (p.hi == 0.0 && x.v != 0.0 && y != 0.0)) ok = false;
        const double e = fabs(y) * x.err + fabs(p.lo) + extra;
        return {p.hi, e == 0.0 ? 0.0 : e * kUp};
    }
    __host__ __device__ static T div(const T& x, const T& y, bool& ok) {
        if (y.v == 0.0 || !(fabs(y.v) > 4.0 * y.err)) {
            ok = false;
            return {0.0, 0.0};
        }
        const double z = x.v / y.v;
        if (!in_range(z) || (z == 0.0 && x.v != 0.0)) ok = false;
        const double r = fma(-z, y.v, x.v);             // x - z y exactly
        double e = fabs(r) / fabs(y.v) * 1.01;
        if (x.err != 0.0 || y.err != 0.0) e += 1.01 * (x.err + fabs(z) * y.err) / (fabs(y.v) - 2.0 * y.err);
        return {z, e == 0.0 ? 0.0 : e * kUp};
    }
    __host__ __device__ static double value(const T& x) { return x.v; }
    __host__ __device__ static double bound(const T& x) { return x.err; }
    // RN32(RN64(exact)) when the bound decides it.  The function changes
    // value only within one float64 unit of a float32 midpoint; f = RN32(v)
    // is the answer when v stays clear of the midpoints around f by more
    // than the bound plus that unit (around a power of two the midpoint
    // below is half as far).
    __host__ __device__ static bool certify(const T& x, double& v64, float& v32) {
        v64 = x.v;
        if (x.err == 0.0) {                         // exact float64 value
            v64 = x.v == 0.0 ? 0.0 : x.v;
            v32 = (float)v64;
            return true;
        }
        const double a = fabs(x.v);
        if (!(a >= 0x1p-100 && a <= 0x1p100)) return false;
        const float f = (float)x.v;
        const double fd = (double)f;
        int e = 0;
        (void)frexp(fabs(fd), &e);                  // |f| in [2^(e-1), 2^e)
        const double up = ldexp(1.0, e - 25);       // half a float32 unit at f
        const double down = fabs(fd) == ldexp(0.5, e) ? 0.5 * up : up;
        const double d_out = fd > 0.0 ? x.v - fd : fd - x.v;   // exact (Sterbenz)
        const double slack = 1.01 * x.err + ldexp(fabs(fd), -51);
        if (!(up - d_out > slack) || !(down + d_out > slack)) return false;
        v32 = f;
        return true;
    }
};

// ---------------------------------------------------------------------------
// 2. double words with an error bound
// ---------------------------------------------------------------------------
// Sum of four float64 terms as a double word whose error is the exact sum
// of the two rounding errors the cascade commits (every other step is an
// error-free transformation).
__host__ __device__ inline DW sum4(double a, double b, double c, double d) {
    const DW s1 = two_sum(a, b);
    const DW s2 = two_sum(c, d);
    const DW h = two_sum(s1.hi, s2.hi);
    const DW l = two_sum(s1.lo, s2.lo);
    const DW m = two_sum(h.lo, l.hi);              // total = h.hi + m.hi + m.lo + l.lo
    const DW t = two_sum(m.lo, l.lo);              // t.hi rounded, error t.lo
    const DW u = two_sum(h.hi, m.hi);              // total = u.hi + u.lo + t.hi + t.lo
    const DW w = two_sum(u.lo, t.hi);              // w.hi rounded, error w.lo
    DW z = two_sum(u.hi, w.hi);                    // total = z.hi + z.lo + t.lo + w.lo
    z.err = 1.01 * (fabs(t.lo) + fabs(w.lo));
    return z;
}

struct ArithDW {
    using T = DW;
    __host__ __device__ static T of(double a) { return {a, 0.0, 0.0}; }
    __host__ __device__ static T neg(const T& x) { return {-x.hi, -x.lo, x.err}; }
    __host__ __device__ static T sum2(double a, double b, bool& ok) {
        const DW s = two_sum(a, b);
        if (!in_range(s.hi)) ok = false;
        return s;
    }
    __host__ __device__ static T prod2(double a, double b, bool& ok) {
        double extra = 0.0;
        DW p = two_prod_b(a, b, extra);
        if (!in_range(p.hi) || (p.hi == 0.0 && a != 0.0 && b != 0.0)) ok = false;
        p.err = extra;
        return p;
    }
    __host__ __device__ static T add(const T& x, const T& y, bool& ok) {
        DW z = sum4(x.hi, y.hi, x.lo, y.lo);
        z.err += 1.01 * (x.err + y.err);
        if (!in_range(z.hi)) ok = false;
        return z;
    }
    // the four-term sum of the exact products hi*y and lo*y
    __host__ __device__ static T mul_d(const T& x, double y, bool& ok) {
        double extra = 0.0;
        const DW p = two_prod_b(x.hi, y, extra);
        const DW q = two_prod_b(x.lo, y, extra);
        DW z = sum4(p.hi, p.lo, q.hi, q.lo);
        z.err += 1.01 * fabs(y) * x.err + extra;
        if (!in_range(z.hi) || (z.hi == 0.0 && x.hi != 0.0 && y != 0.0)) ok = false;
        return z;
    }
    __host__ __device__ static T mul(const T& x, const T& y, bool& ok) {
        if (x.lo == 0.0 && x.err == 0.0) return mul_d(y, x.hi, ok);
        if (y.lo == 0.0 && y.err == 0.0) return mul_d(x, y.hi, ok);
        const DW c = two_prod(x.hi, y.hi);
        const double tl0 = x.lo * y.lo;
        const double tl1 = fma(x.hi, y.lo, tl0);
        const double cl2 = fma(x.lo, y.hi, tl1);
        const double cl3 = c.lo + cl2;
        DW z = fast_two_sum(c.hi, cl3);
        z.err = 1.01 * (fabs(x.hi) * y.err + fabs(y.hi) * x.err + x.err * y.err) + kOpRel * fabs(z.hi);
        if (!in_range(z.hi) || (z.hi == 0.0 && x.hi != 0.0 && y.hi != 0.0)) ok = false;
        return z;
    }
    __host__ __device__ static T div(const T& x, const T& y, bool& ok) {
        if (y.hi == 0.0 || !(fabs(y.hi) > 4.0 * y.err)) {
            ok = false;
            return {0.0, 0.0, 0.0};
        }
        const double th = x.hi / y.hi;
        bool ok_r = true;
        const DW r = mul_d({y.hi, y.lo, 0.0}, th, ok_r);
        const DW pi = two_sum(x.hi, -r.hi);
        const double dh = pi.lo - r.lo;
        const double dl = dh + x.lo;
        const double d = pi.hi + dl;
        const double tl = d / y.hi;
        DW z = fast_two_sum(th, tl);
        z.err = 1.01 * (x.err + fabs(z.hi) * y.err) / (fabs(y.hi) - 2.0 * y.err) + kOpRel * fabs(z.hi);
        if (!in_range(z.hi) || (z.hi == 0.0 && x.hi != 0.0)) ok = false;
        return z;
    }
    __host__ __device__ static double value(const T& x) { return x.hi; }
    __host__ __device__ static double bound(const T& x) { return x.err; }
    // RN64 of the exact value when the bound decides it.  A positive hi is
    // RN64(v) for every v strictly between hi - d_down and hi + d_up, d_up =
    // ulp(hi)/2 and d_down = ulp(hi)/2, or ulp(hi)/4 when hi is a power of
    // two (the binade below has half the spacing); mirrored for a negative
    // hi.  |lo| <= d, so each distance below is exact when it is under d/2
    // (Sterbenz) and far above the bound otherwise.
    __host__ __device__ static bool certify(const T& x, double& v64, float& v32) {
        if (x.err == 0.0) {                        // exact double word
            v64 = x.hi == 0.0 ? 0.0 : x.hi;
            v32 = (float)v64;
            return true;
        }
        const double a = fabs(x.hi);
        if (!(a >= 0x1p-900 && a <= 0x1p900)) return false;
        int e = 0;
        (void)frexp(a, &e);                        // a in [2^(e-1), 2^e)
        const double ulp = ldexp(1.0, e - 53);
        const double up = 0.5 * ulp;
        const double down = a == ldexp(0.5, e) ? 0.25 * ulp : 0.5 * ulp;
        const double lo_out = x.hi > 0.0 ? x.lo : -x.lo;       // component away from zero
        const double err = 1.01 * x.err;
        if (!(up - lo_out > err) || !(down + lo_out > err)) return false;
        v64 = x.hi;
        v32 = (float)x.hi;
        return true;
    }
};

// ---------------------------------------------------------------------------
// One row of a candidate's matrices in a bounded arithmetic
// ---------------------------------------------------------------------------
// Entry layout of a row: A^T column i at [0, M), G row i at [M, M + R), B^T
// row i at [M + R, M + R + A).
template <int M, int R>
struct RowOut {
    static constexpr int kN = M + R + (M + R - 1);
    double v64[kN];
    float v32[kN];
};

// Coefficients (ascending) of prod (x - roots[t]) over the first n roots,
// certified into c64/c32; false when one cannot be decided.  The roots are
// first sorted into zeros (a shift), quadratic factors x^2 - s x + p (pairs
// {a, -a}: s = 0, p = -a^2 exactly; then the rest two at a time, each with
// the remaining root closest to its negative) and at most one linear
// factor; every list is filled with constant indices (no dynamically
// indexed private arrays on the device).
template <class P, int NMAX>
__host__ __device__ inline bool poly_cert(const double* roots, int n, double* c64, float* c32) {
    using T = typename P::T;
    constexpr int NQ = NMAX / 2;
    bool ok = true;
    int zeros = 0, nq = 0;
    unsigned used = 0;
    T qs[NQ > 0 ? NQ : 1], qp[NQ > 0 ? NQ : 1];
    // zero roots and pairs {a, -a}
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j >= n || ((used >> j) & 1u)) continue;
        const double a = roots[j];
        if (a == 0.0) {
            ++zeros;
            used |= 1u << j;
            continue;
        }
        int partner = -1;
#pragma unroll
        for (int k = j + 1; k < NMAX; ++k)
            if (partner < 0 && k < n && !((used >> k) & 1u) && roots[k] == -a) partner = k;
        if (partner < 0) continue;
        used |= (1u << j) | (1u << partner);
        const T pp = P::prod2(a, -a, ok);
#pragma unroll
        for (int f = 0; f < NQ; ++f)
            if (f == nq) {
                qs[f] = P::of(0.0);
                qp[f] = pp;
            }
        ++nq;
    }
    // the rest two at a time, each with the remaining root closest to its
    // negative; a last single root stays linear
    bool has_lin = false;
    double lin = 0.0;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j >= n || ((used >> j) & 1u)) continue;
        used |= 1u << j;
        const double u = roots[j];
        int best = -1;
        double best_gap = 0.0, v = 0.0;
#pragma unroll
        for (int k = j + 1; k < NMAX; ++k) {
            if (k < n && !((used >> k) & 1u)) {
                const double gap = fabs(u + roots[k]);
                if (best < 0 || gap < best_gap) {
                    best = k;
                    best_gap = gap;
                    v = roots[k];
                }
            }
        }
        if (best < 0) {
            has_lin = true;
            lin = u;
            continue;
        }
        used |= 1u << best;
        const T ss = P::sum2(u, v, ok), pp = P::prod2(u, v, ok);
#pragma unroll
        for (int f = 0; f < NQ; ++f)
            if (f == nq) {
                qs[f] = ss;
                qp[f] = pp;
            }
        ++nq;
    }
    // c <- prod of the factors: c[l] <- c[l-2] - s c[l-1] + p c[l]
    T c[NMAX + 1];
#pragma unroll
    for (int l = 0; l <= NMAX; ++l) c[l] = P::of(l == 0 ? 1.0 : 0.0);
#pragma unroll
    for (int f = 0; f < NQ; ++f) {
        if (f >= nq) continue;
        const int deg = 2 * f;
#pragma unroll
        for (int l = 2 * f + 2; l >= 0; --l) {
            T t = l <= deg ? P::mul(qp[f], c[l], ok) : P::of(0.0);
            if (l >= 1 && l - 1 <= deg) t = P::add(t, P::neg(P::mul(qs[f], c[l - 1], ok)), ok);
            if (l >= 2) t = P::add(t, c[l - 2], ok);
            c[l] = t;
        }
    }
    int deg = 2 * nq;
    if (has_lin) {
#pragma unroll
        for (int l = NMAX; l >= 0; --l) {
            if (l > deg + 1) continue;
            const T prod = l <= deg ? P::mul_d(c[l], lin, ok) : P::of(0.0);
            const T prev = l >= 1 ? c[l - 1] : P::of(0.0);
            c[l] = P::add(prev, P::neg(prod), ok);
        }
        ++deg;
    }
    // times x^zeros
#pragma unroll
    for (int l = 0; l <= NMAX; ++l) {
        const int src = l - zeros;
        double v64 = 0.0;
        float v32 = 0.0f;
        if (src >= 0 && src <= deg) {
            T sel{};
#pragma unroll
            for (int q = 0; q <= NMAX; ++q)
                if (q == src) sel = c[q];
            if (!P::certify(sel, v64, v32)) ok = false;
        }
        c64[l] = v64;
        c32[l] = v32;
    }
    return ok;
}

// Row i of a candidate's matrices from its finite points pts[0..NF-1]
// (infinity last): for i < NF column i of A^T, row i of G and row i of B^T
// (the entries point i owns), for i = NF the infinity row and column.
// Returns 0 when every entry is decided, 1 when |RN64(N_i)| < 1e-300 is
// decided (N_i = 0: two points coincide), 2 when something is not decided.
template <class P, int M, int R>
__host__ __device__ inline int row_cert(const double* pts, int i, RowOut<M, R>& o) {
    using T = typename P::T;
    constexpr int A = M + R - 1;
    constexpr int NF = A - 1;
#pragma unroll
    for (int q = 0; q < M + R; ++q) {
        o.v64[q] = 0.0;
        o.v32[q] = 0.0f;
    }
    // the roots of row i: the other points in order (all points for the
    // infinity row), and point i, picked with constant indices (no
    // dynamically indexed private arrays on the device)
    double a = 0.0, roots[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (j == i) a = pts[j];
        roots[j] = (j < i || i == NF) ? pts[j] : (j + 1 < NF ? pts[j + 1] : 0.0);
    }
    const bool poly_ok = poly_cert<P, NF>(roots, i == NF ? NF : NF - 1, o.v64 + M + R, o.v32 + M + R);
    if (i == NF) {
        o.v64[M - 1] = 1.0;
        o.v32[M - 1] = 1.0f;
        o.v64[M + R - 1] = 1.0;
        o.v32[M + R - 1] = 1.0f;
        return poly_ok ? 0 : 2;
    }
    bool ok = in_range(a) && poly_ok;
    T norm = P::of(1.0);
#pragma unroll
    for (int j = 0; j + 1 < NF; ++j) norm = P::mul(norm, P::sum2(a, -roots[j], ok), ok);
    // |RN64(N)| < 1e-300 decided from the bound (1e-300 is a float64 value)
    const double nv = fabs(P::value(norm)), ne = P::bound(norm);
    if (!ok) return 2;
    if (ne == 0.0) {
        if (!(nv >= 1e-300)) return 1;
    } else if (nv + ne < 1e-300 * (1.0 - 0x1p-40)) {
        return 1;
    } else if (!(nv - ne > 1e-300)) {
        return 2;
    }
    T pw = P::of(1.0);
#pragma unroll
    for (int j = 0; j < (M > R ? M : R); ++j) {
        if (j < M && !P::certify(pw, o.v64[j], o.v32[j])) ok = false;
        if (j < R && !P::certify(P::div(pw, norm, ok), o.v64[M + j], o.v32[M + j])) ok = false;
        pw = P::mul_d(pw, a, ok);
    }
    return ok ? 0 : 2;
}

// ---------------------------------------------------------------------------
// 3. Exact integers: sign and magnitude in 32-bit limbs, little-endian
// ---------------------------------------------------------------------------
constexpr int kLimbs = 32;          // 1024 bits

struct Big {
    uint32_t w[kLimbs];
    int n;        // limbs in use (no leading zero limb); 0 means zero
    int neg;
};

__host__ __device__ inline void big_set_u64(Big& b, uint64_t v, int neg) {
    b.w[0] = (uint32_t)v;
    b.w[1] = (uint32_t)(v >> 32);
    b.n = b.w[1] ? 2 : (b.w[0] ? 1 : 0);
    b.neg = b.n ? neg : 0;
}

__host__ __device__ inline void big_zero(Big& b) {
    b.n = 0;
    b.neg = 0;
}

__host__ __device__ inline void big_trim(Big& b) {
    while (b.n > 0 && b.w[b.n - 1] == 0) --b.n;
    if (b.n == 0) b.neg = 0;
}

__host__ __device__ inline int big_bits(const Big& b) {
    if (b.n == 0) return 0;
    uint32_t top = b.w[b.n - 1];
    int nb = 0;
    while (top) {
        ++nb;
        top >>= 1;
    }
    return (b.n - 1) * 32 + nb;
}

__host__ __device__ inline int big_bit(const Big& b, int i) {
    if (i < 0) return 0;
    const int wi = i >> 5;
    return wi < b.n ? (int)((b.w[wi] >> (i & 31)) & 1u) : 0;
}

__host__ __device__ inline int big_cmp_mag(const Big& a, const Big& b) {
    if (a.n != b.n) return a.n < b.n ? -1 : 1;
    for (int i = a.n - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

// r = |a| + |b| (r may alias a or b); false when it outgrows kLimbs
__host__ __device__ inline bool big_add_mag(const Big& a, const Big& b, Big& r) {
    const int na = a.n, nb = b.n;
    const int n = na > nb ? na : nb;
    uint64_t carry = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t s = carry + (i < na ? a.w[i] : 0u) + (i < nb ? b.w[i] : 0u);
        r.w[i] = (uint32_t)s;
        carry = s >> 32;
    }
    r.n = n;
    if (carry) {
        if (n >= kLimbs) return false;
        r.w[n] = (uint32_t)carry;
        r.n = n + 1;
    }
    return true;
}

// r = |a| - |b| for |a| >= |b| (r may alias a or b)
__host__ __device__ inline void big_sub_mag(const Big& a, const Big& b, Big& r) {
    const int na = a.n, nb = b.n;
    int64_t borrow = 0;
    for (int i = 0; i < na; ++i) {
        int64_t d = (int64_t)a.w[i] - (i < nb ? (int64_t)b.w[i] : 0) - borrow;
        borrow = d < 0;
        if (d < 0) d += (int64_t)1 << 32;
        r.w[i] = (uint32_t)d;
    }
    r.n = na;
    big_trim(r);
}

// r = a + (negate_b ? -b : b); r must not alias a or b
__host__ __device__ inline bool big_add(const Big& a, const Big& b, int negate_b, Big& r) {
    const int bneg = b.n ? (b.neg ^ negate_b) : 0;
    if (a.n == 0 || b.n == 0 || a.neg == bneg) {
        const int sign = a.n ? a.neg : bneg;
        if (!big_add_mag(a, b, r)) return false;
        r.neg = sign;
        big_trim(r);
        return true;
    }
    const int c = big_cmp_mag(a, b);
    if (c == 0) {
        big_zero(r);
    } else if (c > 0) {
        big_sub_mag(a, b, r);
        r.neg = r.n ? a.neg : 0;
    } else {
        big_sub_mag(b, a, r);
        r.neg = r.n ? bneg : 0;
    }
    return true;
}

// r = a * b; r must not alias a or b
__host__ __device__ inline bool big_mul(const Big& a, const Big& b, Big& r) {
    if (a.n == 0 || b.n == 0) {
        big_zero(r);
        return true;
    }
    if (a.n + b.n > kLimbs) return false;
    for (int i = 0; i < a.n + b.n; ++i) r.w[i] = 0;
    for (int i = 0; i < a.n; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < b.n; ++j) {
            const uint64_t cur = (uint64_t)a.w[i] * b.w[j] + r.w[i + j] + carry;
            r.w[i + j] = (uint32_t)cur;
            carry = cur >> 32;
        }
        r.w[i + b.n] = (uint32_t)carry;
    }
    r.n = a.n + b.n;
    r.neg = a.neg ^ b.neg;
    big_trim(r);
    return true;
}

// r = |a| * 2^s, s >= 0, sign kept; r must not alias a
__host__ __device__ inline bool big_shl(const Big& a, int s, Big& r) {
    if (a.n == 0) {
        big_zero(r);
        return true;
    }
    const int nbits = big_bits(a) + s;
    if (nbits > kLimbs * 32) return false;
    const int ws = s >> 5, bs = s & 31;
    const int nn = (nbits + 31) >> 5;
    for (int i = 0; i < nn; ++i) r.w[i] = 0;
    for (int i = 0; i < a.n; ++i) {
        r.w[i + ws] |= a.w[i] << bs;
        if (bs && i + ws + 1 < nn) r.w[i + ws + 1] |= a.w[i] >> (32 - bs);
    }
    r.n = nn;
    r.neg = a.neg;
    big_trim(r);
    return true;
}

// Nearest float64 (ties to even) of sign * (q + f) * 2^E, with 2^62 <= q <
// 2^64 an integer and f in [0, 1) (sticky: f > 0).
__host__ __device__ inline double round_q(uint64_t q, int sticky, long E, int neg) {
    const int nb = (q >> 63) ? 64 : 63;
    const long e_top = E + nb - 1;                 // value in [2^e_top, 2^(e_top+1))
    long prec = 53;
    if (e_top < -1022) prec = 53 - (-1022 - e_top);  // subnormal range
    double r;
    if (prec < 0) {
        r = 0.0;
    } else {
        const int drop = nb - (int)prec;           // 10 .. 64
        uint64_t mant = drop >= 64 ? 0 : q >> drop;
        const uint64_t rest = drop >= 64 ? q : q & ((((uint64_t)1) << drop) - 1);
        const uint64_t half = ((uint64_t)1) << (drop - 1);
        bool up = false;
        if (rest > half) up = true;
        else if (rest == half) up = sticky || (mant & 1u);
        if (up) mant += 1;
        r = ldexp((double)mant, (int)(E + drop));
    }
    return neg ? -r : r;
}

// Nearest float64 of P * 2^s: the top 64 bits and a sticky bit.
__host__ __device__ inline double big_round(const Big& P, long s) {
    if (P.n == 0) return 0.0;
    const int nb = big_bits(P);
    uint64_t q = 0;
    int sticky = 0;
    if (nb <= 64) {
        q = (uint64_t)P.w[0] | (P.n > 1 ? (uint64_t)P.w[1] << 32 : 0);
        q <<= 64 - nb;
    } else {
        const int sh = nb - 64, ws = sh >> 5, bs = sh & 31;
        const uint64_t lo = P.w[ws], mid = ws + 1 < P.n ? P.w[ws + 1] : 0u,
                       hi = ws + 2 < P.n ? P.w[ws + 2] : 0u;
        q = bs == 0 ? (lo | (mid << 32)) : ((lo >> bs) | (mid << (32 - bs)) | (hi << (64 - bs)));
        sticky = (lo & ((1u << bs) - 1u)) != 0u;
        for (int k = 0; k < ws; ++k) sticky |= P.w[k] != 0u;
    }
    return round_q(q, sticky, s + nb - 64, P.neg);
}

// Nearest float64 of (P / Q) * 2^s for Q > 0: 64 quotient bits by long
// division, in place, with the remainder as the sticky bit.
__host__ __device__ inline bool big_round_ratio(const Big& P, const Big& Q, long s, double& out, Big& num,
                                                Big& den, Big& rem) {
    if (P.n == 0) {
        out = 0.0;
        return true;
    }
    // num / den in (2^62, 2^64)
    const int t = 63 + big_bits(Q) - big_bits(P);
    if (t >= 0) {
        if (!big_shl(P, t, num)) return false;
        den = Q;
    } else {
        num = P;
        if (!big_shl(Q, -t, den)) return false;
    }
    num.neg = den.neg = 0;
    // rem = num >> 64 (below den: two whole limbs dropped)
    rem.n = num.n > 2 ? num.n - 2 : 0;
    rem.neg = 0;
    for (int i = 0; i < rem.n; ++i) rem.w[i] = num.w[i + 2];
    uint64_t q = 0;
    for (int i = 63; i >= 0; --i) {
        // rem = 2 rem + bit i of num
        uint32_t carry = (uint32_t)big_bit(num, i);
        for (int k = 0; k < rem.n; ++k) {
            const uint32_t w = rem.w[k];
            rem.w[k] = (w << 1) | carry;
            carry = w >> 31;
        }
        if (carry) {
            if (rem.n >= kLimbs) return false;
            rem.w[rem.n++] = carry;
        }
        if (big_cmp_mag(rem, den) >= 0) {
            big_sub_mag(rem, den, rem);
            q |= ((uint64_t)1) << i;
        }
    }
    out = round_q(q, rem.n != 0, s - t, P.neg);
    return true;
}

// Row i of a candidate's matrices (layout of RowOut) from the exact values,
// rounded once to float64 and then to float32.  Returns 0 on success, 1
// when N_i = 0 or |RN64(N_i)| < 1e-300, 3 when an integer outgrows kLimbs
// limbs (nonzero points spanning more than about 2^40 in magnitude).
template <int M, int R>
__host__ __device__ inline int exact_row(const double* pts, int i, RowOut<M, R>& o) {
    constexpr int A = M + R - 1;
    constexpr int NF = A - 1;
    for (int q = 0; q < RowOut<M, R>::kN; ++q) o.v64[q] = 0.0;
    // a_j = I_j 2^-F with integers I_j
    Big I[NF];
    long minE = 0;
    bool any = false;
    for (int j = 0; j < NF; ++j) {
        if (pts[j] != 0.0) {
            int e = 0;
            (void)frexp(pts[j], &e);
            if (!any || e - 53 < minE) minE = e - 53;
            any = true;
        }
    }
    const long F = -minE;
    for (int j = 0; j < NF; ++j) {
        big_zero(I[j]);
        if (pts[j] == 0.0) continue;
        int e = 0;
        const double f = frexp(pts[j], &e);         // |f| in [0.5, 1)
        const int64_t mj = (int64_t)ldexp(f, 53);    // exact 53-bit integer
        Big b;
        big_set_u64(b, (uint64_t)(mj < 0 ? -mj : mj), mj < 0);
        if (!big_shl(b, (int)(e - 53 + F), I[j])) return 3;
    }
    // coefficients of prod (x - I_j) over the roots of this row, in place
    // from the top: C[l] <- C[l-1] - I_j C[l]
    Big C[A + 1], t1, t2;
    big_set_u64(C[0], 1, 0);
    int deg = 0;
    for (int j = 0; j < NF; ++j) {
        if (j == i) continue;
        for (int l = deg + 1; l >= 0; --l) {
            if (l <= deg) {
                if (!big_mul(I[j], C[l], t1)) return 3;
            } else {
                big_zero(t1);
            }
            if (l >= 1) {
                if (!big_add(C[l - 1], t1, 1, t2)) return 3;
                C[l] = t2;
            } else {
                C[0] = t1;
                C[0].neg = t1.n ? !t1.neg : 0;
            }
        }
        ++deg;
    }
    for (int l = 0; l <= deg; ++l) o.v64[M + R + l] = big_round(C[l], -(long)(deg - l) * F);
    if (i == NF) {
        o.v64[M - 1] = 1.0;
        o.v64[M + R - 1] = 1.0;
    } else {
        // D_i = prod_{j != i} (I_i - I_j); N_i = D_i 2^(-(NF-1)F).  The
        // coefficient slots serve as scratch once B^T is rounded (deg =
        // NF - 1 <= A - 2, so slots A-1 and A are free; 0..2 are reused).
        Big& D = C[A];
        big_set_u64(D, 1, 0);
        for (int j = 0; j < NF; ++j) {
            if (j == i) continue;
            if (!big_add(I[i], I[j], 1, t1)) return 3;
            if (!big_mul(D, t1, t2)) return 3;
            D = t2;
        }
        if (D.n == 0) return 1;
        if (!(fabs(big_round(D, -(long)(NF - 1) * F)) >= 1e-300)) return 1;
        const int dneg = D.neg;
        D.neg = 0;
        Big& pw = C[A - 1];
        big_set_u64(pw, 1, 0);
        const int KMAX = M > R ? M : R;
        for (int k = 0; k < KMAX; ++k) {
            if (k < M) o.v64[k] = big_round(pw, -(long)k * F);
            if (k < R) {
                t1 = pw;
                t1.neg = t1.n ? (pw.neg ^ dneg) : 0;
                double v = 0.0;
                if (!big_round_ratio(t1, D, (long)(NF - 1 - k) * F, v, C[0], C[1], t2)) return 3;
                o.v64[M + k] = v;
            }
            if (k + 1 < KMAX) {
                if (!big_mul(pw, I[i], t1)) return 3;
                pw = t1;
            }
        }
    }
    for (int q = 0; q < RowOut<M, R>::kN; ++q) o.v32[q] = (float)o.v64[q];
    return 0;
}

}  // namespace cons
}  // namespace wg
