// Exact construction of the Winograd transform matrices from float64 points.
//
// Every float64 point is a dyadic rational, so the matrices of Sections 4.1
// and 4.2 of arXiv:2201.10369 (Vandermonde A^T, Lagrange numerators B^T, and
// G = Vandermonde / N_i) have exact rational entries.  Writing all points as
// a_j = I_j 2^-F with integers I_j, every entry is an integer, or a ratio of
// two integers, times a power of two:
//   A^T[j][i] = I_i^j 2^(-jF)
//   B^T[i][l] = C_l 2^(-(n-1-l)F),  C_l the coefficients of prod_{j!=i}(x - I_j)
//   N_i       = D_i 2^(-(n-1)F),    D_i = prod_{j!=i}(I_i - I_j)
//   G[i][k]   = (I_i^k / D_i) 2^((n-1-k)F)
// (n finite points).  Each entry is rounded once, to the nearest float64 with
// ties to even.  Cancellations the point families are designed to produce
// (Section 5) therefore give exact zeros.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "wg_internal.h"

namespace wg {
namespace {

using u64 = uint64_t;
using u128 = unsigned __int128;

// Signed arbitrary-precision integer (sign + magnitude, little-endian limbs).
struct Big {
    bool neg = false;
    std::vector<u64> d;   // no leading zero limbs; empty means zero

    static Big from_u64(u64 v, bool negative = false) {
        Big b;
        if (v) {
            b.d.push_back(v);
            b.neg = negative;
        }
        return b;
    }
    bool zero() const { return d.empty(); }
    void trim() {
        while (!d.empty() && d.back() == 0) d.pop_back();
        if (d.empty()) neg = false;
    }
    long bits() const {
        if (d.empty()) return 0;
        return (long)(d.size() - 1) * 64 + (64 - __builtin_clzll(d.back()));
    }
    bool bit(long i) const {
        const size_t w = (size_t)(i / 64);
        return w < d.size() && ((d[w] >> (i % 64)) & 1u);
    }
};

int cmp_mag(const Big& a, const Big& b) {
    if (a.d.size() != b.d.size()) return a.d.size() < b.d.size() ? -1 : 1;
    for (size_t i = a.d.size(); i-- > 0;)
        if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
    return 0;
}

Big add_mag(const Big& a, const Big& b) {
    Big r;
    const size_t n = a.d.size() > b.d.size() ? a.d.size() : b.d.size();
    r.d.resize(n + 1);
    u128 carry = 0;
    for (size_t i = 0; i < n; ++i) {
        u128 s = carry;
        if (i < a.d.size()) s += a.d[i];
        if (i < b.d.size()) s += b.d[i];
        r.d[i] = (u64)s;
        carry = s >> 64;
    }
    r.d[n] = (u64)carry;
    r.trim();
    return r;
}

Big sub_mag(const Big& a, const Big& b) {   // |a| >= |b|
    Big r;
    r.d.resize(a.d.size());
    u64 borrow = 0;
    for (size_t i = 0; i < a.d.size(); ++i) {
        const u64 bi = i < b.d.size() ? b.d[i] : 0;
        const u64 t = a.d[i] - bi;
        const u64 b1 = a.d[i] < bi;
        r.d[i] = t - borrow;
        const u64 b2 = t < borrow;
        borrow = b1 | b2;
    }
    r.trim();
    return r;
}

Big add(const Big& a, const Big& b) {
    if (a.neg == b.neg) {
        Big r = add_mag(a, b);
        r.neg = a.neg && !r.zero();
        return r;
    }
    const int c = cmp_mag(a, b);
    if (c == 0) return Big();
    Big r = c > 0 ? sub_mag(a, b) : sub_mag(b, a);
    r.neg = (c > 0 ? a.neg : b.neg) && !r.zero();
    return r;
}

Big neg(Big a) {
    if (!a.zero()) a.neg = !a.neg;
    return a;
}

Big sub(const Big& a, const Big& b) { return add(a, neg(b)); }

Big mul(const Big& a, const Big& b) {
    if (a.zero() || b.zero()) return Big();
    Big r;
    r.d.assign(a.d.size() + b.d.size(), 0);
    for (size_t i = 0; i < a.d.size(); ++i) {
        u128 carry = 0;
        for (size_t j = 0; j < b.d.size(); ++j) {
            const u128 cur = (u128)a.d[i] * b.d[j] + r.d[i + j] + carry;
            r.d[i + j] = (u64)cur;
            carry = cur >> 64;
        }
        size_t k = i + b.d.size();
        while (carry) {
            const u128 cur = (u128)r.d[k] + carry;
            r.d[k] = (u64)cur;
            carry = cur >> 64;
            ++k;
        }
    }
    r.neg = a.neg != b.neg;
    r.trim();
    return r;
}

Big shl(const Big& a, long s) {   // magnitude shift, keeps the sign
    if (a.zero() || s == 0) return a;
    Big r;
    const size_t w = (size_t)(s / 64);
    const int b = (int)(s % 64);
    r.d.assign(w + a.d.size() + 1, 0);
    for (size_t i = 0; i < a.d.size(); ++i) {
        r.d[i + w] |= a.d[i] << b;
        if (b) r.d[i + w + 1] |= a.d[i] >> (64 - b);
    }
    r.neg = a.neg;
    r.trim();
    return r;
}

// Nearest float64 (ties to even) of (P / Q) * 2^s, Q > 0.
double round_ratio(const Big& P, const Big& Q, long s) {
    if (P.zero()) return 0.0;
    Big num = P, den = Q;
    num.neg = den.neg = false;
    const long t = 66 - (num.bits() - den.bits());   // quotient gets 66 or 67 bits
    if (t >= 0) num = shl(num, t);
    else den = shl(den, -t);
    // binary long division; the quotient is below 2^67
    u128 q = 0;
    Big rem;
    for (long i = num.bits() - 1; i >= 0; --i) {
        rem = shl(rem, 1);
        if (num.bit(i)) {
            if (rem.d.empty()) rem.d.push_back(1);
            else rem.d[0] |= 1;
        }
        if (cmp_mag(rem, den) >= 0) {
            rem = sub_mag(rem, den);
            q |= (u128)1 << i;
        }
    }
    const bool sticky = !rem.zero();
    int nb = 0;
    for (u128 v = q; v; v >>= 1) ++nb;
    const long e_top = s - t + (nb - 1);               // value in [2^e_top, 2^(e_top+1))
    long prec = 53;
    if (e_top < -1022) prec = 53 - (-1022 - e_top);   // subnormal range
    if (prec < 0) return P.neg ? -0.0 : 0.0;
    const int drop = nb - (int)prec;
    u128 mant = q >> drop;
    const u128 rest = q & (((u128)1 << drop) - 1);
    const u128 half = (u128)1 << (drop - 1);
    bool up = false;
    if (rest > half) up = true;
    else if (rest == half) up = sticky || (mant & 1);
    if (up) mant += 1;
    double r = std::ldexp((double)(u64)mant, (int)(s - t + drop));
    return P.neg ? -r : r;
}

// float64 point -> (integer mantissa, exponent) with a = M 2^E exactly.
void split(double a, int64_t& M, int& E) {
    if (a == 0.0) {
        M = 0;
        E = 0;
        return;
    }
    int e = 0;
    const double f = std::frexp(a, &e);   // a = f 2^e, 0.5 <= |f| < 1
    M = (int64_t)std::ldexp(f, 53);       // exact: 53-bit integer
    E = e - 53;
}

// Coefficients (ascending) of prod_t (x - r_t) over big integers.
std::vector<Big> int_product_poly(const std::vector<Big>& roots) {
    std::vector<Big> c(1, Big::from_u64(1));
    for (const Big& a : roots) {
        std::vector<Big> n(c.size() + 1);
        for (size_t i = 0; i < c.size(); ++i) {
            n[i + 1] = add(n[i + 1], c[i]);
            n[i] = sub(n[i], mul(a, c[i]));
        }
        c.swap(n);
    }
    return c;
}

}  // namespace

// Exact matrices rounded to float64; points assumed finite and distinct
// (checked by the caller).  Returns false when some N_i is zero.
bool construct_exact(int m, int r, const double* pts, int nf, bool modified, double* AT, double* G,
                     double* BT) {
    const int alpha = m + r - 1;
    std::vector<int64_t> Ms(nf);
    std::vector<int> Es(nf);
    int minE = 0;
    for (int i = 0; i < nf; ++i) {
        split(pts[i], Ms[i], Es[i]);
        if (Ms[i] != 0 && Es[i] < minE) minE = Es[i];
    }
    const long F = -minE;                  // a_j = I_j 2^-F, I_j integers
    std::vector<Big> I(nf);
    for (int i = 0; i < nf; ++i) {
        const int64_t M = Ms[i];
        Big b = Big::from_u64((u64)(M < 0 ? -M : M), M < 0);
        I[i] = M == 0 ? Big() : shl(b, Es[i] + F);
    }
    const Big one = Big::from_u64(1);
    for (int i = 0; i < m * alpha; ++i) AT[i] = 0.0;
    for (int i = 0; i < alpha * r; ++i) G[i] = 0.0;
    for (int i = 0; i < alpha * alpha; ++i) BT[i] = 0.0;

    for (int i = 0; i < nf; ++i) {
        Big D = one;
        std::vector<Big> others;
        for (int j = 0; j < nf; ++j)
            if (j != i) {
                D = mul(D, sub(I[i], I[j]));
                others.push_back(I[j]);
            }
        if (D.zero()) return false;
        Big Qd = D;
        const bool dneg = Qd.neg;
        Qd.neg = false;
        Big pw = one;                      // I_i^k
        for (int k = 0; k < (m > r ? m : r); ++k) {
            if (k < m) AT[k * alpha + i] = round_ratio(pw, one, -(long)k * F);
            if (k < r) {
                Big num = pw;
                if (dneg) num = neg(num);
                G[i * r + k] = round_ratio(num, Qd, (long)(nf - 1 - k) * F);
            }
            pw = mul(pw, I[i]);
        }
        const std::vector<Big> C = int_product_poly(others);
        const int deg = nf - 1;
        for (int l = 0; l <= deg; ++l) BT[i * alpha + l] = round_ratio(C[l], one, -(long)(deg - l) * F);
    }
    if (modified) {
        const int last = alpha - 1;
        AT[(m - 1) * alpha + last] = 1.0;
        G[last * r + (r - 1)] = 1.0;
        const std::vector<Big> C = int_product_poly(I);
        for (int l = 0; l <= nf; ++l) BT[last * alpha + l] = round_ratio(C[l], one, -(long)(nf - l) * F);
    }
    return true;
}

}  // namespace wg
