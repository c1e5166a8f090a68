// Host build of the device construction (wg_construct.h) checked against
// the library's exact host construction (construct_exact, big integers),
// entry for entry: the float32 entries of the float64 tier, the float64 and
// float32 entries of the double-word tier and of the exact-integer rows,
// whenever a tier reports them decided, and the singular verdicts.
// Point sets: families over c, d in [0.05, 20], random lists, lists of exact
// +-a pairs, dyadic lists, integer lists with cancelling sums, scaled
// Chebyshev nodes, lists spanning 10^12 and quarter-integer lists.
// Prints one line per (size, category); usage: construct_check [sets].
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>

#include "wg_construct.h"
#include "wg_internal.h"

namespace wg {
void set_error(const std::string&) {}
int fail(int status, const std::string&) { return status; }
}  // namespace wg

namespace {

void family(int alpha, double c1, double c2, double* p) {
    const double ic = 1.0 / c1;
    int n = 0;
    if (alpha == 4) { p[n++] = -c1; p[n++] = 0.0; p[n++] = c1; return; }
    if (alpha == 5) { p[n++] = 0.0; p[n++] = -c1; p[n++] = c1; p[n++] = ic; return; }
    p[n++] = -ic; p[n++] = -c1; p[n++] = 0.0; p[n++] = c1; p[n++] = ic;
    const double id = 1.0 / c2;
    if (alpha == 7) { p[n++] = c2; }
    if (alpha == 8) { p[n++] = -c2; p[n++] = c2; }
    if (alpha == 9) { p[n++] = -id; p[n++] = -c2; p[n++] = c2; }
    if (alpha == 10) { p[n++] = -id; p[n++] = -c2; p[n++] = c2; p[n++] = id; }
}

struct Stats {
    long sets = 0, f64_decided = 0, dw_decided = 0, singular = 0, mismatch = 0, status = 0, too_big = 0;
};

bool same64(double a, double b) { return (a == 0.0 && b == 0.0) || std::memcmp(&a, &b, 8) == 0; }
bool same32(float a, float b) { return (a == 0.0f && b == 0.0f) || std::memcmp(&a, &b, 4) == 0; }

// worst row status: 1 (singular) over 2 (undecided) over 0
int worse(int w, int s) { return (w == 1 || s == 1) ? 1 : (s > w ? s : w); }

template <int M, int R>
void check_set(const double* pts, Stats& st) {
    constexpr int A = M + R - 1, NF = A - 1;
    using Row = wg::cons::RowOut<M, R>;
    double eAT[M * A], eG[A * R], eBT[A * A];
    const bool distinct = wg::construct_exact(M, R, pts, NF, true, eAT, eG, eBT);
    ++st.sets;
    int w64 = 0, wdw = 0, wx = 0;
    bool mism = false;
    for (int i = 0; i <= NF; ++i) {
        Row f, d, x;
        const int a = wg::cons::row_cert<wg::cons::ArithF64, M, R>(pts, i, f);
        const int b = wg::cons::row_cert<wg::cons::ArithDW, M, R>(pts, i, d);
        const int c = wg::cons::exact_row<M, R>(pts, i, x);
        w64 = worse(w64, a);
        wdw = worse(wdw, b);
        wx = worse(wx, c == 3 ? 2 : c);
        if (c == 3) ++st.too_big;
        if (!distinct) continue;
        double ref[Row::kN];
        for (int j = 0; j < M; ++j) ref[j] = eAT[j * A + i];
        for (int k = 0; k < R; ++k) ref[M + k] = eG[i * R + k];
        for (int l = 0; l < A; ++l) ref[M + R + l] = eBT[i * A + l];
        for (int q = 0; q < Row::kN; ++q) {
            const float r32 = (float)ref[q];
            if (a == 0 && !same32(f.v32[q], r32)) mism = true;
            if (b == 0 && (!same64(d.v64[q], ref[q]) || !same32(d.v32[q], r32))) mism = true;
            if (c == 0 && (!same64(x.v64[q], ref[q]) || !same32(x.v32[q], r32))) mism = true;
        }
    }
    if (mism) ++st.mismatch;
    // the exact construction fails only for coinciding points; the sweep also
    // flags |RN64(N_i)| < 1e-300, which the exact rows decide
    const int ref_singular = !distinct ? 1 : (wx == 1 ? 1 : 0);
    if (ref_singular) ++st.singular;
    if (ref_singular && (w64 == 0 || wdw == 0)) ++st.status;
    if (!ref_singular && (w64 == 1 || wdw == 1)) ++st.status;
    if (!ref_singular && w64 == 0) ++st.f64_decided;
    if (!ref_singular && wdw == 0) ++st.dw_decided;
}

template <int M, int R>
void run(long n, unsigned seed) {
    constexpr int A = M + R - 1, NF = A - 1;
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const char* cats[] = {"family", "random", "pairs", "dyadic", "cancel", "chebyshev", "wide", "quarter"};
    for (int cat = 0; cat < 8; ++cat) {
        Stats st;
        for (long t = 0; t < n; ++t) {
            double p[NF];
            if (cat == 0) {
                const double c1 = std::exp(std::log(0.05) + U(rng) * std::log(400.0));
                const double c2 = std::exp(std::log(0.05) + U(rng) * std::log(400.0));
                family(A, c1, c2, p);
            } else if (cat == 1) {
                for (int j = 0; j < NF; ++j) p[j] = -3.0 + 6.0 * U(rng);
            } else if (cat == 2) {
                for (int j = 0; j + 1 < NF; j += 2) {
                    p[j] = -3.0 + 6.0 * U(rng);
                    p[j + 1] = -p[j];
                }
                if (NF % 2) p[NF - 1] = (t % 3 == 0) ? 0.0 : -3.0 + 6.0 * U(rng);
                for (int j = NF - 1; j > 0; --j) std::swap(p[j], p[rng() % (j + 1)]);
            } else if (cat == 3) {
                const double vals[] = {0, 1, -1, 2, -2, 0.5, -0.5, 4, -4, 0.25, -0.25, 3, -3, 1.5, -1.5, 0.75};
                int used[16] = {0};
                for (int j = 0; j < NF; ++j) {
                    int k;
                    do { k = (int)(rng() % 16); } while (used[k]);
                    used[k] = 1;
                    p[j] = vals[k];
                }
            } else if (cat == 4) {
                int used[41] = {0};
                for (int j = 0; j < NF; ++j) {
                    int k;
                    do { k = (int)(rng() % 41); } while (used[k]);
                    used[k] = 1;
                    p[j] = k - 20;
                }
                p[NF - 1] = -(p[0] + p[1]);                 // a sum of roots cancels
                for (int j = 0; j + 1 < NF; ++j)
                    if (p[j] == p[NF - 1]) p[NF - 1] = 37.0 + (double)(t % 5);
            } else if (cat == 5) {
                const double s = 0.5 + 3.0 * U(rng);
                for (int j = 0; j < NF; ++j) p[j] = s * std::cos(M_PI * (2 * j + 1) / (2.0 * NF));
            } else if (cat == 6) {
                for (int j = 0; j < NF; ++j)
                    p[j] = (U(rng) < 0.5 ? -1 : 1) * std::exp(std::log(1e-6) + U(rng) * std::log(1e12));
            } else {
                int used[2001] = {0};
                for (int j = 0; j < NF; ++j) {
                    int k;
                    do { k = (int)(rng() % 2001); } while (used[k]);
                    used[k] = 1;
                    p[j] = (k - 1000) / 4.0;
                }
            }
            check_set<M, R>(p, st);
        }
        std::printf("F(%d,%d) %s sets %ld f64 %ld dw %ld singular %ld mismatch %ld status %ld toobig %ld\n", M, R,
                    cats[cat], st.sets, st.f64_decided, st.dw_decided, st.singular, st.mismatch, st.status,
                    st.too_big);
    }
}

}  // namespace

int main(int argc, char** argv) {
    const long n = argc > 1 ? std::atol(argv[1]) : 200;
    run<2, 3>(n, 1); run<3, 3>(n, 2); run<4, 3>(n, 3); run<5, 3>(n, 4); run<6, 3>(n, 5); run<7, 3>(n, 6);
    run<8, 3>(n, 7); run<2, 5>(n, 8); run<3, 5>(n, 9); run<4, 5>(n, 10); run<5, 5>(n, 11); run<6, 5>(n, 12);
    return 0;
}
