// Host side of the Winograd library: float64 construction of the transform
// matrices from points (Sections 4.1 and 4.2 of arXiv:2201.10369), the point
// families of Section 5, layer plans and argument validation for the C ABI.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "wg_internal.h"

namespace wg {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
    set_error(msg);
    return status;
}

// A^T (m x alpha), G (alpha x r), B^T (alpha x alpha), row-major: the exact
// matrices of the points, each entry rounded to the nearest float64.
static int construct(int m, int r, const double* pts, int n_pts, int flags, double* AT,
                     double* G, double* BT) {
    if (m < 1 || r < 2) return fail(WG_EINVAL, "wg_transforms: need m >= 1 and r >= 2");
    const int alpha = m + r - 1;
    if (alpha > kMaxAlpha) return fail(WG_EINVAL, "wg_transforms: alpha = m+r-1 exceeds 16");
    if (flags != WG_MODIFIED && flags != WG_UNMODIFIED)
        return fail(WG_EINVAL, "wg_transforms: flags must be WG_MODIFIED or WG_UNMODIFIED");
    const bool modified = flags == WG_MODIFIED;
    const int nf = modified ? alpha - 1 : alpha;
    if (!pts || !AT || !G || !BT) return fail(WG_EINVAL, "wg_transforms: null pointer");
    if (n_pts != nf)
        return fail(WG_EINVAL, "wg_transforms: expected " + std::to_string(nf) +
                                   " finite points, got " + std::to_string(n_pts));
    for (int i = 0; i < nf; ++i)
        if (!std::isfinite(pts[i])) return fail(WG_EINVAL, "wg_transforms: non-finite point");
    for (int i = 0; i < nf; ++i)
        for (int j = i + 1; j < nf; ++j)
            if (pts[i] == pts[j])
                return fail(WG_ESINGULAR, "wg_transforms: points " + std::to_string(i) + " and " +
                                              std::to_string(j) + " coincide");

    for (int i = 0; i < nf; ++i) {      // reject (near-)singular normalisers N_i
        double prod = 1.0;
        for (int j = 0; j < nf; ++j)
            if (j != i) prod *= (pts[i] - pts[j]);
        if (!(std::fabs(prod) >= 1e-300) || !std::isfinite(prod))
            return fail(WG_ESINGULAR, "wg_transforms: Lagrange normaliser N_" + std::to_string(i) +
                                          " is zero, subnormal or not finite");
    }

    // exact rational construction, each entry rounded once to float64
    double tmpA[kMaxAlpha * kMaxAlpha], tmpG[kMaxAlpha * kMaxAlpha], tmpB[kMaxAlpha * kMaxAlpha];
    if (!construct_exact(m, r, pts, nf, modified, tmpA, tmpG, tmpB))
        return fail(WG_ESINGULAR, "wg_transforms: two points coincide");
    for (int i = 0; i < m * alpha; ++i)
        if (!std::isfinite(tmpA[i])) return fail(WG_ESINGULAR, "wg_transforms: A^T overflows");
    for (int i = 0; i < alpha * r; ++i)
        if (!std::isfinite(tmpG[i])) return fail(WG_ESINGULAR, "wg_transforms: G overflows");
    for (int i = 0; i < alpha * alpha; ++i)
        if (!std::isfinite(tmpB[i])) return fail(WG_ESINGULAR, "wg_transforms: B^T overflows");
    std::memcpy(AT, tmpA, sizeof(double) * m * alpha);
    std::memcpy(G, tmpG, sizeof(double) * alpha * r);
    std::memcpy(BT, tmpB, sizeof(double) * alpha * alpha);
    return WG_OK;
}

static int binary_exponent(double v) {
    if (v == 0.0) return 0;
    int e = 0;
    std::frexp(v, &e);
    return e;
}

int hip_check(int hip_err, const char* what);

}  // namespace wg

using namespace wg;

extern "C" {

const char* wg_last_error(void) { return g_last_error.c_str(); }

int wg_version(void) { return 10000; }

int wg_supported(int m, int r) {
    return (m >= 1 && m <= 8 && (r == 3 || r == 5) && m + r - 1 <= 12) ? 1 : 0;
}

int wg_transforms(int m, int r, const double* pts, int n_pts, int flags, double* AT, double* G,
                  double* BT) {
    return construct(m, r, pts, n_pts, flags, AT, G, BT);
}

int wg_transforms_f32(int m, int r, const double* pts, int n_pts, int flags, float* AT, float* G,
                      float* BT) {
    if (!AT || !G || !BT) return fail(WG_EINVAL, "wg_transforms_f32: null pointer");
    double a[kMaxAlpha * kMaxAlpha], g[kMaxAlpha * kMaxAlpha], b[kMaxAlpha * kMaxAlpha];
    const int st = construct(m, r, pts, n_pts, flags, a, g, b);
    if (st != WG_OK) return st;
    const int alpha = m + r - 1;
    for (int i = 0; i < m * alpha; ++i) AT[i] = static_cast<float>(a[i]);
    for (int i = 0; i < alpha * r; ++i) G[i] = static_cast<float>(g[i]);
    for (int i = 0; i < alpha * alpha; ++i) BT[i] = static_cast<float>(b[i]);
    return WG_OK;
}

int wg_family_points(int alpha, double c1, double c2, double* pts_out) {
    if (!pts_out) return fail(WG_EINVAL, "wg_family_points: null pointer");
    if (alpha < 4 || alpha > 10) return fail(WG_EINVAL, "wg_family_points: alpha must be 4..10");
    if (!std::isfinite(c1) || c1 == 0.0) return fail(WG_EINVAL, "wg_family_points: bad c1");
    if (alpha > 6 && (!std::isfinite(c2) || c2 == 0.0))
        return fail(WG_EINVAL, "wg_family_points: bad c2");
    const double ic = 1.0 / c1;
    int n = 0;
    double* p = pts_out;
    switch (alpha) {
        case 4: p[n++] = -c1; p[n++] = 0.0; p[n++] = c1; return n;
        case 5: p[n++] = 0.0; p[n++] = -c1; p[n++] = c1; p[n++] = ic; return n;
        default: break;
    }
    p[n++] = -ic; p[n++] = -c1; p[n++] = 0.0; p[n++] = c1; p[n++] = ic;
    const double id = 1.0 / c2;
    switch (alpha) {
        case 7: p[n++] = c2; break;
        case 8: p[n++] = -c2; p[n++] = c2; break;
        case 9: p[n++] = -id; p[n++] = -c2; p[n++] = c2; break;
        case 10: p[n++] = -id; p[n++] = -c2; p[n++] = c2; p[n++] = id; break;
        default: break;
    }
    return n;
}

int wg_plan_create(wg_plan** out, int m, int r, const double* pts, int n_pts, int flags, int N,
                   int C, int K, int H, int W, int padding, int dtype) {
    if (!out || !pts) return fail(WG_EINVAL, "wg_plan_create: null pointer");
    if (N <= 0 || C <= 0 || K <= 0 || H <= 0 || W <= 0)
        return fail(WG_EINVAL, "wg_plan_create: sizes must be positive");
    if (padding != WG_SAME && padding != WG_VALID)
        return fail(WG_EINVAL, "wg_plan_create: padding must be WG_SAME or WG_VALID");
    if (dtype != WG_F32 && dtype != WG_F16 && dtype != WG_BF16)
        return fail(WG_EINVAL, "wg_plan_create: dtype must be WG_F32, WG_F16 or WG_BF16");
    if ((flags & ~(WG_UNMODIFIED | WG_F64_TRANSFORMS)) != 0)
        return fail(WG_EINVAL, "wg_plan_create: unknown flags");
    if (flags & WG_UNMODIFIED)
        return fail(WG_EUNSUPPORTED, "wg_plan_create: the layer implements the modified form (WG_MODIFIED) only");
    const bool f64t = (flags & WG_F64_TRANSFORMS) != 0;
    if (f64t && dtype != WG_F32)
        return fail(WG_EINVAL, "wg_plan_create: WG_F64_TRANSFORMS needs dtype WG_F32");
    if (!wg_supported(m, r))
        return fail(WG_EUNSUPPORTED, "wg_plan_create: F(" + std::to_string(m) + "," +
                                         std::to_string(r) + ") is not implemented");
    if (padding == WG_SAME && r % 2 == 0)
        return fail(WG_EUNSUPPORTED, "wg_plan_create: 'same' padding needs an odd kernel size");
    const int pad = padding == WG_SAME ? (r - 1) / 2 : 0;
    const long Hout = (long)H + 2 * pad - r + 1, Wout = (long)W + 2 * pad - r + 1;
    if (Hout < 1 || Wout < 1) return fail(WG_EINVAL, "wg_plan_create: output would be empty");
    const long Th = (Hout + m - 1) / m, Tw = (Wout + m - 1) / m;
    const long P = (long)N * Th * Tw;
    if (P > (1L << 30) || (long)K > 65535 || (long)C > 65535)
        return fail(WG_EUNSUPPORTED, "wg_plan_create: layer too large for this build");
    if (Tw * m > 4096)
        return fail(WG_EUNSUPPORTED, "wg_plan_create: output rows wider than 4096 are not supported");

    Plan* plan = new (std::nothrow) Plan();
    if (!plan) return fail(WG_ENOMEM, "wg_plan_create: out of host memory");
    const int alpha = m + r - 1;
    int st = wg_transforms_f32(m, r, pts, n_pts, WG_MODIFIED, plan->AT, plan->G, plan->BT);
    if (st == WG_OK) st = wg_transforms(m, r, pts, n_pts, WG_MODIFIED, plan->AT64, plan->G64, plan->BT64);
    if (st != WG_OK) {
        delete plan;
        return st;
    }
    plan->f64t = f64t;
    for (int i = 0; i < alpha; ++i) {
        double nb = 0.0, ng = 0.0;
        for (int l = 0; l < alpha; ++l) nb += std::fabs((double)plan->BT[i * alpha + l]);
        for (int k = 0; k < r; ++k) ng += std::fabs((double)plan->G[i * r + k]);
        plan->eB[i] = binary_exponent(nb);
        plan->eG[i] = binary_exponent(ng);
        plan->dB[i] = plan->eB[i] - plan->eG[i];
    }

    // GEMM tiling: 128 x 128 (K x P) blocks when the layer is wide enough,
    // 64 x 64 otherwise; the contraction (channel) step is 128 bytes of each
    // operand row (32 float32 or 64 16-bit channels).
    const bool big = K >= 96 && P >= 512;
    plan->gemm_bm = big ? 128 : 64;
    plan->gemm_bn = big ? 128 : 64;
    plan->gemm_bk = dtype == WG_F32 ? 32 : 64;
    plan->gemm_tpb = 1;

    wg_layout& L = plan->L;
    std::memset(&L, 0, sizeof(L));
    L.alpha = alpha; L.m = m; L.r = r; L.pad = pad;
    L.N = N; L.C = C; L.K = K; L.H = H; L.W = W;
    L.Hout = (int)Hout; L.Wout = (int)Wout; L.Th = (int)Th; L.Tw = (int)Tw;
    L.P = (int)P;
    L.P_pad = (int)round_up(P, plan->gemm_bn);
    L.K_pad = (int)round_up(K, plan->gemm_bm);
    L.C_pad = (int)round_up(C, plan->gemm_bk);
    L.dtype = dtype;
    L.elem_bytes = dtype == WG_F32 ? 4 : 2;
    // kernels address one plane of U', V' and M with 32-bit element offsets
    const unsigned long long lim = 1ull << 32;
    if ((unsigned long long)L.P_pad * L.C_pad >= lim || (unsigned long long)L.K_pad * L.P_pad >= lim ||
        (unsigned long long)L.K_pad * L.C_pad >= lim) {
        delete plan;
        return fail(WG_EUNSUPPORTED, "wg_plan_create: a transformed plane exceeds 2^32 elements");
    }
    const size_t E = (size_t)alpha * alpha;
    const size_t ubytes = E * L.K_pad * L.C_pad * L.elem_bytes;
    L.scale_offset = round_up(ubytes, 256);
    L.chan_offset = round_up(L.scale_offset + E * L.C_pad * sizeof(int32_t), 256);
    // scratch after the per-channel table: partial maxima of |w| per 8 filters
    L.filter_bytes = dtype == WG_F32 ? round_up(ubytes, 256)
                                     : round_up(wpart_offset(L) + (size_t)w_chunks(L) * L.C_pad * sizeof(float), 256);
    L.v_offset = 0;
    L.m_offset = round_up(E * L.P_pad * L.C_pad * L.elem_bytes, 256);
    L.workspace_bytes = round_up(L.m_offset + E * L.K_pad * L.P_pad * sizeof(float), 256);
    *out = reinterpret_cast<wg_plan*>(plan);
    return WG_OK;
}

int wg_plan_destroy(wg_plan* plan) {
    delete reinterpret_cast<Plan*>(plan);
    return WG_OK;
}

int wg_plan_sizes(const wg_plan* plan, size_t* filter_bytes, size_t* workspace_bytes, int* Hout,
                  int* Wout) {
    if (!plan) return fail(WG_EINVAL, "wg_plan_sizes: null plan");
    const wg_layout& L = reinterpret_cast<const Plan*>(plan)->L;
    if (filter_bytes) *filter_bytes = L.filter_bytes;
    if (workspace_bytes) *workspace_bytes = L.workspace_bytes;
    if (Hout) *Hout = L.Hout;
    if (Wout) *Wout = L.Wout;
    return WG_OK;
}

int wg_plan_layout(const wg_plan* plan, wg_layout* out) {
    if (!plan || !out) return fail(WG_EINVAL, "wg_plan_layout: null pointer");
    *out = reinterpret_cast<const Plan*>(plan)->L;
    return WG_OK;
}

int wg_plan_matrices(const wg_plan* plan, float* AT, float* G, float* BT) {
    if (!plan || !AT || !G || !BT) return fail(WG_EINVAL, "wg_plan_matrices: null pointer");
    const Plan* p = reinterpret_cast<const Plan*>(plan);
    const int a = p->L.alpha, m = p->L.m, r = p->L.r;
    std::memcpy(AT, p->AT, sizeof(float) * m * a);
    std::memcpy(G, p->G, sizeof(float) * a * r);
    std::memcpy(BT, p->BT, sizeof(float) * a * a);
    return WG_OK;
}

int wg_plan_set_gemm_tiles(wg_plan* plan, int tiles_per_block) {
    if (!plan) return fail(WG_EINVAL, "wg_plan_set_gemm_tiles: null plan");
    if (tiles_per_block < 1 || tiles_per_block > 16)
        return fail(WG_EINVAL, "wg_plan_set_gemm_tiles: tiles_per_block must be in 1..16");
    reinterpret_cast<Plan*>(plan)->gemm_tpb = tiles_per_block;
    return WG_OK;
}

int wg_plan_gemm_tiles(const wg_plan* plan) {
    if (!plan) return fail(WG_EINVAL, "wg_plan_gemm_tiles: null plan");
    return reinterpret_cast<const Plan*>(plan)->gemm_tpb;
}

int wg_transform_filters(const wg_plan* plan, const float* w, const float* x_absmax, void* U,
                         wg_stream_t stream) {
    if (!plan || !w || !U) return fail(WG_EINVAL, "wg_transform_filters: null pointer");
    return launch_filter_transform(*reinterpret_cast<const Plan*>(plan), w, x_absmax, U, stream);
}

static int check_ws(const Plan& p, const void* ws, size_t ws_bytes, const char* who) {
    if (!ws) return fail(WG_EINVAL, std::string(who) + ": null workspace");
    if (ws_bytes < p.L.workspace_bytes)
        return fail(WG_EWORKSPACE, std::string(who) + ": workspace of " + std::to_string(ws_bytes) +
                                       " bytes, need " + std::to_string(p.L.workspace_bytes));
    return WG_OK;
}

int wg_input_transform(const wg_plan* plan, const float* x, const void* U, void* ws,
                       size_t ws_bytes, wg_stream_t stream) {
    if (!plan || !x || !U) return fail(WG_EINVAL, "wg_input_transform: null pointer");
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_input_transform");
    if (st != WG_OK) return st;
    return launch_input_transform(p, x, U, ws, stream);
}

int wg_filter_maxima(const wg_plan* plan, const float* w, void* U, wg_stream_t stream) {
    if (!plan || !w || !U) return fail(WG_EINVAL, "wg_filter_maxima: null pointer");
    return launch_filter_maxima(*reinterpret_cast<const Plan*>(plan), w, U, stream);
}

int wg_transform_filters_and_input(const wg_plan* plan, const float* w, const float* x_absmax, const float* x,
                                   void* U, void* ws, size_t ws_bytes, wg_stream_t stream) {
    if (!plan || !w || !x || !U) return fail(WG_EINVAL, "wg_transform_filters_and_input: null pointer");
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_transform_filters_and_input");
    if (st != WG_OK) return st;
    return launch_filter_input(p, w, x_absmax, x, U, ws, stream);
}

int wg_layer_maxima(const wg_plan* plan, const float* w, const float* x, void* U, wg_stream_t stream) {
    if (!plan || !w || !x || !U) return fail(WG_EINVAL, "wg_layer_maxima: null pointer");
    return launch_layer_maxima(*reinterpret_cast<const Plan*>(plan), w, x, U, stream);
}

int wg_transform_layer(const wg_plan* plan, const float* w, const float* x, void* U, void* ws, size_t ws_bytes,
                       wg_stream_t stream) {
    if (!plan || !w || !x || !U) return fail(WG_EINVAL, "wg_transform_layer: null pointer");
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_transform_layer");
    if (st != WG_OK) return st;
    return launch_filter_input(p, w, nullptr, x, U, ws, stream, p.L.dtype != WG_F32);
}

int wg_hadamard_gemm(const wg_plan* plan, const void* U, void* ws, size_t ws_bytes,
                     wg_stream_t stream) {
    if (!plan || !U) return fail(WG_EINVAL, "wg_hadamard_gemm: null pointer");
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_hadamard_gemm");
    if (st != WG_OK) return st;
    return launch_hadamard_gemm(p, U, ws, stream);
}

int wg_plan_autotune_gemm(wg_plan* plan, const void* U, void* ws, size_t ws_bytes, int reps, int* chosen,
                          wg_stream_t stream) {
    if (!plan || !U) return fail(WG_EINVAL, "wg_plan_autotune_gemm: null pointer");
    if (reps < 1 || reps > 1000) return fail(WG_EINVAL, "wg_plan_autotune_gemm: reps must be in 1..1000");
    Plan& p = *reinterpret_cast<Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_plan_autotune_gemm");
    if (st != WG_OK) return st;
    return autotune_hadamard_gemm(p, U, ws, reps, chosen, stream);
}

int wg_output_transform(const wg_plan* plan, const void* ws, size_t ws_bytes, float* y,
                        wg_stream_t stream) {
    if (!plan || !y) return fail(WG_EINVAL, "wg_output_transform: null pointer");
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_output_transform");
    if (st != WG_OK) return st;
    return launch_output_transform(p, ws, y, stream);
}

int wg_conv2d_forward(const wg_plan* plan, const float* x, const void* U, float* y, void* ws,
                      size_t ws_bytes, wg_stream_t stream) {
    if (!plan || !x || !U || !y) return fail(WG_EINVAL, "wg_conv2d_forward: null pointer");
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int st = check_ws(p, ws, ws_bytes, "wg_conv2d_forward");
    if (st != WG_OK) return st;
    st = launch_input_transform(p, x, U, ws, stream);
    if (st != WG_OK) return st;
    st = launch_hadamard_gemm(p, U, ws, stream);
    if (st != WG_OK) return st;
    return launch_output_transform(p, ws, y, stream);
}

int wg_channel_absmax(const float* x, int N, int C, int H, int W, float* out, wg_stream_t stream) {
    if (!x || !out) return fail(WG_EINVAL, "wg_channel_absmax: null pointer");
    if (N <= 0 || C <= 0 || H <= 0 || W <= 0)
        return fail(WG_EINVAL, "wg_channel_absmax: sizes must be positive");
    return launch_channel_absmax(x, N, C, H * W, out, stream);
}

int wg_direct_conv_f64(const float* x, const float* w, double* y_ref, int N, int C, int K, int H,
                       int W, int r, int padding, wg_stream_t stream) {
    if (!x || !w || !y_ref) return fail(WG_EINVAL, "wg_direct_conv_f64: null pointer");
    if (N <= 0 || C <= 0 || K <= 0 || H <= 0 || W <= 0 || r < 1 || r > 7)
        return fail(WG_EINVAL, "wg_direct_conv_f64: bad sizes (need positive sizes, 1 <= r <= 7)");
    if (padding != WG_SAME && padding != WG_VALID)
        return fail(WG_EINVAL, "wg_direct_conv_f64: bad padding");
    if (padding == WG_SAME && r % 2 == 0)
        return fail(WG_EINVAL, "wg_direct_conv_f64: 'same' padding needs an odd kernel size");
    const int pad = padding == WG_SAME ? (r - 1) / 2 : 0;
    const int Hout = H + 2 * pad - r + 1, Wout = W + 2 * pad - r + 1;
    if (Hout < 1 || Wout < 1) return fail(WG_EINVAL, "wg_direct_conv_f64: output would be empty");
    return launch_direct_f64(x, w, y_ref, N, C, K, H, W, r, pad, Hout, Wout, stream);
}

size_t wg_score_workspace_bytes(size_t count) { return score_partials(count) * 2 * sizeof(double); }

int wg_score_error(const float* y, const double* y_ref, size_t count, double* out2, void* ws,
                   size_t ws_bytes, wg_stream_t stream) {
    if (!y || !y_ref || !out2 || !ws) return fail(WG_EINVAL, "wg_score_error: null pointer");
    if (count == 0) return fail(WG_EINVAL, "wg_score_error: count must be positive");
    if (ws_bytes < wg_score_workspace_bytes(count))
        return fail(WG_EWORKSPACE, "wg_score_error: workspace too small");
    return launch_score(y, y_ref, count, out2, ws, stream);
}

int wg_score_error_noalloc(const float* y, const double* y_ref, size_t count, double* out2, wg_stream_t stream) {
    if (!y || !y_ref || !out2) return fail(WG_EINVAL, "wg_score_error_noalloc: null pointer");
    if (count == 0) return fail(WG_EINVAL, "wg_score_error_noalloc: count must be positive");
    return launch_score_noalloc(y, y_ref, count, out2, stream);
}

}  // extern "C"
