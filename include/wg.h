/*
 * wg.h - C ABI of the MI355X (gfx950) Winograd / Toom-Cook convolution
 * library with arbitrary interpolation points.
 *
 * Method: Alam, Anderson, Barabasz, Gregg, "Winograd Convolution for Deep
 * Neural Networks: Efficient Point Selection" (arXiv:2201.10369).
 *   - 1D algorithm Y = A^T[(G g) (.) (B^T d)]              (Section 4, eq. conv_1d)
 *   - 2D algorithm Y = A^T[(G g G^T) (.) (B^T d B)] A      (Section 4, eq. conv_2d)
 *   - matrices from points: A^T Vandermonde, G Vandermonde with the Lagrange
 *     normalisation N_i folded in, B^T Lagrange numerators (Section 4.1),
 *     modified with the point at infinity appended last (Section 4.2)
 *   - point families {0, inf, +-c, +-1/c, +-d, +-1/d} and subsets (Section 5)
 *   - float32 error against a float64 direct convolution, L1 norm (Section 6)
 *
 * Conventions for every entry point
 *   - Return value: WG_OK (0) or a negative wg_status.  Nothing throws across
 *     the ABI and nothing aborts.  wg_last_error() describes the last failure
 *     of the calling thread.
 *   - All arguments are validated on the host before anything is launched; a
 *     failed validation launches nothing and writes nothing.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library
 *     keeps no pointer after a call returns (plans keep only their own small
 *     host-side tables).
 *   - Device work is enqueued asynchronously on `stream` (a hipStream_t; NULL
 *     means the default stream); the call returns once it is enqueued.  HIP
 *     launch failures return WG_EHIP with the HIP error string.
 *   - Layouts: x is N x C x H x W, w is K x C x r x r, y is N x K x Hout x Wout,
 *     all float32, dense, row-major (NCHW / KCRS / NKHW).  Stride 1, no bias,
 *     no dilation, no groups.  padding WG_SAME needs odd r (pad (r-1)/2);
 *     WG_VALID pads nothing.
 *   - NaN and Inf in the data propagate unchecked.
 */
#ifndef WG_H
#define WG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t, declared opaquely so this header needs no HIP headers. */
typedef struct ihipStream_t* wg_stream_t;

typedef enum {
    WG_OK = 0,
    WG_EINVAL = -1,        /* bad argument: null pointer, bad size, bad enum */
    WG_ESINGULAR = -2,     /* two points coincide: some N_i = 0 (Section 4.1) */
    WG_EUNSUPPORTED = -3,  /* valid request outside what this build implements */
    WG_EWORKSPACE = -4,    /* caller workspace smaller than required */
    WG_ENOMEM = -5,        /* host or device allocation failed */
    WG_EHIP = -6           /* a HIP runtime call failed */
} wg_status;

/* construction flags */
enum { WG_MODIFIED = 0,    /* alpha-1 finite points + infinity (Section 4.2) */
       WG_UNMODIFIED = 1 };/* alpha finite points (plain Toom-Cook, Section 4.1) */
/* plan flag (or-ed into the flags of wg_plan_create; dtype WG_F32 only):
 * the mixed precision of Section 6, float64 transforms with a float32
 * Hadamard stage.  The filter, input and output transforms use the exact
 * matrices rounded to float64 and take each term as a rounded float64
 * product and a rounded float64 sum in ascending order; U' and V' are
 * rounded to float32, the channel sums are float32, and Y is rounded to
 * float32. */
enum { WG_F64_TRANSFORMS = 4 };
/* padding */
enum { WG_SAME = 0, WG_VALID = 1 };
/* element type of the Hadamard (channel-sum) stage */
enum { WG_F32 = 0, WG_F16 = 1, WG_BF16 = 2 };

/* Description of the last error on the calling thread; valid until the next
 * call on that thread.  Never NULL. */
const char* wg_last_error(void);

/* ABI version (major*10000 + minor*100 + patch). */
int wg_version(void);

/* Limits of this build: 1 <= m <= 8, r in {3, 5}, alpha = m + r - 1 <= 12. */
int wg_supported(int m, int r);   /* 1 if (m, r) is implemented, else 0 */

/* ------------------------------------------------------------------------
 * Points -> transforms (host, synchronous).  Section 4.1 and 4.2.
 *
 * pts: host, the ordered finite points (n_pts of them).  With
 *   flags = WG_MODIFIED, n_pts must be alpha-1 = m+r-2 and the point at
 *   infinity is appended as the last point; with WG_UNMODIFIED, n_pts must be
 *   alpha.  The order of the points is kept (it permutes rows/columns).
 * Outputs (host, caller allocated, row-major):
 *   AT: m x alpha, G: alpha x r, BT: alpha x alpha.
 *   A^T[j][i] = a_i^j;  G[i][k] = a_i^k / N_i;  B^T[i][l] = coefficient of x^l
 *   in prod_{j != i}(x - a_j), with N_i = prod_{j != i}(a_i - a_j); for the
 *   infinity point A^T gets column e_{m-1}, G row e_{r-1} and B^T the row of
 *   coefficients of prod_j (x - a_j).
 * Computed exactly (every float64 point is a dyadic rational; the entries are
 * evaluated in integer arithmetic) and each entry rounded once to the nearest
 * float64, ties to even, so cancellations give exact zeros.
 * Errors: WG_EINVAL (null pointer, m < 1, r < 2,
 * alpha > 16, wrong n_pts, non-finite point), WG_ESINGULAR (two points equal,
 * or some |N_i| < 1e-300).  Nothing is written on error.
 * ---------------------------------------------------------------------- */
int wg_transforms(int m, int r, const double* pts, int n_pts, int flags,
                  double* AT, double* G, double* BT);

/* Same, rounded on to the nearest float32 (ties to even): the matrices the
 * layer kernels use. */
int wg_transforms_f32(int m, int r, const double* pts, int n_pts, int flags,
                      float* AT, float* G, float* BT);

/* Point families of Section 5 (eqs. ps0, ps1, ps2 and the subsets of
 * eq. ps3), one canonical subset per size, c2 playing the role of d:
 *   alpha 4: -c, 0, c          5: 0, -c, c, 1/c       6: -1/c, -c, 0, c, 1/c
 *   alpha 7: (6), d            8: (6), -d, d          9: (6), -1/d, -d, d
 *   alpha 10: (6), -1/d, -d, d, 1/d
 * pts_out (host) receives alpha-1 finite points (infinity is implicit).
 * c2 is ignored for alpha <= 6.  Returns alpha-1, or WG_EINVAL (alpha outside
 * 4..10, c1 or c2 not finite and nonzero where used). */
int wg_family_points(int alpha, double c1, double c2, double* pts_out);

/* ------------------------------------------------------------------------
 * Convolution layer plans (host).
 * A plan fixes the point set, tile size F(m x m, r x r), layer shape, padding
 * and the element type of the Hadamard stage.  It owns only host-side tables
 * (the float32 matrices and their row-norm exponents), is immutable after
 * creation and may be used concurrently from several streams.
 * ---------------------------------------------------------------------- */
typedef struct wg_plan wg_plan;

/* Creates a plan.  flags: WG_MODIFIED, optionally | WG_F64_TRANSFORMS.
 * Errors: WG_EINVAL (null out/pts, non-positive sizes, padding, dtype or
 * flags out of range, WG_F64_TRANSFORMS with a 16-bit dtype, output smaller
 * than 1x1), WG_EUNSUPPORTED
 * ((m, r) not implemented; WG_SAME with even r; WG_UNMODIFIED), WG_ESINGULAR,
 * WG_ENOMEM.  *out is set only on success. */
int wg_plan_create(wg_plan** out, int m, int r, const double* pts, int n_pts, int flags,
                   int N, int C, int K, int H, int W, int padding, int dtype);
int wg_plan_destroy(wg_plan* plan);      /* NULL is accepted */

/* Sizes in bytes of the transformed-filter buffer U and of the forward
 * workspace, and the output size.  Any output pointer may be NULL. */
int wg_plan_sizes(const wg_plan* plan, size_t* filter_bytes, size_t* workspace_bytes,
                  int* Hout, int* Wout);

/* Buffer layout (all offsets in bytes from the start of the buffer named).
 *   U buffer:  U'[e][k][c], e < alpha^2, k < K_pad, c < C_pad, elem_bytes each;
 *              then (WG_F16 / WG_BF16 only) at scale_offset the int32 exponents
 *              s[e][c], c < C_pad; at chan_offset the int32 per-channel parts
 *              t[c] = E(x_absmax[c]) - E(max|w[.][c]|), so that
 *              s[e1*alpha+e2][c] = floor((dB[e1] + dB[e2] + t[c]) / 2) with
 *              dB[i] = E(|B^T row i|_1) - E(|G row i|_1); then library scratch.
 *   workspace: V'[e][p][c] at v_offset (e < alpha^2, p < P_pad, c < C_pad,
 *              elem_bytes each) and M[e][k][p] float32 at m_offset
 *              (k < K_pad, p < P_pad).
 * Tile index p = (n*Th + th)*Tw + tw; tile (th, tw) covers outputs
 * [th*m, th*m+m) x [tw*m, tw*m+m) and reads the input window whose top-left
 * corner is (th*m - pad, tw*m - pad). */
typedef struct {
    int alpha, m, r, pad;
    int N, C, K, H, W, Hout, Wout, Th, Tw;
    int P, P_pad, K_pad, C_pad;
    int dtype, elem_bytes;
    size_t scale_offset, chan_offset, filter_bytes;
    size_t v_offset, m_offset, workspace_bytes;
} wg_layout;
int wg_plan_layout(const wg_plan* plan, wg_layout* out);

/* The float32 matrices of the plan (host outputs, sizes as wg_transforms). */
int wg_plan_matrices(const wg_plan* plan, float* AT, float* G, float* BT);

/* Tuning of a plan's Hadamard GEMM (host only, no effect on results): each
 * thread block takes `tiles_per_block` consecutive output tiles (1..16) and
 * keeps its load pipeline running across them.  wg_plan_gemm_tiles returns
 * the current value (>= 1), or an error code.  Default 1.
 * Errors: WG_EINVAL (null plan, value outside 1..16). */
int wg_plan_set_gemm_tiles(wg_plan* plan, int tiles_per_block);
int wg_plan_gemm_tiles(const wg_plan* plan);

/* Autotuner for the same knob: runs the plan's Hadamard GEMM on the caller's
 * transformed operands (U from wg_transform_filters, V' in `ws` from
 * wg_input_transform) for each candidate in {1, 2, 3, 4, 6, 8}, `reps` timed
 * launches each after one warm-up, and keeps the fastest.  Synchronous on
 * `stream`; overwrites the M part of the workspace (run wg_hadamard_gemm
 * again afterwards).  Writes the chosen value to *chosen if non-null.
 * Errors: WG_EINVAL, WG_EWORKSPACE, WG_EHIP. */
int wg_plan_autotune_gemm(wg_plan* plan, const void* U, void* ws, size_t ws_bytes, int reps,
                          int* chosen, wg_stream_t stream);

/* ------------------------------------------------------------------------
 * Layer (device, asynchronous).  Section 4 eq. conv_2d applied tile by tile
 * to the layer of eq. conv; Section 4.1 notes that the filter and input
 * transforms are amortised and that the channel sum of the Hadamard products
 * is a matrix product.
 *
 * Size limits of the launches (WG_EUNSUPPORTED when exceeded; the kernels
 * address these ranges with 32-bit byte offsets): one image of x padded to
 * C_pad channels below 2 GB; one row of alpha planes of M below 2 GB; 128
 * rows of a plane of M, U' or V' below 2 GB.
 * ---------------------------------------------------------------------- */

/* Filter transform U = G g G^T for every (k, c) (offline, once per weights).
 * w: device, K x C x r x r float32.  U: device, filter_bytes.
 * x_absmax: device, C float32 per-input-channel bounds of |x| used for the
 *   power-of-two scaling of the 16-bit Hadamard stage, or NULL (bound 1).
 *   Ignored for WG_F32.
 * For WG_F16 / WG_BF16 the per (tile element e=(e1,e2), channel c) exponent
 *   s = floor((E_V - E_U) / 2),
 *   E_V = E(|B^T_e1|_1) + E(|B^T_e2|_1) + E(x_absmax[c]),
 *   E_U = E(|G_e1|_1) + E(|G_e2|_1) + E(max_k,u,v |w[k][c][u][v]|),
 * with E(v) the binary exponent of v (v = f 2^E, 0.5 <= f < 1; E(0) = 0) and
 * row norms summed in float64, is stored with U, and U' = RN16(U 2^s).
 * Padding rows/columns of U (k >= K, c >= C) are written as zeros. */
int wg_transform_filters(const wg_plan* plan, const float* w, const float* x_absmax,
                         void* U, wg_stream_t stream);

/* Full forward pass: input transform -> Hadamard/channel-sum GEMM ->
 * output transform.  x: device N x C x H x W.  U: device, from
 * wg_transform_filters with the same plan.  y: device N x K x Hout x Wout.
 * ws: device workspace of at least workspace_bytes (WG_EWORKSPACE otherwise);
 * its contents on return are the V' and M buffers of this pass. */
int wg_conv2d_forward(const wg_plan* plan, const float* x, const void* U, float* y,
                      void* ws, size_t ws_bytes, wg_stream_t stream);

/* The three stages of wg_conv2d_forward, separately (same buffers):
 *   input:  V'[e][p][c] = scaled/rounded (B^T d B)[e] of tile p, channel c
 *   gemm:   M[e][k][p] = sum_c U'[e][k][c] V'[e][p][c]  (float32 accumulation)
 *           for k < K, p < P; the padding of M (k >= K, and p >= P from the
 *           first multiple of 4 at or above P) is left unwritten, and the
 *           padding rows of U' and V' are not read
 *   output: y tile p, channel k = (A^T M[.][k][p] A), outputs past the edge
 *           discarded. */
int wg_input_transform(const wg_plan* plan, const float* x, const void* U,
                       void* ws, size_t ws_bytes, wg_stream_t stream);

/* The first step of wg_transform_filters on its own: for WG_F16 / WG_BF16
 * the maxima of |w| over chunks of filters, per channel, kept in U's buffer
 * (nothing to do for WG_F32).  wg_transform_filters runs it itself;
 * wg_transform_filters_and_input expects it to have run on the same w and U
 * before (in stream order).  Errors: WG_EINVAL, WG_EHIP. */
int wg_filter_maxima(const wg_plan* plan, const float* w, void* U, wg_stream_t stream);

/* The filter transform of w (as wg_transform_filters) and the input
 * transform of x (as wg_input_transform) in one launch, after
 * wg_filter_maxima: both transforms are amortised stages with no
 * dependence on each other (Section 4.1), so the short filter blocks run
 * beside the input transform instead of as a launch of their own.  U and
 * the V' part of ws receive exactly what wg_transform_filters followed by
 * wg_input_transform write (the input blocks derive the 16-bit exponent
 * part t[c] from the same partial maxima as the filter blocks).  Arguments
 * as for the two calls; x_absmax may be NULL.  Errors: WG_EINVAL,
 * WG_EWORKSPACE, WG_EUNSUPPORTED (the limits of both calls), WG_EHIP. */
int wg_transform_filters_and_input(const wg_plan* plan, const float* w, const float* x_absmax,
                                   const float* x, void* U, void* ws, size_t ws_bytes,
                                   wg_stream_t stream);

/* Per-batch 16-bit scaling: the calls a caller makes for every new input
 * when max |x_c| is not known beforehand (the scaling of the Hadamard stage
 * then follows each batch; Section 4.1 amortises both transforms, so they
 * share one launch):
 *   wg_layer_maxima:    for WG_F16 / WG_BF16, in one launch with one block
 *                       per channel: max |x_c| over the batch and max |w_c|
 *                       over the filters, and from them the per-channel part
 *                       t[c] = E(max |x_c|) - E(max |w_c|) and the scale
 *                       table s[e][c] of wg_transform_filters, written into
 *                       U; nothing to do for WG_F32.
 *   wg_transform_layer: then the filter and input transforms in one launch
 *                       as wg_transform_filters_and_input, both reading t[c]
 *                       from U (for WG_F32: wg_transform_filters_and_input
 *                       with x_absmax NULL).
 * U, the scale tables and V' equal bit for bit what wg_channel_absmax,
 * wg_filter_maxima and wg_transform_filters_and_input with those maxima
 * write.  x, w: device float32 as for the other calls; U: device,
 * filter_bytes; ws: device workspace of at least workspace_bytes.
 * Errors: WG_EINVAL (null pointer), WG_EWORKSPACE, WG_EUNSUPPORTED (the
 * limits of wg_transform_filters_and_input), WG_EHIP. */
int wg_layer_maxima(const wg_plan* plan, const float* w, const float* x, void* U, wg_stream_t stream);
int wg_transform_layer(const wg_plan* plan, const float* w, const float* x, void* U, void* ws,
                       size_t ws_bytes, wg_stream_t stream);

int wg_hadamard_gemm(const wg_plan* plan, const void* U, void* ws, size_t ws_bytes,
                     wg_stream_t stream);
int wg_output_transform(const wg_plan* plan, const void* ws, size_t ws_bytes, float* y,
                        wg_stream_t stream);

/* Per-channel max |x| over n, h, w.  x: device N x C x H x W; out: device C. */
int wg_channel_absmax(const float* x, int N, int C, int H, int W, float* out,
                      wg_stream_t stream);

/* ------------------------------------------------------------------------
 * Error scoring (device).  Section 6: the error of a float32 result is its
 * L1 distance to a float64 direct convolution.
 * ---------------------------------------------------------------------- */

/* float64 direct convolution of the float32 inputs (eq. conv as a zero-padded
 * cross-correlation): y_ref[n][k][i][j] = sum_{c,u,v} x[n][c][i+u-p][j+v-p]
 * w[k][c][u][v].  x, w: device float32; y_ref: device float64 N x K x Hout x
 * Wout.  1 <= r <= 7.  Every product is exact in float64; the sums run on the
 * float64 matrix cores in a blocked order (the result is reproducible for
 * given sizes).  Errors: WG_EINVAL. */
int wg_direct_conv_f64(const float* x, const float* w, double* y_ref,
                       int N, int C, int K, int H, int W, int r, int padding,
                       wg_stream_t stream);

/* out2 (device, 2 doubles) = { sum |y - y_ref|, sum |y_ref| } in float64, with
 * a fixed reduction tree (bitwise reproducible for a given count).
 * ws: device, at least wg_score_workspace_bytes(count) bytes.
 * Relative L1 = out2[0]/out2[1]; mean absolute error = out2[0]/count. */
size_t wg_score_workspace_bytes(size_t count);
int wg_score_error(const float* y, const double* y_ref, size_t count, double* out2,
                   void* ws, size_t ws_bytes, wg_stream_t stream);

/* wg_score_error without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels, results bit for bit
 * those of wg_score_error, with the partial sums in a static device array of
 * the library (1024 pairs of doubles, 16 KB, one copy per GPU, held until
 * the process ends; the partial-sum grid never has more than 1024 blocks, so
 * every count fits).  Nothing is allocated and no library routine that
 * allocates is called.  The calling thread's current device must be the
 * device of y, y_ref, out2 and stream; the device address of the array is
 * looked up on the first call on each device.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller.
 * Errors: WG_EINVAL (null pointer, count 0), WG_EHIP. */
int wg_score_error_noalloc(const float* y, const double* y_ref, size_t count, double* out2,
                           wg_stream_t stream);

/* ------------------------------------------------------------------------
 * Batched error sweep (device).  Section 6.1 traces the error of a point
 * family as a function of c; Section 6.3 scores many combinations.  For each
 * candidate (c1[i], c2[i]) the family of wg_family_points for
 * alpha = m + r - 1 is built, its matrices are constructed on the device as
 * the float64 roundings of their exact values (Sections 4.1, 4.2; the same
 * matrices as wg_transforms) and rounded to float32, and float32 Winograd
 * tiles (1D eq. conv_1d or 2D
 * eq. conv_2d, evaluated as the layer's transforms are) are scored on the
 * first counts[i] samples of a shared pool against the float64 direct
 * correlation of each sample.
 * ---------------------------------------------------------------------- */
typedef struct wg_sweep wg_sweep;

/* Creates a sweep for F(m, r) (dims = 1) or F(m x m, r x r) (dims = 2) with
 * alpha = m + r - 1 in 4..10 and r in {3, 5}.
 * d_pool: device, n_pool x alpha (x alpha) float32 input tiles; g_pool:
 * device, n_pool x r (x r) float32 filters; both are read by every run and
 * must stay valid until the sweep is destroyed (the sweep does not copy
 * them).  max_cand bounds n_cand of every run.  The float64 reference of the
 * pool (and an element-major copy of the pool) is computed on `stream` and
 * waited for before returning.  The sweep owns device buffers of about
 * max_cand * (1 KB + 8 * n_pool / 64 B) plus n_pool * (4 * (tile + filter
 * elements) + 8 * (outputs per sample + 2)) bytes.
 * Errors: WG_EINVAL, WG_EUNSUPPORTED, WG_ENOMEM, WG_EHIP. */
int wg_sweep_create(wg_sweep** out, int m, int r, int dims, const float* d_pool,
                    const float* g_pool, int n_pool, int max_cand, wg_stream_t stream);
int wg_sweep_destroy(wg_sweep* sweep);      /* NULL is accepted */

/* Scores n_cand candidates (1 <= n_cand <= max_cand).  c1, c2: device
 * float64 arrays (c2 may be NULL: 1.0 for every candidate; ignored for
 * alpha <= 6); counts: device int32, pool prefix sizes (clamped to
 * [0, n_pool]).  out: device float64 [n_cand][4] =
 *   { sum |y - y_ref| (+inf when flagged), sum |y_ref|,
 *     number of outputs scored, flag (1: c not finite or zero, points
 *     coincide, |N_i| < 1e-300, an entry overflows float32, or the exact
 *     construction below needs integers over 1024 bits) }.
 * mean absolute error = out[0]/out[2]; relative L1 = out[0]/out[1].
 * Every matrix entry is the float64 number nearest (ties to even) to its
 * exact value for the candidate's float64 points, as wg_transforms builds
 * it, and its float32 rounding: the construction evaluates each entry in
 * double-word arithmetic with a rigorous error bound and keeps it when the
 * bound decides the rounding (structural zeros of symmetric point sets come
 * out exact); candidates with an undecided entry are rebuilt in exact
 * multi-limb integer arithmetic by a second launch.
 * The four launches of a run (construct, exact rebuild, persistent
 * evaluation, finalize)
 * are captured in a hipGraph on the first call with a given argument set
 * and replayed on later calls with the same arguments; the result is
 * bitwise reproducible for a given tuning.  Runs on one sweep object must
 * not overlap. */
int wg_sweep_run(wg_sweep* sweep, const double* c1, const double* c2, const int* counts,
                 int n_cand, double* out, wg_stream_t stream);

/* As wg_sweep_run, for explicit point sets instead of a family: the
 * comparison sets of Tables tab:sota_1d and tab:sota_2d, subsets of a base
 * set (Section 5.1, eq. subset_points), or any other ordered list.
 * pts: device float64 [n_cand][alpha - 1], each row the ordered finite
 * points of one candidate (infinity is appended last, the modified form of
 * Section 4.2).  The matrices are built as for a family (Sections 4.1, 4.2)
 * and every term of every product is evaluated (no zero pattern is
 * assumed), so a list equal to a family's points scores exactly as that
 * family.  A candidate is flagged when a point is not finite, two points
 * coincide, |N_i| < 1e-300 or an entry overflows float32.  Shares the
 * tuning and graph cache of wg_sweep_run (a change between the two modes
 * recaptures the graph).  Errors: WG_EINVAL (null pointer, n_cand out of
 * range), WG_EHIP. */
int wg_sweep_run_points(wg_sweep* sweep, const double* pts, const int* counts, int n_cand,
                        double* out, wg_stream_t stream);

/* Times the evaluation over a fixed set of launch shapes (block size,
 * samples per work item, persistent blocks per compute unit) on the given
 * arguments, keeps the fastest for later runs and synchronises `stream`.
 * out receives the last result.  wg_sweep_tuning reports the shape in use;
 * it returns 1 after autotuning, 0 before (default shape). */
int wg_sweep_autotune(wg_sweep* sweep, const double* c1, const double* c2, const int* counts,
                      int n_cand, double* out, wg_stream_t stream);
int wg_sweep_tuning(const wg_sweep* sweep, int* block, int* chunk, int* blocks_per_cu);

/* The float32 matrices the last run built for candidate `cand` (host
 * outputs, sizes as wg_transforms) and its flag: 1 flagged, 2 built by the
 * exact integer construction, 0 built by the certified double-word
 * construction; synchronous. */
int wg_sweep_matrices(const wg_sweep* sweep, int cand, float* AT, float* G, float* BT, int* flag);

/* Precision of the evaluated tiles (Section 6: besides the plain float32
 * evaluation the paper scores a mixed-precision one, float64 transforms with
 * a float32 Hadamard product).
 *   WG_SWEEP_F32   (default): every step in float32, one fused multiply-add
 *                  per term.
 *   WG_SWEEP_MIXED: the float64 matrices (before their float32 rounding)
 *                  transform filter and tile in float64, U and V are rounded
 *                  to float32, multiplied in float32, and Y = A^T M A is
 *                  taken in float64 and rounded to float32; each float64 term
 *                  is a rounded product followed by a rounded sum, in
 *                  ascending index order.
 * Applies to later wg_sweep_run / wg_sweep_run_points calls (the captured
 * graph is rebuilt).  The first switch to WG_SWEEP_MIXED allocates
 * max_cand * 2 KB of device memory, kept until the sweep is destroyed.
 * Errors: WG_EINVAL (null sweep, unknown mode), WG_ENOMEM. */
enum { WG_SWEEP_F32 = 0, WG_SWEEP_MIXED = 1 };
int wg_sweep_set_precision(wg_sweep* sweep, int mode);

/* always = 1: every valid candidate of later runs is built by the exact
 * integer construction (the second launch of a run), bypassing the
 * certified double-word one; always = 0 (default): only candidates the
 * certified construction cannot decide.  Both give the same matrices; the
 * switch serves to check that and to time the exact path.  Later runs
 * rebuild the captured graph.  Errors: WG_EINVAL (null sweep, always not
 * 0 or 1). */
int wg_sweep_set_exact(wg_sweep* sweep, int always);

/* The float64 matrices the last mixed-precision run built for candidate
 * `cand` (host outputs, sizes as wg_transforms); synchronous.  WG_EINVAL if
 * the sweep never ran in mixed precision. */
int wg_sweep_matrices_f64(const wg_sweep* sweep, int cand, double* AT, double* G, double* BT);

/* ------------------------------------------------------------------------
 * Error surrogate (device).  A fully connected network 4 -> 128 -> 128 ->
 * 128 -> 1 with GELU (z * Phi(z); the kernels evaluate the normal tail with
 * the erfc approximation of Abramowitz and Stegun 7.1.26, absolute error at
 * most 1.5e-7, sharing its exponential with the derivative) maps a point-family
 * description to a predicted log10 mean absolute error, so that the smooth
 * error curve (Sections 1 and 6.1) can be searched with few exact sweep
 * evaluations.  Input encoding of a sample (c1, c2, m, r):
 *   (ln c1 / ln 20, ln c2 / ln 20, (m - 5) / 3, r - 4)   (c2 NULL: ln c2 = 0).
 * Parameters: device float32[wg_mlp_param_count()] = 33793, caller owned,
 * layout W1[128][4], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 * W4[1][128], b4[1] (row-major W[out][in]).  Loss: mean over the batch of
 * (prediction - target)^2.  All reductions run in a fixed order, so results
 * are bitwise reproducible.
 * ---------------------------------------------------------------------- */
typedef struct wg_mlp wg_mlp;
int wg_mlp_param_count(void);

/* Training context for batches of at most max_batch samples; owns a device
 * scratch of about 2.3 KB per sample of max_batch (the hidden activations
 * and dL/dZ of a step and per-16-sample partial sums of the small
 * gradients).  Calls on one context share that scratch and must not
 * overlap.  Errors: WG_EINVAL, WG_ENOMEM. */
int wg_mlp_create(wg_mlp** out, int max_batch);
int wg_mlp_destroy(wg_mlp* mlp);            /* NULL is accepted */

/* Data arrays (device): c1, c2 float64 (c2 may be NULL), m, r int32,
 * target float32, all of length n. */

/* Loss gradient over all n samples (n <= max_batch): grad_out (device
 * float32[33793]) and loss_out (device float32[1], may be NULL). */
int wg_mlp_gradient(wg_mlp* mlp, const float* params, const double* c1, const double* c2,
                    const int* m, const int* r, const float* target, int n,
                    float* grad_out, float* loss_out, wg_stream_t stream);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; Kingma and Ba) for
 * `epochs` passes over the n samples in the orders given by perm (device
 * int32[epochs][n]), minibatches of `batch` consecutive entries of perm (the
 * last n % batch entries of each pass are skipped), step counter starting at
 * step0 >= 1.  adam_state: device float32[2 * 33793] (first then second
 * moments; zero before the first step).  losses: device float32
 * [epochs * (n / batch)], the loss of every step before its update.  The
 * context also keeps 20 bytes per sample of the n (the input features and
 * targets of a pass, in minibatch order), allocated on the first call that
 * needs more and held until wg_mlp_destroy (WG_ENOMEM if that allocation
 * fails).  A perm entry outside [0, n) gives NaN features for its sample
 * (so NaN losses), not an out-of-range read. */
int wg_mlp_train(wg_mlp* mlp, float* params, float* adam_state, int step0, float lr,
                 const double* c1, const double* c2, const int* m, const int* r,
                 const float* target, int n, const int* perm, int epochs, int batch,
                 float* losses, wg_stream_t stream);

/* Predictions out (device float32[n]). */
int wg_mlp_predict(const float* params, const double* c1, const double* c2, const int* m,
                   const int* r, int n, float* out, wg_stream_t stream);

/* Indices (device int32[k], ascending values, ties to the smaller index,
 * NaN never chosen, -1 when fewer than k candidates) of the k <= 64
 * smallest entries of v (device float32[n]). */
int wg_topk_min(const float* v, int n, int k, int* idx_out, wg_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* WG_H */
