"""ctypes binding of libwg.so (the C ABI declared in include/wg.h).

Argument marshalling only: every computation happens in the HIP library.
Device buffers are torch tensors on a ROCm device; work is enqueued on the
current torch stream (or the stream passed in).  Raises WGError when the
library reports a failure, and RuntimeError when the library is not built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwg.so")

WG_MODIFIED, WG_UNMODIFIED = 0, 1
WG_SAME, WG_VALID = 0, 1
WG_F32, WG_F16, WG_BF16 = 0, 1, 2
WG_F64_TRANSFORMS = 4
# "mixed": float64 transforms with a float32 Hadamard stage (WG_F32 plan
# with WG_F64_TRANSFORMS)
DTYPES = {"f32": WG_F32, "f16": WG_F16, "bf16": WG_BF16, "mixed": WG_F32}
PADDINGS = {"same": WG_SAME, "valid": WG_VALID}
STATUS = {0: "WG_OK", -1: "WG_EINVAL", -2: "WG_ESINGULAR", -3: "WG_EUNSUPPORTED",
          -4: "WG_EWORKSPACE", -5: "WG_ENOMEM", -6: "WG_EHIP"}

c_int, c_double, c_float, c_size_t, c_void_p = (ctypes.c_int, ctypes.c_double, ctypes.c_float,
                                                ctypes.c_size_t, ctypes.c_void_p)
P_double = ctypes.POINTER(c_double)
P_float = ctypes.POINTER(c_float)
P_int = ctypes.POINTER(c_int)
P_size_t = ctypes.POINTER(c_size_t)


class WGError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Layout(ctypes.Structure):
    _fields_ = [(n, c_int) for n in ("alpha", "m", "r", "pad", "N", "C", "K", "H", "W", "Hout", "Wout",
                                     "Th", "Tw", "P", "P_pad", "K_pad", "C_pad", "dtype", "elem_bytes")] + \
               [(n, c_size_t) for n in ("scale_offset", "chan_offset", "filter_bytes", "v_offset", "m_offset",
                                        "workspace_bytes")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_SIGS = {
    "wg_last_error": (ctypes.c_char_p, []),
    "wg_version": (c_int, []),
    "wg_supported": (c_int, [c_int, c_int]),
    "wg_transforms": (c_int, [c_int, c_int, P_double, c_int, c_int, P_double, P_double, P_double]),
    "wg_transforms_f32": (c_int, [c_int, c_int, P_double, c_int, c_int, P_float, P_float, P_float]),
    "wg_family_points": (c_int, [c_int, c_double, c_double, P_double]),
    "wg_plan_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, P_double, c_int, c_int,
                               c_int, c_int, c_int, c_int, c_int, c_int, c_int]),
    "wg_plan_destroy": (c_int, [c_void_p]),
    "wg_plan_sizes": (c_int, [c_void_p, P_size_t, P_size_t, P_int, P_int]),
    "wg_plan_layout": (c_int, [c_void_p, ctypes.POINTER(Layout)]),
    "wg_plan_matrices": (c_int, [c_void_p, P_float, P_float, P_float]),
    "wg_plan_set_gemm_tiles": (c_int, [c_void_p, c_int]),
    "wg_plan_gemm_tiles": (c_int, [c_void_p]),
    "wg_plan_autotune_gemm": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int, P_int, c_void_p]),
    "wg_transform_filters": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "wg_conv2d_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "wg_input_transform": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "wg_filter_maxima": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "wg_transform_filters_and_input": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                               c_void_p]),
    "wg_layer_maxima": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "wg_transform_layer": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "wg_hadamard_gemm": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "wg_output_transform": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "wg_channel_absmax": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_void_p]),
    "wg_direct_conv_f64": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int,
                                   c_int, c_int, c_void_p]),
    "wg_score_workspace_bytes": (c_size_t, [c_size_t]),
    "wg_sweep_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_int, c_void_p, c_void_p, c_int, c_int,
                                c_void_p]),
    "wg_sweep_destroy": (c_int, [c_void_p]),
    "wg_sweep_run": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "wg_sweep_run_points": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "wg_sweep_set_precision": (c_int, [c_void_p, c_int]),
    "wg_sweep_set_exact": (c_int, [c_void_p, c_int]),
    "wg_sweep_matrices_f64": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "wg_sweep_autotune": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "wg_sweep_tuning": (c_int, [c_void_p, P_int, P_int, P_int]),
    "wg_sweep_matrices": (c_int, [c_void_p, c_int, P_float, P_float, P_float, P_int]),
    "wg_mlp_param_count": (c_int, []),
    "wg_mlp_create": (c_int, [ctypes.POINTER(c_void_p), c_int]),
    "wg_mlp_destroy": (c_int, [c_void_p]),
    "wg_mlp_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                c_void_p, c_void_p, c_void_p]),
    "wg_mlp_train": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_float, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_int, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "wg_mlp_predict": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "wg_topk_min": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "wg_score_error": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p, c_size_t, c_void_p]),
    "wg_score_error_noalloc": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
}

_lib = None


def lib():
    """Load libwg.so (built in-tree); fails loudly when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2201_10369_amd.build")
        # torch first: its HIP runtime is the one the process uses, so the
        # library's launches and torch's memory and streams share a runtime
        # (loading the library first would bring in a second one)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status < 0:
        raise WGError(status, lib().wg_last_error().decode())
    return status


def _dptr(arr):
    return arr.ctypes.data_as(P_double)


def _fptr(arr):
    return arr.ctypes.data_as(P_float)


# ----------------------------------------------------------------------------
# device-buffer helpers
# ----------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _tptr(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous torch tensor on a GPU (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


# ----------------------------------------------------------------------------
# host functions
# ----------------------------------------------------------------------------
def transforms(m, r, pts, modified=True, f32=False):
    """(A^T, G, B^T) from ordered finite points (numpy float64 or float32)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    alpha = m + r - 1
    dt = np.float32 if f32 else np.float64
    AT = np.zeros((m, alpha), dt)
    G = np.zeros((alpha, r), dt)
    BT = np.zeros((alpha, alpha), dt)
    fn = lib().wg_transforms_f32 if f32 else lib().wg_transforms
    conv = _fptr if f32 else _dptr
    _check(fn(m, r, _dptr(pts), len(pts), WG_MODIFIED if modified else WG_UNMODIFIED,
              conv(AT), conv(G), conv(BT)))
    return AT, G, BT


def family_points(alpha, c1, c2=1.0):
    out = np.zeros(16, dtype=np.float64)
    n = _check(lib().wg_family_points(alpha, float(c1), float(c2), _dptr(out)))
    return out[:n].copy()


def supported(m, r):
    return bool(lib().wg_supported(m, r))


class Plan:
    """A Winograd layer plan: points, F(m x m, r x r), layer shape, dtype."""

    def __init__(self, m, r, pts, N, C, K, H, W, padding="same", dtype="f32"):
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        h = c_void_p()
        flags = WG_MODIFIED | (WG_F64_TRANSFORMS if dtype == "mixed" else 0)
        _check(lib().wg_plan_create(ctypes.byref(h), m, r, _dptr(pts), len(pts), flags,
                                    N, C, K, H, W, PADDINGS[padding], DTYPES[dtype]))
        self._h = h
        self.m, self.r, self.dtype, self.padding = m, r, dtype, padding
        lay = Layout()
        _check(lib().wg_plan_layout(self._h, ctypes.byref(lay)))
        self.layout = lay.as_dict()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wg_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def filter_bytes(self):
        return self.layout["filter_bytes"]

    @property
    def workspace_bytes(self):
        return self.layout["workspace_bytes"]

    @property
    def out_hw(self):
        return self.layout["Hout"], self.layout["Wout"]

    def matrices(self):
        L = self.layout
        a, m, r = L["alpha"], L["m"], L["r"]
        AT = np.zeros((m, a), np.float32)
        G = np.zeros((a, r), np.float32)
        BT = np.zeros((a, a), np.float32)
        _check(lib().wg_plan_matrices(self._h, _fptr(AT), _fptr(G), _fptr(BT)))
        return AT, G, BT

    # -- device buffers -----------------------------------------------------
    @property
    def gemm_tiles(self):
        """Output tiles per thread block of the Hadamard GEMM (a tuning knob)."""
        return _check(lib().wg_plan_gemm_tiles(self._h))

    @gemm_tiles.setter
    def gemm_tiles(self, value):
        _check(lib().wg_plan_set_gemm_tiles(self._h, int(value)))

    def empty_filters(self, device="cuda"):
        torch = _torch()
        return torch.empty(self.filter_bytes, dtype=torch.uint8, device=device)

    def empty_workspace(self, device="cuda"):
        torch = _torch()
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def empty_output(self, device="cuda"):
        torch = _torch()
        L = self.layout
        return torch.empty((L["N"], L["K"], L["Hout"], L["Wout"]), dtype=torch.float32, device=device)

    # -- stages ---------------------------------------------------------------
    def transform_filters(self, w, x_absmax=None, U=None, stream=None):
        torch = _torch()
        U = self.empty_filters(w.device) if U is None else U
        _check(lib().wg_transform_filters(self._h, _tptr(w, torch.float32, "w"),
                                          _tptr(x_absmax, torch.float32, "x_absmax"),
                                          _tptr(U, None, "U"), _stream(stream)))
        return U

    def forward(self, x, U, y=None, ws=None, stream=None):
        torch = _torch()
        y = self.empty_output(x.device) if y is None else y
        ws = self.empty_workspace(x.device) if ws is None else ws
        _check(lib().wg_conv2d_forward(self._h, _tptr(x, torch.float32, "x"), _tptr(U, None, "U"),
                                       _tptr(y, torch.float32, "y"), _tptr(ws, None, "ws"),
                                       ws.numel() * ws.element_size(), _stream(stream)))
        return y

    def input_transform(self, x, U, ws, stream=None):
        torch = _torch()
        _check(lib().wg_input_transform(self._h, _tptr(x, torch.float32, "x"), _tptr(U, None, "U"),
                                        _tptr(ws, None, "ws"), ws.numel() * ws.element_size(),
                                        _stream(stream)))

    def filter_maxima(self, w, U, stream=None):
        """The 16-bit partial maxima of |w| into U (no-op for f32)."""
        torch = _torch()
        _check(lib().wg_filter_maxima(self._h, _tptr(w, torch.float32, "w"), _tptr(U, None, "U"),
                                      _stream(stream)))

    def transform_filters_and_input(self, w, x, U, ws, x_absmax=None, stream=None):
        """Filter and input transforms in one launch, after filter_maxima
        (same U and V' as transform_filters followed by input_transform)."""
        torch = _torch()
        _check(lib().wg_transform_filters_and_input(self._h, _tptr(w, torch.float32, "w"),
                                                    _tptr(x_absmax, torch.float32, "x_absmax"),
                                                    _tptr(x, torch.float32, "x"), _tptr(U, None, "U"),
                                                    _tptr(ws, None, "ws"), ws.numel() * ws.element_size(),
                                                    _stream(stream)))

    def layer_maxima(self, w, x, U, stream=None):
        """Per-batch 16-bit scaling, first call: partial maxima of |w| and
        |x| into U (no-op for f32)."""
        torch = _torch()
        _check(lib().wg_layer_maxima(self._h, _tptr(w, torch.float32, "w"), _tptr(x, torch.float32, "x"),
                                     _tptr(U, None, "U"), _stream(stream)))

    def transform_layer(self, w, x, U, ws, stream=None):
        """Per-batch 16-bit scaling, second call: filter and input transforms
        in one launch with max |x_c| from the partial maxima in U."""
        torch = _torch()
        _check(lib().wg_transform_layer(self._h, _tptr(w, torch.float32, "w"), _tptr(x, torch.float32, "x"),
                                        _tptr(U, None, "U"), _tptr(ws, None, "ws"), ws.numel() * ws.element_size(),
                                        _stream(stream)))

    def hadamard_gemm(self, U, ws, stream=None):
        _check(lib().wg_hadamard_gemm(self._h, _tptr(U, None, "U"), _tptr(ws, None, "ws"),
                                      ws.numel() * ws.element_size(), _stream(stream)))

    def autotune_gemm(self, U, ws, reps=10, stream=None):
        """Pick the GEMM's tiles per block by timing the candidates on these
        operands (synchronous; overwrites M in ws).  Returns the choice."""
        chosen = c_int(0)
        _check(lib().wg_plan_autotune_gemm(self._h, _tptr(U, None, "U"), _tptr(ws, None, "ws"),
                                           ws.numel() * ws.element_size(), int(reps), ctypes.byref(chosen),
                                           _stream(stream)))
        return chosen.value

    def output_transform(self, ws, y, stream=None):
        torch = _torch()
        _check(lib().wg_output_transform(self._h, _tptr(ws, None, "ws"), ws.numel() * ws.element_size(),
                                         _tptr(y, torch.float32, "y"), _stream(stream)))

    # -- views of the buffers (for tests) --------------------------------------
    def _elem_dtype(self):
        torch = _torch()
        return {"f32": torch.float32, "mixed": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[self.dtype]

    def view_U(self, U):
        L = self.layout
        E = L["alpha"] ** 2
        n = E * L["K_pad"] * L["C_pad"] * L["elem_bytes"]
        return U[:n].view(self._elem_dtype()).view(E, L["K_pad"], L["C_pad"])

    def view_scales(self, U):
        torch = _torch()
        L = self.layout
        E = L["alpha"] ** 2
        off = L["scale_offset"]
        return U[off:off + E * L["C_pad"] * 4].view(torch.int32).view(E, L["C_pad"])

    def view_V(self, ws):
        L = self.layout
        E = L["alpha"] ** 2
        n = E * L["P_pad"] * L["C_pad"] * L["elem_bytes"]
        off = L["v_offset"]
        return ws[off:off + n].view(self._elem_dtype()).view(E, L["P_pad"], L["C_pad"])

    def view_M(self, ws):
        torch = _torch()
        L = self.layout
        E = L["alpha"] ** 2
        off = L["m_offset"]
        return ws[off:off + E * L["K_pad"] * L["P_pad"] * 4].view(torch.float32).view(E, L["K_pad"], L["P_pad"])


# ----------------------------------------------------------------------------
# scoring
# ----------------------------------------------------------------------------
def direct_conv_f64(x, w, padding="same", y=None, stream=None):
    torch = _torch()
    N, C, H, W = x.shape
    K, _, r, _ = w.shape
    p = (r - 1) // 2 if padding == "same" else 0
    Ho, Wo = H + 2 * p - r + 1, W + 2 * p - r + 1
    y = torch.empty((N, K, Ho, Wo), dtype=torch.float64, device=x.device) if y is None else y
    _check(lib().wg_direct_conv_f64(_tptr(x, torch.float32, "x"), _tptr(w, torch.float32, "w"),
                                    _tptr(y, torch.float64, "y_ref"), N, C, K, H, W, r,
                                    PADDINGS[padding], _stream(stream)))
    return y


def score_error(y, yref, out=None, ws=None, stream=None):
    """Device tensor [sum|y - yref|, sum|yref|] (float64)."""
    torch = _torch()
    count = y.numel()
    if yref.numel() != count:
        raise ValueError("y and yref differ in size")
    out = torch.empty(2, dtype=torch.float64, device=y.device) if out is None else out
    need = lib().wg_score_workspace_bytes(count)
    ws = torch.empty(need, dtype=torch.uint8, device=y.device) if ws is None else ws
    _check(lib().wg_score_error(_tptr(y, torch.float32, "y"), _tptr(yref, torch.float64, "yref"), count,
                                _tptr(out, torch.float64, "out"), _tptr(ws, None, "ws"),
                                ws.numel() * ws.element_size(), _stream(stream)))
    return out


def score_error_noalloc(y, yref, out, stream=None):
    """score_error with the library's static scratch: out (device float64
    [2]) receives [sum|y - yref|, sum|yref|]; nothing is allocated."""
    torch = _torch()
    count = y.numel()
    if yref.numel() != count:
        raise ValueError("y and yref differ in size")
    _check(lib().wg_score_error_noalloc(_tptr(y, torch.float32, "y"), _tptr(yref, torch.float64, "yref"), count,
                                        _tptr(out, torch.float64, "out"), _stream(stream)))
    return out


def channel_absmax(x, out=None, stream=None):
    torch = _torch()
    N, C, H, W = x.shape
    out = torch.empty(C, dtype=torch.float32, device=x.device) if out is None else out
    _check(lib().wg_channel_absmax(_tptr(x, torch.float32, "x"), N, C, H, W,
                                   _tptr(out, torch.float32, "out"), _stream(stream)))
    return out


# ----------------------------------------------------------------------------
# batched error sweep
# ----------------------------------------------------------------------------
class Sweep:
    """Error sweep of F(m, r) (dims 1) or F(m x m, r x r) (dims 2) over the
    point family of alpha = m + r - 1, on a pool of (tile, filter) samples."""

    def __init__(self, m, r, dims, d_pool, g_pool, max_cand, stream=None):
        torch = _torch()
        self.m, self.r, self.dims = m, r, dims
        self.alpha = m + r - 1
        self.n_pool = d_pool.shape[0]
        self.max_cand = max_cand
        self._pool = (d_pool, g_pool)                    # kept alive: the sweep reads them
        h = c_void_p()
        _check(lib().wg_sweep_create(ctypes.byref(h), m, r, dims, _tptr(d_pool, torch.float32, "d_pool"),
                                     _tptr(g_pool, torch.float32, "g_pool"), self.n_pool, max_cand,
                                     _stream(stream)))
        self._h = h
        self._args = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wg_sweep_destroy(h)
            self._h = None

    def _prep(self, c1, c2, counts, out):
        torch = _torch()
        n = c1.numel()
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float64, device=c1.device)
        # the captured graph holds these pointers: keep the tensors alive
        self._args = (c1, c2, counts, out)
        return n, out

    def run(self, c1, c2, counts, out=None, stream=None):
        torch = _torch()
        n, out = self._prep(c1, c2, counts, out)
        _check(lib().wg_sweep_run(self._h, _tptr(c1, torch.float64, "c1"), _tptr(c2, torch.float64, "c2"),
                                  _tptr(counts, torch.int32, "counts"), n, _tptr(out, torch.float64, "out"),
                                  _stream(stream)))
        return out

    def run_points(self, pts, counts, out=None, stream=None):
        """Scores explicit point sets: pts is a device float64 tensor
        [n_cand, alpha - 1] of ordered finite points (infinity implied last)."""
        torch = _torch()
        if pts.dim() != 2 or pts.shape[1] != self.alpha - 1:
            raise ValueError(f"pts must have shape [n_cand, {self.alpha - 1}]")
        n = pts.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float64, device=pts.device)
        self._args = (pts, counts, out)                  # held by the captured graph
        _check(lib().wg_sweep_run_points(self._h, _tptr(pts, torch.float64, "pts"),
                                         _tptr(counts, torch.int32, "counts"), n,
                                         _tptr(out, torch.float64, "out"), _stream(stream)))
        return out

    def autotune(self, c1, c2, counts, out=None, stream=None):
        torch = _torch()
        n, out = self._prep(c1, c2, counts, out)
        _check(lib().wg_sweep_autotune(self._h, _tptr(c1, torch.float64, "c1"), _tptr(c2, torch.float64, "c2"),
                                       _tptr(counts, torch.int32, "counts"), n,
                                       _tptr(out, torch.float64, "out"), _stream(stream)))
        return out

    def tuning(self):
        b, c, k = c_int(), c_int(), c_int()
        tuned = _check(lib().wg_sweep_tuning(self._h, ctypes.byref(b), ctypes.byref(c), ctypes.byref(k)))
        return dict(block=b.value, chunk=c.value, blocks_per_cu=k.value, tuned=bool(tuned))

    def set_precision(self, mode):
        """'f32' (default) or 'mixed' (float64 transforms, float32 Hadamard)."""
        code = {"f32": 0, "mixed": 1}[mode]
        _check(lib().wg_sweep_set_precision(self._h, code))
        self.precision = mode

    def set_exact(self, always):
        """True: build every candidate with the exact integer construction."""
        _check(lib().wg_sweep_set_exact(self._h, 1 if always else 0))

    def matrices_f64(self, cand):
        a, m, r = self.alpha, self.m, self.r
        AT = np.zeros((m, a), np.float64)
        G = np.zeros((a, r), np.float64)
        BT = np.zeros((a, a), np.float64)
        _check(lib().wg_sweep_matrices_f64(self._h, cand, _dptr(AT), _dptr(G), _dptr(BT)))
        return AT, G, BT

    def matrices(self, cand):
        a, m, r = self.alpha, self.m, self.r
        AT = np.zeros((m, a), np.float32)
        G = np.zeros((a, r), np.float32)
        BT = np.zeros((a, a), np.float32)
        flag = c_int()
        _check(lib().wg_sweep_matrices(self._h, cand, _fptr(AT), _fptr(G), _fptr(BT), ctypes.byref(flag)))
        return AT, G, BT, flag.value


# ----------------------------------------------------------------------------
# error surrogate
# ----------------------------------------------------------------------------
def mlp_param_count():
    return lib().wg_mlp_param_count()


def mlp_pack(params):
    """[(W, b), ...] (numpy) -> flat float32 vector in the library's layout."""
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in params]).astype(np.float32)


def mlp_unpack(flat, widths=(4, 128, 128, 128, 1)):
    out, o = [], 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        W = flat[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = flat[o:o + fo]
        o += fo
        out.append((W, b))
    return out


class Mlp:
    """Training context of the surrogate network (parameters are tensors the
    caller owns)."""

    def __init__(self, max_batch):
        h = c_void_p()
        _check(lib().wg_mlp_create(ctypes.byref(h), max_batch))
        self._h = h
        self.max_batch = max_batch

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wg_mlp_destroy(h)
            self._h = None

    def gradient(self, params, c1, c2, m, r, target, stream=None):
        torch = _torch()
        grad = torch.empty_like(params)
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
        _check(lib().wg_mlp_gradient(self._h, _tptr(params, torch.float32, "params"), _tptr(c1, torch.float64, "c1"),
                                     _tptr(c2, torch.float64, "c2"), _tptr(m, torch.int32, "m"),
                                     _tptr(r, torch.int32, "r"), _tptr(target, torch.float32, "target"),
                                     c1.numel(), _tptr(grad, torch.float32, "grad"),
                                     _tptr(loss, torch.float32, "loss"), _stream(stream)))
        return grad, loss

    def train(self, params, adam_state, step0, lr, c1, c2, m, r, target, perm, batch, stream=None):
        torch = _torch()
        n = c1.numel()
        epochs = perm.shape[0]
        losses = torch.empty(epochs * (n // batch), dtype=torch.float32, device=params.device)
        _check(lib().wg_mlp_train(self._h, _tptr(params, torch.float32, "params"),
                                  _tptr(adam_state, torch.float32, "adam_state"), step0, float(lr),
                                  _tptr(c1, torch.float64, "c1"), _tptr(c2, torch.float64, "c2"),
                                  _tptr(m, torch.int32, "m"), _tptr(r, torch.int32, "r"),
                                  _tptr(target, torch.float32, "target"), n, _tptr(perm, torch.int32, "perm"),
                                  epochs, batch, _tptr(losses, torch.float32, "losses"), _stream(stream)))
        return losses


def mlp_predict(params, c1, c2, m, r, out=None, stream=None):
    torch = _torch()
    n = c1.numel()
    out = torch.empty(n, dtype=torch.float32, device=c1.device) if out is None else out
    _check(lib().wg_mlp_predict(_tptr(params, torch.float32, "params"), _tptr(c1, torch.float64, "c1"),
                                _tptr(c2, torch.float64, "c2"), _tptr(m, torch.int32, "m"), _tptr(r, torch.int32, "r"),
                                n, _tptr(out, torch.float32, "out"), _stream(stream)))
    return out


def topk_min(v, k, stream=None):
    torch = _torch()
    idx = torch.empty(k, dtype=torch.int32, device=v.device)
    _check(lib().wg_topk_min(_tptr(v, torch.float32, "v"), v.numel(), k, _tptr(idx, torch.int32, "idx"),
                             _stream(stream)))
    return idx
