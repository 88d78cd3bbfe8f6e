"""Python binding of libvdamp (ctypes).  Argument marshalling only: every step of the
solve runs in the library's HIP kernels; torch supplies device memory and streams.

The names follow the C ABI in ``include/vdamp.h``: ``vdamp_plan``, ``vdamp_solve``,
``vdamp_solve_resume``, ``fista_solve``, ``vdamp_state_export``, ``vdamp_pass_times``,
``vdamp_wavelet``, the
learned denoiser ``vdamp_cnn_*`` and ``vdamp_solve_learned``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvdamp.so")

VDAMP_OK = 0
VDAMP_WAVELET_HAAR = 0
VDAMP_FLAG_DETERMINISTIC = 1 << 0
VDAMP_FLAG_CHECK_FINITE = 1 << 2
VDAMP_FLAG_USE_GRAPH = 1 << 3
VDAMP_FLAG_TIMING = 1 << 5
VDAMP_FLAG_AUTOTUNE = 1 << 6
VDAMP_FLAG_SURE_CONTINUOUS = 1 << 7
VDAMP_FLAG_GROUP_PAIRS = 1 << 8
VDAMP_NOALLOC_MAX_WORKSPACE = 64 << 20
PASS_NAMES = ("prep", "rows_synth", "cols", "rows_anal", "sure", "denoiser", "cnn")
VDAMP_CNN_WS_FORWARD = 0
VDAMP_CNN_WS_TRAIN = 1
VDAMP_CNN_WS_SOLVE = 2
VDAMP_JUDGE_SURE = 0
VDAMP_JUDGE_NONE = 1
# flat parameter order of the learned denoiser
CNN_PARAM_ORDER = ("W1", "b1", "Wt", "W2", "b2", "W3", "b3", "W4", "b4", "W5", "b5", "W6", "b6")
STATUS_NAMES = {0: "VDAMP_OK", 1: "VDAMP_ERR_ARG", 2: "VDAMP_ERR_SHAPE", 3: "VDAMP_ERR_UNSUPPORTED",
                4: "VDAMP_ERR_WORKSPACE", 5: "VDAMP_ERR_HIP", 6: "VDAMP_ERR_NONFINITE",
                7: "VDAMP_ERR_STATE"}

EXPORTED = ("vdamp_plan", "vdamp_plan_destroy", "vdamp_solve", "vdamp_solve_resume", "vdamp_solve_noalloc",
            "fista_solve",
            "vdamp_state_export", "vdamp_pass_times", "vdamp_status_string", "vdamp_last_error",
            "vdamp_cnn_create", "vdamp_cnn_destroy", "vdamp_cnn_param_count", "vdamp_cnn_set_params",
            "vdamp_cnn_get_params", "vdamp_cnn_workspace", "vdamp_cnn_forward", "vdamp_cnn_train_step",
            "vdamp_solve_learned", "vdamp_learned_export", "vdamp_wavelet", "vdamp_plan_describe",
            "vdamp_plan_ortho", "vdamp_wavelet_ws", "vdamp_plan_3d")


class VdampError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {detail}")


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the in-tree libvdamp.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch's HIP context first: torch brings its own HIP runtime, which fails to find the
    # device when the library's runtime initialised it before
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    lib.vdamp_plan.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                               i32, i32, u32, ctypes.POINTER(sz)]
    lib.vdamp_plan.restype = ctypes.c_int
    lib.vdamp_plan_ortho.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     i32, ctypes.POINTER(ctypes.c_double), i32, u32, ctypes.POINTER(sz)]
    lib.vdamp_plan_ortho.restype = ctypes.c_int
    lib.vdamp_plan_3d.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), i32, u32, ctypes.POINTER(sz)]
    lib.vdamp_plan_3d.restype = ctypes.c_int
    lib.vdamp_plan_destroy.argtypes = [vp]
    lib.vdamp_plan_destroy.restype = ctypes.c_int
    lib.vdamp_solve.argtypes = [vp, vp, vp, sz, vp, vp, vp, vp, i32, vp, vp]
    lib.vdamp_solve.restype = ctypes.c_int
    lib.vdamp_solve_resume.argtypes = [vp, vp, vp, sz, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp]
    lib.vdamp_solve_resume.restype = ctypes.c_int
    lib.vdamp_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.vdamp_solve_noalloc.restype = ctypes.c_int
    lib.fista_solve.argtypes = [vp, vp, vp, sz, vp, vp, vp, i32, vp, vp]
    lib.fista_solve.restype = ctypes.c_int
    lib.vdamp_state_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.vdamp_state_export.restype = ctypes.c_int
    lib.vdamp_pass_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64), i32]
    lib.vdamp_pass_times.restype = ctypes.c_int
    lib.vdamp_plan_describe.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    lib.vdamp_plan_describe.restype = ctypes.c_int
    lib.vdamp_status_string.argtypes = [ctypes.c_int]
    lib.vdamp_status_string.restype = ctypes.c_char_p
    lib.vdamp_last_error.argtypes = []
    lib.vdamp_last_error.restype = ctypes.c_char_p
    u64 = ctypes.c_uint64
    sigs = {
        "vdamp_cnn_create": [ctypes.POINTER(vp), i32],
        "vdamp_cnn_destroy": [vp],
        "vdamp_cnn_param_count": [vp, ctypes.POINTER(ctypes.c_int64)],
        "vdamp_cnn_set_params": [vp, vp, vp],
        "vdamp_cnn_get_params": [vp, vp, vp, vp],
        "vdamp_cnn_workspace": [vp, vp, i32, ctypes.POINTER(sz)],
        "vdamp_cnn_forward": [vp, vp, vp, vp, sz, vp, vp, vp, vp, vp, vp],
        "vdamp_cnn_train_step": [vp, vp, vp, vp, sz, vp, vp, vp, vp, ctypes.c_float, vp],
        "vdamp_solve_learned": [vp, vp, vp, vp, sz, vp, sz, vp, vp, vp, vp, i32, i32, i32, u64, vp, vp],
        "vdamp_learned_export": [vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "vdamp_wavelet": [vp, vp, i32, vp, vp],
        "vdamp_wavelet_ws": [vp, vp, vp, sz, i32, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != VDAMP_OK:
        raise VdampError(status, load_library().vdamp_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Plan:
    """A batch of slices (ragged sizes allowed) planned once; see ``vdamp_plan``.  With
    ``lowpass`` (an orthonormal lowpass filter) the plan uses that wavelet instead of
    Haar (``vdamp_plan_ortho``)."""

    def __init__(self, ny: Sequence[int], nx: Sequence[int], levels: int, flags: int = 0,
                 lowpass=None, nz: Optional[Sequence[int]] = None):
        lib = load_library()
        self.ny = [int(v) for v in ny]
        self.nx = [int(v) for v in nx]
        if len(self.ny) != len(self.nx):
            raise ValueError("ny and nx must have the same length")
        self.batch = len(self.ny)
        self.levels = int(levels)
        self.nz = None if nz is None else [int(v) for v in nz]
        self.nbands = 1 + (7 if self.nz is not None else 3) * self.levels
        self.flags = int(flags)
        depth = self.nz if self.nz is not None else [1] * self.batch
        self.offsets = np.concatenate([[0], np.cumsum([c * a * b for c, a, b in zip(depth, self.ny, self.nx)])])
        self.ntot = int(self.offsets[-1])
        a_ny = (ctypes.c_int32 * self.batch)(*self.ny)
        a_nx = (ctypes.c_int32 * self.batch)(*self.nx)
        h = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        if self.nz is not None:
            if lowpass is not None:
                raise ValueError("volumes use the 3D Haar transform")
            a_nz = (ctypes.c_int32 * self.batch)(*self.nz)
            _check(lib.vdamp_plan_3d(ctypes.byref(h), self.batch, a_nz, a_ny, a_nx, self.levels,
                                     self.flags, ctypes.byref(wsb)))
        elif lowpass is None:
            _check(lib.vdamp_plan(ctypes.byref(h), self.batch, a_ny, a_nx, self.levels,
                                  VDAMP_WAVELET_HAAR, self.flags, ctypes.byref(wsb)))
        else:
            taps = [float(v) for v in lowpass]
            a_h = (ctypes.c_double * max(len(taps), 1))(*taps)
            _check(lib.vdamp_plan_ortho(ctypes.byref(h), self.batch, a_ny, a_nx, self.levels,
                                        a_h, len(taps), self.flags, ctypes.byref(wsb)))
        self._h = h
        self.workspace_bytes = int(wsb.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().vdamp_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def vdamp_solve(self, ws, y, mask, p, sigma2, iters, x_hat, trace=None, stream=None):
        _check(load_library().vdamp_solve(self._h, _stream_handle(stream), _ptr(ws), ws.numel(),
                                          _ptr(y), _ptr(mask), _ptr(p), _ptr(sigma2), int(iters),
                                          _ptr(x_hat), _ptr(trace)))

    def vdamp_solve_resume(self, ws, y, mask, p, sigma2, r_init, theta_init, theta2_init, alpha_init,
                           iters, x_hat, trace=None, x_monitor=None, stream=None):
        _check(load_library().vdamp_solve_resume(
            self._h, _stream_handle(stream), _ptr(ws), ws.numel(), _ptr(y), _ptr(mask), _ptr(p),
            _ptr(sigma2), _ptr(r_init), _ptr(theta_init), _ptr(theta2_init), _ptr(alpha_init),
            int(iters), _ptr(x_hat), _ptr(trace), _ptr(x_monitor)))

    def vdamp_solve_noalloc(self, y, mask, p, sigma2, iters, x_hat, trace=None, stream=None):
        _check(load_library().vdamp_solve_noalloc(self._h, _stream_handle(stream), _ptr(y), _ptr(mask),
                                                  _ptr(p), _ptr(sigma2), int(iters), _ptr(x_hat),
                                                  _ptr(trace)))

    def fista_solve(self, ws, y, mask, lam, iters, x_hat, objective=None, stream=None):
        _check(load_library().fista_solve(self._h, _stream_handle(stream), _ptr(ws), ws.numel(),
                                          _ptr(y), _ptr(mask), _ptr(lam), int(iters), _ptr(x_hat),
                                          _ptr(objective)))

    def vdamp_state_export(self, ws, r=None, theta=None, alpha=None, tau=None, theta2=None,
                           stream=None):
        _check(load_library().vdamp_state_export(self._h, _stream_handle(stream), _ptr(ws),
                                                 _ptr(r), _ptr(theta), _ptr(theta2), _ptr(alpha),
                                                 _ptr(tau)))

    def vdamp_pass_times(self):
        n = len(PASS_NAMES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(load_library().vdamp_pass_times(self._h, ms, cnt, n))
        return {PASS_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}

    def describe(self) -> str:
        """The plan's launch configuration (and the tuner's measurements) as text."""
        lib = load_library()
        need = ctypes.c_size_t(0)
        _check(lib.vdamp_plan_describe(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.vdamp_plan_describe(self._h, buf, need.value, None))
        return buf.value.decode()

    def vdamp_wavelet(self, x, out, inverse, stream=None):
        _check(load_library().vdamp_wavelet(self._h, _stream_handle(stream), int(bool(inverse)),
                                            _ptr(x), _ptr(out)))

    def vdamp_wavelet_ws(self, ws, x, out, inverse, stream=None):
        _check(load_library().vdamp_wavelet_ws(self._h, _stream_handle(stream), _ptr(ws), ws.numel(),
                                               int(bool(inverse)), _ptr(x), _ptr(out)))

    def vdamp_solve_learned(self, cnn, ws, cnn_ws, y, mask, p, sigma2, iters, seed, x_hat,
                            trace=None, judge=0, learned_from=0, stream=None):
        _check(load_library().vdamp_solve_learned(
            self._h, cnn._h, _stream_handle(stream), _ptr(ws), ws.numel(), _ptr(cnn_ws),
            cnn_ws.numel(), _ptr(y), _ptr(mask), _ptr(p), _ptr(sigma2), int(iters),
            int(learned_from), int(judge), ctypes.c_uint64(int(seed)), _ptr(x_hat), _ptr(trace)))

    # ---- marshalling helpers (host numpy <-> packed device tensors)
    def pack(self, arrays, dtype):
        """Concatenate per-slice 2D numpy arrays in plan order into one flat array."""
        out = np.concatenate([np.asarray(a).reshape(-1) for a in arrays]).astype(dtype)
        if out.size != self.ntot:
            raise ValueError("arrays do not match the plan's slice sizes")
        return out

    def unpack(self, flat):
        """Split a flat per-pixel array into per-slice 2D (or per-volume 3D) arrays."""
        flat = np.asarray(flat)
        shape = (lambda b: (self.ny[b], self.nx[b])) if self.nz is None else \
            (lambda b: (self.nz[b], self.ny[b], self.nx[b]))
        return [flat[self.offsets[b]:self.offsets[b + 1]].reshape(shape(b)) for b in range(self.batch)]


def to_device(plan: Plan, slices, device="cuda"):
    """Pack a list of synth.Slice objects into the device tensors vdamp_solve reads."""
    import torch
    y = torch.from_numpy(plan.pack([s.y for s in slices], np.complex64)).to(device)
    mask = torch.from_numpy(plan.pack([s.mask for s in slices], np.uint8)).to(device)
    p = torch.from_numpy(plan.pack([s.p for s in slices], np.float32)).to(device)
    sigma2 = torch.tensor([s.sigma2 for s in slices], dtype=torch.float32, device=device)
    return y, mask, p, sigma2


class Cnn:
    """The learned denoiser (``vdamp_cnn_*``): FP32 master parameters, BF16 kernels."""

    def __init__(self, nbands: int):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.vdamp_cnn_create(ctypes.byref(h), int(nbands)))
        self._h = h
        self.nbands = int(nbands)
        n = ctypes.c_int64()
        _check(lib.vdamp_cnn_param_count(self._h, ctypes.byref(n)))
        self.param_count = int(n.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().vdamp_cnn_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat, stream=None):
        _check(load_library().vdamp_cnn_set_params(self._h, _stream_handle(stream), _ptr(flat)))

    def get_params(self, params=None, grad=None, stream=None):
        _check(load_library().vdamp_cnn_get_params(self._h, _stream_handle(stream), _ptr(params),
                                                   _ptr(grad)))

    def workspace(self, plan: Plan, kind: int, device="cuda"):
        import torch
        b = ctypes.c_size_t()
        _check(load_library().vdamp_cnn_workspace(self._h, plan._h, int(kind), ctypes.byref(b)))
        return torch.empty(int(b.value), dtype=torch.uint8, device=device)

    def forward(self, plan: Plan, ws, x, tau, s0, x_out, tangent=None, jvp_out=None, stream=None):
        _check(load_library().vdamp_cnn_forward(self._h, plan._h, _stream_handle(stream), _ptr(ws),
                                                ws.numel(), _ptr(x), _ptr(tau), _ptr(s0), _ptr(x_out),
                                                _ptr(tangent), _ptr(jvp_out)))

    def train_step(self, plan: Plan, ws, x, tau, s0, x0, lr, loss, stream=None):
        _check(load_library().vdamp_cnn_train_step(self._h, plan._h, _stream_handle(stream), _ptr(ws),
                                                   ws.numel(), _ptr(x), _ptr(tau), _ptr(s0), _ptr(x0),
                                                   ctypes.c_float(float(lr)), _ptr(loss)))

    def learned_export(self, plan: Plan, cnn_ws, sel=None, s0=None, sure_cnn=None, alpha_cnn=None,
                       sure_soft=None, stream=None):
        _check(load_library().vdamp_learned_export(self._h, plan._h, _stream_handle(stream), _ptr(cnn_ws),
                                                   _ptr(sel), _ptr(s0), _ptr(sure_cnn), _ptr(alpha_cnn),
                                                   _ptr(sure_soft)))


def cnn_flatten(params) -> np.ndarray:
    """Flatten a dict of denoiser parameters (W1..W6, b1..b6, Wt) in the library's order."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k in CNN_PARAM_ORDER])


def cnn_unflatten(flat, nbands: int, channels: int = 48):
    """Inverse of cnn_flatten."""
    flat = np.asarray(flat)
    shapes = {"W1": (channels, 2, 3, 3), "b1": (channels,), "Wt": (channels, nbands)}
    for l in range(2, 6):
        shapes[f"W{l}"] = (channels, channels, 3, 3)
        shapes[f"b{l}"] = (channels,)
    shapes["W6"] = (2, channels, 3, 3)
    shapes["b6"] = (2,)
    out, o = {}, 0
    for k in CNN_PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = flat[o:o + n].reshape(shapes[k])
        o += n
    if o != flat.size:
        raise ValueError("flat parameter vector has the wrong length")
    return out
