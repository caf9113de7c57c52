"""Python binding of the gfx950 Radon NUFFT library (``libradon.so``).

Argument marshalling only: every step of the transform runs in the HIP
kernels behind the C ABI declared in ``include/radon.h``. PyTorch supplies
device memory and the current stream. If the library is not built the import
of the binding still works, but every call raises ``RuntimeError``; there is
no CPU fallback.

    plan = Plan(n, angles, n_det, sigma=2.0, W=6)
    sino = plan.forward(img)        # img: (n, n) float32 CUDA tensor
    back = plan.adjoint(sino)       # exact transpose of forward
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libradon.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "radon.h")

RADON_OK, RADON_ERR_INVALID, RADON_ERR_UNSUPPORTED, RADON_ERR_OOM, RADON_ERR_DEVICE = range(5)

_lib = None

_c_int, _c_i64, _c_dbl, _vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
_SIGS = {
    "radon_plan": (_c_int, [ctypes.POINTER(_vp), _c_int, ctypes.POINTER(_c_dbl), _c_int, _c_int, _c_dbl, _c_int]),
    "radon_forward": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_adjoint": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_fbp": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_forward_batched": (_c_int, [_vp, _c_int, _vp, _vp, _vp]),
    "radon_adjoint_batched": (_c_int, [_vp, _c_int, _vp, _vp, _vp]),
    "radon_plan_sort_indices": (_c_int, [_vp, _vp, _c_i64, _vp, _c_i64]),
    "radon_plan_info": (_c_int, [_vp, ctypes.POINTER(_c_i64), _c_int]),
    "radon_plan_device_bytes": (ctypes.c_size_t, [_vp]),
    "radon_plan_destroy": (None, [_vp]),
    "radon_supported_length": (_c_int, [_c_int]),
    "radon_status_string": (ctypes.c_char_p, [_c_int]),
    "radon_last_error": (ctypes.c_char_p, []),
    "radon_plan_set_profiling": (_c_int, [_vp, _c_int]),
    "radon_plan_stage_times": (_c_int, [_vp, ctypes.POINTER(_c_dbl), ctypes.POINTER(_c_i64), _c_int]),
    "radon_stage_count": (_c_int, []),
    "radon_stage_name": (ctypes.c_char_p, [_c_int]),
    "radon_debug_forward_grid": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_debug_adjoint_grid": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_fft_test": (_c_int, [_c_int, _c_int, _c_int, _vp, _vp, _vp]),
    "radon_ring_filter": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_ring_filter_noalloc": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_solve_bpdn": (_c_int, [_vp, _vp, _vp, ctypes.c_void_p, ctypes.c_void_p, _vp]),
    "radon_project_l1": (_c_int, [_vp, _c_i64, _c_dbl, _vp, ctypes.POINTER(_c_dbl), _vp]),
    "radon_plan_tuned": (_c_int, [ctypes.POINTER(_vp), _c_int, ctypes.POINTER(_c_dbl), _c_int, _c_int, _c_dbl,
                                  _c_int, ctypes.c_void_p]),
    "radon_plan_tuning": (_c_int, [_vp, ctypes.c_void_p]),
    "radon_autotune": (_c_int, [_c_int, ctypes.POINTER(_c_dbl), _c_int, _c_int, _c_dbl, _c_int, _c_int,
                                ctypes.c_void_p, ctypes.POINTER(_c_dbl), ctypes.POINTER(_c_dbl), _vp]),
    "radon_batch_create": (_c_int, [ctypes.POINTER(_vp), _c_int, ctypes.POINTER(_vp), _c_int]),
    "radon_batch_forward": (_c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "radon_batch_adjoint": (_c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "radon_batch_graphs_recorded": (_c_int, [_vp]),
    "radon_batch_destroy": (None, [_vp]),
    "radon_cnn_create": (_c_int, [ctypes.POINTER(_vp), _c_int, _c_int, _c_int, ctypes.c_uint64]),
    "radon_cnn_destroy": (None, [_vp]),
    "radon_cnn_forward": (_c_int, [_vp, _vp, _vp, _vp]),
    "radon_cnn_train_step": (_c_int, [_vp, _vp, _vp, ctypes.c_float, ctypes.POINTER(ctypes.c_float), _vp, _vp]),
    "radon_cnn_param_count": (_c_i64, [_vp]),
    "radon_cnn_get_params": (_c_int, [_vp, _vp, _c_i64]),
    "radon_cnn_set_params": (_c_int, [_vp, _vp, _c_i64]),
    "radon_cnn_get_grads": (_c_int, [_vp, _vp, _c_i64]),
    "radon_cnn_conv_test": (_c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _c_int, _vp, _vp, _vp, _vp, _c_int, _c_int,
                                     _c_int, _c_int, _c_int, _vp]),
}


class Tuning(ctypes.Structure):
    """Work decomposition of a plan: bin tile side, most visits per spreading
    item, most samples per forward-interpolation item (0 = default)."""
    _fields_ = [("tile", ctypes.c_int), ("a2_chunk", ctypes.c_int), ("f3_chunk", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveOpts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("opt_tol", ctypes.c_double), ("bp_tol", ctypes.c_double),
                ("dec_tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("ring_filter", ctypes.c_int),
                ("warm_start", ctypes.c_int), ("fallback_iters", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("rnorm", ctypes.c_double), ("tau", ctypes.c_double), ("x_l1", ctypes.c_double),
                ("seconds", ctypes.c_double), ("iterations", ctypes.c_int), ("n_forward", ctypes.c_int),
                ("n_adjoint", ctypes.c_int), ("status", ctypes.c_int), ("fallback", ctypes.c_int),
                ("warm_iterations", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RadonError(RuntimeError):
    """A failing library call; ``status`` is the radon_status_t value."""

    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


def lib():
    """Load libradon.so (once). Raises RuntimeError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1009_1380_amd.build.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def declared_functions(header: str = HEADER_PATH):
    """Names of the functions that include/radon.h declares."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(radon_[a-z0-9_]+)\s*\(", text)))


def _check(status: int, what: str):
    if status != RADON_OK:
        name = lib().radon_status_string(status).decode()
        detail = lib().radon_last_error().decode()
        msg = f"{what}: {name}: {detail}"
        if status in (RADON_ERR_INVALID, RADON_ERR_UNSUPPORTED):
            err = ValueError(msg)
            err.status = status
            raise err
        raise RadonError(status, msg)


def supported_length(length: int) -> bool:
    return bool(lib().radon_supported_length(int(length)))


def stage_names():
    L = lib()
    return [L.radon_stage_name(i).decode() for i in range(L.radon_stage_count())]


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_ptr(t, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor, got {t.device}")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Plan of the forward / adjoint Radon NUFFT for one geometry.

    n: image side; angles: view angles in radians (float64, copied); n_det:
    detector bins; sigma: oversampling (2); W: Kaiser-Bessel width (4, 6, 8).
    The plan lives on the current CUDA device.
    """

    INFO_KEYS = ("n", "n_views", "n_det", "W", "G", "T", "n_samples", "n_bins",
                 "n_items", "n_slots", "device_bytes", "n_fitems")

    def __init__(self, n: int, angles, n_det: int, sigma: float = 2.0, W: int = 6, tuning=None):
        ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).ravel())
        self.n, self.n_det, self.n_views = int(n), int(n_det), int(ang.size)
        self.sigma, self.W = float(sigma), int(W)
        self.angles = ang.copy()
        h = ctypes.c_void_p()
        angp = ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if tuning is None:
            st = lib().radon_plan(ctypes.byref(h), self.n, angp, self.n_views, self.n_det, self.sigma, self.W)
        else:
            t = Tuning(int(tuning.get("tile", 0)), int(tuning.get("a2_chunk", 0)), int(tuning.get("f3_chunk", 0)))
            st = lib().radon_plan_tuned(ctypes.byref(h), self.n, angp, self.n_views, self.n_det, self.sigma,
                                        self.W, ctypes.byref(t))
        _check(st, "radon_plan")
        self._h = h

    def tuning(self) -> dict:
        """The work decomposition this plan uses (defaults resolved)."""
        t = Tuning()
        _check(lib().radon_plan_tuning(self._h, ctypes.byref(t)), "radon_plan_tuning")
        return t.as_dict()

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().radon_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- transforms
    def forward(self, img, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n_views, self.n_det), dtype=torch.float32, device=img.device)
        _check(lib().radon_forward(self._h, _dev_ptr(img, (self.n, self.n), "img"),
                                   _dev_ptr(out, (self.n_views, self.n_det), "out"), _stream_ptr(stream)),
               "radon_forward")
        return out

    def adjoint(self, sino, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n, self.n), dtype=torch.float32, device=sino.device)
        _check(lib().radon_adjoint(self._h, _dev_ptr(sino, (self.n_views, self.n_det), "sino"),
                                   _dev_ptr(out, (self.n, self.n), "out"), _stream_ptr(stream)),
               "radon_adjoint")
        return out

    def fbp(self, sino, out=None, stream=None):
        """Filtered adjoint (ramp-weighted back-projection)."""
        torch = _torch()
        if out is None:
            out = torch.empty((self.n, self.n), dtype=torch.float32, device=sino.device)
        _check(lib().radon_fbp(self._h, _dev_ptr(sino, (self.n_views, self.n_det), "sino"),
                               _dev_ptr(out, (self.n, self.n), "out"), _stream_ptr(stream)),
               "radon_fbp")
        return out

    def forward_batched(self, imgs, out=None, stream=None):
        torch = _torch()
        b = int(imgs.shape[0])
        if out is None:
            out = torch.empty((b, self.n_views, self.n_det), dtype=torch.float32, device=imgs.device)
        _check(lib().radon_forward_batched(self._h, b, _dev_ptr(imgs, (b, self.n, self.n), "imgs"),
                                           _dev_ptr(out, (b, self.n_views, self.n_det), "out"),
                                           _stream_ptr(stream)), "radon_forward_batched")
        return out

    def adjoint_batched(self, sinos, out=None, stream=None):
        torch = _torch()
        b = int(sinos.shape[0])
        if out is None:
            out = torch.empty((b, self.n, self.n), dtype=torch.float32, device=sinos.device)
        _check(lib().radon_adjoint_batched(self._h, b, _dev_ptr(sinos, (b, self.n_views, self.n_det), "sinos"),
                                           _dev_ptr(out, (b, self.n, self.n), "out"), _stream_ptr(stream)),
               "radon_adjoint_batched")
        return out

    # -- reconstruction (the paper's basis-pursuit problem)
    def ring_filter(self, sino, out=None, stream=None):
        """Cubic-polynomial ring filter F of the sinogram (a symmetric projection)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(sino)
        _check(lib().radon_ring_filter(self._h, _dev_ptr(sino, (self.n_views, self.n_det), "sino"),
                                       _dev_ptr(out, (self.n_views, self.n_det), "out"), _stream_ptr(stream)),
               "radon_ring_filter")
        return out

    def ring_filter_noalloc(self, sino, out=None, stream=None):
        """The ring filter without any device allocation (scratch in a static
        device array shared by all calls on the GPU; stream-ordered)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(sino)
        _check(lib().radon_ring_filter_noalloc(self._h, _dev_ptr(sino, (self.n_views, self.n_det), "sino"),
                                               _dev_ptr(out, (self.n_views, self.n_det), "out"),
                                               _stream_ptr(stream)), "radon_ring_filter_noalloc")
        return out

    def solve_bpdn(self, sino, sigma: float, x0=None, opt_tol: float = 1e-4, bp_tol: float = 1e-6,
                   dec_tol: float = 1e-4, max_iter: int = 500, ring_filter: bool = True, stream=None,
                   fallback_iters: int = 100):
        """min ||x||_1 s.t. ||F(A x - sino)||_2 <= sigma (SPGL1). x0: optional
        warm-start image; the library falls back to a cold solve when the warm
        run misbehaves (stats["fallback"] says why, 0 if it did not).
        Returns (x, stats dict)."""
        torch = _torch()
        if x0 is None:
            x = torch.zeros((self.n, self.n), dtype=torch.float32, device=sino.device)
        else:
            x = x0.clone()
        opts = SolveOpts(float(sigma), float(opt_tol), float(bp_tol), float(dec_tol), int(max_iter),
                         int(bool(ring_filter)), int(x0 is not None), int(fallback_iters))
        stats = SolveStats()
        _check(lib().radon_solve_bpdn(self._h, _dev_ptr(sino, (self.n_views, self.n_det), "sino"),
                                      _dev_ptr(x, (self.n, self.n), "x"), ctypes.byref(opts), ctypes.byref(stats),
                                      _stream_ptr(stream)), "radon_solve_bpdn")
        return x, stats.as_dict()

    # -- introspection and test hooks
    def info(self) -> dict:
        arr = (ctypes.c_int64 * len(self.INFO_KEYS))()
        _check(lib().radon_plan_info(self._h, arr, len(self.INFO_KEYS)), "radon_plan_info")
        return dict(zip(self.INFO_KEYS, [int(v) for v in arr]))

    def sort_indices(self):
        inf = self.info()
        perm = np.empty(inf["n_samples"], dtype=np.int32)
        offs = np.empty(4 * inf["n_bins"] + 1, dtype=np.int32)
        _check(lib().radon_plan_sort_indices(self._h, perm.ctypes.data_as(ctypes.c_void_p), perm.size,
                                             offs.ctypes.data_as(ctypes.c_void_p), offs.size),
               "radon_plan_sort_indices")
        return perm, offs

    def set_profiling(self, enable: bool = True):
        _check(lib().radon_plan_set_profiling(self._h, int(bool(enable))), "radon_plan_set_profiling")

    def stage_times(self) -> dict:
        k = lib().radon_stage_count()
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int64 * k)()
        _check(lib().radon_plan_stage_times(self._h, ms, cnt, k), "radon_plan_stage_times")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(stage_names())}

    def debug_forward_grid(self, img, stream=None):
        torch = _torch()
        G = 2 * self.n
        out = torch.empty((self.n + 1, G, 2), dtype=torch.float32, device=img.device)
        _check(lib().radon_debug_forward_grid(self._h, _dev_ptr(img, (self.n, self.n), "img"),
                                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "radon_debug_forward_grid")
        return torch.view_as_complex(out)

    def debug_adjoint_grid(self, sino, stream=None):
        torch = _torch()
        G = 2 * self.n
        out = torch.empty((self.n + 1, G, 2), dtype=torch.float32, device=sino.device)
        _check(lib().radon_debug_adjoint_grid(self._h, _dev_ptr(sino, (self.n_views, self.n_det), "sino"),
                                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "radon_debug_adjoint_grid")
        return torch.view_as_complex(out)


def fft_test(x, inverse: bool = False, stream=None):
    """Batched LDS FFT of the rows of a complex64 CUDA tensor (batch, len)."""
    torch = _torch()
    if x.dtype != torch.complex64 or x.dim() != 2 or not x.is_contiguous() or x.device.type != "cuda":
        raise ValueError("x must be a contiguous (batch, len) complex64 device tensor")
    out = torch.empty_like(x)
    _check(lib().radon_fft_test(int(x.shape[1]), int(x.shape[0]), int(bool(inverse)),
                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                _stream_ptr(stream)), "radon_fft_test")
    return out


def project_l1(v, tau: float, stream=None):
    """Euclidean projection of a float32 device tensor (contiguous, numel a
    multiple of 4) onto {||x||_1 <= tau}; returns (projection, lam), the
    projection sign(v) max(|v| - lam, 0) in v's shape."""
    torch = _torch()
    flat = v.reshape(-1)
    _dev_ptr(flat, (flat.numel(),), "v")
    out = torch.empty_like(v)
    lam = ctypes.c_double(0.0)
    _check(lib().radon_project_l1(ctypes.c_void_p(flat.data_ptr()), int(flat.numel()), float(tau),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.byref(lam), _stream_ptr(stream)),
           "radon_project_l1")
    return out, lam.value


def autotune(n: int, angles, n_det: int, sigma: float = 2.0, W: int = 6, repeats: int = 5, stream=None):
    """Time candidate work decompositions of a geometry on the device and
    return (best tuning dict, best ms per forward+adjoint pair, default ms)."""
    ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).ravel())
    best, best_ms, def_ms = Tuning(), ctypes.c_double(), ctypes.c_double()
    _check(lib().radon_autotune(int(n), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(ang.size),
                                int(n_det), float(sigma), int(W), int(repeats), ctypes.byref(best),
                                ctypes.byref(best_ms), ctypes.byref(def_ms), _stream_ptr(stream)),
           "radon_autotune")
    return best.as_dict(), best_ms.value, def_ms.value


class Batch:
    """Uneven slices (distinct plans of any sizes) run together: each
    direction is recorded once per set of buffers into one HIP graph whose
    branches run slices side by side, then replayed with a single launch."""

    def __init__(self, plans, n_branches: int = 4):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().radon_batch_create(ctypes.byref(h), len(self.plans), arr, int(n_branches)),
               "radon_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().radon_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def graphs_recorded(self) -> int:
        return int(lib().radon_batch_graphs_recorded(self._h))

    def _ptrs(self, tensors, shapes, name):
        if len(tensors) != len(self.plans):
            raise ValueError(f"{name}: {len(tensors)} tensors for {len(self.plans)} slices")
        return (ctypes.c_void_p * len(tensors))(*[_dev_ptr(t, s, f"{name}[{i}]").value
                                                 for i, (t, s) in enumerate(zip(tensors, shapes))])

    def forward(self, imgs, outs, stream=None):
        ins = self._ptrs(imgs, [(p.n, p.n) for p in self.plans], "imgs")
        ous = self._ptrs(outs, [(p.n_views, p.n_det) for p in self.plans], "outs")
        _check(lib().radon_batch_forward(self._h, ins, ous, _stream_ptr(stream)), "radon_batch_forward")
        return outs

    def adjoint(self, sinos, outs, stream=None):
        ins = self._ptrs(sinos, [(p.n_views, p.n_det) for p in self.plans], "sinos")
        ous = self._ptrs(outs, [(p.n, p.n) for p in self.plans], "outs")
        _check(lib().radon_batch_adjoint(self._h, ins, ous, _stream_ptr(stream)), "radon_batch_adjoint")
        return outs


def _ptr_or_null(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _check_dev(t, dtype, name):
    torch = _torch()
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")


class WarmStartNet:
    """The learned warm start's encoder-decoder (radon_cnn_*): bf16 matrix-core
    convolutions, float32 parameters and Adam state, fixed batch and size."""

    def __init__(self, batch: int, height: int, width: int, seed: int = 0):
        self.batch, self.height, self.width = int(batch), int(height), int(width)
        h = ctypes.c_void_p()
        _check(lib().radon_cnn_create(ctypes.byref(h), self.batch, self.height, self.width, int(seed)),
               "radon_cnn_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().radon_cnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self):
        return (self.batch, self.height, self.width)

    def forward(self, x, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self._shape(), dtype=torch.float32, device=x.device)
        _check(lib().radon_cnn_forward(self._h, _dev_ptr(x, self._shape(), "x"), _dev_ptr(out, self._shape(), "out"),
                                       _stream_ptr(stream)), "radon_cnn_forward")
        return out

    def train_step(self, x, target, lr: float, pred=None, stream=None) -> float:
        torch = _torch()
        if pred is None:
            pred = torch.empty(self._shape(), dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        _check(lib().radon_cnn_train_step(self._h, _dev_ptr(x, self._shape(), "x"),
                                          _dev_ptr(target, self._shape(), "target"), float(lr), ctypes.byref(loss),
                                          _dev_ptr(pred, self._shape(), "pred"), _stream_ptr(stream)),
               "radon_cnn_train_step")
        return float(loss.value)

    def param_count(self) -> int:
        return int(lib().radon_cnn_param_count(self._h))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.param_count(), dtype=np.float32)
        _check(lib().radon_cnn_get_params(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size), "radon_cnn_get_params")
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.size != self.param_count():
            raise ValueError(f"need {self.param_count()} parameters, got {a.size}")
        _check(lib().radon_cnn_set_params(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size), "radon_cnn_set_params")

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.param_count(), dtype=np.float32)
        _check(lib().radon_cnn_get_grads(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size), "radon_cnn_get_grads")
        return a


def cnn_conv_test(x16, w, bias=None, res16=None, relu=False, gout16=None, want_out16=False, stream=None):
    """Test hook over radon_cnn_conv_test: bf16 tensors are torch.int16 views of
    bfloat16 bits (B, C, H, W); w float32 (Cout, Cin, 3, 3) on the device.
    Returns (out32, out16 or None, gin16 or None, gw, gb)."""
    torch = _torch()
    B, Cin, H, W = (int(v) for v in x16.shape)
    Cout = int(w.shape[0])
    _check_dev(x16, torch.int16, "x16")
    _check_dev(w, torch.float32, "w")
    _check_dev(bias, torch.float32, "bias")
    _check_dev(res16, torch.int16, "res16")
    _check_dev(gout16, torch.int16, "gout16")
    dev = x16.device
    out32 = torch.empty((B, Cout, H, W), dtype=torch.float32, device=dev)
    out16 = torch.empty((B, Cout, H, W), dtype=torch.int16, device=dev) if want_out16 else None
    gin = gw = gb = None
    if gout16 is not None:
        gin = torch.empty((B, Cin, H, W), dtype=torch.int16, device=dev)
        gw = torch.empty((Cout, Cin, 3, 3), dtype=torch.float32, device=dev)
        gb = torch.empty((Cout,), dtype=torch.float32, device=dev)
    _check(lib().radon_cnn_conv_test(_ptr_or_null(x16), _ptr_or_null(w), _ptr_or_null(bias), _ptr_or_null(res16),
                                     _ptr_or_null(out16), _ptr_or_null(out32), int(bool(relu)), _ptr_or_null(gout16),
                                     _ptr_or_null(gin), _ptr_or_null(gw), _ptr_or_null(gb), B, Cin, Cout, H, W,
                                     _stream_ptr(stream)), "radon_cnn_conv_test")
    return out32, out16, gin, gw, gb
