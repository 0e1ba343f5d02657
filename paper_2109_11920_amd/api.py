"""Python binding of libboac on torch device tensors: argument marshalling only. Every step of the
candidate evaluation runs in the library's HIP kernels; torch provides device memory and streams."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

import numpy as np

from . import _lib
from ._lib import BoacError, BoacGeom, BoacGpInfo, BoacSlice, check

DEFAULT_TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

STATUS_ZERO_PROJECTION = 1
STATUS_NONFINITE = 2
STATUS_NEGATIVE_RADIUS = 4
STATUS_NEGATIVE_COUNTS = 8

GRAD_MODES = {"unrolled": 0, "envelope": 1}


@dataclass(frozen=True)
class Geometry:
    """n x n image with pixel (cm); n_angles over 360 deg; n_bins bins; n_samples samples per ray."""
    n: int
    n_angles: int
    n_bins: int
    n_samples: int
    pixel: float

    def c(self) -> BoacGeom:
        return BoacGeom(self.n, self.n_angles, self.n_bins, self.n_samples, float(self.pixel))

    @property
    def image_shape(self):
        return (self.n, self.n)

    @property
    def sino_shape(self):
        return (self.n_angles, self.n_bins)


def _ptr(t: Optional[torch.Tensor], name: str, dtype=torch.float32, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A libboac context on one GPU (scratch, launch plans, graphs, instrumentation)."""

    def __init__(self, device: int = 0, tune_cache: Optional[str] = None):
        """tune_cache: plan cache written by the autotuner; default: the package's tune_cache.json
        when present (or $BOAC_TUNE_CACHE, read by the library)."""
        self.lib = _lib.load()
        if tune_cache is None and os.path.exists(DEFAULT_TUNE_CACHE) and not os.environ.get("BOAC_TUNE_CACHE"):
            tune_cache = DEFAULT_TUNE_CACHE
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        check(self.lib.boac_ctx_create(device, tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.boac_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- entry points -------------------------------------------------------------------------
    def rasterize_mu(self, geom: Geometry, cand: torch.Tensor, delta_r: float, out=None) -> torch.Tensor:
        C = cand.shape[0]
        out = out if out is not None else torch.empty((C, geom.n, geom.n), device=self.device)
        check(self.lib.boac_rasterize_mu(self.handle, ctypes.byref(geom.c()), _ptr(cand, "cand", shape=(C, 8)),
                                         C, float(delta_r), _ptr(out, "mu", shape=(C, geom.n, geom.n)),
                                         _stream(self.device)))
        return out

    def project(self, geom: Geometry, mu: torch.Tensor, img: torch.Tensor, out=None) -> torch.Tensor:
        C = mu.shape[0]
        out = out if out is not None else torch.empty((C,) + geom.sino_shape, device=self.device)
        check(self.lib.boac_project(self.handle, ctypes.byref(geom.c()), _ptr(mu, "mu", shape=(C,) + geom.image_shape),
                                    _ptr(img, "img", shape=(C,) + geom.image_shape), C,
                                    _ptr(out, "sino", shape=(C,) + geom.sino_shape), _stream(self.device)))
        return out

    def backproject(self, geom: Geometry, mu: torch.Tensor, sino: torch.Tensor, out=None) -> torch.Tensor:
        C = mu.shape[0]
        out = out if out is not None else torch.empty((C,) + geom.image_shape, device=self.device)
        check(self.lib.boac_backproject(self.handle, ctypes.byref(geom.c()),
                                        _ptr(mu, "mu", shape=(C,) + geom.image_shape),
                                        _ptr(sino, "sino", shape=(C,) + geom.sino_shape), C,
                                        _ptr(out, "img", shape=(C,) + geom.image_shape), _stream(self.device)))
        return out

    def mlem(self, geom: Geometry, mu: torch.Tensor, meas: torch.Tensor, n_iter: int,
             img: Optional[torch.Tensor] = None) -> torch.Tensor:
        C = mu.shape[0]
        img = img if img is not None else torch.ones((C,) + geom.image_shape, device=self.device)
        check(self.lib.boac_mlem(self.handle, ctypes.byref(geom.c()), _ptr(mu, "mu", shape=(C,) + geom.image_shape),
                                 _ptr(meas, "meas", shape=geom.sino_shape), C, int(n_iter),
                                 _ptr(img, "img", shape=(C,) + geom.image_shape), _stream(self.device)))
        return img

    def objective(self, geom: Geometry, meas: torch.Tensor, cand: torch.Tensor, delta_r: float, n_iter: int,
                  want_image: bool = False, obj=None, status=None):
        """Returns (J [C], F^K [C,n,n] or None, status [C] int32)."""
        C = cand.shape[0]
        obj = obj if obj is not None else torch.empty(C, device=self.device)
        status = status if status is not None else torch.empty(C, device=self.device, dtype=torch.int32)
        img = torch.empty((C,) + geom.image_shape, device=self.device) if want_image else None
        check(self.lib.boac_objective(self.handle, ctypes.byref(geom.c()), _ptr(meas, "meas", shape=geom.sino_shape),
                                      _ptr(cand, "cand", shape=(C, 8)), C, float(delta_r), int(n_iter),
                                      _ptr(obj, "obj", shape=(C,)), _ptr(img, "img"),
                                      _ptr(status, "status", dtype=torch.int32, shape=(C,)), _stream(self.device)))
        return obj, img, status

    def objective_noalloc(self, geom: Geometry, meas: torch.Tensor, cand: torch.Tensor, delta_r: float,
                          n_iter: int, obj: torch.Tensor, status: torch.Tensor, img: Optional[torch.Tensor] = None):
        """boac_objective_noalloc: as objective(), with the library's fixed per-device scratch and no device
        allocation by the library; the caller provides every output. Returns (obj, img, status)."""
        C = cand.shape[0]
        check(self.lib.boac_objective_noalloc(self.handle, ctypes.byref(geom.c()),
                                              _ptr(meas, "meas", shape=geom.sino_shape),
                                              _ptr(cand, "cand", shape=(C, 8)), C, float(delta_r), int(n_iter),
                                              _ptr(obj, "obj", shape=(C,)),
                                              _ptr(img, "img", shape=(C,) + geom.image_shape),
                                              _ptr(status, "status", dtype=torch.int32, shape=(C,)),
                                              _stream(self.device)))
        return obj, img, status

    def objective_grad(self, geom: Geometry, meas: torch.Tensor, cand: torch.Tensor, delta_r: float, n_iter: int,
                       ckpt_every: int = 5, obj=None, grad=None, status=None):
        """Returns (J [C], dJ/dtheta [C, 8], status [C] int32)."""
        C = cand.shape[0]
        obj = obj if obj is not None else torch.empty(C, device=self.device)
        grad = grad if grad is not None else torch.empty((C, 8), device=self.device)
        status = status if status is not None else torch.empty(C, device=self.device, dtype=torch.int32)
        check(self.lib.boac_objective_grad(self.handle, ctypes.byref(geom.c()),
                                           _ptr(meas, "meas", shape=geom.sino_shape),
                                           _ptr(cand, "cand", shape=(C, 8)), C, float(delta_r), int(n_iter),
                                           int(ckpt_every), _ptr(obj, "obj", shape=(C,)),
                                           _ptr(grad, "grad", shape=(C, 8)),
                                           _ptr(status, "status", dtype=torch.int32, shape=(C,)),
                                           _stream(self.device)))
        return obj, grad, status

    def objective_grad_ex(self, geom: Geometry, meas: torch.Tensor, cand: torch.Tensor, delta_r: float,
                          n_iter: int, ckpt_every: int = 5, mode: str = "unrolled", obj=None, grad=None, status=None):
        """Returns (J [C], dJ/d(c_0..c_5, mu_b, mu_c, dR) [C, 9], status [C] int32). mode "unrolled": the
        exact gradient through the MLEM iterations; "envelope": the reconstruction F^K held fixed."""
        if mode not in GRAD_MODES:
            raise ValueError(f"mode must be one of {sorted(GRAD_MODES)}")
        C = cand.shape[0]
        obj = obj if obj is not None else torch.empty(C, device=self.device)
        grad = grad if grad is not None else torch.empty((C, 9), device=self.device)
        status = status if status is not None else torch.empty(C, device=self.device, dtype=torch.int32)
        check(self.lib.boac_objective_grad_ex(self.handle, ctypes.byref(geom.c()),
                                              _ptr(meas, "meas", shape=geom.sino_shape),
                                              _ptr(cand, "cand", shape=(C, 8)), C, float(delta_r), int(n_iter),
                                              int(ckpt_every), GRAD_MODES[mode], _ptr(obj, "obj", shape=(C,)),
                                              _ptr(grad, "grad", shape=(C, 9)),
                                              _ptr(status, "status", dtype=torch.int32, shape=(C,)),
                                              _stream(self.device)))
        return obj, grad, status

    def gp_ei(self, model: "GpModel", q: torch.Tensor, best: float, xi: float, want_mu_sigma: bool = False):
        """Expected improvement (and optionally posterior mean and standard deviation) of the fitted
        surrogate at unit-box queries q [M, d] (float64 device tensor). Returns ei [M] or (ei, mu, sigma)."""
        M = q.shape[0]
        dm = model.on(self.device)
        ei = torch.empty(M, device=self.device, dtype=torch.float64)
        mu = torch.empty(M, device=self.device, dtype=torch.float64) if want_mu_sigma else None
        sd = torch.empty(M, device=self.device, dtype=torch.float64) if want_mu_sigma else None
        f64 = torch.float64
        check(self.lib.boac_gp_ei(self.handle, ctypes.byref(model.info),
                                  _ptr(dm["u"], "u", f64), _ptr(dm["linv"], "linv", f64),
                                  _ptr(dm["alpha"], "alpha", f64), _ptr(q, "q", f64, (M, model.info.d)), M,
                                  float(best), float(xi), _ptr(mu, "mu", f64), _ptr(sd, "sigma", f64),
                                  _ptr(ei, "ei", f64), _stream(self.device)))
        return (ei, mu, sd) if want_mu_sigma else ei

    def gp_chaos_local(self, model: "GpModel", best: float, xi: float, z: torch.Tensor, centres: torch.Tensor,
                       centre_ei: torch.Tensor, radius0: float, shrink: float, n_local: int):
        """The acquisition search's local stage on the device (boac_gp_chaos_local): z [P, d], centres [nc, d]
        and centre_ei [nc] (float64 device tensors) are updated in place; returns the rounds' points
        [n_local, per * nc, d] and EI values [n_local, per * nc], per = P // nc."""
        P, d = z.shape
        nc = centres.shape[0]
        m = (P // max(nc, 1)) * nc
        dm = model.on(self.device)
        f64 = torch.float64
        pts = torch.empty((n_local, m, d), device=self.device, dtype=f64)
        vals = torch.empty((n_local, m), device=self.device, dtype=f64)
        check(self.lib.boac_gp_chaos_local(self.handle, ctypes.byref(model.info),
                                           _ptr(dm["u"], "u", f64), _ptr(dm["linv"], "linv", f64),
                                           _ptr(dm["alpha"], "alpha", f64), float(best), float(xi),
                                           _ptr(z, "z", f64, (P, model.info.d)), P,
                                           _ptr(centres, "centres", f64, (nc, model.info.d)),
                                           _ptr(centre_ei, "centre_ei", f64, (nc,)), nc, float(radius0),
                                           float(shrink), int(n_local), _ptr(pts, "pts", f64),
                                           _ptr(vals, "vals", f64), _stream(self.device)))
        return pts, vals

    def gp_chaos_search(self, model: "GpModel", best: float, xi: float, z: torch.Tensor, taken: Optional[torch.Tensor],
                        q: int, *, n_global: int, n_local: int, centres: int, radius0: float, shrink: float,
                        exclusion: float, per_step: int):
        """The whole acquisition search on the device (boac_gp_chaos_search): chains z [P, d] (float64 device
        tensor, not modified), taken [T, d] or None. Returns (proposals [count, d] device tensor, largest EI
        evaluated, number of EI evaluations)."""
        P, d = z.shape
        f64 = torch.float64
        dm = model.on(self.device)
        props = torch.empty((q, d), device=self.device, dtype=f64)
        T = 0 if taken is None else taken.shape[0]
        count, vmax, nq = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int64()
        check(self.lib.boac_gp_chaos_search(self.handle, ctypes.byref(model.info), _ptr(dm["u"], "u", f64),
                                            _ptr(dm["linv"], "linv", f64), _ptr(dm["alpha"], "alpha", f64),
                                            float(best), float(xi), _ptr(z, "z", f64, (P, model.info.d)), P,
                                            int(n_global), int(n_local), int(centres), int(q), float(radius0),
                                            float(shrink), float(exclusion), int(per_step),
                                            _ptr(taken, "taken", f64, (T, model.info.d)) if T else None, T,
                                            _ptr(props, "props", f64), ctypes.byref(count), ctypes.byref(vmax),
                                            ctypes.byref(nq), _stream(self.device)))
        return props[: count.value], float(vmax.value), int(nq.value)

    def evaluate_batch(self, slices: Sequence["SliceBatch"], delta_r: float, n_iter: int, ckpt_every: int = 5):
        arr = (BoacSlice * len(slices))()
        for i, s in enumerate(slices):
            C = s.cand.shape[0]
            arr[i] = BoacSlice(s.geom.c(), _ptr(s.meas, "meas", shape=s.geom.sino_shape),
                               _ptr(s.cand, "cand", shape=(C, 8)), C, _ptr(s.obj, "obj", shape=(C,)),
                               _ptr(s.grad, "grad"), _ptr(s.status, "status", dtype=torch.int32))
        check(self.lib.boac_evaluate_batch(self.handle, arr, len(slices), float(delta_r), int(n_iter),
                                           int(ckpt_every), _stream(self.device)))

    def set_batch_mode(self, mode: str, spin_limit: int = 0):
        """evaluate_batch execution: "lanes" (stream lanes captured in a graph) or "persistent" (one
        persistent launch with a device work queue; spin_limit bounds each dependency wait)."""
        modes = {"lanes": 0, "persistent": 1}
        if mode not in modes:
            raise ValueError(f"mode must be one of {sorted(modes)}")
        check(self.lib.boac_ctx_set_batch_mode(self.handle, modes[mode], int(spin_limit)))

    # ---- instrumentation ------------------------------------------------------------------------
    def set_profiling(self, on: bool):
        check(self.lib.boac_ctx_set_profiling(self.handle, 1 if on else 0))

    def kernel_stats(self, kind: str):
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        check(self.lib.boac_ctx_kernel_stats(self.handle, _lib.KERNEL_KINDS[kind], ctypes.byref(cnt),
                                             ctypes.byref(ms), ctypes.byref(by)))
        return int(cnt.value), float(ms.value), float(by.value)

    def reset_stats(self):
        check(self.lib.boac_ctx_reset_stats(self.handle))

    def graph_stats(self):
        """(graphs held, captures, replays, scratch generation) of the batch graph cache."""
        v = [ctypes.c_int64() for _ in range(4)]
        check(self.lib.boac_ctx_graph_stats(self.handle, *[ctypes.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)


@dataclass
class SliceBatch:
    """One slice of an uneven batch with its output tensors (grad None = objective only)."""
    geom: Geometry
    meas: torch.Tensor
    cand: torch.Tensor
    obj: torch.Tensor
    grad: Optional[torch.Tensor] = None
    status: Optional[torch.Tensor] = None

    @staticmethod
    def make(geom: Geometry, meas: torch.Tensor, cand: torch.Tensor, with_grad: bool) -> "SliceBatch":
        C = cand.shape[0]
        dev = cand.device
        return SliceBatch(geom, meas, cand, torch.empty(C, device=dev),
                          torch.empty((C, 8), device=dev) if with_grad else None,
                          torch.empty(C, device=dev, dtype=torch.int32))


class GpModel:
    """A fitted surrogate (boac_gp_fit): selection info, L^-1 and K^-1 z as host arrays, and the inputs;
    device copies are made once per device on first use."""

    def __init__(self, info: BoacGpInfo, u: np.ndarray, linv: np.ndarray, alpha: np.ndarray):
        self.info, self.u, self.linv, self.alpha = info, u, linv, alpha
        self._dev = {}

    def on(self, device: torch.device):
        key = str(device)
        if key not in self._dev:
            self._dev[key] = {k: torch.as_tensor(v, device=device).contiguous()
                              for k, v in (("u", self.u), ("linv", self.linv), ("alpha", self.alpha))}
        return self._dev[key]


def gp_fit(u: np.ndarray, y: np.ndarray, lengths: Sequence[float], n_select: int = 0,
           noise: float = 1e-6) -> GpModel:
    """Fit the surrogate on the host (native FP64, boac_gp_fit). u [n, d] unit-box inputs, y [n]."""
    lib = _lib.load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    lengths = np.ascontiguousarray(lengths, dtype=np.float64)
    n, d = u.shape
    if y.shape != (n,):
        raise ValueError(f"y has shape {y.shape}, expected ({n},)")
    linv = np.empty((n, n), dtype=np.float64)
    alpha = np.empty(n, dtype=np.float64)
    info = BoacGpInfo()
    p = lambda a: ctypes.c_void_p(a.ctypes.data)
    check(lib.boac_gp_fit(p(u), p(y), n, d, p(lengths), len(lengths), int(n_select), float(noise), p(linv),
                          p(alpha), ctypes.byref(info)))
    return GpModel(info, u, linv, alpha)


class BoacObjective(torch.autograd.Function):
    """J(theta) for a batch of candidates theta [C, 8] with an exact hand-written adjoint.

    forward(ctx_obj, geom, meas, delta_r, n_iter, ckpt_every, theta) -> J [C]; when theta requires a
    gradient it is computed together with J by the library's reverse sweep and applied in backward,
    otherwise only the objective is evaluated."""

    @staticmethod
    def forward(fctx, boac: Context, geom: Geometry, meas: torch.Tensor, delta_r: float, n_iter: int,
                ckpt_every: int, theta: torch.Tensor):
        th = theta.detach().to(torch.float32).contiguous()
        if fctx.needs_input_grad[6]:
            J, grad, status = boac.objective_grad(geom, meas, th, delta_r, n_iter, ckpt_every)
            fctx.save_for_backward(grad)
        else:
            J, _, status = boac.objective(geom, meas, th, delta_r, n_iter)
            fctx.save_for_backward(None)
        fctx.status = status
        return J.to(theta.dtype)

    @staticmethod
    def backward(fctx, gJ):
        (grad,) = fctx.saved_tensors
        return None, None, None, None, None, None, (gJ[:, None] * grad).to(gJ.dtype)


def objective(boac: Context, geom: Geometry, meas: torch.Tensor, theta: torch.Tensor, delta_r: float,
              n_iter: int, ckpt_every: int = 5) -> torch.Tensor:
    """Differentiable J(theta) (see BoacObjective)."""
    return BoacObjective.apply(boac, geom, meas, float(delta_r), int(n_iter), int(ckpt_every), theta)


__all__ = ["Context", "Geometry", "SliceBatch", "BoacObjective", "BoacError", "GpModel", "gp_fit", "objective"]
