"""Torch-facing wrappers of the HIP library. PyTorch supplies device memory and
the stream; every step of the shooting and of its adjoint runs in the
library's kernels.

* :class:`Plan`        - a bound plan over a list of pairs (CUDA float32 tensors)
* :class:`ShootCost`   - ``torch.autograd.Function`` whose forward evaluates the
                         cost and dH/dp0 with the hand-written adjoint and whose
                         backward returns ``g * dH/dp0``
* :func:`shoot_cost`   - functional form of :class:`ShootCost`
* :func:`gradient_descent` - batched fixed-step descent on p0
"""
from __future__ import annotations

import ctypes
import os
from collections import OrderedDict
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (SHOOT_CHECK_FINITE, SHOOT_FORCE_GLOBAL_SCATTER, SHOOT_FULL_STORE, SHOOT_LANES,  # noqa: F401
                   SHOOT_NO_GRAPH, SHOOT_SCHEME_EULERIAN, SHOOT_SCHEME_MIXED, SHOOT_UNFUSED, ShootError)

__all__ = ["PairSpec", "Plan", "ShootCost", "shoot_cost", "gradient_descent",
           "SHOOT_FULL_STORE", "SHOOT_UNFUSED", "SHOOT_NO_GRAPH", "SHOOT_FORCE_GLOBAL_SCATTER", "SHOOT_LANES",
           "SHOOT_CHECK_FINITE"]


@dataclass
class PairSpec:
    """One pair: source ``image``, ``target`` (optional for forward only),
    initial momentum ``p0``, and the scalars rho, sigma, lam."""

    image: torch.Tensor
    p0: torch.Tensor
    rho: float
    sigma: float
    lam: float = 0.01
    target: Optional[torch.Tensor] = None


def _check_field(t: torch.Tensor, name: str, device: torch.device, shape=None) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device or t.device.type != "cuda":
        raise ValueError(f"{name} must live on {device} (a GPU device)")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """A plan for a batch of pairs sharing T, bound to a workspace.

    Output tensors are allocated here and stay fixed (captured graphs replay
    their addresses): ``out_image``, ``out_momentum``, ``out_grad`` (lists,
    one tensor per pair), ``out_cost`` (tensor [n_pairs, 3] =
    (H, data, reg)) and, when "deformation" is among the outputs,
    ``out_deformation`` (list of [ndim, *shape] tensors, psi_T of forward()). Input tensors must stay alive and in place; their
    contents may change between calls (e.g. p0 updated in place).
    """

    def __init__(self, pairs: Sequence[PairSpec], T: int, flags: int = 0, budget_bytes: int = 0,
                 stream: Optional[torch.cuda.Stream] = None, outputs: Sequence[str] = ("image", "momentum",
                                                                                       "grad", "cost"),
                 scratch: bool = False):
        self._lib = _lib.load()
        self._plan = None
        if len(pairs) == 0:
            raise ValueError("at least one pair is needed")
        device = pairs[0].image.device
        self.device = device
        self.T = int(T)
        self.flags = int(flags)
        self.pairs = list(pairs)
        n = len(self.pairs)
        outs = set(outputs)
        with torch.cuda.device(device):
            self.out_cost = torch.zeros((n, 3), dtype=torch.float32, device=device) if "cost" in outs else None
            self.out_image, self.out_momentum, self.out_grad, self.out_deformation = [], [], [], []
            arr = (_lib.ShootPair * n)()
            for i, ps in enumerate(self.pairs):
                shp = tuple(ps.image.shape)
                if len(shp) not in (2, 3):
                    raise ValueError(f"pair {i}: image must be 2-D or 3-D")
                _check_field(ps.image, f"pair {i} image", device)
                _check_field(ps.p0, f"pair {i} p0", device, shp)
                if ps.target is not None:
                    _check_field(ps.target, f"pair {i} target", device, shp)
                oi = torch.empty_like(ps.image) if "image" in outs else None
                om = torch.empty_like(ps.image) if "momentum" in outs else None
                og = torch.empty_like(ps.image) if "grad" in outs else None
                od = (torch.empty((len(shp),) + shp, dtype=torch.float32, device=device)
                      if "deformation" in outs else None)
                self.out_deformation.append(od)
                self.out_image.append(oi)
                self.out_momentum.append(om)
                self.out_grad.append(og)
                d = arr[i]
                d.ndim = len(shp)
                for a in range(3):
                    d.shape[a] = shp[a] if a < len(shp) else 0
                d.rho = float(ps.rho)
                d.sigma = float(ps.sigma)
                d.lambda_ = float(ps.lam)
                d.image = ps.image.data_ptr()
                d.target = ps.target.data_ptr() if ps.target is not None else None
                d.p0 = ps.p0.data_ptr()
                d.out_image = oi.data_ptr() if oi is not None else None
                d.out_momentum = om.data_ptr() if om is not None else None
                d.out_grad = og.data_ptr() if og is not None else None
                d.out_cost = (self.out_cost.data_ptr() + 12 * i) if self.out_cost is not None else None
                d.out_deformation = od.data_ptr() if od is not None else None
            self._desc = arr
            handle = ctypes.c_void_p()
            _lib.check(self._lib.shoot_plan_create(ctypes.cast(arr, ctypes.c_void_p), n, self.T, self.flags,
                                                   int(budget_bytes), ctypes.byref(handle)), "shoot_plan_create")
            self._plan = handle
            nbytes = ctypes.c_size_t()
            _lib.check(self._lib.shoot_plan_workspace_bytes(self._plan, ctypes.byref(nbytes)),
                       "shoot_plan_workspace_bytes")
            self.workspace_bytes = int(nbytes.value)
            if scratch:
                # the library's static scratch: no workspace is allocated here
                self._raw = self.workspace = None
                _lib.check(self._lib.shoot_plan_bind_scratch(self._plan, _stream_ptr(stream)),
                           "shoot_plan_bind_scratch")
            else:
                raw = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
                shift = (-raw.data_ptr()) % 256
                self._raw = raw
                self.workspace = raw[shift:shift + self.workspace_bytes]
                _lib.check(self._lib.shoot_plan_bind(self._plan, self.workspace.data_ptr(), self.workspace_bytes,
                                                     _stream_ptr(stream)), "shoot_plan_bind")

    @property
    def waves(self) -> int:
        w = ctypes.c_int32()
        _lib.check(self._lib.shoot_plan_waves(self._plan, ctypes.byref(w)), "shoot_plan_waves")
        return int(w.value)

    @property
    def lanes(self) -> int:
        """Largest number of concurrent lanes of an admission wave."""
        n = ctypes.c_int32()
        _lib.check(self._lib.shoot_plan_lanes(self._plan, ctypes.byref(n)), "shoot_plan_lanes")
        return int(n.value)

    def _call(self, fn, name, stream):
        if self._plan is None:
            raise RuntimeError("plan is closed")
        with torch.cuda.device(self.device):
            _lib.check(fn(self._plan, _stream_ptr(stream)), name)

    def forward(self, stream=None) -> None:
        """I_T, z_T (and the cost where a target is given)."""
        self._call(self._lib.shoot_forward, "shoot_forward", stream)

    def cost(self, stream=None) -> None:
        self._call(self._lib.shoot_cost, "shoot_cost", stream)

    def grad(self, stream=None) -> None:
        """Cost and dH/dp0 of every pair (hand-written discrete adjoint)."""
        self._call(self._lib.shoot_grad_p0, "shoot_grad_p0", stream)

    def cost_and_grad(self, stream=None):
        """grad(), then (costs [n_pairs] = H of every pair, list of dH/dp0 per
        pair): views of the plan's output tensors, valid until the next call."""
        if self.out_cost is None or self.out_grad is None:
            raise ValueError("cost_and_grad needs the 'cost' and 'grad' outputs")
        self.grad(stream)
        return self.out_cost[:, 0], list(self.out_grad)

    def descend(self, eta0: float = 1.0, reset: bool = False, stream=None) -> None:
        """One gradient-descent iteration on every pair's p0 (in place, on the
        device): cost and dH/dp0 at the current p0, then p0 -= eta_i dH/dp0,
        with eta_i halved when the pair's cost rose (reset: eta_i = eta0)."""
        if self._plan is None:
            raise RuntimeError("plan is closed")
        with torch.cuda.device(self.device):
            st = self._lib.shoot_descend(self._plan, float(eta0), 1 if reset else 0, _stream_ptr(stream))
        _lib.check(st, "shoot_descend")

    def autotune(self, stream=None) -> list:
        """Time both options of every launch-shape choice and keep the faster
        ones (bit-identical results); returns the chosen tuning."""
        self._call(self._lib.shoot_autotune, "shoot_autotune", stream)
        return self.tuning

    def autotune_cached(self, path, stream=None):
        """Autotune through the JSON cache at ``path`` (keyed by the device's
        gcnArchName and the plan's shape class); returns (tuning, hit)."""
        hit = ctypes.c_int32(0)
        _lib.check(self._lib.shoot_autotune_cached(self._plan, os.fsencode(path), ctypes.byref(hit),
                                                   _stream_ptr(stream)), "shoot_autotune_cached")
        return self.tuning, bool(hit.value)

    @property
    def tune_class(self) -> str:
        """The plan's shape class (the plan's part of a tuning-cache key)."""
        buf = ctypes.create_string_buffer(256)
        _lib.check(self._lib.shoot_plan_tune_class(self._plan, buf, len(buf)), "shoot_plan_tune_class")
        return buf.value.decode()

    @property
    def tuning(self) -> list:
        """The plan's launch-shape choices (SHOOT_TUNE_COUNT values, each 0 or 1)."""
        arr = (ctypes.c_int32 * _lib.SHOOT_TUNE_COUNT)()
        _lib.check(self._lib.shoot_plan_get_tuning(self._plan, arr), "shoot_plan_get_tuning")
        return [int(v) for v in arr]

    @tuning.setter
    def tuning(self, choices) -> None:
        vals = [int(v) for v in choices]
        if len(vals) != _lib.SHOOT_TUNE_COUNT:
            raise ValueError(f"expected {_lib.SHOOT_TUNE_COUNT} tuning choices, got {len(vals)}")
        arr = (ctypes.c_int32 * _lib.SHOOT_TUNE_COUNT)(*vals)
        _lib.check(self._lib.shoot_plan_set_tuning(self._plan, arr), "shoot_plan_set_tuning")

    def set_active(self, active=None, stream=None) -> None:
        """Evaluate only the pairs whose entry of ``active`` is true (None: all);
        the others keep the outputs of the last call that evaluated them."""
        if active is None:
            arr = None
        else:
            vals = [1 if v else 0 for v in active]
            if len(vals) != len(self.pairs):
                raise ValueError(f"expected {len(self.pairs)} flags, got {len(vals)}")
            arr = (ctypes.c_int32 * len(vals))(*vals)
        _lib.check(self._lib.shoot_plan_set_active(self._plan, arr, _stream_ptr(stream)), "shoot_plan_set_active")

    def displacements(self, stream=None) -> np.ndarray:
        """[n_pairs, T] largest |dt v| of every pair and step of the last
        execution call (synchronises the stream)."""
        n = len(self.pairs)
        out = np.zeros((n, self.T), dtype=np.float32)
        _lib.check(self._lib.shoot_plan_displacements(self._plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                      _stream_ptr(stream)), "shoot_plan_displacements")
        return out

    def set_profiling(self, enable: bool) -> None:
        """Eager launches with a HIP event pair around each kernel (diagnostics)."""
        _lib.check(self._lib.shoot_plan_set_profiling(self._plan, 1 if enable else 0), "shoot_plan_set_profiling")

    def reset_stats(self) -> None:
        _lib.check(self._lib.shoot_plan_reset_stats(self._plan), "shoot_plan_reset_stats")

    def kernel_stats(self) -> dict:
        """{kernel family: (launches, total milliseconds)} since the last reset."""
        out = {}
        i = 0
        while True:
            name = ctypes.c_char_p()
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            st = self._lib.shoot_plan_kernel_stats(self._plan, i, ctypes.byref(name), ctypes.byref(n),
                                                   ctypes.byref(ms))
            if st != _lib.SHOOT_OK:
                break
            out[name.value.decode()] = (int(n.value), float(ms.value))
            i += 1
        return out

    def close(self) -> None:
        if self._plan is not None:
            self._lib.shoot_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LBFGS:
    """Batched L-BFGS on the p0 of every pair of a plan (shoot_lbfgs_*): the
    plan needs "grad" and "cost" outputs and every pair a target; p0 tensors
    are overwritten with the iterates."""

    def __init__(self, plan: Plan, m: int = 5, c1: float = 1e-4, trials: int = 8, stream=None):
        self._lib = plan._lib
        self.plan = plan
        self._opt = None
        h = ctypes.c_void_p()
        _lib.check(self._lib.shoot_lbfgs_create(plan._plan, int(m), float(c1), int(trials), ctypes.byref(h)),
                   "shoot_lbfgs_create")
        self._opt = h
        nb = ctypes.c_size_t()
        _lib.check(self._lib.shoot_lbfgs_workspace_bytes(self._opt, ctypes.byref(nb)), "shoot_lbfgs_workspace_bytes")
        with torch.cuda.device(plan.device):
            raw = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=plan.device)
            shift = (-raw.data_ptr()) % 256
            self._raw = raw
            self.workspace = raw[shift:shift + int(nb.value)]
            _lib.check(self._lib.shoot_lbfgs_bind(self._opt, self.workspace.data_ptr(), int(nb.value),
                                                  _stream_ptr(stream)), "shoot_lbfgs_bind")

    def step(self, stream=None):
        """One iteration for every pair; returns (cost at the start of the
        step per pair, gradient evaluations used)."""
        with torch.cuda.device(self.plan.device):
            _lib.check(self._lib.shoot_lbfgs_step(self._opt, _stream_ptr(stream)), "shoot_lbfgs_step")
        n = len(self.plan.pairs)
        costs = (ctypes.c_double * n)()
        ev = ctypes.c_int32()
        _lib.check(self._lib.shoot_lbfgs_last_step(self._opt, costs, ctypes.byref(ev)), "shoot_lbfgs_last_step")
        return [float(c) for c in costs], int(ev.value)

    def close(self):
        if self._opt is not None:
            self._lib.shoot_lbfgs_destroy(self._opt)
            self._opt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbfgs(pairs: Sequence[PairSpec], T: int, iters: int, m: int = 5, c1: float = 1e-4, trials: int = 8,
          flags: int = 0):
    """L-BFGS on every pair's p0 (updated in place). Returns the plan, the cost
    history [iters, n_pairs] (cost at the start of each iteration) and the
    gradient evaluations of each iteration."""
    plan = Plan(pairs, T, flags, outputs=("grad", "cost"))
    opt = LBFGS(plan, m, c1, trials)
    hist, evals = [], []
    for _ in range(iters):
        c, e = opt.step()
        hist.append(c)
        evals.append(e)
    opt.close()
    return plan, hist, evals


# ---------------------------------------------------------------- autograd

_PLAN_CACHE: "OrderedDict[tuple, Plan]" = OrderedDict()
_PLAN_CACHE_SIZE = 8


def _cached_plan(S, J, p0, rho, sigma, lam, T, flags):
    key = (S.data_ptr(), J.data_ptr(), p0.data_ptr(), tuple(S.shape), float(rho), float(sigma), float(lam),
           int(T), int(flags), S.device.index)
    plan = _PLAN_CACHE.get(key)
    if plan is None:
        plan = Plan([PairSpec(S, p0, rho, sigma, lam, J)], T, flags, outputs=("grad", "cost"))
        plan._keep = (S, J, p0)
        _PLAN_CACHE[key] = plan
        while len(_PLAN_CACHE) > _PLAN_CACHE_SIZE:
            _PLAN_CACHE.popitem(last=False)[1].close()
    else:
        _PLAN_CACHE.move_to_end(key)
    return plan


class ShootCost(torch.autograd.Function):
    """H(p0) for one pair; the gradient comes from the library's adjoint."""

    @staticmethod
    def forward(ctx, S, J, p0, rho, sigma, lam, T, flags=0):
        plan = _cached_plan(S.detach(), J.detach(), p0.detach(), rho, sigma, lam, T, flags)
        plan.grad()
        ctx.save_for_backward(plan.out_grad[0].clone())
        return plan.out_cost[0, 0].clone()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return None, None, g * grad, None, None, None, None, None


def shoot_cost(S, J, p0, rho, sigma, lam=0.01, T=10, flags=0):
    """Differentiable (w.r.t. p0) cost H of Eq. 4 for one pair."""
    return ShootCost.apply(S, J, p0, rho, sigma, lam, T, flags)


def gradient_descent(pairs: Sequence[PairSpec], T: int, iters: int, eta: float = 1.0, flags: int = 0):
    """Fixed-step gradient descent on every pair's p0 (updated in place on the
    device by shoot_descend), with the step of a pair halved whenever its cost
    rises. Returns the plan and the cost history [iters, n_pairs] (the cost at
    the p0 each iteration started from)."""
    plan = Plan(pairs, T, flags, outputs=("grad", "cost"))
    hist = []
    for it in range(iters):
        plan.descend(eta, reset=(it == 0))
        hist.append(plan.out_cost[:, 0].clone())
    return plan, torch.stack(hist) if hist else None


def stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst <- src through the library's streaming copy kernel (the bandwidth
    reference of the measurements); contiguous device tensors of equal size,
    a multiple of 16 bytes."""
    if src.device.type != "cuda" or dst.device != src.device:
        raise ValueError("src and dst must be on the same GPU")
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous")
    nbytes = src.numel() * src.element_size()
    if nbytes != dst.numel() * dst.element_size():
        raise ValueError("src and dst sizes differ")
    lib = _lib.load()
    _lib.check(lib.shoot_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream_ptr(stream)), "shoot_stream_copy")
