"""Python binding of libodp.so.  Argument marshalling only: every step runs in the
HIP kernels; PyTorch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import (ODP_BALANCE_R, ODP_FFT_F32, ODP_STOP_NONE, BatchEntry, PlanInfo, Problem, StateLayout, StopStatus,
                   Tuning, check, lib)


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _c64(t: torch.Tensor, shape=None) -> torch.Tensor:
    if t.dtype != torch.complex64:
        raise TypeError("expected complex64")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def prox_stagm(y: torch.Tensor, sqrt_f: torch.Tensor, eps: float, lam: float,
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Elementwise Prox_{G_eps; lam}(y) against sqrt(f) (odp_prox_stagm)."""
    _c64(y)
    if sqrt_f.dtype != torch.float32 or sqrt_f.numel() != y.numel():
        raise ValueError("sqrt_f must be float32 with y's element count")
    z = torch.empty_like(y) if out is None else out
    check(lib().odp_prox_stagm(_ptr(y), _ptr(sqrt_f), y.numel(), float(eps), float(lam), _ptr(z),
                               _stream(stream)))
    return z


def blind_initial_probe_static(sqrt_f: torch.Tensor, out: torch.Tensor | None = None,
                               stream=None) -> torch.Tensor:
    """w0 = (1/J) sum_j F*(sqrt f_j) from amplitudes [J, p, p] without a plan
    (odp_blind_initial_probe_static: no workspace, the library's static scratch)."""
    if sqrt_f.dtype != torch.float32 or sqrt_f.dim() != 3 or sqrt_f.shape[1] != sqrt_f.shape[2]:
        raise ValueError("sqrt_f must be float32 [J, p, p]")
    if not sqrt_f.is_contiguous():
        raise ValueError("sqrt_f must be contiguous")
    J, p = int(sqrt_f.shape[0]), int(sqrt_f.shape[1])
    out = torch.empty((p, p), dtype=torch.complex64, device=sqrt_f.device) if out is None else out
    _c64(out, (p, p))
    check(lib().odp_blind_initial_probe_static(_ptr(sqrt_f), J, p, _ptr(out), _stream(stream)))
    return out


@dataclass
class Geometry:
    rects: np.ndarray      # [D,4] (r0, c0, r1, c1)
    usub_off: np.ndarray   # [D]
    pairs: np.ndarray      # [n_pairs, 6] (i1, i2, r0, c0, r1, c1)
    lam_off: np.ndarray    # [n_pairs]
    cover: np.ndarray      # [H, W]


class State:
    """One device state buffer of a plan (u_d, Gamma, Lam; blind: w, w_d, Delta)."""

    def __init__(self, plan: "Plan", buf: torch.Tensor):
        self.plan = plan
        self.buf = buf

    def _view(self, off: int, n: int) -> torch.Tensor:
        return self.buf[off: off + 8 * n].view(torch.complex64)

    def u_sub(self) -> list[torch.Tensor]:
        g = self.plan.geometry()
        out = []
        for d in range(self.plan.info.D):
            r0, c0, r1, c1 = (int(v) for v in g.rects[d])
            base = self.plan.layout.u_sub + 8 * int(g.usub_off[d])
            out.append(self._view(base, (r1 - r0) * (c1 - c0)).view(r1 - r0, c1 - c0))
        return out

    def gamma(self) -> torch.Tensor:
        i = self.plan.info
        return self._view(self.plan.layout.gamma, i.J * i.p * i.p).view(i.J, i.p, i.p)

    def lam(self) -> dict:
        """{(a, b): Lam_{a,b}} on Omega_a cap Omega_b for both orders of every pair."""
        g = self.plan.geometry()
        out = {}
        for q in range(len(g.pairs)):
            a, b, r0, c0, r1, c1 = (int(v) for v in g.pairs[q])
            h, w = r1 - r0, c1 - c0
            both = self._view(self.plan.layout.lam + 8 * int(g.lam_off[q]), 2 * h * w).view(2, h, w)
            out[(a, b)] = both[0]
            out[(b, a)] = both[1]
        return out

    def probe(self) -> torch.Tensor:
        p = self.plan.info.p
        return self._view(self.plan.layout.w, p * p).view(p, p)

    def probe_copies(self) -> torch.Tensor:
        i = self.plan.info
        return self._view(self.plan.layout.w_sub, i.D * i.p * i.p).view(i.D, i.p, i.p)

    def probe_multipliers(self) -> torch.Tensor:
        i = self.plan.info
        return self._view(self.plan.layout.delta, i.D * i.p * i.p).view(i.D, i.p, i.p)

    def clone(self) -> "State":
        return State(self.plan, self.buf.clone())


def _problem(H, W, p, offsets, frame_sub, D, eps, eta, r, mu, gamma, transform, blind, probe_fmask):
    """(odp_problem, keep-alive arrays) for one problem."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 2))
    sub = np.ascontiguousarray(np.asarray(frame_sub, dtype=np.int32).reshape(-1))
    mask = None if probe_fmask is None else np.ascontiguousarray(np.asarray(probe_fmask, dtype=np.uint8))
    if D is None:
        D = int(sub.max()) + 1 if len(sub) else 0
    prob = Problem(H=H, W=W, p=p, J=len(off), offsets=off.ctypes.data_as(C.POINTER(C.c_int32)), D=D,
                   frame_sub=sub.ctypes.data_as(C.POINTER(C.c_int32)), eps=eps, eta=eta, r=r, mu=mu,
                   gamma=gamma, transform=transform, blind=1 if blind else 0,
                   probe_fmask=mask.ctypes.data_as(C.POINTER(C.c_uint8)) if mask is not None else None)
    return prob, (off, sub, mask)


class Plan:
    """A validated problem (odp_plan) plus its device workspace once bound."""

    def __init__(self, H: int, W: int, p: int, offsets, frame_sub, D: int | None = None,
                 eps: float = 0.5, eta: float = 0.1, r: float = 0.0, mu: float = 0.0,
                 gamma: float = 0.0, transform: int = ODP_FFT_F32, blind: bool = False,
                 probe_fmask=None, _handle=None):
        L = lib()
        if _handle is None:
            prob, self._arrays = _problem(H, W, p, offsets, frame_sub, D, eps, eta, r, mu, gamma, transform,
                                          blind, probe_fmask)
            h = C.c_void_p()
            check(L.odp_plan_create(C.byref(prob), C.byref(h)))
        else:
            h = _handle
        self._h = h
        self.info = PlanInfo()
        check(L.odp_plan_get_info(self._h, C.byref(self.info)))
        self.layout = StateLayout()
        check(L.odp_state_get_layout(self._h, C.byref(self.layout)))
        self.params = dict(eps=eps, eta=eta, r=r, mu=mu, gamma=gamma)
        self.blind = blind
        self._geom = None
        self.workspace = None
        self._keep = ()

    @classmethod
    def batch(cls, problems: list[dict]) -> "Plan":
        """One plan over independent problems (dicts with the Plan() keyword arguments)."""
        arr = (Problem * len(problems))()
        keep = []
        for i, pb in enumerate(problems):
            kw = dict(D=None, eps=0.5, eta=0.1, r=0.0, mu=0.0, gamma=0.0, transform=ODP_FFT_F32, blind=False,
                      probe_fmask=None)
            kw.update(pb)
            prob, k = _problem(kw.pop("H"), kw.pop("W"), kw.pop("p"), kw.pop("offsets"), kw.pop("frame_sub"),
                               **kw)
            arr[i] = prob
            keep.append(k)
        h = C.c_void_p()
        check(lib().odp_batch_plan_create(arr, len(problems), C.byref(h)))
        p0 = problems[0]
        plan = cls(0, 0, p0["p"], None, None, eps=p0.get("eps", 0.5), eta=p0.get("eta", 0.1),
                   transform=p0.get("transform", ODP_FFT_F32), _handle=h)
        plan._arrays = keep
        return plan

    def n_problems(self) -> int:
        n = 0
        e = BatchEntry()
        while lib().odp_batch_get_entry(self._h, n, C.byref(e)) == 0:
            n += 1
        return n

    def entry(self, i: int) -> BatchEntry:
        e = BatchEntry()
        check(lib().odp_batch_get_entry(self._h, int(i), C.byref(e)))
        return e

    def set_penalties(self, r, stream=None) -> None:
        rr = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
        check(lib().odp_batch_set_penalties(self._h, rr.ctypes.data, _stream(stream)))

    def tuning(self) -> Tuning:
        t = Tuning()
        check(lib().odp_plan_get_tuning(self._h, C.byref(t)))
        return t

    def set_tuning(self, transform: int, xcd_slice: int, tiling: int, stream=None) -> None:
        check(lib().odp_plan_set_tuning(self._h, int(transform), int(xcd_slice), int(tiling), _stream(stream)))

    def set_streaming(self, mode: int = -1) -> None:
        """Cache policy of the frame arrays: 1 streaming (non-temporal) kernel variants, 0
        ordinary accesses, -1 by size (the default); identical results either way."""
        check(lib().odp_plan_set_streaming(self._h, int(mode)))

    def set_pixel_pairs(self, mode: int = 1) -> None:
        """Pixel-update pull width: 1 (default) one 16-byte load for a thread's two row
        neighbours wherever the plan's window columns allow it, 0 one load per pixel;
        identical iterates either way (``get_tuning().pixel_pairs`` reports the choice)."""
        check(lib().odp_plan_set_pixel_pairs(self._h, int(mode)))

    def set_stopping(self, measure: int = ODP_STOP_NONE, tol: float = 0.0, max_iter: int = 0,
                     every: int = 1) -> None:
        """Device-side stopping rule of Sec. 4 (ODP_STOP_RF / ODP_STOP_RE, tolerance,
        iteration cap), checked after every `every`-th iteration; applies to later
        iterations and graphs created afterwards."""
        check(lib().odp_plan_set_stopping(self._h, int(measure), float(tol), int(max_iter), int(every)))

    def set_balancing(self, mu: float = 10.0, tau: float = 2.0, period: int = 0, until: int = 0,
                      which: int = ODP_BALANCE_R) -> None:
        """Penalties by residual balancing every `period` iterations (0: off): the overlap
        penalties (ODP_BALANCE_R), the data penalty (ODP_BALANCE_ETA) or both."""
        check(lib().odp_plan_set_balancing(self._h, float(mu), float(tau), int(period), int(until), int(which)))

    def eta(self) -> float:
        """The current data penalty (changed by balancing)."""
        return float(lib().odp_plan_get_eta(self._h))

    def penalties(self) -> list[float]:
        """The overlap penalty r of each problem (changed by balancing)."""
        return [self.entry(i).r for i in range(self.n_problems())]

    def stop_status(self, state: "State", stream=None) -> list[dict]:
        """Per problem: iterations run, whether it stopped, and its last RF, RE, G."""
        n = self.n_problems()
        arr = (StopStatus * n)()
        check(lib().odp_state_get_stop_status(self._h, _ptr(state.buf), C.cast(arr, C.c_void_p), _stream(stream)))
        return [dict(iters=e.iters, stopped=bool(e.stopped), rf=e.rf, re=e.re, g=e.g) for e in arr]

    def autotune(self, scratch: "State", iters: int = 5, stream=None) -> Tuning:
        t = Tuning()
        check(lib().odp_plan_autotune(self._h, _ptr(scratch.buf), int(iters), _stream(stream), C.byref(t)))
        return t

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().odp_plan_destroy(h)
            except (AttributeError, TypeError, ImportError):
                pass   # interpreter shutdown: module state is gone and the process frees the plan
            self._h = None

    # ---- geometry exports (host, no device needed) ----
    def geometry(self) -> Geometry:
        if self._geom is None:
            i = self.info
            rects = np.zeros((i.D, 4), np.int32)
            uoff = np.zeros(i.D, np.int64)
            pairs = np.zeros((max(i.n_pairs, 0), 6), np.int32)
            loff = np.zeros(max(i.n_pairs, 0), np.int64)
            cover = np.zeros((i.H, i.W), np.int32)
            L = lib()
            check(L.odp_plan_get_rects(self._h, rects.ctypes.data, uoff.ctypes.data))
            if i.n_pairs:
                check(L.odp_plan_get_pairs(self._h, pairs.ctypes.data, loff.ctypes.data))
            check(L.odp_plan_get_cover(self._h, cover.ctypes.data))
            self._geom = Geometry(rects, uoff, pairs, loff, cover)
        return self._geom

    # ---- device side ----
    def bind(self, sqrt_f: torch.Tensor, w: torch.Tensor, stream=None,
             workspace: torch.Tensor | None = None) -> "Plan":
        """w: [p, p] probe, or [n, p, p] probes of a batch plan (one per problem).
        workspace: optional uint8 device buffer of at least info.workspace_bytes,
        256-byte aligned (allocated here when omitted)."""
        i = self.info
        if sqrt_f.dtype != torch.float32 or tuple(sqrt_f.shape) != (i.J, i.p, i.p):
            raise ValueError("sqrt_f must be float32 [J, p, p]")
        if w.dim() == 3:
            _c64(w, (self.n_problems(), i.p, i.p))
        else:
            _c64(w, (i.p, i.p))
        if workspace is None:
            workspace = torch.empty(i.workspace_bytes, dtype=torch.uint8, device=sqrt_f.device)
        elif workspace.dtype != torch.uint8 or workspace.numel() < i.workspace_bytes:
            raise ValueError("workspace must be uint8 with at least workspace_bytes elements")
        self.workspace = workspace
        check(lib().odp_plan_bind(self._h, _ptr(self.workspace), _ptr(sqrt_f), _ptr(w), _stream(stream)))
        self._keep = (sqrt_f, w)
        return self

    def illum_max(self) -> float:
        v = C.c_double()
        check(lib().odp_plan_illum_max(self._h, C.byref(v)))
        return v.value

    def set_params(self, stream=None, **kw) -> None:
        self.params.update(kw)
        p = self.params
        check(lib().odp_plan_set_params(self._h, p["eps"], p["eta"], p["r"], p["mu"], p["gamma"],
                                        _stream(stream)))

    def forward(self, u: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        i = self.info
        _c64(u, (i.H, i.W))
        _c64(w, (i.p, i.p))
        out = torch.empty((i.J, i.p, i.p), dtype=torch.complex64, device=u.device) if out is None else out
        _c64(out, (i.J, i.p, i.p))
        check(lib().odp_forward(self._h, _ptr(u), _ptr(w), _ptr(out), _stream(stream)))
        return out

    def adjoint(self, frames: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        i = self.info
        _c64(frames, (i.J, i.p, i.p))
        _c64(w, (i.p, i.p))
        out = torch.empty((i.H, i.W), dtype=torch.complex64, device=frames.device) if out is None else out
        _c64(out, (i.H, i.W))
        check(lib().odp_adjoint(self._h, _ptr(frames), _ptr(w), _ptr(out), _stream(stream)))
        return out

    def new_state(self, w0: torch.Tensor | None = None, device=None, stream=None) -> State:
        dev = device if device is not None else self.workspace.device
        buf = torch.empty(self.info.state_bytes, dtype=torch.uint8, device=dev)
        check(lib().odp_state_init(self._h, _ptr(buf), _ptr(w0), _stream(stream)))
        return State(self, buf)

    def iterate(self, state: State, n_iter: int, stats: bool = False, stream=None):
        st = (torch.empty((n_iter, 3), dtype=torch.float64, device=state.buf.device)
              if stats and n_iter > 0 else None)
        check(lib().odp_admm_iterate(self._h, _ptr(state.buf), int(n_iter), _ptr(st), _stream(stream)))
        return st

    def set_sweep_events(self, events, stride: int = 1) -> None:
        """events: list of (start, stop) torch.cuda.Event(enable_timing=True), each recorded
        once beforehand (which creates it); of the next len(events)*stride sweeps, sweep
        i*stride records pair i at its kernel's own start and end, so elapsed_time gives
        the kernel time."""
        n = len(events)
        s = (C.c_void_p * max(n, 1))(*[e[0].cuda_event for e in events])
        t = (C.c_void_p * max(n, 1))(*[e[1].cuda_event for e in events])
        check(lib().odp_plan_set_sweep_events(self._h, s, t, n, int(stride)))

    def frame_sweep(self, state: State, stats: torch.Tensor | None = None, stream=None) -> None:
        check(lib().odp_frame_sweep(self._h, _ptr(state.buf), _ptr(stats), _stream(stream)))

    def blind_initial_probe(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """w0 = (1/J) sum_j F*(sqrt f_j) from the bound amplitudes: [p, p], or [n, p, p] for
        a batch plan (one per problem)."""
        i = self.info
        n = self.n_problems()
        shape = (n, i.p, i.p) if n > 1 else (i.p, i.p)
        out = torch.empty(shape, dtype=torch.complex64, device=self.workspace.device) if out is None else out
        _c64(out, shape)
        check(lib().odp_blind_initial_probe(self._h, _ptr(out), _stream(stream)))
        return out

    def probe_update(self, state: State, stream=None) -> None:
        check(lib().odp_probe_update(self._h, _ptr(state.buf), _stream(stream)))

    def pixel_update(self, state: State, stats: torch.Tensor | None = None, stream=None) -> None:
        check(lib().odp_pixel_update(self._h, _ptr(state.buf), _ptr(stats), _stream(stream)))

    def merge(self, state: State, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        i = self.info
        out = torch.empty((i.H, i.W), dtype=torch.complex64, device=state.buf.device) if out is None else out
        check(lib().odp_merge(self._h, _ptr(state.buf), _ptr(out), _stream(stream)))
        return out

    def amp_loss(self, u: torch.Tensor, w: torch.Tensor, grad_u: bool = True, grad_w: bool = True,
                 stream=None):
        i = self.info
        _c64(u, (i.H, i.W))
        _c64(w, (i.p, i.p))
        loss = torch.empty(1, dtype=torch.float64, device=u.device)
        gu = torch.empty_like(u) if grad_u else None
        gw = torch.empty_like(w) if grad_w else None
        check(lib().odp_amp_loss(self._h, _ptr(u), _ptr(w), _ptr(loss), _ptr(gu), _ptr(gw), _stream(stream)))
        return loss, gu, gw


class Graph:
    """n_iter iterations of several (plan, state) pairs captured into one HIP graph."""

    def __init__(self, plans: list, states: list, n_iter: int):
        n = len(plans)
        ph = (C.c_void_p * n)(*[pl._h.value for pl in plans])
        sh = (C.c_void_p * n)(*[st.buf.data_ptr() for st in states])
        g = C.c_void_p()
        check(lib().odp_graph_create(ph, sh, n, int(n_iter), C.byref(g)))
        self._g = g
        self._keep = (plans, states)

    def launch(self, stream=None) -> None:
        check(lib().odp_graph_launch(self._g, _stream(stream)))

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value:
            try:
                lib().odp_graph_destroy(g)
            except (AttributeError, TypeError, ImportError):
                pass   # interpreter shutdown
            self._g = None
