"""Python binding of the C ABI.  PyTorch provides device memory and streams;
every step of the solver runs in the HIP library (libhopf.so).

    prob = Problem(A, hkind="l2_wl1", w=w, precision="bf16_refined", tol=1e-12)
    out = prob.eval(x, t)          # x: (npts, n) float32 cuda tensor, t: (npts,)
    out["phi"], out["grad"], out["dphidt"], out["iters"], out["kstar"]
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check


def set_deterministic(on: bool) -> None:
    """Deterministic mode of the dense evaluations (hopf_set_deterministic): every later launch,
    and every plan created later, gives the same bits on every run; False restores the fastest
    schedule (results agree to the parity tolerances, not bit for bit).  Process-wide."""
    check(_lib.load().hopf_set_deterministic(1 if on else 0))


def deterministic() -> bool:
    """The current deterministic-mode setting (hopf_get_deterministic)."""
    return bool(_lib.load().hopf_get_deterministic())


def _stream_ptr(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host64(a, shape=None):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _device_array(a: torch.Tensor, dtype, name, shape):
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if a.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, a.dtype))
    if tuple(a.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(a.shape), tuple(shape)))
    return a.contiguous()


class Problem:
    """One problem: J(y) = 1/2 y^T A^{-1} y (or the min over K translated copies / ellipsoid
    level sets c_k + {u^T A^{-1} u <= 1}), H in {"wl1", "l2", "l2_wl1", "wl2", "al2"} with weights w
    ("wl2": sqrt(<p, diag(w) p>); "al2": sqrt(<p, HA p>) with the SPD matrix HA; "linf": |p|_inf;
    "linctrl": the time-dependent H of the linear control system dx/ds = diag(drift) x + diag(w) beta,
    beta in [-1, 1]^n, whose points are the transformed states z = e^{-sM} x).
    jkind "quad" is J(y) = 1/2 y^T A^{-1} y; "l1sq" and "linfsq" are 1/2 |y|_1^2 and 1/2 |y|_inf^2
    (A unused: pass n=...)."""

    def __init__(self, A=None, *, n: Optional[int] = None, diagonal: bool = False, centres=None,
                 level_set: bool = False, hkind: str = "wl1", w=None, lam: float = 1.0,
                 tol: float = 1e-12, max_iter: int = 20000, precision: str = "bf16_refined",
                 HA=None, jkind: str = "quad", drift=None, stream=None, _handle=None):
        self._lib = _lib.load()
        A64 = _host64(A)
        if n is None:
            if A64 is None:
                raise ValueError("give A or n")
            n = A64.shape[0]
        if A64 is not None:
            if diagonal:
                A64 = A64.reshape(n)
            else:
                A64 = A64.reshape(n, n)
        self.n = int(n)
        self.diagonal = bool(diagonal) or A64 is None
        self.A = A64
        self.centres = _host64(centres, (-1, self.n)) if centres is not None else None
        self.K = 1 if self.centres is None else self.centres.shape[0]
        self.level_set = bool(level_set)
        self.hkind = hkind
        self.w = _host64(w, (self.n,)) if w is not None else None
        self.HA = _host64(HA, (self.n, self.n)) if HA is not None else None
        self.drift = _host64(drift, (self.n,)) if drift is not None else None
        self.jkind = jkind
        self.lam, self.tol, self.max_iter = float(lam), float(tol), int(max_iter)
        self.precision = precision
        self.io_dtype = torch.float64 if precision == "f64" else torch.float32
        self._handle = None
        if _handle is not None:
            self._handle = _handle
            return
        h = ctypes.c_void_p()
        desc = self._desc()
        check(self._lib.hopf_problem_create(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(h)))
        self._handle = h

    def _desc(self):
        return _lib.ProblemDesc(
            self.n, None if self.A is None else self.A.ctypes.data, int(self.diagonal), self.K,
            None if self.centres is None else self.centres.ctypes.data, int(self.level_set),
            _lib.HKIND[self.hkind], None if self.w is None else self.w.ctypes.data, self.lam, self.tol,
            self.max_iter, _lib.PRECISION[self.precision], None if self.HA is None else self.HA.ctypes.data,
            _lib.JKIND[self.jkind], None if self.drift is None else self.drift.ctypes.data)

    @classmethod
    def batch(cls, specs: Sequence[dict], stream=None):
        """Create many problems with one batched factorisation (ragged batches)."""
        lib = _lib.load()
        objs = [cls.__new__(cls) for _ in specs]
        descs = (_lib.ProblemDesc * len(specs))()
        for o, s, i in zip(objs, specs, range(len(specs))):
            cls.__init__(o, **s, _handle=ctypes.c_void_p(0))
            descs[i] = o._desc()
        out = (ctypes.c_void_p * len(specs))()
        check(lib.hopf_problem_create_batch(len(specs), descs, _stream_ptr(stream), out))
        for o, i in zip(objs, range(len(specs))):
            o._handle = ctypes.c_void_p(out[i])
        return objs

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            try:
                self._lib.hopf_problem_destroy(h)
            except Exception:
                pass
            self._handle = None

    # ------------------------------------------------------------------ calls
    def eval(self, x: torch.Tensor, t: torch.Tensor, stream=None, out=None):
        npts = x.shape[0]
        x = _device_array(x, self.io_dtype, "x", (npts, self.n))
        t = _device_array(t, self.io_dtype, "t", (npts,))
        dev = x.device
        if out is None:
            out = dict(
                phi=torch.empty(npts, dtype=self.io_dtype, device=dev),
                grad=torch.empty(npts, self.n, dtype=self.io_dtype, device=dev),
                dphidt=torch.empty(npts, dtype=self.io_dtype, device=dev),
                iters=torch.empty(npts, dtype=torch.int32, device=dev),
                kstar=torch.empty(npts, dtype=torch.int32, device=dev),
            )
        check(self._lib.hopf_eval(self._handle, npts, _ptr(x), _ptr(t), _ptr(out["phi"]), _ptr(out["grad"]),
                                  _ptr(out["dphidt"]), _ptr(out["iters"]), _ptr(out["kstar"]),
                                  _stream_ptr(stream)))
        return out

    def closest_point(self, y: torch.Tensor, s_tol: float = 1e-6, stream=None):
        npts = y.shape[0]
        y = _device_array(y, torch.float32, "y", (npts, self.n))
        dev = y.device
        out = dict(
            dist=torch.empty(npts, dtype=torch.float32, device=dev),
            cp=torch.empty(npts, self.n, dtype=torch.float32, device=dev),
            kstar=torch.empty(npts, dtype=torch.int32, device=dev),
            inside=torch.empty(npts, dtype=torch.int32, device=dev),
            newton=torch.empty(npts, dtype=torch.int32, device=dev),
        )
        check(self._lib.hopf_closest_point(self._handle, npts, _ptr(y), float(s_tol), _ptr(out["dist"]),
                                           _ptr(out["cp"]), _ptr(out["kstar"]), _ptr(out["inside"]),
                                           _ptr(out["newton"]), _stream_ptr(stream)))
        return out

    def backward(self, gphi, grad, dphidt, kstar=None, want=("gx", "gt", "gA", "gc"), stream=None,
                 noalloc=False):
        """Envelope-theorem gradients (C ABI hopf_backward; hopf_backward_noalloc with noalloc=True,
        which keeps its partial sums in the library's fixed device array instead of allocating)."""
        npts = grad.shape[0]
        dev = grad.device
        gphi = _device_array(gphi, torch.float32, "gphi", (npts,))
        grad = _device_array(grad, torch.float32, "grad", (npts, self.n))
        dphidt = _device_array(dphidt, torch.float32, "dphidt", (npts,))
        out = {}
        if "gx" in want:
            out["gx"] = torch.empty(npts, self.n, dtype=torch.float32, device=dev)
        if "gt" in want:
            out["gt"] = torch.empty(npts, dtype=torch.float32, device=dev)
        if "gA" in want:
            out["gA"] = torch.empty(self.n, self.n, dtype=torch.float32, device=dev)
        if "gc" in want:
            out["gc"] = torch.empty(self.K, self.n, dtype=torch.float32, device=dev)
        fn = self._lib.hopf_backward_noalloc if noalloc else self._lib.hopf_backward
        check(fn(self._handle, npts, _ptr(gphi), _ptr(grad), _ptr(dphidt), _ptr(kstar),
                                      _ptr(out.get("gx")), _ptr(out.get("gt")), _ptr(out.get("gA")),
                                      _ptr(out.get("gc")), _stream_ptr(stream)))
        return out

    def control(self, x, t, grad, kstar=None, stream=None):
        """Optimal control beta and terminal value xT of each point from an evaluation's grad and
        kstar (C ABI hopf_control)."""
        npts = x.shape[0]
        x = _device_array(x, self.io_dtype, "x", (npts, self.n))
        t = _device_array(t, self.io_dtype, "t", (npts,))
        grad = _device_array(grad, self.io_dtype, "grad", (npts, self.n))
        out = dict(beta=torch.empty(npts, self.n, dtype=self.io_dtype, device=x.device),
                   xT=torch.empty(npts, self.n, dtype=self.io_dtype, device=x.device))
        check(self._lib.hopf_control(self._handle, npts, _ptr(x), _ptr(t), _ptr(grad), _ptr(kstar),
                                     _ptr(out["beta"]), _ptr(out["xT"]), _stream_ptr(stream)))
        return out

    def inverse(self) -> np.ndarray:
        out = np.empty((self.n, self.n))
        check(self._lib.hopf_problem_get_inverse(self._handle, out.ctypes.data))
        return out

    def iterations(self, reset: bool = False) -> int:
        """Passes of the dense solvers summed over every column (every copy, every Newton solve)
        of this problem's calls since creation or the last reset (hopf_problem_iterations)."""
        v = ctypes.c_int64()
        check(self._lib.hopf_problem_iterations(self._handle, ctypes.byref(v), 1 if reset else 0))
        return v.value

    def info(self):
        v = [ctypes.c_int32() for _ in range(4)]
        check(self._lib.hopf_problem_info(self._handle, *[ctypes.byref(x) for x in v]))
        return dict(n=v[0].value, n_pad=v[1].value, K=v[2].value, precision=v[3].value)


def closest_point_ragged(problems: Sequence[Problem], ys: Sequence[torch.Tensor], s_tol: float = 1e-6, stream=None):
    """Closest points and distances for a ragged batch of ellipsoid level-set problems in one call
    (hopf_closest_point_ragged)."""
    lib = _lib.load()
    nprob = len(problems)
    counts = [int(y.shape[0]) for y in ys]
    off = np.zeros(nprob + 1, np.int64)
    off[1:] = np.cumsum(counts)
    y_packed = torch.cat([y.reshape(-1) for y in ys]).contiguous()
    dev = y_packed.device
    tot = int(off[-1])
    dist = torch.empty(tot, dtype=torch.float32, device=dev)
    cp = torch.empty_like(y_packed)
    kstar = torch.empty(tot, dtype=torch.int32, device=dev)
    inside = torch.empty(tot, dtype=torch.int32, device=dev)
    newton = torch.empty(tot, dtype=torch.int32, device=dev)
    handles = (ctypes.c_void_p * nprob)(*[p._handle.value for p in problems])
    offs = (ctypes.c_int64 * (nprob + 1))(*off.tolist())
    check(lib.hopf_closest_point_ragged(nprob, handles, offs, _ptr(y_packed), float(s_tol), _ptr(dist), _ptr(cp),
                                        _ptr(kstar), _ptr(inside), _ptr(newton), _stream_ptr(stream)))
    cps, o = [], 0
    for p, c in zip(problems, counts):
        cps.append(cp[o:o + c * p.n].view(c, p.n))
        o += c * p.n
    return dict(dist=dist, cp=cps, kstar=kstar, inside=inside, newton=newton, offsets=off)


class RaggedPlan:
    """A ragged evaluation bound to its problems, inputs and (owned) outputs once
    (hopf_ragged_plan_create); launch() enqueues kernels only (hopf_ragged_plan_launch), so it can
    be captured in a HIP graph.  The inputs are packed into buffers the plan owns; refill them in
    place (x_packed, t) to evaluate other points of the same shape."""

    def __init__(self, problems: Sequence[Problem], xs: Sequence[torch.Tensor], ts: Sequence[torch.Tensor]):
        self._lib = _lib.load()
        self.problems = list(problems)
        nprob = len(self.problems)
        counts = [int(x.shape[0]) for x in xs]
        off = np.zeros(nprob + 1, np.int64)
        off[1:] = np.cumsum(counts)
        self.offsets = off
        self.x_packed = torch.cat([x.reshape(-1) for x in xs]).contiguous()
        self.t = torch.cat(list(ts)).contiguous()
        dev = self.x_packed.device
        tot = int(off[-1])
        self.phi = torch.empty(tot, dtype=torch.float32, device=dev)
        self.grad_packed = torch.empty_like(self.x_packed)
        self.dphidt = torch.empty(tot, dtype=torch.float32, device=dev)
        self.iters = torch.empty(tot, dtype=torch.int32, device=dev)
        self.kstar = torch.empty(tot, dtype=torch.int32, device=dev)
        handles = (ctypes.c_void_p * nprob)(*[p._handle.value for p in self.problems])
        offs = (ctypes.c_int64 * (nprob + 1))(*off.tolist())
        self._handle = ctypes.c_void_p()
        check(self._lib.hopf_ragged_plan_create(nprob, handles, offs, _ptr(self.x_packed), _ptr(self.t),
                                                _ptr(self.phi), _ptr(self.grad_packed), _ptr(self.dphidt),
                                                _ptr(self.iters), _ptr(self.kstar), ctypes.byref(self._handle)))

    def launch(self, stream=None):
        check(self._lib.hopf_ragged_plan_launch(self._handle, _stream_ptr(stream)))

    def grads(self):
        out, o = [], 0
        for p, c in zip(self.problems, np.diff(self.offsets)):
            out.append(self.grad_packed[o:o + int(c) * p.n].view(int(c), p.n))
            o += int(c) * p.n
        return out

    def __del__(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self._lib.hopf_ragged_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()


def eval_ragged(problems: Sequence[Problem], xs: Sequence[torch.Tensor], ts: Sequence[torch.Tensor],
                stream=None):
    """Evaluate a ragged batch (each problem its own n, A, K, w; points packed) in one call."""
    lib = _lib.load()
    nprob = len(problems)
    counts = [int(x.shape[0]) for x in xs]
    off = np.zeros(nprob + 1, np.int64)
    off[1:] = np.cumsum(counts)
    x_packed = torch.cat([x.reshape(-1) for x in xs]).contiguous()
    t_all = torch.cat(list(ts)).contiguous()
    dev = x_packed.device
    tot = int(off[-1])
    phi = torch.empty(tot, dtype=torch.float32, device=dev)
    grad = torch.empty_like(x_packed)
    dphidt = torch.empty(tot, dtype=torch.float32, device=dev)
    iters = torch.empty(tot, dtype=torch.int32, device=dev)
    kstar = torch.empty(tot, dtype=torch.int32, device=dev)
    handles = (ctypes.c_void_p * nprob)(*[p._handle.value for p in problems])
    offs = (ctypes.c_int64 * (nprob + 1))(*off.tolist())
    check(lib.hopf_eval_ragged(nprob, handles, offs, _ptr(x_packed), _ptr(t_all), _ptr(phi), _ptr(grad),
                               _ptr(dphidt), _ptr(iters), _ptr(kstar), _stream_ptr(stream)))
    grads, o = [], 0
    for p, c in zip(problems, counts):
        grads.append(grad[o:o + c * p.n].view(c, p.n))
        o += c * p.n
    return dict(phi=phi, grad=grads, dphidt=dphidt, iters=iters, kstar=kstar, offsets=off)


def max_over_hamiltonians(outs: Sequence[dict], stream=None):
    """phi for H = min_i H_i from the evaluations outs[i] (same points, same J, Hamiltonian H_i):
    max_i phi_i with the grad and dphidt of the attaining i (C ABI hopf_max_over_hamiltonians)."""
    lib = _lib.load()
    k = len(outs)
    npts, n = outs[0]["grad"].shape
    dt = outs[0]["phi"].dtype
    for o in outs:
        for key in ("phi", "grad", "dphidt"):
            if o[key].dtype != dt or not o[key].is_contiguous():
                raise ValueError("the evaluations must share one dtype and be contiguous")
    arr = lambda key: (ctypes.c_void_p * k)(*[o[key].data_ptr() for o in outs])
    dev = outs[0]["phi"].device
    res = dict(phi=torch.empty(npts, dtype=dt, device=dev), grad=torch.empty(npts, n, dtype=dt, device=dev),
               dphidt=torch.empty(npts, dtype=dt, device=dev), istar=torch.empty(npts, dtype=torch.int32, device=dev))
    check(lib.hopf_max_over_hamiltonians(k, npts, n, int(dt == torch.float64), arr("phi"), arr("grad"), arr("dphidt"),
                                         _ptr(res["phi"]), _ptr(res["grad"]), _ptr(res["dphidt"]), _ptr(res["istar"]),
                                         _stream_ptr(stream)))
    return res


def _held_like(problem: Problem, which: str, like: torch.Tensor) -> torch.Tensor:
    """The problem's own A (n x n, or its n diagonal entries) or centres (K x n), as a tensor of
    like's dtype and device: what the forward actually solves with."""
    if which == "A":
        if problem.A is None:
            held = np.eye(problem.n) if like.dim() == 2 else np.ones(problem.n)
        elif problem.diagonal and like.dim() == 2:
            held = np.diag(problem.A)
        else:
            held = problem.A
    else:
        held = problem.centres if problem.centres is not None else np.zeros((problem.K, problem.n))
    return torch.as_tensor(np.asarray(held), dtype=like.dtype, device=like.device)


def _check_held(problem: Problem, which: str, value):
    """The autograd inputs A and centres must be the problem's own: the forward solves with the
    matrices the problem was created with, so a different tensor would get phi and gradients of
    another problem."""
    if value is None:
        return
    if not isinstance(value, torch.Tensor):
        raise TypeError("%s must be a tensor" % which)
    held = _held_like(problem, which, value.detach())
    if tuple(value.shape) != tuple(held.shape):
        raise ValueError("%s has shape %s; the problem holds %s" % (which, tuple(value.shape), tuple(held.shape)))
    if not torch.equal(value.detach(), held):
        raise ValueError("%s differs from the problem's own (create a new Problem for new values)" % which)


class HopfValue(torch.autograd.Function):
    """phi(x, t; A, centres) with envelope-theorem gradients wrt x, t, A and centres.
    Only phi is differentiable; grad and dphidt are returned detached.  A and centres must hold
    the problem's own values (checked); gA comes back in A's shape and dtype (the diagonal of the
    gradient for a diagonal A given as a vector)."""

    @staticmethod
    def forward(ctx, x, t, A, centres, problem: Problem):
        _check_held(problem, "A", A)
        _check_held(problem, "centres", centres)
        out = problem.eval(x.detach(), t.detach())
        ctx.problem = problem
        ctx.a_meta = None if A is None else (tuple(A.shape), A.dtype)
        ctx.c_dtype = None if centres is None else centres.dtype
        ctx.save_for_backward(out["grad"], out["dphidt"], out["kstar"])
        ctx.mark_non_differentiable(out["grad"], out["dphidt"])
        return out["phi"], out["grad"], out["dphidt"]

    @staticmethod
    def backward(ctx, gphi, _g1, _g2):
        grad, dphidt, kstar = ctx.saved_tensors
        prob = ctx.problem
        want = []
        if ctx.needs_input_grad[0]:
            want.append("gx")
        if ctx.needs_input_grad[1]:
            want.append("gt")
        if ctx.needs_input_grad[2]:
            want.append("gA")
        if ctx.needs_input_grad[3]:
            want.append("gc")
        b = prob.backward(gphi.contiguous().float(), grad, dphidt, kstar, want=tuple(want))
        gA = b.get("gA")
        if gA is not None:
            shape, dt = ctx.a_meta
            gA = (torch.diagonal(gA) if len(shape) == 1 else gA).to(dt)
        gc = b.get("gc")
        if gc is not None:
            gc = gc.to(ctx.c_dtype)
        return b.get("gx"), b.get("gt"), gA, gc, None


def hopf_value(x, t, A, centres, problem: Problem):
    return HopfValue.apply(x, t, A, centres, problem)
