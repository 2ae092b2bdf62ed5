"""ctypes wrapper of the C oracle plus the parts that are library primitives.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``oracle_eval``: Hopf value, gradient and time derivative by split Bregman
  (paper eqs. (3.3), (3.4a)-(3.4c), stopping test of section 4.5), min over
  translated initial data (section 2, min over initial data), in C.
* ``oracle_distance_newton``: distance / closest point to a union of
  ellipsoids by the level-set route of section 3.2 (eikonal Hopf evaluation
  and Newton on s, eq. (Newton_zero)), in C.
* ``oracle_distance_secular``: the same distance by the textbook ellipsoid
  projection of section 4.3 (Lagrange multiplier, Newton on mu); the
  eigendecomposition A = Q diag(sigma) Q^T is a library primitive
  (``numpy.linalg.eigh``).
* ``oracle_eval_linear_control``: the time-dependent Hamiltonian of linear controls (section
  2.2, some extensions and future work) for diagonal drift and input matrices and box controls,
  by the time-integrated Hopf formula over ``oracle_eval``.
* ``oracle_backward``: envelope-theorem gradients of phi with respect to x, t,
  A and the centres (phi is the optimal value of eq. (3.3), whose objective is
  affine in x, t, A and c at fixed p).  Parity unpinned by any printed value:
  pinned by central finite differences of ``oracle_eval``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hopf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_hopf.so")

OH_WL1, OH_L2, OH_L2_WL1, OH_WL2, OH_AL2, OH_LINF = 0, 1, 2, 3, 4, 5
_HKIND = {"wl1": OH_WL1, "l2": OH_L2, "l2_wl1": OH_L2_WL1, "wl2": OH_WL2, "al2": OH_AL2,
          "linf": OH_LINF}
_JKIND = {"quad": 0, "l1sq": 1, "linfsq": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def available() -> bool:
    return os.path.exists(_LIB)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("A", ctypes.c_void_p), ("K", ctypes.c_int32),
        ("centres", ctypes.c_void_p), ("level_set", ctypes.c_int32), ("hkind", ctypes.c_int32),
        ("w", ctypes.c_void_p), ("lam", ctypes.c_double), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("HA", ctypes.c_void_p), ("HQ", ctypes.c_void_p),
        ("Hsig", ctypes.c_void_p), ("jkind", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str):
    """Load an oracle shared library built from hopf_oracle.c and declare its signatures."""
    lib = ctypes.CDLL(path)
    P, V, I64, I32, D = (ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_int64,
                         ctypes.c_int32, ctypes.c_double)
    lib.oh_eval.argtypes = [P, I64, V, V, V, V, V, V, V, V, ctypes.c_int]
    lib.oh_distance_newton.argtypes = [P, I64, V, D, I32, V, V, V, V, V, ctypes.c_int]
    lib.oh_distance_secular.argtypes = [I32, V, V, I32, V, I64, V, V, V, V, V]
    for f in (lib.oh_eval, lib.oh_distance_newton, lib.oh_distance_secular):
        f.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load_library(_LIB)
    return _lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _problem(A, hkind, w, centres, level_set, lam, tol, max_iter, HA=None, jkind="quad"):
    A = _f64(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be n x n")
    w = _f64(w)
    centres = None if centres is None else _f64(centres).reshape(-1, n)
    K = 1 if centres is None else centres.shape[0]
    hk = _HKIND[hkind] if isinstance(hkind, str) else int(hkind)
    HQ = Hsig = None
    if HA is not None:
        # H(p) = sqrt(p^T HA p): its eigendecomposition is a library primitive (numpy.linalg.eigh)
        HA = _f64(HA)
        Hsig, HQ = np.linalg.eigh(0.5 * (HA + HA.T))
        HQ, Hsig = np.ascontiguousarray(HQ), np.ascontiguousarray(Hsig)
    pb = _Problem(n, _ptr(A), K, _ptr(centres), int(bool(level_set)), hk, _ptr(w),
                  float(lam), float(tol), int(max_iter), _ptr(HA), _ptr(HQ), _ptr(Hsig), _JKIND[jkind])
    return pb, (A, w, centres, HA, HQ, Hsig), n, K


def _threads(nthreads):
    if nthreads is None or nthreads <= 0:
        return os.cpu_count() or 1
    return int(nthreads)


def oracle_eval(A, x, t, hkind="wl1", w=None, centres=None, level_set=False, lam=1.0,
                tol=1e-28, max_iter=100000, nthreads=None, with_gap=False, HA=None, jkind="quad"):
    """Hopf evaluation of every point of x (npts x n) at times t (npts).  hkind "al2" takes the
    SPD matrix HA of H(p) = sqrt(p^T HA p); "linf" is H = |p|_inf.  jkind "quad" is
    J(y) = 1/2 y^T A^{-1} y; "l1sq" J = 1/2 |y|_1^2 and "linfsq" J = 1/2 |y|_inf^2 (A is then
    only used for its size: pass the identity)."""
    lib = _load()
    pb, keep, n, K = _problem(A, hkind, w, centres, level_set, lam, tol, max_iter, HA, jkind)
    x = _f64(x).reshape(-1, n)
    t = _f64(t).reshape(-1)
    m = x.shape[0]
    if t.shape[0] != m:
        raise ValueError("t must have one entry per point")
    phi = np.empty(m); grad = np.empty((m, n)); dphidt = np.empty(m)
    iters = np.empty(m, np.int32); kstar = np.empty(m, np.int32)
    gap = np.empty(m) if with_gap else None
    rc = lib.oh_eval(ctypes.byref(pb), m, _ptr(x), _ptr(t), _ptr(phi), _ptr(grad), _ptr(dphidt),
                     _ptr(iters), _ptr(kstar), _ptr(gap), _threads(nthreads))
    if rc == -2:
        raise np.linalg.LinAlgError("A + lambda I (or A) is not symmetric positive definite")
    if rc:
        raise ValueError("oracle_eval: invalid arguments")
    out = dict(phi=phi, grad=grad, dphidt=dphidt, iters=iters, kstar=kstar)
    if with_gap:
        out["gap"] = gap
    return out


def oracle_distance_newton(A, y, centres=None, lam=1.0, tol=1e-28, max_iter=100000,
                           s_tol=1e-13, max_newton=100, nthreads=None):
    """Distance / closest point from each y to the union of ellipsoids c_k + {u^T A^{-1} u <= 1}."""
    lib = _load()
    pb, keep, n, K = _problem(A, "l2", None, centres, True, lam, tol, max_iter)
    y = _f64(y).reshape(-1, n)
    m = y.shape[0]
    dist = np.empty(m); cp = np.empty((m, n))
    kstar = np.empty(m, np.int32); inside = np.empty(m, np.int32); newton = np.empty(m, np.int32)
    rc = lib.oh_distance_newton(ctypes.byref(pb), m, _ptr(y), float(s_tol), int(max_newton),
                                _ptr(dist), _ptr(cp), _ptr(kstar), _ptr(inside), _ptr(newton),
                                _threads(nthreads))
    if rc:
        raise ValueError("oracle_distance_newton failed (%d)" % rc)
    return dict(dist=dist, cp=cp, kstar=kstar, inside=inside, newton=newton)


def oracle_distance_secular(A, y, centres=None):
    """Same distance via the eigenbasis projection (section 4.3)."""
    lib = _load()
    A = _f64(A)
    n = A.shape[0]
    sigma, Q = np.linalg.eigh(0.5 * (A + A.T))
    Q = np.ascontiguousarray(Q)
    sigma = np.ascontiguousarray(sigma)
    centres = None if centres is None else _f64(centres).reshape(-1, n)
    K = 1 if centres is None else centres.shape[0]
    y = _f64(y).reshape(-1, n)
    m = y.shape[0]
    dist = np.empty(m); cp = np.empty((m, n))
    kstar = np.empty(m, np.int32); inside = np.empty(m, np.int32)
    rc = lib.oh_distance_secular(n, _ptr(Q), _ptr(sigma), K, _ptr(centres), m, _ptr(y),
                                 _ptr(dist), _ptr(cp), _ptr(kstar), _ptr(inside))
    if rc:
        raise ValueError("oracle_distance_secular failed (%d)" % rc)
    return dict(dist=dist, cp=cp, kstar=kstar, inside=inside)


def oracle_backward(grad, kstar, t_h, gphi, K=1):
    """Envelope-theorem gradients of L = sum_j gphi_j phi_j.

    phi_j = -F_j(p_j) with F_j(p) = 1/2 p^T A p + <c_k, p> + t_j H(p) - <x_j, p> (+ const),
    which is affine in (x_j, t_j, A, c_k) at fixed p, so at the minimiser p_j (= grad phi_j):
      d phi_j / d x_j = p_j,  d phi_j / d t_j = -H(p_j),
      d phi_j / d A = -1/2 p_j p_j^T,  d phi_j / d c_{k*} = -p_j  (0 for the other k).
    ``t_h`` carries H(p_j) (i.e. -dphidt).
    """
    grad = np.asarray(grad, np.float64)
    gphi = np.asarray(gphi, np.float64).reshape(-1)
    m, n = grad.shape
    gx = gphi[:, None] * grad
    gt = -gphi * np.asarray(t_h, np.float64).reshape(-1)
    gA = -0.5 * (grad * gphi[:, None]).T @ grad
    gc = np.zeros((K, n))
    for k in range(K):
        sel = np.asarray(kstar) == k
        gc[k] = -(gphi[sel, None] * grad[sel]).sum(0)
    return dict(gx=gx, gt=gt, gA=gA, gc=gc)


def oracle_control(A, x, t, grad, kstar=None, centres=None):
    """Optimal-control read-out of section 2 (optimal control and HJ-PDE): the terminal value
    x(T) = ybar, the Hopf-Lax minimiser, for which grad phi = p* lies in dJ(ybar) -- for the
    quadratic J_k(y) = 1/2 (y - c_k)^T A^{-1} (y - c_k) that is ybar = c_k + A p* -- and the
    control beta = (x - x(T)) / t, which is grad H(p*) wherever H is differentiable at p* (the
    paper's beta = grad H(grad phi) and x(T) = x - t grad H(grad phi)), and otherwise the element of
    dH(p*) that the optimality of p* selects (x' - A p* = t beta).  Definition written out."""
    A = _f64(A)
    x = _f64(x)
    p = _f64(grad)
    t = _f64(t).reshape(-1)
    c = np.zeros_like(x)
    if centres is not None:
        C = _f64(centres).reshape(-1, x.shape[1])
        c = C[np.zeros(x.shape[0], np.int64) if kstar is None else np.asarray(kstar)]
    xT = c + p @ A.T
    beta = (x - xT) / t[:, None]
    return dict(beta=beta, xT=xT)


def oracle_max_over_hamiltonians(A, x, t, hkinds, ws=None, **kw):
    """The min-of-Hamiltonians fact of section 2 (extensions): phi for H = min_i H_i with one
    convex J is max_i phi_i, each phi_i the Hopf value for H_i; grad phi and dphi/dt are those of
    the attaining i (the lowest index on ties).  Definition written out over oracle_eval."""
    ws = ws if ws is not None else [None] * len(hkinds)
    rs = [oracle_eval(A, x, t, hk, w=w, **kw) for hk, w in zip(hkinds, ws)]
    phis = np.stack([r["phi"] for r in rs])
    istar = np.argmax(phis, axis=0)
    j = np.arange(phis.shape[1])
    return dict(phi=phis[istar, j], grad=np.stack([r["grad"] for r in rs])[istar, j],
                dphidt=np.stack([r["dphidt"] for r in rs])[istar, j], istar=istar.astype(np.int32))


def linear_control_weights(t, drift, nu):
    """W_i(t) = integral over s in [0, t] of |(e^{-sM} N)_ii| = |nu_i| (1 - e^{-t m_i}) / m_i
    (t |nu_i| for m_i = 0), M = diag(m), N = diag(nu); one row per entry of t."""
    t = _f64(t).reshape(-1, 1)
    m = _f64(drift).reshape(1, -1)
    a = np.abs(_f64(nu)).reshape(1, -1)
    tm = t * m
    safe = np.where(m != 0.0, m, 1.0)
    return a * np.where(m != 0.0, -np.expm1(-tm) / safe, t)


def oracle_eval_linear_control(A, z, t, drift, nu, centres=None, level_set=False, lam=1.0, tol=1e-28,
                               max_iter=100000, nthreads=None):
    """Section 2.2 (some extensions and future work), Hamiltonians of linear controls: the state
    follows dx/ds = M x + N beta(s) with beta(s) in C; with z(s) = e^{-sM} x(s) the Hamiltonian
    becomes H(p, s) = -min_{c in C} <e^{-sM} N c, p>, and for convex J
        phi(z, t) = -min_u ( J*(u) + int_0^t H(u, s) ds - <z, u> ).
    Here M = diag(drift), N = diag(nu) and C = [-1, 1]^n, so H(p, s) = sum_i e^{-s m_i} |nu_i| |p_i|
    and the integral is sum_i W_i(t) |u_i| (``linear_control_weights``).  For each point the
    minimisation is the weighted-l1 Hopf problem (split Bregman, ``oracle_eval``) with weights
    W_i(t) / t at its time t, so that t H = sum_i W_i(t) |u_i|.  grad phi = the minimiser u*;
    dphi/dt = -H(grad phi, t), the HJ equation at time t (the integrand at s = t, not the
    integral).  z is the state in the transformed coordinates; J(y) = 1/2 y^T A^{-1} y (min over
    the translated copies with centres)."""
    from concurrent.futures import ThreadPoolExecutor

    A = _f64(A)
    n = A.shape[0]
    z = _f64(z).reshape(-1, n)
    t = _f64(t).reshape(-1)
    m = z.shape[0]
    if t.shape[0] != m:
        raise ValueError("t must have one entry per point")
    W = linear_control_weights(t, drift, nu)

    def one(j):
        if not (t[j] > 0.0 and np.isfinite(t[j])):  # no evaluation: flagged as invalid
            return dict(phi=np.full(1, np.nan), grad=np.full((1, n), np.nan), dphidt=np.full(1, np.nan),
                        iters=np.full(1, -1, np.int32), kstar=np.full(1, -1, np.int32))
        return oracle_eval(A, z[j:j + 1], t[j:j + 1], "wl1", w=W[j] / t[j], centres=centres,
                           level_set=level_set, lam=lam, tol=tol, max_iter=max_iter, nthreads=1)

    with ThreadPoolExecutor(_threads(nthreads)) as ex:
        rs = list(ex.map(one, range(m)))
    out = {k: np.concatenate([r[k] for r in rs]) for k in ("phi", "grad", "dphidt", "iters", "kstar")}
    inst = np.abs(_f64(nu)).reshape(1, -1) * np.exp(-t.reshape(-1, 1) * _f64(drift).reshape(1, -1))
    ok = np.isfinite(out["phi"])
    out["dphidt"] = np.where(ok, -(inst * np.abs(out["grad"])).sum(1), np.nan)
    return out

