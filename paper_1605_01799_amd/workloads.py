"""Seeded synthetic inputs for the five workloads (and the scaled n=8 variant).

This module only draws inputs.  It holds none of the method's arithmetic and is
the one piece shared by the oracle side (tests, CPU baseline) and the HIP side
(tests, benchmark).  The paper measures on synthetic data only (section 4.5:
points uniform in a box, times uniform); the shapes and distributions here are
those of the five workload definitions, written out in ``WORKLOADS``.

Floating-point inputs are drawn in float64.  Workloads that run in FP32 round
x and t to float32 (``round_inputs``); the oracle is handed those rounded
values upcast to float64, so input rounding is never charged to a kernel.
The problem data (A, w, centres) are float64 on the host on both sides.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 160501799


def rng_for(index: int, *sub: int) -> np.random.Generator:
    """PCG64 generator for workload ``index`` (1..5, or 6 for the scaled n=8 case)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + index, *sub]))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    column signs fixed by sign(diag R) (Mezzadri 2007)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def spd_from_spectrum(Q: np.ndarray, spectrum: np.ndarray) -> np.ndarray:
    """A = Q diag(spectrum) Q^T, symmetrised."""
    A = (Q * spectrum) @ Q.T
    return 0.5 * (A + A.T)


def log_uniform(lo: float, hi: float, size, rng: np.random.Generator) -> np.ndarray:
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


@dataclasses.dataclass
class Problem:
    """One problem: J(y) = 1/2 y^T A^{-1} y (or the min over K translated
    ellipsoid level-set functions), H = hkind with weights w, and its points."""
    n: int
    A: np.ndarray                 # n x n float64 SPD
    hkind: str                    # "wl1" | "l2" | "l2_wl1" | "wl2" | "al2"
    w: Optional[np.ndarray]       # n float64 (None: all ones)
    x: np.ndarray                 # npts x n
    t: np.ndarray                 # npts
    centres: Optional[np.ndarray] = None   # K x n float64
    level_set: bool = False
    A_is_diagonal: bool = False
    spectrum: Optional[np.ndarray] = None  # eigenvalues of A (for reference only)
    HA: Optional[np.ndarray] = None        # n x n SPD matrix of H for hkind "al2"
    drift: Optional[np.ndarray] = None     # n drift diagonal for hkind "linctrl"

    @property
    def npts(self) -> int:
        return self.x.shape[0]

    @property
    def K(self) -> int:
        return 1 if self.centres is None else self.centres.shape[0]


def round_inputs(p: Problem) -> Problem:
    """FP32 workloads: x and t are float32 values (returned as float32 arrays)."""
    return dataclasses.replace(p, x=p.x.astype(np.float32), t=p.t.astype(np.float32))


# --------------------------------------------------------------------------
# The workloads.  Sizes are the full ones; tests take leading slices.
# --------------------------------------------------------------------------
WORKLOADS = {
    1: "n=8, A=I, H=l1, J=1/2|x|^2, 1024 points x~N(0,1)^8, t~U(0.1,2), FP64, lambda=1, "
       "cap 500 iterations, squared residual <= 1e-24",
    2: "n=64, A=Q diag(s) Q^T (Q Haar, s log-uniform [0.1,10]), H=sum w_i|p_i|, w~U(0.5,2), "
       "2^20 points x~N(0,4I), t~U(0.05,3), FP32 inputs",
    3: "n=1024, A as workload 2, H=||p||_2 + sum w_i|p_i|, w~U(0.5,2), 2^16 points x~N(0,4I), "
       "t~U(0.05,3), FP32 inputs, BF16 MFMA products refined by exact anchor products",
    4: "4096 problems, n=round(logU[4,2048]), A=Q diag(a^2) Q^T (a~U(0.5,3)), w~U(0.5,2), one "
       "t~U(0.05,3) per problem, round(logU[1,4096]) points x~N(0,4I), J=min over K=8 ellipsoid "
       "level sets with centres ~N(0,9I); phi (H=wl1), closest point + distance; FP32",
    5: "n=256, A=Q diag(a^2) Q^T (a~U(0.5,3)), J=min over K=4 ellipsoid level sets (centres "
       "~N(0,9I)), H=sum w_i|p_i|, w~U(0.5,2), 2^18 points x~N(0,4I), t~U(0.05,3); forward + "
       "backward wrt x, t, A, centres; FP32",
    6: "workload 1 scaled to 2^24 points (same distributions) for the HBM roofline of the "
       "elementwise path",
}


def workload1(npts: int = 1024) -> Problem:
    rng = rng_for(1)
    n = 8
    x = rng.standard_normal((1024, n))
    t = rng.uniform(0.1, 2.0, 1024)
    return Problem(n=n, A=np.eye(n), hkind="wl1", w=np.ones(n), x=x[:npts], t=t[:npts],
                   A_is_diagonal=True, spectrum=np.ones(n))


def workload_scaled_n8(npts: int = 1 << 24) -> Problem:
    rng = rng_for(6)
    n = 8
    x = rng.standard_normal((npts, n))
    t = rng.uniform(0.1, 2.0, npts)
    return Problem(n=n, A=np.eye(n), hkind="wl1", w=np.ones(n), x=x, t=t,
                   A_is_diagonal=True, spectrum=np.ones(n))


def _dense_problem(index: int, n: int, npts_full: int, npts: int, hkind: str) -> Problem:
    rng = rng_for(index)
    Q = haar_orthogonal(n, rng)
    s = log_uniform(0.1, 10.0, n, rng)
    A = spd_from_spectrum(Q, s)
    w = rng.uniform(0.5, 2.0, n)
    # points drawn in blocks so a prefix never depends on npts
    prng = rng_for(index, 1)
    x = prng.normal(0.0, 2.0, (npts, n))
    trng = rng_for(index, 2)
    t = trng.uniform(0.05, 3.0, npts_full)[:npts]
    return Problem(n=n, A=A, hkind=hkind, w=w, x=x, t=t, spectrum=s)


def workload2(npts: int = 1 << 20) -> Problem:
    return _dense_problem(2, 64, 1 << 20, npts, "wl1")


def workload2_wl2(npts: int = 1 << 20) -> Problem:
    """The n = 64 dense workload with H = sqrt(<p, diag(w) p>) instead of the weighted l1."""
    return _dense_problem(2, 64, 1 << 20, npts, "wl2")


def workload_paper_d(n: int = 16, npts: int = 1 << 20, j_is_d: bool = True) -> Problem:
    """The setting of the paper's timing tables (section 4.5) for the ||.||_D column:
    D_ii = 1 + (i-1)/(n-1), H = sqrt(<p, D p>), J = 1/2 <y, D^{-1} y> (A = D, diagonal) or
    J = 1/2 |y|^2 (A = I); (x, t) uniform in [-10, 10]^n x (0, 10]."""
    rng = rng_for(7, n)
    D = 1.0 + np.arange(n) / (n - 1)
    x = rng.uniform(-10.0, 10.0, (npts, n))
    t = 10.0 - rng.uniform(0.0, 10.0, npts)   # in (0, 10]
    A = D.copy() if j_is_d else np.ones(n)
    return Problem(n=n, A=np.diag(A), hkind="wl2", w=D.copy(), x=x, t=t, A_is_diagonal=True,
                   spectrum=A.copy())


def workload_paper_a(n: int = 16, npts: int = 1 << 20) -> Problem:
    """The paper's timing-table setting (section 4.5) for the ||.||_A column with
    J = 1/2 <y, D^{-1} y>: D_ii = 1 + (i-1)/(n-1), H = sqrt(<p, HA p>) with HA = I + 1 1^T,
    (x, t) uniform in [-10, 10]^n x (0, 10]."""
    rng = rng_for(8, n)
    D = 1.0 + np.arange(n) / (n - 1)
    x = rng.uniform(-10.0, 10.0, (npts, n))
    t = 10.0 - rng.uniform(0.0, 10.0, npts)
    HA = np.eye(n) + np.ones((n, n))
    return Problem(n=n, A=np.diag(D), hkind="al2", w=None, x=x, t=t, A_is_diagonal=True,
                   spectrum=D.copy(), HA=HA)


def workload_paper_norms(n: int = 16, npts: int = 1 << 20, hkind: str = "linf") -> Problem:
    """The paper's timing tables for the squared-norm initial data (section 4.5; Table 5 is
    J = 1/2 |y|_1^2 with H = |p|_inf): (x, t) uniform in [-10, 10]^n x (0, 10].  J is not part of
    the record (the caller picks the squared norm); A is the identity placeholder."""
    rng = rng_for(9, n)
    x = rng.uniform(-10.0, 10.0, (npts, n))
    t = 10.0 - rng.uniform(0.0, 10.0, npts)
    return Problem(n=n, A=np.eye(n), hkind=hkind, w=None, x=x, t=t, A_is_diagonal=True, spectrum=np.ones(n))


def workload_linear_control(n: int = 16, npts: int = 1 << 20) -> Problem:
    """Linear controls with a time-dependent Hamiltonian (section 2.2, extensions; no workload in
    the paper): diagonal A with entries U(0.5, 3), drift diagonal U(-1, 2) with every fifth entry 0,
    input weights U(0.2, 2), transformed states z ~ N(0, 4I), t ~ U(0.05, 3)."""
    rng = rng_for(10, n)
    a = rng.uniform(0.5, 3.0, n)
    drift = rng.uniform(-1.0, 2.0, n)
    drift[::5] = 0.0
    w = rng.uniform(0.2, 2.0, n)
    x = rng.normal(0.0, 2.0, (npts, n))
    t = rng.uniform(0.05, 3.0, npts)
    return Problem(n=n, A=np.diag(a), hkind="linctrl", w=w, x=x, t=t, A_is_diagonal=True, spectrum=a.copy(),
                   drift=drift)


def workload3(npts: int = 1 << 16) -> Problem:
    return _dense_problem(3, 1024, 1 << 16, npts, "l2_wl1")


def workload3_wl2(npts: int = 1 << 16) -> Problem:
    """Workload 3 with H = sqrt(<p, diag(w) p>) (the same A, weights and points)."""
    return _dense_problem(3, 1024, 1 << 16, npts, "wl2")


def workload5(npts: int = 1 << 18) -> Problem:
    rng = rng_for(5)
    n, K = 256, 4
    Q = haar_orthogonal(n, rng)
    a = rng.uniform(0.5, 3.0, n)
    A = spd_from_spectrum(Q, a * a)
    w = rng.uniform(0.5, 2.0, n)
    centres = rng.normal(0.0, 3.0, (K, n))
    x = rng_for(5, 1).normal(0.0, 2.0, (npts, n))
    t = rng_for(5, 2).uniform(0.05, 3.0, 1 << 18)[:npts]
    return Problem(n=n, A=A, hkind="wl1", w=w, x=x, t=t, centres=centres, level_set=True,
                   spectrum=a * a)


# Workload 4: a ragged batch.  Problem sizes are drawn first (cheap) so that any
# subset of problems can be materialised on its own.
W4_PROBLEMS = 4096
W4_K = 8


def workload4_sizes() -> tuple:
    rng = rng_for(4)
    n = np.rint(log_uniform(4, 2048, W4_PROBLEMS, rng)).astype(np.int64)
    P = np.rint(log_uniform(1, 4096, W4_PROBLEMS, rng)).astype(np.int64)
    return n, P


def workload4_problem(i: int, build_A=None) -> Problem:
    """Problem i of workload 4.  build_A(G, spectrum), if given, replaces the host QR and product
    of haar_orthogonal / spd_from_spectrum (same draws, same definition: A = Q diag(spectrum) Q^T
    with Q the sign-fixed QR factor of the Gaussian G), e.g. by a device implementation."""
    n_all, P_all = workload4_sizes()
    n, P = int(n_all[i]), int(P_all[i])
    rng = rng_for(4, 10 + i)
    if build_A is None:
        Q = haar_orthogonal(n, rng)
        a = rng.uniform(0.5, 3.0, n)
        A = spd_from_spectrum(Q, a * a)
    else:
        G = rng.standard_normal((n, n))
        a = rng.uniform(0.5, 3.0, n)
        A = build_A(G, a * a)
    w = rng.uniform(0.5, 2.0, n)
    t = float(rng.uniform(0.05, 3.0))
    centres = rng.normal(0.0, 3.0, (W4_K, n))
    x = rng.normal(0.0, 2.0, (P, n))
    return Problem(n=n, A=A, hkind="wl1", w=w, x=x, t=np.full(P, t), centres=centres,
                   level_set=True, spectrum=a * a)


def workload4(indices=None) -> List[Problem]:
    if indices is None:
        indices = range(W4_PROBLEMS)
    return [workload4_problem(int(i)) for i in indices]
