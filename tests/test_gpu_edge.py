"""Edge cases of the HIP path through the C ABI: empty and one-point calls, invalid points
(t <= 0, non-finite inputs) mixed with valid ones, the iteration cap, padding at every
residue of n modulo the tile, the largest n, the diagonal path beyond its register sizes,
empty problems inside a ragged batch, points inside the union, and argument errors."""
import ctypes

import numpy as np
import pytest

from tests.helpers import rand_problem, rel_err_phi, rel_err_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1605_01799_amd import _lib  # noqa: E402
from paper_1605_01799_amd import hopf as H  # noqa: E402
from paper_1605_01799_amd import workloads as W  # noqa: E402

DEV = "cuda:0"
REFINED_TOL = 1e-6
FP32_TOL = 1e-6   # FP32 increments on exact anchors (test_gpu_parity)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("precision", ["bf16_refined", "f32"])
def test_zero_and_one_point(oracle_lib, precision):
    rng = np.random.default_rng(1)
    n = 40
    A = rand_problem(n, rng)
    prob = H.Problem(A, hkind="l2", precision=precision, tol=1e-16 * n)
    out = prob.eval(torch.empty(0, n, device=DEV), torch.empty(0, device=DEV))
    torch.cuda.synchronize()
    assert out["phi"].numel() == 0
    x = rng.normal(0, 2, (1, n)).astype(np.float32)
    t = np.array([0.7], np.float32)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    ref = oracle_lib.oracle_eval(A, x.astype(np.float64), t.astype(np.float64), "l2", tol=1e-28)
    bound = REFINED_TOL if precision == "bf16_refined" else FP32_TOL
    assert rel_err_phi(out["phi"].cpu().numpy(), ref["phi"]).max() <= bound


@pytest.mark.parametrize("precision", ["bf16_refined", "f32"])
def test_invalid_points_are_flagged(oracle_lib, precision):
    rng = np.random.default_rng(2)
    n, npts = 70, 80
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    bad_t = [3, 17, 18, 79]
    t[3], t[17], t[18], t[79] = 0.0, -1.0, np.nan, np.inf
    x[40, 5] = np.nan
    x[41, 0] = np.inf
    bad = sorted(bad_t + [40, 41])
    good = np.setdiff1d(np.arange(npts), bad)
    prob = H.Problem(A, hkind="l2_wl1", w=w, precision=precision,
                     tol=1e-16 * n)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    it = out["iters"].cpu().numpy()
    assert np.all(it[bad] == -1)
    assert np.all(np.isnan(out["phi"].cpu().numpy()[bad]))
    assert np.all(np.isnan(out["grad"].cpu().numpy()[bad]))
    assert np.all(it[good] > 0)
    ref = oracle_lib.oracle_eval(A, x[good].astype(np.float64), t[good].astype(np.float64), "l2_wl1", w=w,
                                 tol=1e-28)
    bound = REFINED_TOL if precision == "bf16_refined" else FP32_TOL
    assert rel_err_vec(out["grad"].cpu().numpy()[good], ref["grad"]).max() <= bound


@pytest.mark.parametrize("precision", ["bf16_refined", "f32"])
def test_iteration_cap(precision):
    rng = np.random.default_rng(3)
    n, npts = 50, 65
    A = rand_problem(n, rng)
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    prob = H.Problem(A, hkind="wl1", precision=precision, tol=0.0, max_iter=7)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    assert np.all(out["iters"].cpu().numpy() == -2)
    assert np.all(np.isfinite(out["phi"].cpu().numpy()))
    assert np.all(np.isfinite(out["grad"].cpu().numpy()))


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 31, 32, 33, 63, 65, 127, 129, 255, 257])
def test_padding_residues(oracle_lib, n):
    rng = np.random.default_rng(100 + n)
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    npts = 67
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    prob = H.Problem(A, hkind="l2_wl1", w=w, precision="bf16_refined", tol=1e-16 * n)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    ref = oracle_lib.oracle_eval(A, x.astype(np.float64), t.astype(np.float64), "l2_wl1", w=w, tol=1e-28)
    assert rel_err_vec(out["grad"].cpu().numpy(), ref["grad"]).max() <= REFINED_TOL
    assert rel_err_phi(out["phi"].cpu().numpy(), ref["phi"]).max() <= REFINED_TOL


def test_refined_wide_scales(oracle_lib):
    """The refined anchors take M and every right-hand side in integer slices under one
    power-of-two scale per row and per column: coordinates spread over three decades (per
    coordinate) put small and large entries in the same right-hand side."""
    rng = np.random.default_rng(4242)
    n, npts = 96, 64
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    scale = 10.0 ** rng.uniform(-1.5, 1.5, n)
    x = (rng.normal(0, 2, (npts, n)) * scale).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    print("case wide scales n=%d npts=%d bf16_refined" % (n, npts), flush=True)
    # the stopping rule is absolute: scaled with the largest coordinate scale squared
    prob = H.Problem(A, hkind="l2_wl1", w=w, precision="bf16_refined", tol=1e-16 * n * scale.max() ** 2,
                     max_iter=20000)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    assert (out["iters"].cpu().numpy() != -1).all()
    ref = oracle_lib.oracle_eval(A, x.astype(np.float64), t.astype(np.float64), "l2_wl1", w=w, tol=1e-28)
    assert rel_err_vec(out["grad"].cpu().numpy(), ref["grad"]).max() <= REFINED_TOL
    assert rel_err_phi(out["phi"].cpu().numpy(), ref["phi"]).max() <= REFINED_TOL


def test_largest_n(oracle_lib):
    rng = np.random.default_rng(2048)
    n, npts = 2048, 40
    Q = W.haar_orthogonal(n, rng)
    A = W.spd_from_spectrum(Q, W.log_uniform(0.1, 10, n, rng))
    w = rng.uniform(0.5, 2, n)
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    prob = H.Problem(A, hkind="l2_wl1", w=w, precision="bf16_refined", tol=1e-16 * n)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    idx = np.array([0, 1, 2, npts - 1])
    ref = oracle_lib.oracle_eval(A, x[idx].astype(np.float64), t[idx].astype(np.float64), "l2_wl1", w=w,
                                 tol=1e-28, nthreads=4)
    assert rel_err_vec(out["grad"].cpu().numpy()[idx], ref["grad"]).max() <= REFINED_TOL
    assert rel_err_phi(out["phi"].cpu().numpy()[idx], ref["phi"]).max() <= REFINED_TOL
    with pytest.raises(_lib.HopfError) as e:
        H.Problem(n=2049, precision="f32")
    assert e.value.status == _lib.HOPF_EINVAL


@pytest.mark.parametrize("n", [3, 8, 9, 16, 17, 32, 33, 100])
@pytest.mark.parametrize("hk", ["wl1", "l2", "l2_wl1"])
def test_diagonal_fp64_union(oracle_lib, n, hk):
    """Diagonal A in FP64 (n <= 32: one thread per point and copy; larger n: the dense path
    is refused for FP64) with a union of level sets."""
    rng = np.random.default_rng(7 * n)
    a = rng.uniform(0.3, 4, n)
    w = rng.uniform(0.5, 2, n)
    C = rng.normal(0, 2, (3, n))
    npts = 130
    x = rng.normal(0, 2, (npts, n))
    t = rng.uniform(0.05, 3, npts)
    if n > 32:
        with pytest.raises(_lib.HopfError):
            prob = H.Problem(a, diagonal=True, centres=C, level_set=True, hkind=hk, w=w, precision="f64")
            prob.eval(dev(x), dev(t))
        return
    prob = H.Problem(a, diagonal=True, centres=C, level_set=True, hkind=hk, w=w, precision="f64", tol=1e-26,
                     max_iter=100000)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    ref = oracle_lib.oracle_eval(np.diag(a), x, t, hk, w=w, centres=C, level_set=True, tol=1e-28)
    assert rel_err_phi(out["phi"].cpu().numpy(), ref["phi"]).max() <= 1e-10
    ks = out["kstar"].cpu().numpy()
    agree = ks == ref["kstar"]
    assert agree.mean() >= 0.97
    assert rel_err_vec(out["grad"].cpu().numpy()[agree], ref["grad"][agree]).max() <= 1e-8


def test_diagonal_large_n_f32(oracle_lib):
    """A diagonal A beyond the per-thread sizes runs on the dense path as a dense matrix."""
    rng = np.random.default_rng(9)
    n, npts = 200, 70
    a = rng.uniform(0.3, 4, n)
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    prob = H.Problem(a, diagonal=True, hkind="wl1", precision="bf16_refined", tol=1e-16 * n)
    out = prob.eval(dev(x), dev(t))
    torch.cuda.synchronize()
    pcf = np.sign(x) * np.maximum(np.abs(x.astype(np.float64)) - t[:, None], 0) / a
    assert rel_err_vec(out["grad"].cpu().numpy(), pcf).max() <= REFINED_TOL


def test_ragged_with_empty_problems(oracle_lib):
    rng = np.random.default_rng(11)
    specs, xs, ts, refs = [], [], [], []
    for q, (n, P) in enumerate([(5, 0), (40, 3), (17, 0), (100, 70), (3, 1), (64, 0)]):
        A = rand_problem(n, rng)
        w = rng.uniform(0.5, 2, n)
        specs.append(dict(A=A, hkind="wl1", w=w, precision="bf16_refined", tol=1e-16 * n))
        x = rng.normal(0, 2, (P, n)).astype(np.float32)
        t = rng.uniform(0.05, 3, P).astype(np.float32)
        xs.append(dev(x))
        ts.append(dev(t))
        refs.append(oracle_lib.oracle_eval(A, x.astype(np.float64), t.astype(np.float64), "wl1", w=w, tol=1e-28)
                    if P else None)
    probs = H.Problem.batch(specs)
    out = H.eval_ragged(probs, xs, ts)
    torch.cuda.synchronize()
    off = out["offsets"]
    for q, r in enumerate(refs):
        if r is None:
            continue
        assert rel_err_vec(out["grad"][q].cpu().numpy(), r["grad"]).max() <= REFINED_TOL
        assert rel_err_phi(out["phi"].cpu().numpy()[off[q]:off[q + 1]], r["phi"]).max() <= REFINED_TOL


def test_closest_point_inside_and_unit_ball():
    n = 12
    # unit ball: dist = |y| - 1, cp = y / |y|
    prob = H.Problem(np.eye(n), centres=np.zeros((1, n)), level_set=True, hkind="l2", precision="bf16_refined",
                     tol=1e-16 * n)
    rng = np.random.default_rng(12)
    y = rng.normal(0, 1, (50, n))
    y *= (rng.uniform(0.2, 5, 50) / np.linalg.norm(y, axis=1))[:, None]
    y = y.astype(np.float32)
    out = prob.closest_point(dev(y), s_tol=1e-7)
    torch.cuda.synchronize()
    r = np.linalg.norm(y.astype(np.float64), axis=1)
    inside = r <= 1
    assert np.array_equal(out["inside"].cpu().numpy().astype(bool), inside)
    d = out["dist"].cpu().numpy()
    assert np.all(d[inside] == 0)
    assert np.abs(d[~inside] - (r[~inside] - 1)).max() <= 1e-5
    cp = out["cp"].cpu().numpy()
    assert np.array_equal(cp[inside], y[inside])
    assert np.abs(cp[~inside] - y[~inside] / r[~inside, None]).max() <= 1e-5


def test_argument_errors():
    lib = _lib.load()
    dense = np.eye(4) + 0.1
    for A, kw in ((None, dict(n=0)), (None, dict(n=4, lam=0.0)), (None, dict(n=4, lam=-1.0)),
                  (None, dict(n=4, tol=-1.0)), (None, dict(n=4, max_iter=0)),
                  (dense, dict(precision="f64")),                     # FP64 is the diagonal path only
                  (dense - 0.2 * np.tri(4, k=-1), dict(precision="f32")),   # not symmetric
                  (np.full(4, -1.0), dict(diagonal=True, precision="f32")),  # not positive
                  (None, dict(n=4, w=-np.ones(4), precision="f32"))):
        with pytest.raises(_lib.HopfError) as e:
            H.Problem(A, **kw)
        assert e.value.status in (_lib.HOPF_EINVAL, _lib.HOPF_ENOTSPD)
    prob = H.Problem(np.eye(4), precision="f32")
    st = lib.hopf_eval(prob._handle, 5, None, None, None, None, None, None, None, None)
    assert st == _lib.HOPF_EINVAL
    assert b"NULL" in lib.hopf_last_error() or len(lib.hopf_last_error()) > 0
    st = lib.hopf_eval(prob._handle, -1, None, None, None, None, None, None, None, None)
    assert st == _lib.HOPF_EINVAL
    # a level-set distance on a problem that is not a level set is refused
    y = torch.zeros(3, 4, device=DEV)
    with pytest.raises(_lib.HopfError):
        prob.closest_point(y)
    # K = 0 through the raw descriptor
    d = prob._desc()
    d.K = 0
    h = ctypes.c_void_p()
    assert lib.hopf_problem_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.HOPF_EINVAL
