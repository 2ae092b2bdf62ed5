"""GPU parity for the time-dependent Hamiltonian of linear controls (section 2.2, some extensions
and future work; ABI kind HOPF_H_LINCTRL): dx/ds = M x + N beta, beta in [-1, 1]^n,
M = diag(drift), N = diag(w); in the variables z = e^{-sM} x, H(p, s) = sum e^{-s m_i} w_i |p_i|
and phi(z, t) = -min_u (J*(u) + int_0^t H(u, s) ds - <z, u>).  The per-thread kernel through the
C ABI against the FP64 oracle (oracle_eval_linear_control) element by element: FP64 at n in
{4, 8, 16, 32} with drifts of both signs and zero (1e-10), FP32 I/O (1e-6), translated level
sets (the union), A = I, invalid times; against the separable closed form for diagonal A; the
no-drift case against the static weighted-l1 path; and the calls that refuse the kind."""
import numpy as np
import pytest

from tests.helpers import rel_err_phi, rel_err_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1605_01799_amd import hopf as H  # noqa: E402

DEV = "cuda:0"
FP64_TOL = 1e-10
FP32_TOL = 1e-6


def make(n, npts, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 3, n)
    drift = rng.uniform(-1.0, 2.0, n)
    drift[::5] = 0.0
    w = rng.uniform(0.2, 2.0, n)
    z = rng.normal(0, 2, (npts, n))
    t = rng.uniform(0.05, 3, npts)
    return a, drift, w, z, t


def gpu(prob, z, t, dtype):
    out = prob.eval(torch.from_numpy(z.astype(dtype)).to(DEV), torch.from_numpy(t.astype(dtype)).to(DEV))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(out, ref, bound, label):
    ep = rel_err_vec(out["grad"], ref["grad"])
    ef = rel_err_phi(out["phi"], ref["phi"])
    et = rel_err_phi(out["dphidt"], ref["dphidt"])
    print("  %s: max err grad %.2e phi %.2e dphidt %.2e iters med %d" %
          (label, ep.max(), ef.max(), et.max(), np.median(out["iters"])), flush=True)
    assert ep.max() <= bound and ef.max() <= bound and et.max() <= bound


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_fp64(oracle_lib, n):
    a, drift, w, z, t = make(n, 400, 7000 + n)
    print("case linctrl fp64 n=%d" % n, flush=True)
    prob = H.Problem(a, diagonal=True, hkind="linctrl", w=w, drift=drift, precision="f64", tol=1e-26,
                     max_iter=20000)
    out = gpu(prob, z, t, np.float64)
    ref = oracle_lib.oracle_eval_linear_control(np.diag(a), z, t, drift, w, tol=1e-26)
    assert np.all(out["iters"] > 0)
    check(out, ref, FP64_TOL, "linctrl fp64 n=%d" % n)
    # the separable closed form: u_i = shrink(z_i, W_i) / a_i, phi = sum (|z_i| - W_i)_+^2 / (2 a_i)
    W = np.abs(w)[None, :] * np.where(drift != 0, -np.expm1(-t[:, None] * drift[None, :]) /
                                      np.where(drift != 0, drift, 1.0)[None, :], t[:, None])
    m = np.maximum(np.abs(z) - W, 0)
    assert rel_err_phi(out["phi"], (m ** 2 / (2 * a)).sum(1)).max() <= FP64_TOL
    assert rel_err_vec(out["grad"], np.sign(z) * m / a).max() <= FP64_TOL


def test_fp32_io(oracle_lib):
    a, drift, w, z, t = make(16, 400, 7100)
    z32, t32 = z.astype(np.float32), t.astype(np.float32)
    prob = H.Problem(a, diagonal=True, hkind="linctrl", w=w, drift=drift, precision="f32", tol=1e-24,
                     max_iter=20000)
    out = gpu(prob, z32, t32, np.float32)
    ref = oracle_lib.oracle_eval_linear_control(np.diag(a), z32.astype(np.float64), t32.astype(np.float64),
                                                drift, w, tol=1e-26)
    check(out, ref, FP32_TOL, "linctrl fp32 I/O")


def test_union_and_identity(oracle_lib):
    n, K = 12, 3
    a, drift, w, z, t = make(n, 300, 7200)
    C = np.random.default_rng(7201).normal(0, 2, (K, n))
    prob = H.Problem(a, diagonal=True, hkind="linctrl", w=w, drift=drift, centres=C, level_set=True,
                     precision="f64", tol=1e-26, max_iter=20000)
    out = gpu(prob, z, t, np.float64)
    ref = oracle_lib.oracle_eval_linear_control(np.diag(a), z, t, drift, w, centres=C, level_set=True, tol=1e-26)
    check(out, ref, FP64_TOL, "linctrl union K=3")
    assert np.array_equal(out["kstar"], ref["kstar"])
    prob = H.Problem(None, n=n, hkind="linctrl", w=w, drift=drift, precision="f64", tol=1e-26, max_iter=20000)
    out = gpu(prob, z, t, np.float64)
    ref = oracle_lib.oracle_eval_linear_control(np.eye(n), z, t, drift, w, tol=1e-26)
    check(out, ref, FP64_TOL, "linctrl A = I")


def test_no_drift_is_the_static_problem():
    a, drift, w, z, t = make(8, 300, 7300)
    lc = H.Problem(a, diagonal=True, hkind="linctrl", w=w, drift=np.zeros(8), precision="f64", tol=1e-26,
                   max_iter=20000)
    st = H.Problem(a, diagonal=True, hkind="wl1", w=w, precision="f64", tol=1e-26, max_iter=20000)
    o1, o2 = gpu(lc, z, t, np.float64), gpu(st, z, t, np.float64)
    for k in ("phi", "grad", "dphidt"):
        assert np.allclose(o1[k], o2[k], rtol=1e-12, atol=1e-12), k


def test_invalid_times_and_refusals():
    a, drift, w, z, t = make(8, 6, 7400)
    t[1] = 0.0
    t[2] = np.nan
    prob = H.Problem(a, diagonal=True, hkind="linctrl", w=w, drift=drift, precision="f64", tol=1e-26,
                     max_iter=20000)
    out = gpu(prob, z, t, np.float64)
    assert np.isnan(out["phi"][1]) and np.isnan(out["phi"][2]) and out["iters"][1] == -1
    assert np.isfinite(out["phi"][[0, 3, 4, 5]]).all()
    with pytest.raises(H._lib.HopfError):   # no drift given
        H.Problem(a, diagonal=True, hkind="linctrl", w=w, precision="f64")
    with pytest.raises(H._lib.HopfError):   # dense A: not on the per-thread path
        H.Problem(np.diag(a), hkind="linctrl", w=w, drift=drift, precision="f32")
    f32 = H.Problem(a, diagonal=True, hkind="linctrl", w=w, drift=drift, precision="f32")
    x = torch.from_numpy(z.astype(np.float32)).to(DEV)
    tt = torch.from_numpy(np.abs(t).astype(np.float32) + 0.1).to(DEV)
    with pytest.raises(H._lib.HopfError):   # ragged batches run the dense kernels
        H.eval_ragged([f32], [x], [tt])
