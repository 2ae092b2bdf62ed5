"""Pins of the oracle's time-dependent Hamiltonian for linear controls (section 2.2, some
extensions and future work): dx/ds = M x + N beta, beta in [-1, 1]^n, M = diag(m), N = diag(nu);
with z = e^{-sM} x, H(p, s) = sum_i e^{-s m_i} |nu_i| |p_i| and
phi(z, t) = -min_u (J*(u) + int_0^t H(u, s) ds - <z, u>).

Each pin is fixed by something other than the oracle's own formulas:
* the integral by numerical quadrature (scipy.integrate.quad) of the definition of H(p, s);
* diagonal A: the minimisation separates per coordinate, u_i = shrink(z_i, W_i) / a_i and
  phi = sum (|z_i| - W_i)_+^2 / (2 a_i), with W_i from the quadrature;
* dense A at n = 2: brute-force minimisation over a fine grid, W_i from the quadrature;
* the HJ equation: central differences of phi in t against dphi/dt = -H(grad phi, t), the
  integrand at s = t (this separates the integral from t H(., t));
* no drift (m = 0): the static weighted-l1 problem with w = |nu| at time t;
and a set of planted mistakes (each a plausible slip in the formula) fails at least one pin."""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from tests.helpers import rand_problem

M_DRIFT = np.array([0.0, 0.8, -0.4, 2.5, 0.05])
NU = np.array([1.0, -1.5, 0.7, 2.0, -0.3])


def quad_weights(t, m, nu):
    return np.array([quad(lambda s, mi=mi, ai=ai: abs(np.exp(-s * mi) * ai), 0.0, t, epsabs=1e-14,
                          epsrel=1e-13)[0] for mi, ai in zip(m, nu)])


def pin_integral(impl_w):
    for t in (0.3, 1.0, 2.7):
        W = impl_w([t], M_DRIFT, NU)[0]
        if not np.allclose(W, quad_weights(t, M_DRIFT, NU), rtol=1e-11, atol=0):
            return False
    return True


def pin_separable(impl):
    rng = np.random.default_rng(11)
    n = len(M_DRIFT)
    a = rng.uniform(0.5, 3, n)
    z = rng.normal(0, 2, (30, n))
    t = rng.uniform(0.05, 3, 30)
    r = impl(np.diag(a), z, t, M_DRIFT, NU)
    for j in range(30):
        W = quad_weights(t[j], M_DRIFT, NU)
        u = np.sign(z[j]) * np.maximum(np.abs(z[j]) - W, 0) / a
        phi = np.sum(np.maximum(np.abs(z[j]) - W, 0) ** 2 / (2 * a))
        dt = -np.sum(np.exp(-t[j] * M_DRIFT) * np.abs(NU) * np.abs(u))
        if not (abs(r["phi"][j] - phi) <= 1e-10 * max(1, abs(phi)) and np.allclose(r["grad"][j], u, atol=1e-9)
                and abs(r["dphidt"][j] - dt) <= 1e-9 * max(1, abs(dt))):
            return False
    return True


def pin_brute_force(impl):
    rng = np.random.default_rng(12)
    A = rand_problem(2, rng)
    m, nu = np.array([0.9, -0.3]), np.array([1.2, -0.8])
    z = np.array([[1.5, -2.0], [0.3, 2.5], [-2.2, -0.4]])
    t = np.array([0.7, 1.9, 1.2])
    r = impl(A, z, t, m, nu)
    g = np.linspace(-8, 8, 3201)
    U1, U2 = np.meshgrid(g, g, indexing="ij")
    for j in range(3):
        W = quad_weights(t[j], m, nu)
        f = (0.5 * (A[0, 0] * U1 ** 2 + 2 * A[0, 1] * U1 * U2 + A[1, 1] * U2 ** 2) + W[0] * np.abs(U1)
             + W[1] * np.abs(U2) - z[j, 0] * U1 - z[j, 1] * U2)
        if abs(r["phi"][j] - (-f.min())) > 2e-4:
            return False
    return True


def pin_pde(impl):
    rng = np.random.default_rng(13)
    n = len(M_DRIFT)
    A = rand_problem(n, rng)
    z = rng.normal(0, 3, (12, n))
    t = rng.uniform(0.3, 2.5, 12)
    h = 1e-5
    r = impl(A, z, t, M_DRIFT, NU)
    rp = impl(A, z, t + h, M_DRIFT, NU)
    rm = impl(A, z, t - h, M_DRIFT, NU)
    fd = (rp["phi"] - rm["phi"]) / (2 * h)
    return bool(np.all(np.abs(fd - r["dphidt"]) <= 1e-6 * np.maximum(1, np.abs(fd))))


def pin_no_drift(impl):
    rng = np.random.default_rng(14)
    n = len(NU)
    A = rand_problem(n, rng)
    z = rng.normal(0, 2, (20, n))
    t = rng.uniform(0.05, 3, 20)
    r = impl(A, z, t, np.zeros(n), NU)
    s = oracle.oracle_eval(A, z, t, "wl1", w=np.abs(NU), tol=1e-28)
    return bool(np.allclose(r["phi"], s["phi"], rtol=1e-12, atol=1e-12)
                and np.allclose(r["grad"], s["grad"], rtol=1e-10, atol=1e-10)
                and np.allclose(r["dphidt"], s["dphidt"], rtol=1e-10, atol=1e-10))


def all_pins(impl, impl_w):
    """Each pin's result (a pin whose implementation raises counts as failed)."""
    def run(f, arg):
        try:
            return f(arg)
        except (ValueError, FloatingPointError, np.linalg.LinAlgError):
            return False
    return dict(integral=run(pin_integral, impl_w), separable=run(pin_separable, impl),
                brute=run(pin_brute_force, impl), pde=run(pin_pde, impl), no_drift=run(pin_no_drift, impl))


def test_oracle_passes_every_pin():
    res = all_pins(oracle.oracle_eval_linear_control, oracle.linear_control_weights)
    assert all(res.values()), res


def test_invalid_time_is_flagged():
    r = oracle.oracle_eval_linear_control(np.eye(5), np.ones((2, 5)), [0.0, 1.0], M_DRIFT, NU)
    assert np.isnan(r["phi"][0]) and np.isnan(r["dphidt"][0]) and np.isfinite(r["phi"][1])


# ---- planted mistakes: each variant must fail at least one pin
def _variant(weights, inst):
    def impl(A, z, t, drift, nu, **kw):
        t = np.asarray(t, float).reshape(-1)
        W = weights(t, drift, nu)
        rs = [oracle.oracle_eval(A, z[j:j + 1], t[j:j + 1], "wl1", w=W[j] / t[j], tol=1e-28) for j in range(len(t))]
        out = {k: np.concatenate([r[k] for r in rs]) for k in ("phi", "grad")}
        out["dphidt"] = -(inst(t, drift, nu) * np.abs(out["grad"])).sum(1)
        return out
    return impl


def _w_ok(t, m, nu):
    return oracle.linear_control_weights(t, m, nu)


def _inst_ok(t, m, nu):
    return np.abs(nu)[None, :] * np.exp(-np.asarray(t).reshape(-1, 1) * m[None, :])


MISTAKES = {
    # t H(., t) in place of the integral
    "rectangle rule": (lambda t, m, nu: np.asarray(t).reshape(-1, 1) * _inst_ok(t, m, nu), _inst_ok),
    # e^{+sM} (the wrong direction of the change of variables)
    "drift sign": (lambda t, m, nu: oracle.linear_control_weights(t, -np.asarray(m), nu),
                   lambda t, m, nu: np.abs(nu)[None, :] * np.exp(np.asarray(t).reshape(-1, 1) * m[None, :])),
    # nu without its absolute value (the box's support function is |.|)
    "signed nu": (lambda t, m, nu: oracle.linear_control_weights(t, m, np.abs(nu)) * np.sign(nu)[None, :],
                  lambda t, m, nu: nu[None, :] * np.exp(-np.asarray(t).reshape(-1, 1) * m[None, :])),
    # dphi/dt from the time-averaged weights instead of the integrand at s = t
    "averaged dphi/dt": (_w_ok, lambda t, m, nu: oracle.linear_control_weights(t, m, nu) /
                         np.asarray(t).reshape(-1, 1)),
}


@pytest.mark.parametrize("name", list(MISTAKES))
def test_planted_mistake_is_caught(name):
    wf, inst = MISTAKES[name]
    impl = _variant(lambda t, m, nu: wf(t, m, nu), inst)
    res = all_pins(impl, wf)
    assert not all(res.values()), (name, res)
