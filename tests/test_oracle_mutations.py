"""Planted mistakes: each mutant of the oracle source (a dropped term, a flipped sign, a
transposed operand, a wrong index or comparison) must fail at least one pin.  The mutants
are compiled into a temporary directory on the CPU and never touch the real oracle."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle.oracle as O

SRC = os.path.join(os.path.dirname(O.__file__), "hopf_oracle.c")

MUTANTS = {
    "bregman_update_sign": ("s->b[i] + s->vn[i] - s->dn[i]", "s->b[i] - s->vn[i] + s->dn[i]"),
    "rhs_drops_lambda": ("xp[i] + lam * (s->d[i] - s->b[i])", "xp[i] + (s->d[i] - s->b[i])"),
    "rhs_sign_b": ("lam * (s->d[i] - s->b[i])", "lam * (s->d[i] + s->b[i])"),
    "threshold_times_lambda": ("const double theta = t / lam;", "const double theta = t * lam;"),
    "shrink2_sign": ("(nr - theta > 0.0 ? nr - theta : 0.0) / nr", "(nr + theta > 0.0 ? nr + theta : 0.0) / nr"),
    "shrink1_ignores_weights": ("d[i] = shrink1(z[i], theta * wgt(w, i));", "d[i] = shrink1(z[i], theta);"),
    "backsolve_transposed": ("ks_add(&k, -L[(size_t)m * n + i] * out[m]);", "ks_add(&k, -L[(size_t)i * n + m] * out[m]);"),
    "cholesky_sign": ("ks_add(&k, -L[(size_t)j * n + m] * L[(size_t)j * n + m]);", "ks_add(&k, L[(size_t)j * n + m] * L[(size_t)j * n + m]);"),
    "value_drops_H": ("ks_add(&F, t * ham(pb, hkind, p));", "ks_add(&F, 0.0);"),
    "value_half_missing": ("ks_add(&F, 0.5 * quad(n, pb->A, p));", "ks_add(&F, quad(n, pb->A, p));"),
    "union_max_not_min": ("if (val < best || kb < 0)", "if (val > best || kb < 0)"),
    "level_set_offset_sign": ("if (pb->level_set) val -= 0.5;", "if (pb->level_set) val += 0.5;"),
    "newton_step_sign": ("sv += ds;", "sv -= ds;"),
    "dphidt_sign": ("J->dphidt[j] = -ham(", "J->dphidt[j] = ham("),
    "centre_sign": ("xp[i] = x[i] - (pb->centres", "xp[i] = x[i] + (pb->centres"),
    "wl2_multiplier_equation_rhs": ("ks_add(&g, 1.0);", "ks_add(&g, 0.5);"),
    "wl2_prox_wrong_factor": ("d[i] = mu * z[i] / (s + mu);", "d[i] = s * z[i] / (s + mu);"),
    "wl2_hamiltonian_unweighted": ("ks_add(&k, wgt(w, i) * p[i] * p[i]);", "ks_add(&k, p[i] * p[i]);"),
    "al2_rotation_transposed": ("ks_add(&k, Q[(size_t)i * n + a] * z[i]);", "ks_add(&k, Q[(size_t)a * n + i] * z[i]);"),
    "al2_back_rotation_dropped": ("ks_add(&k, Q[(size_t)i * n + a] * du[a]);", "ks_add(&k, (i == a) * du[a]);"),
    "linf_ball_radius": ("const double mu = breakpoint_root(n, z, 1.0, 0.0, theta, bp);",
                         "const double mu = breakpoint_root(n, z, 1.0, 0.0, 0.5 * theta, bp);"),
    "l1sq_threshold_equation": ("breakpoint_root(n, z, alpha, 1.0, 0.0, bp)", "breakpoint_root(n, z, 1.0, alpha, 0.0, bp)"),
    "linfsq_conjugate_scale": ("prox_l1sq(n, 1.0 / alpha, z, tmp, bp);", "prox_l1sq(n, alpha, z, tmp, bp);"),
    "breakpoint_interpolation": ("return lo + flo * (hi - lo) / (flo - fhi);", "return lo + fhi * (hi - lo) / (flo - fhi);"),
    "secular_projection_index": ("us[a] = sigma[a] * u[a] / (sigma[a] + mu);", "us[a] = sigma[a] * u[a] / (sigma[a] + mu * mu);"),
}


def battery(lib):
    """Quick pins; returns the names of those that fail."""
    old = O._lib
    O._lib = lib
    fails = []
    rng = np.random.default_rng(0)
    try:
        def check(name, fn):
            try:
                if not fn():
                    fails.append(name)
            except Exception:
                fails.append(name)

        n = 6
        a = rng.uniform(0.5, 3, n)
        w = rng.uniform(0.5, 2, n)
        x = rng.normal(0, 3, (8, n))
        t = rng.uniform(0.1, 2, 8)

        def ellipsoid_cf():
            r = O.oracle_eval(np.diag(a * a), x, t, "wl1", w=w, level_set=True, tol=1e-26, max_iter=20000)
            ex = np.maximum(np.abs(x) - t[:, None] * w, 0)
            ok = np.allclose(r["phi"], -0.5 + 0.5 * ((ex / a) ** 2).sum(1), atol=1e-9)
            ok &= np.allclose(r["dphidt"], -(w * np.abs(r["grad"])).sum(1), atol=1e-9)
            return ok and np.allclose(r["grad"], np.sign(x) * ex / (a * a), atol=1e-9)
        check("ellipsoid_cf", ellipsoid_cf)

        def sphere_cf():
            r = O.oracle_eval(np.eye(n), x, t, "l2", level_set=True, tol=1e-26, max_iter=20000)
            nx = np.linalg.norm(x, axis=1)
            return np.allclose(r["phi"], np.where(nx > t, 0.5 * (nx - t) ** 2 - 0.5, -0.5), atol=1e-9)
        check("sphere_cf", sphere_cf)

        Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
        A = (Q * rng.uniform(0.2, 5, n)) @ Q.T
        A = 0.5 * (A + A.T)

        def kkt():
            from tests.test_oracle_pins import kkt_residual
            ok = True
            for hk in ("wl1", "l2", "l2_wl1", "wl2"):
                for lam in (1.0, 0.4):
                    r = O.oracle_eval(A, x, t, hk, w=w, lam=lam, tol=1e-26, max_iter=20000)
                    ok &= all(kkt_residual(A, x[j], t[j], r["grad"][j], hk, w) < 1e-7 for j in range(8))
            return ok
        check("kkt", kkt)

        def wl2_scaled_l2():
            r = O.oracle_eval(A, x, t, "wl2", w=np.full(n, 2.0), tol=1e-26, max_iter=20000)
            r2 = O.oracle_eval(A, x, np.sqrt(2.0) * t, "l2", tol=1e-26, max_iter=20000)
            ok = np.allclose(r["phi"], r2["phi"], atol=1e-9) and np.allclose(r["grad"], r2["grad"], atol=1e-9)
            return ok and np.allclose(r["dphidt"], -np.sqrt(2.0) * np.linalg.norm(r["grad"], axis=1), atol=1e-9)
        check("wl2_scaled_l2", wl2_scaled_l2)

        def al2_kkt():
            from tests.test_oracle_pins import al2_kkt_residual
            HA = (Q * rng.uniform(0.5, 3, n)) @ Q.T
            HA = 0.5 * (HA + HA.T)
            A2 = np.diag(rng.uniform(0.5, 2, n))
            r = O.oracle_eval(A2, x, t, "al2", HA=HA, tol=1e-26, max_iter=20000)
            return all(al2_kkt_residual(A2, HA, x[j], t[j], r["grad"][j]) < 1e-7 for j in range(8))
        check("al2_kkt", al2_kkt)

        def norm_family():
            ok = True
            y = rng.uniform(-10, 10, (8, n))
            for jk in ("l1sq", "linfsq"):
                for hk, lam in (("linf", 1.0), ("linf", 0.5), ("l2", 1.0)):
                    r = O.oracle_eval(np.eye(n), y, 3 * t, hk, jkind=jk, lam=lam, tol=1e-26, max_iter=20000,
                                      with_gap=True)
                    ok &= bool(np.all(np.abs(r["gap"]) <= 1e-9 * np.maximum(1, np.abs(r["phi"]))))
            r = O.oracle_eval(np.eye(n), y, 3 * t, "linf", tol=1e-26, max_iter=20000, with_gap=True)
            return ok and bool(np.all(np.abs(r["gap"]) <= 1e-9 * np.maximum(1, np.abs(r["phi"]))))
        check("norm_family", norm_family)

        def union_translation():
            C = rng.normal(0, 2, (2, n))
            r = O.oracle_eval(A, x, t, "wl1", w=w, centres=C, tol=1e-26, max_iter=20000)
            r0 = O.oracle_eval(A, x - C[0], t, "wl1", w=w, tol=1e-26, max_iter=20000)
            r1 = O.oracle_eval(A, x - C[1], t, "wl1", w=w, tol=1e-26, max_iter=20000)
            return np.allclose(r["phi"], np.minimum(r0["phi"], r1["phi"]), atol=1e-9)
        check("union_translation", union_translation)

        def distances():
            C = rng.normal(0, 3, (2, n))
            y = rng.normal(0, 5, (6, n))
            r1 = O.oracle_distance_newton(A, y, centres=C, tol=1e-26, max_iter=20000, max_newton=60)
            yb = rng.normal(0, 3, (6, n))
            yb = yb[np.linalg.norm(yb, axis=1) > 1.1]
            rb = O.oracle_distance_newton(np.eye(n), yb, tol=1e-26, max_iter=20000, max_newton=60)
            ok = np.allclose(rb["dist"], np.linalg.norm(yb, axis=1) - 1, atol=1e-8)
            r2 = O.oracle_distance_secular(A, y, centres=C)
            ok &= np.array_equal(r1["inside"], r2["inside"])
            ok &= np.allclose(r1["dist"], r2["dist"], atol=1e-8)
            out = r2["inside"] == 0
            for j in np.nonzero(out)[0]:  # closest point on the boundary of its ellipsoid
                u = r2["cp"][j] - C[r2["kstar"][j]]
                ok &= abs(u @ np.linalg.solve(A, u) - 1) < 1e-8
            return ok
        check("distances", distances)
    finally:
        O._lib = old
    return fails


def _compile(src_text, d, name):
    c = os.path.join(d, name + ".c")
    so = os.path.join(d, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-I", os.path.dirname(SRC), "-o", so, c, "-lm", "-lpthread"])
    return O.load_library(so)


def test_unmutated_passes_battery(oracle_lib):
    assert battery(O._load()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(oracle_lib, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        lib = _compile(src.replace(old, new), d, "m_" + name)
        assert battery(lib), "planted mistake %s not caught" % name


def test_control_mistakes_are_caught(oracle_lib):
    """Planted mistakes in the control read-out (written in Python): a flipped sign of A p*, a
    transposed A, a dropped centre, the control's sign: each breaks a pin of the read-out."""
    from tests.test_oracle_pins import in_wulff
    rng = np.random.default_rng(71)
    n, K = 6, 2
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = (Q * rng.uniform(0.2, 5, n)) @ Q.T
    A = 0.5 * (A + A.T)
    N = rng.normal(size=(n, n))          # a non-symmetric perturbation for the transposed variant
    w = rng.uniform(0.5, 2, n)
    C = rng.normal(0, 2, (K, n))
    x = rng.normal(0, 3, (20, n))
    t = rng.uniform(0.1, 2, 20)
    r = O.oracle_eval(A, x, t, "wl1", w=w, centres=C, level_set=True, tol=1e-26, max_iter=20000)
    Ainv = np.linalg.inv(A)

    def pins(xT, beta):
        ok = True
        for j in range(20):
            u = xT[j] - C[r["kstar"][j]]
            ok &= abs(0.5 * (u @ Ainv @ u - 1) - r["phi"][j]) <= 1e-8 * max(1, abs(r["phi"][j]))
            ok &= bool(in_wulff(beta[j], "wl1", w))
            ok &= abs(beta[j] @ r["grad"][j] + r["dphidt"][j]) <= 1e-8 * max(1, abs(r["dphidt"][j]))
        return ok

    good = O.oracle_control(A, x, t, r["grad"], r["kstar"], C)
    assert pins(good["xT"], good["beta"])
    c = C[r["kstar"]]
    p = r["grad"]
    for xT in (c - p @ A.T, p @ A.T, c + p @ (A + 0.1 * N)):
        assert not pins(xT, (x - xT) / t[:, None])
    assert not pins(good["xT"], -good["beta"])
