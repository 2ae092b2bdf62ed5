"""Shared test helpers: error metrics and problem builders (no method arithmetic)."""
import numpy as np

from paper_1605_01799_amd import workloads as W


def rel_err_phi(phi_hat, phi):
    """|phi_hat - phi| / max(|phi|, 1), per point."""
    phi_hat = np.asarray(phi_hat, np.float64)
    phi = np.asarray(phi, np.float64)
    return np.abs(phi_hat - phi) / np.maximum(np.abs(phi), 1.0)


def rel_err_vec(v_hat, v):
    """|v_hat - v|_2 / max(|v|_2, 1), per row."""
    v_hat = np.asarray(v_hat, np.float64)
    v = np.asarray(v, np.float64)
    return np.linalg.norm(v_hat - v, axis=-1) / np.maximum(np.linalg.norm(v, axis=-1), 1.0)


def rand_problem(n, rng, lo=0.1, hi=10.0):
    Q = W.haar_orthogonal(n, rng)
    s = W.log_uniform(lo, hi, n, rng)
    return W.spd_from_spectrum(Q, s)
