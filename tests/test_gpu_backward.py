"""GPU parity of the backward kernels (C ABI hopf_backward) against the oracle's envelope
formulas, on seeded saved outputs of every shape class the kernels distinguish: n below, at and
above the 64-wide gA tiles and the 256-thread points pass, n not a multiple of 4 (element loads),
K beyond the register sums (K > 8), point counts from 0 to several splits with ragged tails, and
every subset of the requested outputs.

The backward takes the forward's saved outputs (p*, dphidt, k*) as plain arrays, so these tests
feed seeded arrays of the forward's shape and value range directly; workload 5's end-to-end
backward is in test_gpu_workloads.

Bars: gx and gt are one FP32 product per element (1e-6 relative); gA and gc are sums over the
points (FP32 MFMA partials over at most a few thousand points, combined in FP64) and are held to
1e-5 of the largest entry, as the workload test does."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1605_01799_amd import hopf as H  # noqa: E402
from paper_1605_01799_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def saved_outputs(n, K, npts, seed):
    """Seeded stand-ins for a forward's saved outputs: p* ~ N(0, 1) with a few exact zeros (as
    shrinks produce), H(p*) > 0, k* uniform over the copies."""
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(npts, n)).astype(np.float32)
    p[rng.random((npts, n)) < 0.2] = 0.0
    dphidt = -rng.uniform(0.1, 5.0, npts).astype(np.float32)
    kstar = rng.integers(0, K, npts).astype(np.int32)
    g = rng.normal(size=npts).astype(np.float32)
    return p, dphidt, kstar, g


def make_problem(n, K, seed):
    rng = np.random.default_rng(seed)
    A = W.spd_from_spectrum(W.haar_orthogonal(n, rng), W.log_uniform(0.5, 3.0, n, rng))
    C = rng.normal(0, 3, (K, n))
    return H.Problem(A, hkind="wl1", w=np.ones(n), centres=C, level_set=True, precision="f32")


def run_backward(prob, p, dphidt, kstar, g, want):
    t = lambda a: torch.from_numpy(a).to(DEV)  # noqa: E731
    out = prob.backward(t(g), t(p), t(dphidt), t(kstar), want=want)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def check_against_oracle(oracle_lib, b, p, dphidt, kstar, g, K):
    ob = oracle_lib.oracle_backward(p.astype(np.float64), kstar, -dphidt.astype(np.float64), g, K=K)
    if "gx" in b:
        scale = np.maximum(np.abs(ob["gx"]), 1.0)
        assert (np.abs(b["gx"] - ob["gx"]) / scale).max() <= 1e-6
    if "gt" in b:
        assert (np.abs(b["gt"] - ob["gt"]) / np.maximum(np.abs(ob["gt"]), 1.0)).max() <= 1e-6
    for key in ("gA", "gc"):
        if key in b:
            ref = ob[key]
            tol = 1e-5 * max(np.abs(ref).max(), 1.0)
            assert np.abs(b[key] - ref).max() <= tol, (key, np.abs(b[key] - ref).max(), tol)
    if "gA" in b:
        assert np.array_equal(b["gA"], b["gA"].T) or np.abs(b["gA"] - b["gA"].T).max() <= 1e-6 * np.abs(b["gA"]).max()


@pytest.mark.parametrize("n,K,npts", [
    (1, 1, 1), (5, 3, 700), (63, 1, 4097), (64, 4, 2048), (65, 2, 3001), (130, 9, 1500),
    (256, 4, 70000), (300, 3, 2500), (701, 2, 1200),
])
def test_backward_shapes(oracle_lib, n, K, npts):
    p, dphidt, kstar, g = saved_outputs(n, K, npts, 100 + n + K)
    prob = make_problem(n, K, n)
    b = run_backward(prob, p, dphidt, kstar, g, ("gx", "gt", "gA", "gc"))
    check_against_oracle(oracle_lib, b, p, dphidt, kstar, g, K)


@pytest.mark.parametrize("want", [("gA",), ("gc",), ("gx",), ("gt",), ("gx", "gc"), ("gt", "gA")])
def test_backward_output_subsets(oracle_lib, want):
    n, K, npts = 96, 3, 5000
    p, dphidt, kstar, g = saved_outputs(n, K, npts, 7)
    prob = make_problem(n, K, 8)
    b = run_backward(prob, p, dphidt, kstar, g, want)
    assert set(b) == set(want)
    check_against_oracle(oracle_lib, b, p, dphidt, kstar, g, K)


def test_backward_no_points():
    """Sums over no points are zero (written by the library, not left as they were)."""
    n, K = 70, 2
    prob = make_problem(n, K, 9)
    e = torch.empty(0, device=DEV)
    out = prob.backward(e, torch.empty(0, n, device=DEV), e, torch.empty(0, dtype=torch.int32, device=DEV),
                        want=("gA", "gc"))
    torch.cuda.synchronize()
    assert out["gA"].shape == (n, n) and not out["gA"].abs().max().item()
    assert out["gc"].shape == (K, n) and not out["gc"].abs().max().item()


def test_backward_deterministic():
    """The reductions have a fixed order: two calls give identical bits."""
    n, K, npts = 256, 4, 20000
    p, dphidt, kstar, g = saved_outputs(n, K, npts, 11)
    prob = make_problem(n, K, 12)
    a = run_backward(prob, p, dphidt, kstar, g, ("gA", "gc"))
    b = run_backward(prob, p, dphidt, kstar, g, ("gA", "gc"))
    assert np.array_equal(a["gA"], b["gA"]) and np.array_equal(a["gc"], b["gc"])
