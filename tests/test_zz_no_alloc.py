"""The allocation-free backward (C ABI hopf_backward_noalloc) against hopf_backward on the same
saved outputs: calls in a row through the fixed device array, each with fewer columns and a
smaller problem than the one before (the array keeps the first call's contents; the second must not read
them), each compared with the allocating entry point's results to the backward's bar (gx, gt
1e-6 relative; gA, gc 1e-5 of the largest entry; identical bits where both use the same split
counts).  Every problem the library accepts fits the array (n <= 2048), so its size
refusal cannot be reached through a problem handle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1605_01799_amd import hopf as H  # noqa: E402
from paper_1605_01799_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def setup(n, K, npts, seed):
    rng = np.random.default_rng(seed)
    A = W.spd_from_spectrum(W.haar_orthogonal(n, rng), W.log_uniform(0.5, 3.0, n, rng))
    prob = H.Problem(A, hkind="wl1", w=np.ones(n), centres=rng.normal(0, 3, (K, n)), level_set=True,
                     precision="f32")
    p = rng.normal(size=(npts, n)).astype(np.float32)
    p[rng.random((npts, n)) < 0.2] = 0.0
    t = lambda a: torch.from_numpy(a).to(DEV)  # noqa: E731
    saved = (t(rng.normal(size=npts).astype(np.float32)), t(p),
             t(-rng.uniform(0.1, 5.0, npts).astype(np.float32)), t(rng.integers(0, K, npts).astype(np.int32)))
    return prob, saved


def compare(a, b):
    for k in ("gx", "gt"):
        x, y = a[k].cpu().numpy().astype(np.float64), b[k].cpu().numpy().astype(np.float64)
        assert (np.abs(x - y) / np.maximum(np.abs(y), 1.0)).max() <= 1e-6, k
    for k in ("gA", "gc"):
        x, y = a[k].cpu().numpy().astype(np.float64), b[k].cpu().numpy().astype(np.float64)
        assert np.abs(x - y).max() <= 1e-5 * max(np.abs(y).max(), 1.0), k


def test_noalloc_matches_backward_in_a_row():
    """Three calls in a row, each smaller than the one before: the first (n = 2048, K = 8) needs
    fewer point ranges than hopf_backward takes, the others use the same ranges."""
    for (n, K, npts, seed, same) in [(2048, 8, 20000, 1, False), (256, 4, 70000, 2, True), (130, 3, 3001, 3, True)]:
        prob, saved = setup(n, K, npts, seed)
        ref = prob.backward(*saved)
        got = prob.backward(*saved, noalloc=True)
        torch.cuda.synchronize()
        compare(got, ref)
        if same:
            for k in ref:
                assert torch.equal(got[k], ref[k]), k
