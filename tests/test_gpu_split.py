"""GPU parity of the tile kernel's split contraction (FP32 refined mode, launch shapes whose FP32
right-hand sides do not fit LDS whole: the products run over one half of the rows at a time, the
first half's partial sums going through the workgroup's staging).  The shape is forced with
HOPF_DENSE_VARIANT (32 columns at n_pad = 2048, 64 columns at n_pad = 704), on unions of level
sets and a single problem, against the FP64 oracle (1e-6) and against the default shape."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from tests.helpers import rand_problem, rel_err_phi, rel_err_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1605_01799_amd import hopf as H  # noqa: E402

DEV = "cuda:0"
TOL = 1e-6


def evaluate(prob, x, t, variant):
    old = os.environ.get("HOPF_DENSE_VARIANT")
    try:
        if variant:
            os.environ["HOPF_DENSE_VARIANT"] = variant
        else:
            os.environ.pop("HOPF_DENSE_VARIANT", None)
        out = prob.eval(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV))
        torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("HOPF_DENSE_VARIANT", None)
        else:
            os.environ["HOPF_DENSE_VARIANT"] = old
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("n,variant,K", [(2000, "32:1:4", 2), (700, "64:1:4", 1), (1030, "32:1:4", 1)])
def test_split_contraction(oracle_lib, n, variant, K):
    rng = np.random.default_rng(8000 + n)
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    C = rng.normal(0, 3, (K, n)) if K > 1 else None
    npts = 70
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    print("case split n=%d shape %s K=%d" % (n, variant, K), flush=True)
    prob = H.Problem(A, hkind="l2_wl1", w=w, centres=C, level_set=C is not None, precision="f32",
                     tol=1e-16 * n, max_iter=20000)
    out = evaluate(prob, x, t, variant)
    base = evaluate(prob, x, t, None)
    print("  GPU evaluations done (iters med %d); oracle on %d points" % (np.median(out["iters"]), len(range(0, npts, 7))),
          flush=True)
    assert np.all(out["iters"] > 0)
    assert rel_err_phi(out["phi"], base["phi"]).max() <= TOL
    idx = np.arange(0, npts, 7)

    # at n ~ 2000 the oracle's FP64 steps stall near 1e-27 (rounding), so it stops at 1e-24 (steps of
    # 1e-12, far inside the bar)
    def one(j):
        return oracle_lib.oracle_eval(A, x[j:j + 1].astype(np.float64), t[j:j + 1].astype(np.float64), "l2_wl1", w=w,
                                      centres=C, level_set=C is not None, tol=1e-24, nthreads=1)
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(one, idx))
    ref_phi = np.concatenate([r["phi"] for r in refs])
    ref_grad = np.concatenate([r["grad"] for r in refs])
    ef = rel_err_phi(out["phi"][idx], ref_phi).max()
    ep = rel_err_vec(out["grad"][idx], ref_grad).max()
    print("  err phi %.2e grad %.2e iters med %d" % (ef, ep, np.median(out["iters"])), flush=True)
    assert ef <= TOL and ep <= TOL
