"""GPU parity of the refined BF16 solver with the column state on chip (one point per column,
64 <= n_pad <= 1024): the HIP path through the C ABI against the FP64 oracle on seeded inputs.

Covered: ragged batches of such problems (so one persistent launch switches problems, and both
row-tile shapes of the kernel run: largest n_pad <= 512 and up to 1024), each kind of H that
the kernel takes (l1, l2, l2 + weighted l1), a centre (a single shifted level set), point counts
that leave a ragged last tile, and a point count large enough that every workgroup refills its
column slots many times (checked on sampled points, all points for finiteness and iterations).
Bar: 1e-6 relative, the refined path's target."""
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
REFINED_TOL = 1e-6
HK = ["wl1", "l2", "l2_wl1"]


def make_case(n, npts, seed, hk, centre):
    rng = np.random.default_rng(seed)
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    C = rng.normal(0, 3, (1, n)) if centre else None
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    return dict(A=A, w=w, C=C, x=x, t=t, hk=hk, n=n)


def oracle_rows(oracle_lib, c, idx):
    return oracle_lib.oracle_eval(c["A"], c["x"][idx].astype(np.float64), c["t"][idx].astype(np.float64), c["hk"],
                                  w=c["w"], centres=c["C"], level_set=c["C"] is not None, tol=1e-28, nthreads=1)


def sample(npts, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, npts - 1], rng.choice(npts, min(k, npts), replace=False)]))


@pytest.mark.parametrize("ns", [(64, 100, 300, 513, 1024), (64, 129, 257, 500)])
def test_ragged_refined_batch(oracle_lib, ns):
    cases = [make_case(n, 70 + 13 * q, 9000 + n, HK[q % 3], q % 2 == 1) for q, n in enumerate(ns)]
    print("case rs ragged n=%s" % (list(ns),), flush=True)
    probs = H.Problem.batch([dict(A=c["A"], hkind=c["hk"], w=c["w"], centres=c["C"], level_set=c["C"] is not None,
                                  precision="bf16_refined", tol=1e-16 * c["n"], max_iter=20000) for c in cases])
    out = H.eval_ragged(probs, [torch.from_numpy(c["x"]).to(DEV) for c in cases],
                        [torch.from_numpy(c["t"]).to(DEV) for c in cases])
    torch.cuda.synchronize()
    off = out["offsets"]
    phi, it = out["phi"].cpu().numpy(), out["iters"].cpu().numpy()
    assert np.all(it > 0)

    def check(q):
        c = cases[q]
        npts = c["x"].shape[0]
        idx = np.arange(npts) if c["n"] <= 300 else sample(npts, 6, q)
        ref = oracle_rows(oracle_lib, c, idx)
        g = out["grad"][q].cpu().numpy()[idx]
        return (c["n"], rel_err_phi(phi[off[q]:off[q + 1]][idx], ref["phi"]).max(),
                rel_err_vec(g, ref["grad"]).max())

    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(check, range(len(cases))))
    for r in res:
        print("  n=%4d err phi %.2e grad %.2e" % r, flush=True)
    assert max(r[1] for r in res) <= REFINED_TOL and max(r[2] for r in res) <= REFINED_TOL


def test_many_refills(oracle_lib):
    """Several column tiles per workgroup: slots are refilled while others iterate."""
    c = make_case(128, 40000, 9100, "l2_wl1", False)
    print("case rs many refills n=128 npts=40000", flush=True)
    prob = H.Problem(c["A"], hkind="l2_wl1", w=c["w"], precision="bf16_refined", tol=1e-16 * 128, max_iter=20000)
    out = prob.eval(torch.from_numpy(c["x"]).to(DEV), torch.from_numpy(c["t"]).to(DEV))
    torch.cuda.synchronize()
    it = out["iters"].cpu().numpy()
    assert np.all(it > 0)
    assert torch.isfinite(out["grad"]).all().item() and torch.isfinite(out["phi"]).all().item()
    idx = sample(40000, 40, 5)
    ref = oracle_rows(oracle_lib, c, idx)
    ep = rel_err_vec(out["grad"].cpu().numpy()[idx], ref["grad"]).max()
    ef = rel_err_phi(out["phi"].cpu().numpy()[idx], ref["phi"]).max()
    print("  err phi %.2e grad %.2e iters med %d max %d" % (ef, ep, np.median(it), it.max()), flush=True)
    assert ep <= REFINED_TOL and ef <= REFINED_TOL

