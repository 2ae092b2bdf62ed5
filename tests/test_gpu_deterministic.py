"""Deterministic mode of the dense evaluations (hopf_set_deterministic): with it on, repeated
launches on the same inputs give the same bits in every output (phi, grad, dphidt, iters, kstar;
dist, cp, newton for closest points), on each dense kernel (the tile kernel in its FP32 and BF16
refined modes, the on-chip kernel, the wave-local kernel), for a ragged plan replayed from a HIP
graph, and for closest points.  Launches are separated by other GPU work, so the workgroups'
timing differs between them.  The mode changes only which workgroup takes which chunk of columns:
its results are checked against the default mode to the parity bar (1e-6) and on sampled points
against the FP64 oracle."""
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


@pytest.fixture
def det_mode():
    H.set_deterministic(True)
    try:
        yield
    finally:
        H.set_deterministic(False)


def host(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items() if isinstance(v, torch.Tensor)}


def busy():
    """Unrelated GPU work between launches (shifts the workgroups' timing)."""
    a = torch.randn(2048, 2048, device=DEV)
    for _ in range(3):
        a = a @ a.T
        a = a / a.abs().max()
    torch.cuda.synchronize()


def same_bits(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, k
        assert a[k].tobytes() == b[k].tobytes(), "output %s differs between launches" % k


CASES = {
    # (precision, n, K, points): the kernel each shape runs on
    "tile_f32": ("f32", 200, 3, 6000),            # tile kernel, FP32 refined, union of 3
    "tile_bf16": ("bf16_refined", 300, 2, 3000),  # tile kernel, BF16 refined, union of 2
    "onchip_bf16": ("bf16_refined", 256, 1, 8000),  # on-chip kernel (K = 1)
    "wavelocal_f32": ("f32", 40, 2, 20000),       # wave-local kernel (n_pad <= 64)
}


@pytest.mark.parametrize("name", list(CASES))
def test_repeat_bitwise(oracle_lib, det_mode, name):
    precision, n, K, npts = CASES[name]
    print("case deterministic %s n=%d K=%d points=%d" % (name, n, K, npts), flush=True)
    rng = np.random.default_rng(9100 + n)
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    C = rng.normal(0, 3, (K, n)) if K > 1 else None
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    prob = H.Problem(A, hkind="l2_wl1", w=w, centres=C, level_set=C is not None, precision=precision,
                     tol=1e-16 * n, max_iter=20000)
    first = host(prob.eval(xd, td))
    torch.cuda.synchronize()
    assert np.all(first["iters"] > 0)
    for rep in range(2):
        busy()
        again = host(prob.eval(xd, td))
        torch.cuda.synchronize()
        same_bits(first, again)
        print("  launch %d: same bits" % (rep + 2), flush=True)
    # the default schedule: the same results to the parity bar
    H.set_deterministic(False)
    dflt = host(prob.eval(xd, td))
    torch.cuda.synchronize()
    ef = rel_err_phi(first["phi"], dflt["phi"]).max()
    eg = rel_err_vec(first["grad"], dflt["grad"]).max()
    print("  vs the default schedule: phi %.2e grad %.2e" % (ef, eg), flush=True)
    assert ef <= TOL and eg <= TOL
    idx = np.linspace(0, npts - 1, 4).astype(int)
    ref = oracle_lib.oracle_eval(A, x[idx].astype(np.float64), t[idx].astype(np.float64), "l2_wl1", w=w,
                                 centres=C, level_set=C is not None, tol=1e-24, nthreads=4)
    assert rel_err_phi(first["phi"][idx], ref["phi"]).max() <= TOL
    assert rel_err_vec(first["grad"][idx], ref["grad"]).max() <= TOL


def test_plan_graph_replay_bitwise(det_mode):
    print("case deterministic ragged plan, graph replays", flush=True)
    rng = np.random.default_rng(9200)
    specs, xs, ts = [], [], []
    for q, (n, prec) in enumerate([(24, "f32"), (90, "f32"), (300, "f32"), (700, "f32")]):
        A = rand_problem(n, rng)
        specs.append(dict(A=A, hkind="l2_wl1", w=rng.uniform(0.5, 2, n), centres=rng.normal(0, 3, (2, n)),
                          level_set=True, precision=prec, tol=1e-16 * n, max_iter=20000))
        npts = 500 + 300 * q
        xs.append(torch.from_numpy(rng.normal(0, 2, (npts, n)).astype(np.float32)).to(DEV))
        ts.append(torch.from_numpy(rng.uniform(0.05, 3, npts).astype(np.float32)).to(DEV))
    hp = H.Problem.batch(specs)
    plan = H.RaggedPlan(hp, xs, ts)
    plan.launch()
    torch.cuda.synchronize()

    def snap():
        return dict(phi=plan.phi.cpu().numpy().copy(), grad=plan.grad_packed.cpu().numpy().copy(),
                    iters=plan.iters.cpu().numpy().copy())
    eager = snap()
    assert (eager["iters"] > 0).all()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch()
    torch.cuda.synchronize()
    for k in range(3):
        plan.phi.fill_(float("nan"))
        plan.grad_packed.fill_(float("nan"))
        plan.iters.fill_(0)
        busy()
        graph.replay()
        torch.cuda.synchronize()
        same_bits(eager, snap())
        print("  replay %d: same bits as the eager launch" % k, flush=True)
    del graph
    del plan


def test_closest_point_bitwise(det_mode):
    print("case deterministic closest points", flush=True)
    rng = np.random.default_rng(9300)
    n, K, npts = 120, 3, 3000
    A = rand_problem(n, rng, 0.5, 4.0)
    C = rng.normal(0, 3, (K, n))
    y = torch.from_numpy(rng.normal(0, 4, (npts, n)).astype(np.float32)).to(DEV)
    prob = H.Problem(A, hkind="l2", centres=C, level_set=True, precision="f32", tol=1e-16 * n, max_iter=20000)
    first = host(prob.closest_point(y, s_tol=1e-7))
    torch.cuda.synchronize()
    busy()
    again = host(prob.closest_point(y, s_tol=1e-7))
    torch.cuda.synchronize()
    same_bits(first, again)
    assert np.isfinite(first["dist"]).all()
