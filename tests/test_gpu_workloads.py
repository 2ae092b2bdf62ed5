"""GPU parity at the workloads' own shapes: the HIP path (through the C ABI) against the FP64
oracle on seeded samples of the full-size runs, plus properties that hold at any size
(checked on every point).

* workload 2: n = 64, 2^20 points, H = weighted l1, FP32 products.
* workload 3: n = 1024, 2^16 points, H = l2 + weighted l1, BF16 products refined by FP64
  anchors (the benchmark's configuration and launch).
* workload 4: a ragged batch of problems (own n, A, w, t, K = 8 ellipsoid level sets each)
  in one launch, and the closest point / distance to each union.  A subset of the 4096
  problems: the largest n, the most points, the smallest problems, and a seeded draw.
* workload 5: n = 256, 2^18 points, K = 4 level sets, forward and the envelope-theorem
  backward (x, t, A, centres), against the oracle and against central finite differences of
  oracle values (directional, as the sampled derivative check of the gradient wrt A).
"""
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
from paper_1605_01799_amd import workloads as W  # noqa: E402

DEV = "cuda:0"
REFINED_TOL = 1e-6
FP32_TOL = 1e-6          # FP32 increments on exact anchors (test_gpu_parity)
THREADS = max(1, min(16, os.cpu_count() or 1))


def sample(npts, m, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(npts, size=min(m, npts), replace=False)
    return np.unique(np.concatenate([idx, [0, npts - 1]]))


def ham(grad, hk, w):
    g = np.asarray(grad, np.float64)
    h = np.zeros(g.shape[0])
    if hk in ("wl1", "l2_wl1"):
        h += np.abs(g) @ np.asarray(w, np.float64)
    if hk in ("l2", "l2_wl1"):
        h += np.linalg.norm(g, axis=1)
    return h


def clear_union_gap(oracle_lib, A, x, t, hk, w, C):
    """Points whose best two copies differ by more than 1e-5 relative (unique minimiser)."""
    per_k = np.stack([oracle_lib.oracle_eval(A, x - C[k], t, hk, w=w, level_set=True, tol=1e-28,
                                             nthreads=THREADS)["phi"] for k in range(C.shape[0])])
    srt = np.sort(per_k, axis=0)
    return (srt[1] - srt[0]) > 1e-5 * np.maximum(1, np.abs(srt[0]))


# ----------------------------------------------------------------------------- workload 2
def test_workload2_full_size(oracle_lib):
    p = W.round_inputs(W.workload2())
    print("case workload2 n=%d npts=%d f32" % (p.n, p.npts), flush=True)
    prob = H.Problem(p.A, hkind="wl1", w=p.w, precision="f32", tol=1e-12, max_iter=20000)
    out = prob.eval(torch.from_numpy(p.x).to(DEV), torch.from_numpy(p.t).to(DEV))
    torch.cuda.synchronize()
    grad = out["grad"].cpu().numpy()
    phi = out["phi"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    # every point: finite, converged, phi >= 0 (J* >= 0 and J*(0) = 0), dphidt = -H(grad)
    assert np.all(it > 0), "unconverged points: %d" % int(np.sum(it <= 0))
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(grad))
    assert phi.min() >= -1e-5
    h = ham(grad, "wl1", p.w)
    assert rel_err_phi(-out["dphidt"].cpu().numpy(), h).max() <= 1e-6
    idx = sample(p.npts, 256, 2)
    ref = oracle_lib.oracle_eval(p.A, p.x[idx].astype(np.float64), p.t[idx].astype(np.float64), "wl1", w=p.w,
                                 tol=1e-28, nthreads=THREADS)
    ep, ef = rel_err_vec(grad[idx], ref["grad"]), rel_err_phi(phi[idx], ref["phi"])
    print("  sampled %d: max err grad %.2e phi %.2e; iters mean %.1f max %d" %
          (len(idx), ep.max(), ef.max(), it.mean(), it.max()), flush=True)
    assert ep.max() <= FP32_TOL and ef.max() <= FP32_TOL


# ----------------------------------------------------------------------------- workload 3
def test_workload3_full_size(oracle_lib):
    p = W.round_inputs(W.workload3())
    print("case workload3 n=%d npts=%d bf16_refined tol 1e-12" % (p.n, p.npts), flush=True)
    prob = H.Problem(p.A, hkind="l2_wl1", w=p.w, precision="bf16_refined", tol=1e-12, max_iter=20000)
    out = prob.eval(torch.from_numpy(p.x).to(DEV), torch.from_numpy(p.t).to(DEV))
    torch.cuda.synchronize()
    grad = out["grad"].cpu().numpy()
    phi = out["phi"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert np.all(it > 0), "unconverged points: %d" % int(np.sum(it <= 0))
    assert phi.min() >= -1e-5
    assert rel_err_phi(-out["dphidt"].cpu().numpy(), ham(grad, "l2_wl1", p.w)).max() <= 1e-6
    idx = sample(p.npts, 64, 3)
    ref = oracle_lib.oracle_eval(p.A, p.x[idx].astype(np.float64), p.t[idx].astype(np.float64), "l2_wl1",
                                 w=p.w, tol=1e-28, nthreads=THREADS)
    ep, ef = rel_err_vec(grad[idx], ref["grad"]), rel_err_phi(phi[idx], ref["phi"])
    et = rel_err_phi(out["dphidt"].cpu().numpy()[idx], ref["dphidt"])
    print("  sampled %d: max err grad %.2e phi %.2e dphidt %.2e" % (len(idx), ep.max(), ef.max(), et.max()),
          flush=True)
    assert ep.max() <= REFINED_TOL and ef.max() <= REFINED_TOL and et.max() <= REFINED_TOL


# ----------------------------------------------------------------------------- workload 4
def w4_subset():
    n, P = W.workload4_sizes()
    fixed = [int(np.argmax(n)), int(np.argmax(P)), int(np.argmin(n * 10000 + P)), 1294]
    rng = np.random.default_rng(44)
    rest = [int(i) for i in rng.choice(W.W4_PROBLEMS, 20, replace=False) if int(i) not in fixed]
    return fixed + rest


_W4 = {}


def w4_problems():
    if "p" not in _W4:
        _W4["p"] = [W.round_inputs(W.workload4_problem(i)) for i in w4_subset()]
    return _W4["p"]


def w4_tol(precision, n):
    # both precisions resolve steps to FP64-anchored accuracy (increments on exact anchors)
    return 1e-16 * n


@pytest.mark.parametrize("precision", ["bf16_refined", "f32"])
def test_workload4_ragged(oracle_lib, precision):
    probs = w4_problems()
    print("case workload4 ragged: %d problems, n = %s, %s" %
          (len(probs), [p.n for p in probs], precision), flush=True)
    hp = H.Problem.batch([dict(A=p.A, centres=p.centres, level_set=True, hkind="wl1", w=p.w,
                               precision=precision, tol=w4_tol(precision, p.n), max_iter=20000)
                          for p in probs])
    xs = [torch.from_numpy(p.x).to(DEV) for p in probs]
    ts = [torch.from_numpy(p.t).to(DEV) for p in probs]
    out = H.eval_ragged(hp, xs, ts)
    torch.cuda.synchronize()
    off = out["offsets"]
    phi_all, it_all, ks_all = (out[k].cpu().numpy() for k in ("phi", "iters", "kstar"))
    assert np.all(it_all != -1)
    bound = REFINED_TOL if precision == "bf16_refined" else FP32_TOL

    def check(q):
        p = probs[q]
        idx = sample(p.npts, 3, 400 + q)
        x = p.x[idx].astype(np.float64)
        t = p.t[idx].astype(np.float64)
        ref = oracle_lib.oracle_eval(p.A, x, t, "wl1", w=p.w, centres=p.centres, level_set=True, tol=1e-28,
                                     nthreads=1)
        clear = clear_union_gap(oracle_lib, p.A, x, t, "wl1", p.w, p.centres)
        g = out["grad"][q].cpu().numpy()[idx]
        sl = slice(off[q], off[q + 1])
        ef = rel_err_phi(phi_all[sl][idx], ref["phi"]).max()
        ep = rel_err_vec(g[clear], ref["grad"][clear]).max() if clear.any() else 0.0
        ks = bool(np.all(ks_all[sl][idx][clear] == ref["kstar"][clear]))
        return p.n, p.npts, ef, ep, ks

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(check, range(len(probs))))
    for r in res:
        print("  n=%4d P=%4d  err phi %.2e grad %.2e kstar ok %s" % r, flush=True)
    assert all(r[4] for r in res)
    assert max(r[2] for r in res) <= bound and max(r[3] for r in res) <= bound


@pytest.mark.parametrize("precision", ["bf16_refined", "f32"])
def test_workload4_closest_point(oracle_lib, precision):
    probs = w4_problems()
    bound = REFINED_TOL if precision == "bf16_refined" else FP32_TOL
    results = []
    for q, p in enumerate(probs):
        print("case workload4 closest point: problem %d n=%d P=%d %s" % (q, p.n, p.npts, precision), flush=True)
        prob = H.Problem(p.A, centres=p.centres, level_set=True, hkind="l2", precision=precision,
                         tol=w4_tol(precision, p.n), max_iter=20000)
        o = prob.closest_point(torch.from_numpy(p.x).to(DEV), s_tol=1e-7)
        torch.cuda.synchronize()
        results.append({k: v.cpu().numpy() for k, v in o.items()})

    def check(q):
        p, o = probs[q], results[q]
        idx = sample(p.npts, 4, 500 + q)
        ref = oracle_lib.oracle_distance_secular(p.A, p.x[idx].astype(np.float64), centres=p.centres)
        ins = bool(np.array_equal(o["inside"][idx], ref["inside"]))
        ed = rel_err_phi(o["dist"][idx], ref["dist"]).max()
        outp = ref["inside"] == 0
        ec = rel_err_vec(o["cp"][idx][outp], ref["cp"][outp]).max() if outp.any() else 0.0
        return p.n, p.npts, ed, ec, ins

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(check, range(len(probs))))
    for r in res:
        print("  n=%4d P=%4d  err dist %.2e cp %.2e inside ok %s" % r, flush=True)
    assert all(r[4] for r in res)
    assert max(r[2] for r in res) <= bound and max(r[3] for r in res) <= 10 * bound


# ----------------------------------------------------------------------------- workload 5
_W5 = {}


def w5_forward():
    if "out" not in _W5:
        p = W.round_inputs(W.workload5())
        prob = H.Problem(p.A, centres=p.centres, level_set=True, hkind="wl1", w=p.w, precision="f32",
                         tol=1e-12, max_iter=20000)
        x = torch.from_numpy(p.x).to(DEV)
        t = torch.from_numpy(p.t).to(DEV)
        out = prob.eval(x, t)
        torch.cuda.synchronize()
        _W5.update(p=p, prob=prob, x=x, t=t, out=out)
    return _W5


def test_workload5_forward(oracle_lib):
    d = w5_forward()
    p, out = d["p"], d["out"]
    print("case workload5 forward n=%d npts=%d K=%d" % (p.n, p.npts, p.K), flush=True)
    it = out["iters"].cpu().numpy()
    assert np.all(it > 0)
    idx = sample(p.npts, 96, 5)
    x, t = p.x[idx].astype(np.float64), p.t[idx].astype(np.float64)
    ref = oracle_lib.oracle_eval(p.A, x, t, "wl1", w=p.w, centres=p.centres, level_set=True, tol=1e-28,
                                 nthreads=THREADS)
    clear = clear_union_gap(oracle_lib, p.A, x, t, "wl1", p.w, p.centres)
    phi = out["phi"].cpu().numpy()[idx]
    grad = out["grad"].cpu().numpy()[idx]
    assert np.all(out["kstar"].cpu().numpy()[idx][clear] == ref["kstar"][clear])
    ef, ep = rel_err_phi(phi, ref["phi"]).max(), rel_err_vec(grad[clear], ref["grad"][clear]).max()
    print("  sampled %d (%d clear): max err phi %.2e grad %.2e" % (len(idx), clear.sum(), ef, ep), flush=True)
    assert ef <= FP32_TOL and ep <= FP32_TOL


def test_workload5_backward_full_size():
    """The backward kernels against the envelope formulas applied (in FP64) to the forward's
    own outputs, on every point of the full-size run."""
    d = w5_forward()
    p, prob, out = d["p"], d["prob"], d["out"]
    g = torch.from_numpy(np.random.default_rng(55).normal(size=p.npts).astype(np.float32)).to(DEV)
    b = prob.backward(g, out["grad"], out["dphidt"], out["kstar"])
    torch.cuda.synchronize()
    gn = g.cpu().numpy().astype(np.float64)
    grad = out["grad"].cpu().numpy().astype(np.float64)
    dphidt = out["dphidt"].cpu().numpy().astype(np.float64)
    ks = out["kstar"].cpu().numpy()
    assert rel_err_vec(b["gx"].cpu().numpy(), gn[:, None] * grad).max() <= 1e-6
    assert rel_err_phi(b["gt"].cpu().numpy(), gn * dphidt).max() <= 1e-6
    gA = -0.5 * (grad * gn[:, None]).T @ grad
    assert np.abs(b["gA"].cpu().numpy() - gA).max() <= 1e-5 * np.abs(gA).max()
    gc = np.stack([-(gn[ks == k, None] * grad[ks == k]).sum(0) for k in range(p.K)])
    assert np.abs(b["gc"].cpu().numpy() - gc).max() <= 1e-5 * np.abs(gc).max()


def test_workload5_backward_vs_oracle_and_fd(oracle_lib):
    """Autograd through the forward/backward pair on a sample of points, against the oracle's
    envelope gradients and against central differences of oracle values (h = 1e-6): t exactly,
    x along 8 random and 8 coordinate directions, A along 8 random symmetric directions and
    the centres along 8 random directions."""
    d = w5_forward()
    p = d["p"]
    idx = sample(p.npts, 32, 6)
    x64, t64 = p.x[idx].astype(np.float64), p.t[idx].astype(np.float64)
    gw = np.random.default_rng(66).normal(size=len(idx))
    # GPU: a fresh forward on the sampled points through the autograd function
    A_t = torch.tensor(p.A, dtype=torch.float32, device=DEV, requires_grad=True)
    C_t = torch.tensor(p.centres, dtype=torch.float32, device=DEV, requires_grad=True)
    xs = torch.from_numpy(p.x[idx]).to(DEV).requires_grad_(True)
    ts = torch.from_numpy(p.t[idx]).to(DEV).requires_grad_(True)
    phi, _, _ = H.hopf_value(xs, ts, A_t, C_t, d["prob"])
    (phi.double() * torch.from_numpy(gw).to(DEV)).sum().backward()
    gx, gt = xs.grad.cpu().numpy().astype(np.float64), ts.grad.cpu().numpy().astype(np.float64)
    gA, gc = A_t.grad.cpu().numpy().astype(np.float64), C_t.grad.cpu().numpy().astype(np.float64)

    def L(A=p.A, C=p.centres, x=x64, t=t64):
        r = oracle_lib.oracle_eval(A, x, t, "wl1", w=p.w, centres=C, level_set=True, tol=1e-28,
                                   nthreads=THREADS)
        return float(np.dot(gw, r["phi"])), r

    L0, r0 = L()
    ob = oracle_lib.oracle_backward(r0["grad"], r0["kstar"], -r0["dphidt"], gw, K=p.K)
    clear = clear_union_gap(oracle_lib, p.A, x64, t64, "wl1", p.w, p.centres)
    assert clear.all(), "a sampled point sits on a union tie; pick another seed"
    # against the oracle's envelope gradients
    for name, mine, ref in (("gx", gx, ob["gx"]), ("gt", gt, ob["gt"]), ("gA", gA, ob["gA"]), ("gc", gc, ob["gc"])):
        e = np.abs(mine - ref).max() / max(1.0, np.abs(ref).max())
        print("  %s vs oracle envelope gradient: %.2e" % (name, e), flush=True)
        assert e <= FP32_TOL
    # against central differences of oracle values
    h = 1e-6
    rng = np.random.default_rng(67)
    checks = [("t", (L(t=t64 + h)[0] - L(t=t64 - h)[0]) / (2 * h), gt.sum())]
    for k in range(8):
        E = rng.normal(size=x64.shape)
        checks.append(("x rand", (L(x=x64 + h * E)[0] - L(x=x64 - h * E)[0]) / (2 * h), np.sum(gx * E)))
        E = np.zeros_like(x64)
        E[:, rng.integers(p.n)] = 1.0
        checks.append(("x coord", (L(x=x64 + h * E)[0] - L(x=x64 - h * E)[0]) / (2 * h), np.sum(gx * E)))
        S = rng.normal(size=(p.n, p.n))
        S = 0.5 * (S + S.T)
        checks.append(("A sym", (L(A=p.A + h * S)[0] - L(A=p.A - h * S)[0]) / (2 * h), np.sum(gA * S)))
        Ec = rng.normal(size=p.centres.shape)
        checks.append(("centres", (L(C=p.centres + h * Ec)[0] - L(C=p.centres - h * Ec)[0]) / (2 * h),
                       np.sum(gc * Ec)))
    for name, fd, an in checks:
        e = abs(fd - an) / max(1.0, abs(fd))
        print("  FD %-8s fd %+.6e gpu %+.6e rel %.2e" % (name, fd, an, e), flush=True)
        assert e <= 1e-4


@pytest.mark.parametrize("precision", ["bf16_refined", "f32"])
def test_workload4_closest_point_ragged(oracle_lib, precision):
    """The ragged closest-point call (one call for the whole batch) against the oracle's
    secular-equation route, on the problems of the ragged evaluation (H is ignored: distances
    use the l2 norm)."""
    probs = w4_problems()
    bound = REFINED_TOL if precision == "bf16_refined" else FP32_TOL
    print("case workload4 ragged closest point: %d problems, %s" % (len(probs), precision), flush=True)
    hp = H.Problem.batch([dict(A=p.A, centres=p.centres, level_set=True, hkind="wl1", w=p.w, precision=precision,
                               tol=w4_tol(precision, p.n), max_iter=20000) for p in probs])
    out = H.closest_point_ragged(hp, [torch.from_numpy(p.x).to(DEV) for p in probs], s_tol=1e-7)
    torch.cuda.synchronize()
    off = out["offsets"]
    dist, inside = out["dist"].cpu().numpy(), out["inside"].cpu().numpy()

    def check(q):
        p = probs[q]
        idx = sample(p.npts, 4, 600 + q)
        ref = oracle_lib.oracle_distance_secular(p.A, p.x[idx].astype(np.float64), centres=p.centres)
        sl = slice(off[q], off[q + 1])
        ins = bool(np.array_equal(inside[sl][idx], ref["inside"]))
        ed = rel_err_phi(dist[sl][idx], ref["dist"]).max()
        outp = ref["inside"] == 0
        cp = out["cp"][q].cpu().numpy()[idx]
        ec = rel_err_vec(cp[outp], ref["cp"][outp]).max() if outp.any() else 0.0
        return p.n, p.npts, ed, ec, ins

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(check, range(len(probs))))
    for r in res:
        print("  n=%4d P=%4d  err dist %.2e cp %.2e inside ok %s" % r, flush=True)
    assert all(r[4] for r in res)
    assert max(r[2] for r in res) <= bound and max(r[3] for r in res) <= 10 * bound
    assert all(p.iterations() > 0 for p in hp)


@pytest.mark.parametrize("precision,n", [("bf16_refined", 300), ("bf16_refined", 1024), ("f32", 40), ("f32", 200)])
def test_iteration_counter_matches_iters(precision, n):
    """hopf_problem_iterations: with one copy per point and no capped point, the passes summed
    on the device equal the per-point iteration counts summed on the host."""
    rng = np.random.default_rng(7000 + n)
    A = rand_problem(n, rng)
    w = rng.uniform(0.5, 2, n)
    x = torch.from_numpy(rng.normal(0, 2, (777, n)).astype(np.float32)).to(DEV)
    t = torch.from_numpy(rng.uniform(0.05, 3, 777).astype(np.float32)).to(DEV)
    prob = H.Problem(A, hkind="l2_wl1", w=w, precision=precision, tol=1e-16 * n, max_iter=20000)
    prob.iterations(reset=True)
    out = prob.eval(x, t)
    it = out["iters"].cpu().numpy()
    assert np.all(it > 0)
    assert prob.iterations(reset=True) == int(it.astype(np.int64).sum())
    assert prob.iterations() == 0
