"""GPU parity for H = sqrt(<p, HA p>) with a full SPD matrix HA (section 4.3, the norm ||.||_A).
FP32: the problem is diagonalised on the device (FP64 Jacobi), solved in HA's eigenbasis by the
wave-local FP32 kernel and rotated back.  FP64 (diagonal A, n <= 32, the paper's timing-table
setting): the per-thread kernel in the caller's basis, its prox rotating into HA's eigenbasis
and back every iteration.  Compared element by element with the FP64 oracle (which projects in
the eigenbasis and rotates back every iteration, as the paper states it)."""
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
FP32_TOL = 1e-6   # FP32 increments on exact anchors (test_gpu_parity); the rotations add FP32 roundings only
FP64_TOL = 1e-10


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(out, ref, label):
    ep = rel_err_vec(out["grad"], ref["grad"])
    ef = rel_err_phi(out["phi"], ref["phi"])
    et = rel_err_phi(out["dphidt"], ref["dphidt"])
    print("  %s: max err grad %.2e phi %.2e dphidt %.2e iters med %d" %
          (label, ep.max(), ef.max(), et.max(), np.median(out["iters"])), flush=True)
    assert ep.max() <= FP32_TOL and ef.max() <= FP32_TOL and et.max() <= FP32_TOL


@pytest.mark.parametrize("n", [5, 16, 33, 64])
def test_dense(oracle_lib, n):
    rng = np.random.default_rng(5000 + n)
    A = rand_problem(n, rng)
    HA = rand_problem(n, rng, 0.5, 3.0)
    npts = 300
    x = rng.normal(0, 2, (npts, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, npts).astype(np.float32)
    x[:6] *= 0.01   # inside t C
    t[:6] = 2.5
    print("case al2 dense n=%d" % n, flush=True)
    prob = H.Problem(A, hkind="al2", HA=HA, precision="f32", tol=1e-16 * n, max_iter=6000)
    out = to_np(prob.eval(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)))
    ref = oracle_lib.oracle_eval(A, x.astype(np.float64), t.astype(np.float64), "al2", HA=HA, tol=1e-28)
    assert np.all(ref["grad"][:6] == 0)
    assert np.abs(out["grad"][:6]).max() <= 1e-6   # zero in the eigenbasis, rotated back in FP32
    check(out, ref, "al2 dense")


@pytest.mark.parametrize("n", [4, 8, 16])
def test_paper_table_matrices(oracle_lib, n):
    """HA = I + 1 1^T (section 4.5's A) with J = 1/2 |.|^2 (A = I) and J = 1/2 <., D^{-1} .>
    (diagonal A = D): the diagonal inputs become dense in HA's eigenbasis."""
    HA = np.eye(n) + np.ones((n, n))
    D = 1 + np.arange(n) / (n - 1)
    rng = np.random.default_rng(5100 + n)
    x = rng.uniform(-10, 10, (400, n)).astype(np.float32)
    t = rng.uniform(0.01, 10, 400).astype(np.float32)
    for Adiag in (np.ones(n), D):
        prob = H.Problem(Adiag, diagonal=True, hkind="al2", HA=HA, precision="f32", tol=1e-16 * n, max_iter=6000)
        out = to_np(prob.eval(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)))
        ref = oracle_lib.oracle_eval(np.diag(Adiag), x.astype(np.float64), t.astype(np.float64), "al2", HA=HA,
                                     tol=1e-28)
        check(out, ref, "paper matrices n=%d" % n)


@pytest.mark.parametrize("n", [4, 8, 12, 16, 32])
def test_paper_table_fp64(oracle_lib, n):
    """Section 4.5's FP64 setting for the ||.||_A column: D_ii = 1 + (i-1)/(n-1),
    J = 1/2 <y, D^{-1} y>, HA = I + 1 1^T, (x, t) uniform in [-10, 10]^n x (0, 10]."""
    p = W.workload_paper_a(n, 2000)
    print("case al2 fp64 paper table n=%d" % n, flush=True)
    prob = H.Problem(np.diag(p.A).copy(), diagonal=True, hkind="al2", HA=p.HA, precision="f64", tol=1e-26,
                     max_iter=20000)
    out = to_np(prob.eval(torch.from_numpy(p.x).to(DEV), torch.from_numpy(p.t).to(DEV)))
    ref = oracle_lib.oracle_eval(p.A, p.x, p.t, "al2", HA=p.HA, tol=1e-26, max_iter=20000)
    ep = rel_err_vec(out["grad"], ref["grad"])
    ef = rel_err_phi(out["phi"], ref["phi"])
    et = rel_err_phi(out["dphidt"], ref["dphidt"])
    print("  max err grad %.2e phi %.2e dphidt %.2e iters med %d" % (ep.max(), ef.max(), et.max(),
                                                                    np.median(out["iters"])), flush=True)
    assert np.all(out["iters"] > 0)
    assert ep.max() <= FP64_TOL and ef.max() <= FP64_TOL and et.max() <= FP64_TOL


def test_fp64_random_HA_union(oracle_lib):
    """FP64 per-thread path with a random SPD HA, weights ignored, and a union of 3 shifted level
    sets (the copy loop and the minimum over copies)."""
    rng = np.random.default_rng(5500)
    n, K = 11, 3
    a = rng.uniform(0.5, 3, n)
    HA = rand_problem(n, rng, 0.5, 3.0)
    C = rng.normal(0, 3, (K, n))
    x = rng.normal(0, 2, (300, n))
    t = rng.uniform(0.05, 3, 300)
    prob = H.Problem(a, diagonal=True, hkind="al2", HA=HA, centres=C, level_set=True, precision="f64",
                     tol=1e-26, max_iter=20000)
    out = to_np(prob.eval(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)))
    ref = oracle_lib.oracle_eval(np.diag(a), x, t, "al2", HA=HA, centres=C, level_set=True, tol=1e-26,
                                 max_iter=20000)
    per_k = [oracle_lib.oracle_eval(np.diag(a), x - C[k], t, "al2", HA=HA, level_set=True, tol=1e-26,
                                    max_iter=20000)["phi"] for k in range(K)]
    srt = np.sort(np.stack(per_k), axis=0)
    clear = (srt[1] - srt[0]) > 1e-8 * np.maximum(1, np.abs(srt[0]))
    assert np.all(out["kstar"][clear] == ref["kstar"][clear])
    assert rel_err_phi(out["phi"], ref["phi"]).max() <= FP64_TOL
    assert rel_err_vec(out["grad"][clear], ref["grad"][clear]).max() <= FP64_TOL


def test_union_and_ragged(oracle_lib):
    rng = np.random.default_rng(5200)
    n, K = 12, 3
    Q = W.haar_orthogonal(n, rng)
    a = rng.uniform(0.5, 3, n)
    A = W.spd_from_spectrum(Q, a * a)
    HA = rand_problem(n, rng, 0.5, 3.0)
    C = rng.normal(0, 3, (K, n))
    x = rng.normal(0, 2, (150, n)).astype(np.float32)
    t = rng.uniform(0.05, 3, 150).astype(np.float32)
    prob = H.Problem(A, hkind="al2", HA=HA, centres=C, level_set=True, precision="f32", tol=1e-16 * n,
                     max_iter=6000)
    out = to_np(prob.eval(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)))
    ref = oracle_lib.oracle_eval(A, x.astype(np.float64), t.astype(np.float64), "al2", HA=HA, centres=C,
                                 level_set=True, tol=1e-28)
    per_k = [oracle_lib.oracle_eval(A, x.astype(np.float64) - C[k], t.astype(np.float64), "al2", HA=HA,
                                    level_set=True, tol=1e-28)["phi"] for k in range(K)]
    srt = np.sort(np.stack(per_k), axis=0)
    clear = (srt[1] - srt[0]) > 1e-5 * np.maximum(1, np.abs(srt[0]))
    assert np.all(out["kstar"][clear] == ref["kstar"][clear])
    assert rel_err_phi(out["phi"], ref["phi"]).max() <= FP32_TOL
    assert rel_err_vec(out["grad"][clear], ref["grad"][clear]).max() <= FP32_TOL
    # a ragged batch mixing this problem with a weighted-l1 one
    A2 = rand_problem(20, rng)
    w2 = rng.uniform(0.5, 2, 20)
    probs = H.Problem.batch([dict(A=A, hkind="al2", HA=HA, centres=C, level_set=True, precision="f32",
                                  tol=1e-16 * n, max_iter=6000),
                             dict(A=A2, hkind="wl1", w=w2, precision="f32", tol=1e-16 * n, max_iter=6000)])
    x2 = rng.normal(0, 2, (90, 20)).astype(np.float32)
    t2 = rng.uniform(0.05, 3, 90).astype(np.float32)
    r = H.eval_ragged(probs, [torch.from_numpy(x).to(DEV), torch.from_numpy(x2).to(DEV)],
                      [torch.from_numpy(t).to(DEV), torch.from_numpy(t2).to(DEV)])
    torch.cuda.synchronize()
    cut = lambda v, a, b: v[a:b].cpu().numpy()
    o0 = dict(phi=cut(r["phi"], 0, 150), grad=r["grad"][0].cpu().numpy(), dphidt=cut(r["dphidt"], 0, 150),
              iters=cut(r["iters"], 0, 150))
    o1 = dict(phi=cut(r["phi"], 150, 240), grad=r["grad"][1].cpu().numpy(), dphidt=cut(r["dphidt"], 150, 240),
              iters=cut(r["iters"], 150, 240))
    assert rel_err_phi(o0["phi"], ref["phi"]).max() <= FP32_TOL
    assert rel_err_vec(o0["grad"][clear], ref["grad"][clear]).max() <= FP32_TOL
    ref2 = oracle_lib.oracle_eval(A2, x2.astype(np.float64), t2.astype(np.float64), "wl1", w=w2, tol=1e-28)
    check(o1, ref2, "ragged wl1 partner")


def test_closest_point_rotated(oracle_lib):
    """Distances do not depend on H; an HA problem answers them in its rotated frame."""
    rng = np.random.default_rng(5300)
    n, K = 9, 2
    Q = W.haar_orthogonal(n, rng)
    a = rng.uniform(0.5, 3, n)
    A = W.spd_from_spectrum(Q, a * a)
    HA = rand_problem(n, rng, 0.5, 3.0)
    C = rng.normal(0, 3, (K, n))
    y = rng.normal(0, 4, (60, n)).astype(np.float32)
    prob = H.Problem(A, hkind="al2", HA=HA, centres=C, level_set=True, precision="f32", tol=1e-16 * n,
                     max_iter=20000)
    out = to_np(prob.closest_point(torch.from_numpy(y).to(DEV), s_tol=1e-7))
    ref = oracle_lib.oracle_distance_secular(A, y.astype(np.float64), centres=C)
    assert np.array_equal(out["inside"], ref["inside"])
    assert rel_err_phi(out["dist"], ref["dist"]).max() <= FP32_TOL
    o = ref["inside"] == 0
    assert rel_err_vec(out["cp"][o], ref["cp"][o]).max() <= 10 * FP32_TOL


def test_rejected():
    rng = np.random.default_rng(5400)
    HA = rand_problem(8, rng, 0.5, 3.0)
    with pytest.raises(H._lib.HopfError) as e:   # FP64 needs diagonal A
        H.Problem(rand_problem(8, rng), hkind="al2", HA=HA, precision="f64")
    assert e.value.status == H._lib.HOPF_EINVAL
    with pytest.raises(H._lib.HopfError) as e:   # FP64 beyond the per-thread kernel's n <= 32
        H.Problem(np.ones(40), diagonal=True, hkind="al2", HA=rand_problem(40, rng), precision="f64")
    assert e.value.status == H._lib.HOPF_EINVAL
    with pytest.raises(H._lib.HopfError) as e:   # HA missing
        H.Problem(rand_problem(8, rng), hkind="al2", precision="f32")
    assert e.value.status == H._lib.HOPF_EINVAL
    bad = HA.copy()
    bad[0, 0] = -50.0
    with pytest.raises(H._lib.HopfError) as e:   # HA indefinite
        H.Problem(rand_problem(8, rng), hkind="al2", HA=bad, precision="f32")
    assert e.value.status == H._lib.HOPF_ENOTSPD
