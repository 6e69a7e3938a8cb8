"""The interior point driver on the GPU (qdmf_ipm_solve) against the reference interior point
method (oracle/ipm.py, same readings) and against SciPy's HiGHS optimum, on LPs in standard
form and with lower and upper bounds."""
import numpy as np
import pytest

from oracle import ipm as I
from paper_2508_04370_amd import workloads as W

pytestmark = pytest.mark.gpu
scipy_optimize = pytest.importorskip("scipy.optimize")


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_04370_amd import qdmf as Q
    Q.lib()
    return torch


def gpu_ipm(torch, lp, b, c, l=None, u=None, **opt):
    from paper_2508_04370_amd import qdmf as Q
    s = Q.Solver(lp, device=0)
    dev = "cuda:0"
    t = lambda v: None if v is None else torch.from_numpy(np.ascontiguousarray(v, np.float64)).to(dev)
    x = torch.empty(lp["n"], dtype=torch.float64, device=dev)
    zl = torch.empty(lp["n"], dtype=torch.float64, device=dev)
    zu = torch.empty(lp["n"], dtype=torch.float64, device=dev)
    y = torch.empty(lp["m"], dtype=torch.float64, device=dev)
    info, hist = Q.qdmf_ipm_solve(s.h, t(b), t(c), x, y, zl, Q.qdmf_ipm_default_options(**opt), l=t(l), u=t(u),
                                  zu=zu)
    torch.cuda.synchronize()
    out = dict(info=info, hist=hist, x=x.cpu().numpy(), y=y.cpu().numpy(), zl=zl.cpu().numpy(),
               zu=zu.cpu().numpy())
    s.close()
    return out


def host_converged(A, b, c, l, u, g, tau):
    """The termination test on the driver's last iterate, with the slacks x - l and u - x."""
    hasu = np.isfinite(u)
    st = I.State(g["x"], g["x"] - l, np.where(hasu, u - g["x"], 0.0), g["y"], g["zl"], g["zu"])
    return I.converged(A, b, c, l, u, st, tau)[0]


def highs_bounds(l, u):
    return [(lo, None if np.isinf(hi) else hi) for lo, hi in zip(l, u)]


@pytest.mark.parametrize("m,n,d,seed", [(50, 100, 0.05, 0), (120, 300, 0.02, 1), (80, 240, 0.03, 2)])
def test_ipm_matches_reference_iterations(torch_dev, m, n, d, seed):
    base = W.ne_random(m=m, n=n, density=d, seed=10 + seed)
    lp, b, c = W.feasible_lp(base, seed=seed)
    print(f"[gpu case] ipm m={m} n={n} seed={seed}", flush=True)
    g = gpu_ipm(torch_dev, lp, b, c, correctors=2)
    A = W.lp_dense(lp)
    r = I.ipm(A, b, c, k=2)
    ref = scipy_optimize.linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    info = g["info"]
    print(f"  gpu: status {info['status']} iters {info['iters']} obj {info['primal_obj']:.12g} "
          f"{info['ms']:.1f} ms; reference iters {r['iters']} obj {r['fp']:.12g}; highs {ref.fun:.12g}")
    assert info["status"] == 0 and r["status"] == "optimal"
    assert abs(info["iters"] - r["iters"]) <= 1
    assert abs(info["primal_obj"] - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    # the first iterations follow the reference closely: same corrector counts, mu and steps
    hg, hr = g["hist"], np.array(r["history"])
    for it in range(3):
        assert hg[it, 3] == hr[it, 3], it
        assert np.allclose(hg[it, :3], hr[it, :3], rtol=1e-8, atol=0), (it, hg[it], hr[it])
    # the driver's termination test holds for its own iterate, recomputed on the host
    assert host_converged(A, b, c, np.zeros(n), np.full(n, np.inf), g, 1e-8)
    assert np.all(g["zu"] == 0)


def test_ipm_default_correctors_on_staircase_lp(torch_dev):
    base = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10, seed=12)
    lp, b, c = W.feasible_lp(base, seed=5)
    print("[gpu case] ipm staircase 200 x 400", flush=True)
    g = gpu_ipm(torch_dev, lp, b, c)
    A = W.lp_dense(lp)
    ref = scipy_optimize.linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    info = g["info"]
    print(f"  gpu: status {info['status']} iters {info['iters']} correctors {info['correctors']} "
          f"obj {info['primal_obj']:.12g} highs {ref.fun:.12g} {info['ms']:.1f} ms")
    assert info["status"] == 0 and info["correctors"] >= 1
    assert abs(info["primal_obj"] - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    assert np.all(g["x"] > 0) and np.all(g["zl"] > 0)


def test_ipm_iteration_limit_is_reported(torch_dev):
    from paper_2508_04370_amd import qdmf as Q
    base = W.ne_random(m=50, n=100, density=0.05, seed=10)
    lp, b, c = W.feasible_lp(base, seed=0)
    g = gpu_ipm(torch_dev, lp, b, c, max_iter=3)
    assert g["info"]["status"] == Q.QDMF_WARN_NOT_CONVERGED and g["info"]["iters"] == 3


@pytest.mark.parametrize("m,n,d,seed,upper", [(50, 100, 0.05, 0, 0.5), (120, 300, 0.02, 1, 1.0),
                                              (80, 240, 0.03, 2, 0.2)])
def test_bounded_ipm_matches_reference_iterations(torch_dev, m, n, d, seed, upper):
    base = W.ne_random(m=m, n=n, density=d, seed=20 + seed)
    lp, b, c, l, u = W.bounded_lp(base, seed=seed, upper=upper)
    print(f"[gpu case] bounded ipm m={m} n={n} seed={seed} upper={upper}", flush=True)
    g = gpu_ipm(torch_dev, lp, b, c, l, u, correctors=2)
    A = W.lp_dense(lp)
    r = I.ipm(A, b, c, l, u, k=2)
    ref = scipy_optimize.linprog(c, A_eq=A, b_eq=b, bounds=highs_bounds(l, u), method="highs")
    info = g["info"]
    print(f"  gpu: status {info['status']} iters {info['iters']} obj {info['primal_obj']:.12g} "
          f"{info['ms']:.1f} ms; reference iters {r['iters']} obj {r['fp']:.12g}; highs {ref.fun:.12g}")
    assert info["status"] == 0 and r["status"] == "optimal"
    assert abs(info["iters"] - r["iters"]) <= 1
    assert abs(info["primal_obj"] - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    hg, hr = g["hist"], np.array(r["history"])
    for it in range(3):
        assert hg[it, 3] == hr[it, 3], it
        assert np.allclose(hg[it, :3], hr[it, :3], rtol=1e-8, atol=0), (it, hg[it], hr[it])
    hasu = np.isfinite(u)
    assert np.all(g["x"] > l) and np.all(g["x"][hasu] < u[hasu])
    assert np.all(g["zu"][~hasu] == 0)
    assert host_converged(A, b, c, l, u, g, 1e-8)


def test_bounded_ipm_rejects_bad_bounds(torch_dev):
    from paper_2508_04370_amd import qdmf as Q
    base = W.ne_random(m=50, n=100, density=0.05, seed=20)
    lp, b, c, l, u = W.bounded_lp(base, seed=0)
    for bad in ("l_inf", "u_below"):
        l2, u2 = l.copy(), u.copy()
        if bad == "l_inf":
            l2[3] = -np.inf
        else:
            j = int(np.flatnonzero(np.isfinite(u))[0])
            u2[j] = l2[j]
        with pytest.raises(Q.QdmfError) as e:
            gpu_ipm(torch_dev, lp, b, c, l2, u2)
        assert e.value.code == Q.QDMF_ERR_INVALID_ARG


@pytest.mark.parametrize("m,n,d,seed,upper", [(50, 100, 0.05, 0, 0.5), (80, 240, 0.03, 2, 0.0)])
def test_qp_ipm_matches_reference_iterations(torch_dev, m, n, d, seed, upper):
    """A quadratic program (Q from workloads.with_hessian) through qdmf_analyse_qp: the driver
    against the reference method with the same Q, iteration by iteration, and the optimality
    conditions of the convex QP at its last iterate."""
    base = W.ne_random(m=m, n=n, density=d, seed=60 + seed)
    lpq = W.with_hessian(W.LP(dict(base, mode=W.AS)), seed=seed, window=10)
    lp, b, c, l, u = W.bounded_lp(lpq, seed=seed, upper=upper)
    print(f"[gpu case] qp ipm m={m} n={n} seed={seed} upper={upper}", flush=True)
    g = gpu_ipm(torch_dev, lp, b, c, l, u, correctors=2)
    A, Qm = W.lp_dense(lp), W.q_dense(lp)
    r = I.ipm(A, b, c, l, u, k=2, Q=Qm)
    info = g["info"]
    print(f"  gpu: status {info['status']} iters {info['iters']} obj {info['primal_obj']:.12g} "
          f"{info['ms']:.1f} ms; reference iters {r['iters']} obj {r['fp']:.12g}")
    assert info["status"] == 0 and r["status"] == "optimal"
    assert abs(info["iters"] - r["iters"]) <= 1
    assert abs(info["primal_obj"] - r["fp"]) <= 1e-7 * (1 + abs(r["fp"]))
    hg, hr = g["hist"], np.array(r["history"])
    for it in range(3):
        assert hg[it, 3] == hr[it, 3], it
        assert np.allclose(hg[it, :3], hr[it, :3], rtol=1e-8, atol=0), (it, hg[it], hr[it])
    hasu = np.isfinite(u)
    x, y, zl, zu = g["x"], g["y"], g["zl"], g["zu"]
    scale = 1 + max(np.abs(b).max(), np.abs(c).max())
    assert np.abs(A @ x - b).max() <= 1e-6 * scale
    assert np.all(x > l) and np.all(x[hasu] < u[hasu]) and np.all(zl > 0) and np.all(zu[hasu] > 0)
    assert np.abs(c + Qm @ x - A.T @ y - zl + zu).max() <= 1e-6 * scale
    assert np.abs((x - l) * zl).max() <= 1e-6 * scale
