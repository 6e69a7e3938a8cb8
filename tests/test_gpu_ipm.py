"""The interior point driver on the GPU (qdmf_ipm_solve) against the reference interior point
method (oracle/ipm.py, same readings) and against SciPy's HiGHS optimum."""
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


def gpu_ipm(torch, lp, b, c, **opt):
    from paper_2508_04370_amd import qdmf as Q
    s = Q.Solver(lp, device=0)
    dev = "cuda:0"
    bd = torch.from_numpy(b).to(dev)
    cd = torch.from_numpy(c).to(dev)
    x = torch.empty(lp["n"], dtype=torch.float64, device=dev)
    z = torch.empty(lp["n"], dtype=torch.float64, device=dev)
    y = torch.empty(lp["m"], dtype=torch.float64, device=dev)
    info, hist = Q.qdmf_ipm_solve(s.h, bd, cd, x, y, z, Q.qdmf_ipm_default_options(**opt))
    torch.cuda.synchronize()
    out = dict(info=info, hist=hist, x=x.cpu().numpy(), y=y.cpu().numpy(), z=z.cpu().numpy())
    s.close()
    return out


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
    ok, _, _ = I.converged(A, b, c, g["x"], g["y"], g["z"], 1e-8)
    assert ok


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
    assert np.all(g["x"] > 0) and np.all(g["z"] > 0)


def test_ipm_iteration_limit_is_reported(torch_dev):
    from paper_2508_04370_amd import qdmf as Q
    base = W.ne_random(m=50, n=100, density=0.05, seed=10)
    lp, b, c = W.feasible_lp(base, seed=0)
    g = gpu_ipm(torch_dev, lp, b, c, max_iter=3)
    assert g["info"]["status"] == Q.QDMF_WARN_NOT_CONVERGED and g["info"]["iters"] == 3
