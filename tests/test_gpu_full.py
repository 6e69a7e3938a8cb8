"""Full-size workloads on the GPU: properties that hold at any size, checked with the oracle's
own residual against K_static (formed from A, Theta, rho and delta on the CPU), the
inertia a quasi-definite (AS) or positive definite (NE) matrix must have, and, for batches,
every system on its own.  Sizes are those of the benchmark workloads."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_04370_amd import qdmf as Q
    Q.lib()
    return torch, "cuda:0"


def run(torch_dev, lp, prec, systems=None, **opts):
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    print(f"[gpu case] {lp['name']} prec={prec} opts={opts}", flush=True)
    s = Q.Solver(lp, device=0, systems=systems, **opts)
    th = torch.from_numpy(np.ascontiguousarray(lp["theta"])).to(dev)
    s.factorise(th, lp["rho"], lp["delta"], prec)
    r1 = Q.to_device_colmajor(lp["r1"], dev)
    r7 = Q.to_device_colmajor(lp["r7"], dev) if lp.get("r7") is not None else None
    dx, dy = s.solve(r7, r1)
    torch.cuda.synchronize()
    nrhs = r1.shape[1]
    out = dict(dx=dx.cpu().numpy(), dy=dy.cpu().numpy(), fs=s.factor_stats(), ss=s.solve_stats(nrhs),
               bs=s.batch_stats(nrhs) if systems else None, sym=s.sym)
    s.close()
    return out


def berr_columns(lp, g):
    out = []
    for c in range(lp["r1"].shape[1]):
        r7 = lp["r7"][:, c] if lp.get("r7") is not None else None
        x = np.concatenate([g["dx"][:, c], g["dy"][:, c]]) if lp["mode"] == W.AS else g["dy"][:, c]
        b = O.system_rhs(lp, r7, lp["r1"][:, c], lp["theta"])
        _, nw, _, _ = O.residual(lp, lp["theta"], lp["rho"], lp["delta"], x, b)
        out.append(nw)
    return np.array(out)


def test_grid_ne_full_fp64_and_mixed(torch_dev):
    """The 50 x 50 x 40 grid NE workload with 8 right-hand sides (geometric nested
    dissection): FP64 to 1e-12; the mixed path never ends worse than it started, reports
    its true backward error, and flags a miss of 1e-10."""
    from paper_2508_04370_amd import qdmf as Q
    lp = W.ne_grid(nrhs=8)
    lp["r7"] = None
    g = run(torch_dev, lp, 0, ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"])
    nw = berr_columns(lp, g)
    print(f"grid fp64: max f {g['sym']['max_front']} berr per rhs {nw}")
    assert nw.max() <= 1e-12
    assert (g["fs"]["nneg"], g["fs"]["npos"]) == (0, lp["m"])
    gm = run(torch_dev, lp, 1, ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"])
    nwm = berr_columns(lp, gm)
    ss = gm["ss"]
    print(f"grid mixed: initial {ss['berr_nw_initial']:.2e} final {ss['berr_nw']:.2e} oracle {nwm.max():.2e} "
          f"steps {ss['max_steps']} status {ss['status']}")
    assert ss["berr_nw"] <= ss["berr_nw_initial"]
    # the reported error is the true one up to the residual's own rounding (rows of up to 25
    # entries: at most 26 u of the normalising denominator)
    assert abs(nwm.max() - ss["berr_nw"]) <= 0.1 * nwm.max() + 26 * U
    assert nwm.max() <= 1e-10 and ss["berr_nw"] <= 1e-10 and ss["status"] == 0


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_full_512_systems(torch_dev, prec):
    """All 512 systems of the batched workload (m in [50, 2000], n = 2m, AMD per system):
    FP64, every system to 1e-12 against its own K_static with its own inertia; mixed precision,
    every system to 1e-10 (inertia may differ through FP32-updated 2x2 blocks, which the
    library reports)."""
    lps = W.as_batch(512)
    cat = W.concat_systems(lps)
    cat["theta"] = np.concatenate([W.as_batch_theta(q, s, 0) for s, q in enumerate(lps)])
    rs = [W.as_batch_rhs(q, s, 0, 0) for s, q in enumerate(lps)]
    cat["r7"] = np.concatenate([r[0] for r in rs]).reshape(-1, 1)
    cat["r1"] = np.concatenate([r[1] for r in rs]).reshape(-1, 1)
    g = run(torch_dev, cat, prec, systems=lps, ordering=0)
    bs = g["bs"]
    tol = 1e-12 if prec == 0 else 1e-10
    worst = 0.0
    for q, lp in enumerate(lps):
        c0, c1 = cat["col_off"][q], cat["col_off"][q + 1]
        r0, r1 = cat["row_off"][q], cat["row_off"][q + 1]
        x = np.concatenate([g["dx"][c0:c1, 0], g["dy"][r0:r1, 0]])
        th = cat["theta"][c0:c1]
        b = O.system_rhs(lp, cat["r7"][c0:c1, 0], cat["r1"][r0:r1, 0], th)
        _, nw, _, _ = O.residual(lp, th, lp["rho"], lp["delta"], x, b)
        worst = max(worst, nw)
        assert nw <= tol, (q, nw)
        if prec == 0:
            assert tuple(bs["inertia"][q][:2]) == (lp["n"], lp["m"]), q
    print(f"batch 512 prec {prec}: worst system berr {worst:.2e}, reported worst {bs['berr_nw'].max():.2e}")
    assert bs["berr_nw"].max() <= tol


def test_dense_column_as_full_fp64(torch_dev):
    """The 80 x 50 x 50 grid AS workload with 20 dense columns (N = 600000), geometric
    nested dissection with the dense columns last: FP64 to 1e-12 and inertia (n, m)."""
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_dense_cols()
    g = run(torch_dev, lp, 0, ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"])
    nw = berr_columns(lp, g)
    print(f"dense columns: max f {g['sym']['max_front']} berr {nw}")
    assert nw.max() <= 1e-12
    assert (g["fs"]["nneg"], g["fs"]["npos"]) == (lp["n"], lp["m"])
    assert abs(nw.max() - g["ss"]["berr_nw"]) <= 0.1 * nw.max() + 64 * U


def test_dense_column_as_full_mixed(torch_dev):
    """The same workload in mixed precision: FP32 Schur updates on fronts of order >= 1024,
    refined in FP64 to a normwise backward error <= 1e-10 against the oracle's residual."""
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_dense_cols()
    g = run(torch_dev, lp, 1, ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"])
    nw = berr_columns(lp, g)
    ss = g["ss"]
    print(f"dense columns mixed: initial {ss['berr_nw_initial']:.2e} final {ss['berr_nw']:.2e} oracle {nw.max():.2e} "
          f"steps {ss['max_steps']}")
    assert nw.max() <= 1e-10 and ss["berr_nw"] <= 1e-10 and ss["status"] == 0
    assert abs(nw.max() - ss["berr_nw"]) <= 0.1 * nw.max() + 64 * U
