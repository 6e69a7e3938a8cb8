"""GPU path vs the CPU oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

import parity_bounds as PB

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


def gpu_solve(torch_dev, lp, prec=0, theta=None, r7=None, r1=None, perm=None, **opts):
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    theta = lp["theta"] if theta is None else theta
    r1 = lp["r1"] if r1 is None else r1
    if r7 is None and lp["mode"] == W.AS:
        r7 = lp["r7"]
    print(f"[gpu case] {lp['name']} N={lp['n'] + lp['m'] if lp['mode'] else lp['m']} prec={prec} "
          f"opts={opts} user_perm={perm is not None}", flush=True)
    s = Q.Solver(lp, device=0, perm=perm, **opts)
    th = torch.from_numpy(np.ascontiguousarray(theta)).to(dev)
    s.factorise(th, lp["rho"], lp["delta"], prec)
    r1d = Q.to_device_colmajor(r1, dev)
    r7d = None if r7 is None else Q.to_device_colmajor(r7, dev)
    dx, dy = s.solve(r7d, r1d)
    torch.cuda.synchronize()
    nrhs = r1d.shape[1]
    out = dict(dx=dx.cpu().numpy(), dy=dy.cpu().numpy(), fstats=s.factor_stats(),
               sstats=s.solve_stats(nrhs), solver=s)
    return out


def system_x(lp, dx, dy):
    return np.concatenate([dx, dy]) if lp["mode"] == W.AS else dy


def oracle_berr(lp, theta, x, r7, r1):
    b = O.system_rhs(lp, r7, r1, theta)
    _, nw, cw, _ = O.residual(lp, theta, lp["rho"], lp["delta"], x, b)
    return nw, cw


def check_solution_gap(lp, theta, x, xo, b, N_max=3000):
    """||x - x_oracle||_inf within ||K^-1||_inf times the two residuals (the exact form of the
    kappa-times-backward-error bound, tests/parity_bounds.py), for systems of order <= N_max
    where K_static can be written out densely."""
    if len(x) > N_max or len(x) == 0:
        return None
    K = PB.dense_k_static(lp, theta, lp["rho"], lp["delta"])
    gap, bound = PB.solution_gap_bound(K, b, x, xo)
    assert gap <= bound, (gap, bound)
    return gap / max(np.abs(xo).max(), 1e-300), bound / max(np.abs(xo).max(), 1e-300)


def check_against_oracle(lp, g, berr=1e-12):
    theta = lp["theta"]
    r7 = lp.get("r7") if lp["mode"] == W.AS else None
    S = O.Sym(lp)
    F = O.Num(S, lp["val"], theta, lp["rho"], lp["delta"])
    ro = F.solve(r7, lp["r1"])
    nrhs = lp["r1"].shape[1]
    for c in range(nrhs):
        x = system_x(lp, g["dx"][:, c], g["dy"][:, c])
        r7c = None if r7 is None else r7[:, c]
        nw, _ = oracle_berr(lp, theta, x, r7c, lp["r1"][:, c])
        assert nw <= berr, (c, nw)
        xo = system_x(lp, ro["dx"][:, c], ro["dy"][:, c])
        rel = np.abs(x - xo).max() / max(np.abs(xo).max(), 1e-300)
        b = O.system_rhs(lp, r7c, lp["r1"][:, c], theta)
        gb = check_solution_gap(lp, theta, x, xo, b)
        print(f"  rhs {c}: berr_nw={nw:.2e} gpu_reported={g['sstats']['berr_nw_per_rhs'][c]:.2e} "
              f"steps={g['sstats']['steps_per_rhs'][c]} |x-x_oracle|/|x_oracle|={rel:.2e}"
              + ("" if gb is None else f" (bound {gb[1]:.2e})"))
    st = F.stats()
    fs = g["fstats"]
    assert (fs["nneg"], fs["npos"], fs["nzero"]) == (st["nneg"], st["npos"], st["nzero"])
    if lp["mode"] == W.AS:
        assert (fs["nneg"], fs["npos"]) == (lp["n"], lp["m"])
    else:
        assert (fs["nneg"], fs["npos"]) == (0, lp["m"])
    assert np.isclose(fs["knorm"], F.knorm(), rtol=1e-13)
    return ro


def test_ne_random_fp64(torch_dev):
    lp = W.ne_random()
    g = gpu_solve(torch_dev, lp)
    check_against_oracle(lp, g)


def test_small_staircase_fp64(torch_dev):
    lp = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10)
    g = gpu_solve(torch_dev, lp)
    check_against_oracle(lp, g)


def test_dense_ne_large_front_windows(torch_dev):
    """A nearly dense normal-equations matrix: one front of order ~200 factorised by the
    windowed kernels (assembly, diagonal block, panel, MFMA update, row swaps)."""
    lp = W.ne_random(m=200, n=400, density=0.08, seed=21)
    g = gpu_solve(torch_dev, lp)
    assert g["solver"].sym["max_front"] > 64
    check_against_oracle(lp, g)


@pytest.mark.parametrize("split", [1024, 1])
@pytest.mark.parametrize("case", ["dense_ne", "staircase"])
def test_mid_size_fronts_solves(torch_dev, case, split):
    """Fronts of order 256..1024 with more than 32 pivots: the one-workgroup solve kernels take
    several trips over the rows below each block (and several blocks); with split_solve_front
    = 1 the multi-workgroup solves take them in 256-pivot blocks (two or more, the last
    partial); solution and backward error against the oracle."""
    if case == "dense_ne":
        lp = W.ne_random(m=420, n=840, density=0.05, seed=23)
    else:
        lp = W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24)
    if split == 1:
        lp = W.LP(dict(lp, r1=np.hstack([lp["r1"]] * 3), r7=np.hstack([lp["r7"]] * 3)))
        lp["r1"][:, 1] *= -2.0
        lp["r1"][:, 2] = W.rng(25).standard_normal(lp["m"])
    g = gpu_solve(torch_dev, lp, split_solve_front=split)
    sym = g["solver"].sym
    print(f"  max front {sym['max_front']}")
    assert 256 < sym["max_front"] < 1024
    check_against_oracle(lp, g)


def test_ne_with_r7_recovers_dx(torch_dev):
    lp = W.ne_random(m=120, n=240, density=0.03, seed=5, rho=1e-6)
    g7 = W.rng(77)
    r7 = g7.standard_normal((lp["n"], 1))
    g = gpu_solve(torch_dev, lp, r7=r7)
    S = O.Sym(lp)
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"])
    ro = F.solve(r7, lp["r1"])
    for key in ("dx", "dy"):
        a, b = g[key][:, 0], ro[key][:, 0]
        print(key, np.abs(a - b).max() / np.abs(b).max())
    # the augmented system built from the same data is solved by (dx, dy)
    lpa = W.LP(dict(lp, mode=W.AS))
    nw, _ = oracle_berr(lpa, lp["theta"], np.concatenate([g["dx"][:, 0], g["dy"][:, 0]]), r7[:, 0],
                        lp["r1"][:, 0])
    assert nw <= 1e-11, nw


@pytest.mark.parametrize("trange,reg", [((1e-10, 1e10), 1e-10), ((1e-1, 1e1), 1e-2)])
def test_matched_mode_reproduces_oracle_pivots(torch_dev, trange, reg):
    """Oracle ordering fed to the GPU with fundamental supernodes: same supernodes and
    windows, so every pivot decision (order, 1x1/2x2, regularisation flags) must match the
    oracle exactly.  Pivot values agree to rounding amplified by conditioning: on the
    well-conditioned case they must agree to 1e-12 relative."""
    lp = W.as_staircase(periods=3, rows=40, cols=80, link_cols=8, seed=9, theta_range=trange,
                        rho=reg, delta=reg)
    S = O.Sym(lp)
    perm = S.perm()
    g = gpu_solve(torch_dev, lp, perm=perm, amalgamate=0)
    s = g["solver"]
    assert np.array_equal(s.sym["perm"], perm)
    assert np.array_equal(s.sym["sn_ptr"], S.snptr())
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"])
    ex = F.export()
    gd = s.export_d()
    agree = np.mean(gd["pivot_order"] == ex["fperm"])
    print("pivot order agreement", agree)
    assert agree == 1.0
    assert np.array_equal(gd["ptype"], ex["ptype"])
    assert np.array_equal(s.export_flags(), ex["eflag"].astype(np.uint8))
    check_pivot_values(lp, S, F, ex, gd)
    if trange[0] >= 1e-1:  # well conditioned: the bound itself is at the rounding level
        rel = np.abs(gd["d"] - ex["d"]) / np.abs(ex["d"])
        assert rel.max() <= 1e-12


def check_pivot_values(lp, S, F, ex, gd, upto=None):
    """D, the 2x2 off-diagonals and E_dyn of the GPU's factor against the oracle's, for the
    same pivot sequence, within the first-order rounding bounds of tests/parity_bounds.py
    (positions before `upto` only, when the sequences part there)."""
    K = PB.dense_k_static(lp, lp["theta"], lp["rho"], lp["delta"])
    sigma, shift = PB.signs_shifts(lp, ex["fperm"])
    dE = gd["edyn"] - ex["edyn"]
    bd, bo, be, _ = PB.pivot_bounds(K, ex, sigma, shift, S.snptr(), F.knorm(), dE)
    if upto is not None:
        keep = np.arange(len(bd)) < upto
        bd, bo, be = np.where(keep, bd, np.inf), np.where(keep, bo, np.inf), np.where(keep, be, np.inf)
        gd = dict(gd, edyn=np.where(keep, gd["edyn"], ex["edyn"]))
        dE = gd["edyn"] - ex["edyn"]
    dd = np.abs(gd["d"] - ex["d"])
    if upto is not None:
        dd = np.where(np.arange(len(dd)) < upto, dd, 0.0)
    k = int(np.argmax(dd / bd))
    print(f"  |d_gpu - d_oracle| / bound: max {dd[k] / bd[k]:.3e} at {k} (d {ex['d'][k]:.6e}, "
          f"ptype {ex['ptype'][k]}, flag {ex['eflag'][k]})")
    assert np.all(dd <= bd), np.nonzero(dd > bd)[0][:10]
    two = ex["ptype"] == 1
    assert np.all(np.abs(gd["doff"] - ex["doff"])[two] <= bo[two])
    fl = ex["eflag"] != 0
    assert np.all(gd["edyn"][~fl] == 0) and np.all(ex["edyn"][~fl] == 0)
    if fl.any():
        print(f"  |E_gpu - E_oracle| / bound: max {np.max(np.abs(dE)[fl] / be[fl]):.3e} over {int(fl.sum())} pivots")
    assert np.all(np.abs(dE)[fl] <= be[fl])


def test_matched_mode_without_presort(torch_dev):
    """The same with the presort swap switched off on both sides: the window's pivot steps take
    positions in order, and every decision must still match the oracle's."""
    lp = W.as_staircase(periods=3, rows=40, cols=80, link_cols=8, seed=9, theta_range=(1e-1, 1e1),
                        rho=1e-2, delta=1e-2)
    S = O.Sym(lp)
    g = gpu_solve(torch_dev, lp, perm=S.perm(), amalgamate=0, presort=0)
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"], opts=O.default_opts(presort=0))
    ex = F.export()
    gd = g["solver"].export_d()
    assert np.array_equal(gd["pivot_order"], ex["fperm"])
    assert np.array_equal(gd["ptype"], ex["ptype"])
    assert np.array_equal(g["solver"].export_flags(), ex["eflag"].astype(np.uint8))
    check_pivot_values(lp, S, F, ex, gd)
    rel = np.abs(gd["d"] - ex["d"]) / np.abs(ex["d"])
    print("max relative pivot difference", rel.max())
    assert rel.max() <= 1e-12


def test_full_staircase_fp64(torch_dev):
    lp = W.as_staircase()
    g = gpu_solve(torch_dev, lp)
    fs = g["fstats"]
    print("factor stats", fs)
    assert (fs["nneg"], fs["npos"]) == (lp["n"], lp["m"])
    x = system_x(lp, g["dx"][:, 0], g["dy"][:, 0])
    nw, cw = oracle_berr(lp, lp["theta"], x, lp["r7"][:, 0], lp["r1"][:, 0])
    print(f"full staircase: berr_nw={nw:.2e} berr_cw={cw:.2e} gpu={g['sstats']}")
    assert nw <= 1e-12


def test_determinism_bitwise(torch_dev):
    lp = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10)
    a = gpu_solve(torch_dev, lp)
    b = gpu_solve(torch_dev, lp)
    assert np.array_equal(a["dx"], b["dx"]) and np.array_equal(a["dy"], b["dy"])
    da, db = a["solver"].export_d(), b["solver"].export_d()
    assert np.array_equal(da["d"], db["d"])


def _dense_factor(s, N):
    gd = s.export_d()
    po = gd["pivot_order"]
    pos = np.empty(N, np.int64)
    pos[po] = np.arange(N)
    L = np.eye(N)
    D = np.diag(gd["d"])
    for k in np.nonzero(gd["ptype"] == 1)[0]:
        D[k, k + 1] = D[k + 1, k] = gd["doff"][k]
    snp = s.sym["sn_ptr"]
    for sidx in range(len(snp) - 1):
        panel, rows = s.export_front(sidx)
        f, p = panel.shape
        for k in range(p):
            L[pos[rows[k + 1:]], snp[sidx] + k] = panel[k + 1:, k]
    return po, L, D, gd["edyn"]


@pytest.mark.parametrize("amalgamate,split", [(0, 1024), (1, 1024), (1, 1)])
def test_factor_backward_stable_and_solve_matches_its_factor(torch_dev, amalgamate, split):
    """||P K P^T - L D L^T|| small (no dynamic regularisation here), and the GPU solve
    (no refinement) equals a dense solve with the GPU's own factor; split = 1 sends every
    supernode through the multi-workgroup solves."""
    from test_oracle import dense_K
    lp = W.as_staircase(periods=3, rows=40, cols=80, link_cols=8, seed=9, theta_range=(1e-2, 1e2))
    g = gpu_solve(torch_dev, lp, amalgamate=amalgamate, max_refine=0, split_solve_front=split)
    s = g["solver"]
    N = s.N
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    po, L, D, ed = _dense_factor(s, N)
    R = K[np.ix_(po, po)] + np.diag(ed) - L @ D @ L.T
    scale = np.abs(L) @ np.abs(D) @ np.abs(L).T
    print("reconstruction error / (|L||D||L^T|)_max:", np.abs(R).max() / scale.max())
    assert np.abs(R).max() <= 100 * s.sym["max_front"] * U * scale.max()
    # the GPU's forward/D/backward solves are backward stable for its own factor:
    # ||b - L D L^T x||_inf <= c f u (|| |L||D||L^T| ||_inf ||x||_inf + ||b||_inf)
    b = np.concatenate([lp["r7"][:, 0], lp["r1"][:, 0]])[po]
    x = system_x(lp, g["dx"][:, 0], g["dy"][:, 0])[po]
    r = b - L @ (D @ (L.T @ x))
    bound = np.abs(scale).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()
    print("solve backward error vs own factor:", np.abs(r).max() / bound)
    assert np.abs(r).max() <= 100 * s.sym["max_front"] * U * bound


@pytest.mark.parametrize("case", ["dense_ne", "staircase_20rhs"])
def test_split_solves_match_oracle(torch_dev, case):
    """Multi-workgroup solves on every supernode (split_solve_front = 1, all right-hand
    sides per launch, per-rhs refinement flags): same backward-error target, inertia and
    norm as the oracle.  dense_ne has a front of order ~200 (several 64-pivot blocks and
    256-row chunks); 20 right-hand sides cross the kernels' groups of 8 and 16."""
    if case == "dense_ne":
        lp = W.ne_random(m=200, n=400, density=0.08, seed=21)
    else:
        lp = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10, nrhs=20)
    g = gpu_solve(torch_dev, lp, split_solve_front=1)
    check_against_oracle(lp, g)


def test_joined_split_solves_match_oracle(torch_dev):
    """A level that holds a front of at least split_solve_front rows takes its other fronts of
    at least 128 rows (with no more 64-pivot blocks) into the same multi-workgroup launches:
    a staircase whose levels mix both kinds, against the oracle."""
    lp = W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24, nrhs=3)
    split = 200
    g = gpu_solve(torch_dev, lp, split_solve_front=split)
    sym = g["solver"].sym
    f, lv = np.asarray(sym["sn_front"]), np.asarray(sym["sn_level"])
    nblk = (np.diff(np.asarray(sym["sn_ptr"])) + 63) // 64
    joined = 0
    for level in np.unique(lv):
        on = lv == level
        big = on & (f >= split)
        if big.any():
            joined += int((on & (f >= 128) & (f < split) & (nblk <= nblk[big].max())).sum())
    print(f"  fronts joining split launches: {joined}")
    assert joined > 0
    check_against_oracle(lp, g)


def test_split_solves_wide_theta_own_factor(torch_dev):
    """Theta over [1e-10, 1e10] (2x2 pivots and tiny pivots possible): with no refinement
    the multi-workgroup solves are backward stable for the GPU's own factor, like the
    one-workgroup solves."""
    lp = W.as_staircase(periods=3, rows=40, cols=80, link_cols=8, seed=9, theta_range=(1e-10, 1e10),
                        rho=1e-10, delta=1e-10)
    for split in (1024, 1):
        g = gpu_solve(torch_dev, lp, max_refine=0, split_solve_front=split, amalgamate=0)
        s = g["solver"]
        po, L, D, _ = _dense_factor(s, s.N)
        print(f"split {split}: 2x2 pivots {int((s.export_d()['ptype'] == 1).sum())}")
        scale = np.abs(L) @ np.abs(D) @ np.abs(L).T
        b = np.concatenate([lp["r7"][:, 0], lp["r1"][:, 0]])[po]
        x = system_x(lp, g["dx"][:, 0], g["dy"][:, 0])[po]
        r = b - L @ (D @ (L.T @ x))
        bound = np.abs(scale).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()
        print("solve backward error vs own factor:", np.abs(r).max() / bound)
        assert np.abs(r).max() <= 100 * s.sym["max_front"] * U * bound
        s.close()


def test_multiple_rhs(torch_dev):
    lp = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10, nrhs=3)
    g = gpu_solve(torch_dev, lp)
    check_against_oracle(lp, g)


@pytest.mark.parametrize("lpname", ["dense_ne", "staircase"])
def test_mixed_precision_refines_to_target(torch_dev, lpname):
    """FP32 MFMA Schur updates on every large front (f_mix lowered so they apply here);
    FP64 refinement must bring the normwise backward error to <= 1e-10."""
    if lpname == "dense_ne":
        lp = W.ne_random(m=300, n=600, density=0.08, seed=22)
    else:
        lp = W.as_staircase(periods=6, rows=120, cols=240, link_cols=30, seed=23)
    g64 = gpu_solve(torch_dev, lp, prec=0, f_mix=65)
    gmx = gpu_solve(torch_dev, lp, prec=1, f_mix=65)
    assert gmx["solver"].sym["max_front"] >= 65
    ss = gmx["sstats"]
    print(f"mixed: initial berr {ss['berr_nw_initial']:.2e} final {ss['berr_nw']:.2e} steps {ss['max_steps']}; "
          f"fp64 initial {g64['sstats']['berr_nw_initial']:.2e}")
    r7 = lp["r7"][:, 0] if lp["mode"] == W.AS else None
    x = system_x(lp, gmx["dx"][:, 0], gmx["dy"][:, 0])
    nw, _ = oracle_berr(lp, lp["theta"], x, r7, lp["r1"][:, 0])
    assert nw <= 1e-10, nw
    # the FP32 updates really ran: the unrefined mixed solution is less accurate
    assert ss["berr_nw_initial"] > g64["sstats"]["berr_nw_initial"]
    from paper_2508_04370_amd import qdmf as Q
    if lp["mode"] == W.AS:
        fs = g64["fstats"]
        assert (fs["nneg"], fs["npos"]) == (lp["n"], lp["m"])
        fs = gmx["fstats"]
        if (fs["nneg"], fs["npos"]) != (lp["n"], lp["m"]):
            # 1x1 pivots keep their expected signs (sign rule); a 2x2 block formed from
            # FP32-updated entries can carry the other inertia, which the library reports
            print("  mixed inertia", fs["nneg"], fs["npos"], "2x2 blocks", fs["n2x2"], "status", fs["rc"])
            assert fs["n2x2"] > 0 and fs["rc"] in (Q.QDMF_WARN_INERTIA, Q.QDMF_WARN_LARGE_REG)
            assert fs["nneg"] + fs["npos"] == lp["n"] + lp["m"]


@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_precision_hard_case_is_safe(torch_dev, seed):
    """Theta over [1e-8, 1e8] and a nearly dense front above f_mix: FP32 Schur updates may
    leave the factor too inaccurate for the refinement to reach 1e-10.  What must hold:
    refinement never returns a worse iterate than it started from, the reported backward
    error is the true one (the oracle's residual against K_static), and a miss of the
    target is reported as QDMF_WARN_NOT_CONVERGED."""
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_batch_system(seed, seed=61, mrange=(1100, 1200), drange=(0.02, 0.03))
    lp["theta"] = W.as_batch_theta(lp, seed, 0, seed=61)
    r7, r1 = W.as_batch_rhs(lp, seed, 0, 0, seed=61)
    lp["r7"], lp["r1"] = r7.reshape(-1, 1), r1.reshape(-1, 1)
    gmx = gpu_solve(torch_dev, lp, prec=1)
    assert gmx["solver"].sym["max_front"] >= 1024
    ss = gmx["sstats"]
    x = system_x(lp, gmx["dx"][:, 0], gmx["dy"][:, 0])
    nw, _ = oracle_berr(lp, lp["theta"], x, r7, r1)
    print(f"mixed hard: initial berr {ss['berr_nw_initial']:.2e} final {ss['berr_nw']:.2e} "
          f"(oracle residual {nw:.2e}) steps {ss['max_steps']} status {ss['status']}")
    assert ss["berr_nw"] <= ss["berr_nw_initial"]
    assert abs(nw - ss["berr_nw"]) <= 0.1 * max(nw, 1e-300)
    assert (ss["status"] == Q.QDMF_WARN_NOT_CONVERGED) == (ss["berr_nw"] > 1e-10)


@pytest.mark.parametrize("case", ["small", "one_graph", "grouped", "lookahead"])
def test_graph_replay_matches_eager(torch_dev, case):
    """factorise + 2 solves captured once; replays read refreshed Theta and rhs in place
    and must reproduce the eager results bitwise, every replay.  "grouped": fronts of up to
    ~300 rows with their trailing updates grouped three windows at a time; "lookahead": the
    same with the updates past the next group on the second stream, which the capture forks
    and joins; "one_graph": the capture is not cut at the refinement decisions (graph_poll =
    0), so every pass is in the graph and finished ones return at once."""
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    if case in ("small", "one_graph"):
        lp, opts = W.as_staircase(periods=4, rows=50, cols=100, link_cols=10), {}
        if case == "one_graph":
            opts["graph_poll"] = 0
    else:
        lp = W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24)
        opts = dict(syrk_group_front=64, syrk_group=3)
        if case == "lookahead":
            opts["lookahead_front"] = 64
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = Q.Solver(lp, device=0, stream=stream.cuda_stream, **opts)
        th = torch.empty(lp["n"], dtype=torch.float64, device=dev)
        r7 = torch.empty((1, lp["n"]), dtype=torch.float64, device=dev).T
        r1 = torch.empty((1, lp["m"]), dtype=torch.float64, device=dev).T
        dx = torch.empty((1, lp["n"]), dtype=torch.float64, device=dev).T
        dy = torch.empty((1, lp["m"]), dtype=torch.float64, device=dev).T

        def refresh(k):
            g = W.rng(55, k)
            th.copy_(torch.from_numpy(W.log_uniform(g, 1e-10, 1e10, lp["n"])))
            r7.copy_(torch.from_numpy(g.standard_normal((lp["n"], 1))))
            r1.copy_(torch.from_numpy(g.standard_normal((lp["m"], 1))))

        refresh(0)
        Q.qdmf_graph_capture(s.h, th, lp["rho"], lp["delta"], 0, 2, 1, r7, r1, dx, dy)
        for k in range(3):
            refresh(k)
            stream.synchronize()
            Q.qdmf_graph_launch(s.h)
            stream.synchronize()
            gx, gy = dx.cpu().numpy().copy(), dy.cpu().numpy().copy()
            # eager on a fresh handle with the same inputs
            e = Q.Solver(lp, device=0, stream=stream.cuda_stream, **opts)
            e.factorise(th, lp["rho"], lp["delta"], 0)
            ex, ey = e.solve(r7, r1)
            e.solve(r7, r1, ex, ey)
            stream.synchronize()
            assert np.array_equal(gx, ex.cpu().numpy()) and np.array_equal(gy, ey.cpu().numpy()), k
            x = np.concatenate([gx[:, 0], gy[:, 0]])
            nw, _ = oracle_berr(lp, th.cpu().numpy(), x, r7.cpu().numpy()[:, 0], r1.cpu().numpy()[:, 0])
            assert nw <= 1e-12
            e.close()
        s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_dense_columns_small(torch_dev, prec):
    """The dense-column augmented system at a size the oracle solves in seconds (rows on a
    10 x 8 x 8 grid, 5 dense columns of ~320 entries): the residual and the Krylov products sum
    those long columns with one workgroup each.  FP64: backward error <= 1e-12 and the solution
    against the oracle's; mixed (f_mix lowered): <= 1e-10.  Both: the backward error the library
    reports is the true one (the oracle's residual) up to the residual's own rounding."""
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_dense_cols(10, 8, 8, ndense=5)
    assert (np.diff(lp["colptr"]) > 128).sum() == 5
    g = gpu_solve(torch_dev, lp, prec=prec, ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"], f_mix=64)
    x = system_x(lp, g["dx"][:, 0], g["dy"][:, 0])
    nw, _ = oracle_berr(lp, lp["theta"], x, lp["r7"][:, 0], lp["r1"][:, 0])
    rep = g["sstats"]["berr_nw"]
    print(f"  dense columns prec {prec}: berr {nw:.2e} reported {rep:.2e} steps {g['sstats']['max_steps']}")
    assert abs(nw - rep) <= 0.1 * nw + 64 * U
    if prec == 0:
        check_against_oracle(lp, g)
    else:
        assert nw <= 1e-10
