"""Batches of independent systems analysed as one block-diagonal pattern."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import qdmf as Q
from paper_2508_04370_amd import workloads as W

import parity_bounds as PB
from test_analyse import _brute_structure


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(Q.LIB_PATH):
        from paper_2508_04370_amd import build as B
        B.build()
    O.build(force=False)


def small_batch(count, seed=41, mode=W.AS):
    lps = W.as_batch(count, seed=seed, mrange=(12, 40), drange=(0.05, 0.15))
    if mode == W.NE:
        for lp in lps:
            lp["mode"] = W.NE
            lp["delta"] = 1e-8
            lp["rho"] = 0.0
    return lps


def analysed(lps):
    h = Q.qdmf_create(-1, None, Q.qdmf_default_options())
    Q.qdmf_batch_analyse(h, lps, lps[0]["mode"])
    return h


@pytest.mark.parametrize("mode", [W.AS, W.NE])
def test_batch_offsets_and_block_structure(mode):
    lps = small_batch(5, mode=mode)
    h = analysed(lps)
    ro, co = Q.qdmf_batch_offsets(h, len(lps))
    assert np.array_equal(ro, np.concatenate([[0], np.cumsum([lp["m"] for lp in lps])]))
    assert np.array_equal(co, np.concatenate([[0], np.cumsum([lp["n"] for lp in lps])]))
    sy = Q.qdmf_symbolic(h)
    cat = W.concat_systems(lps)
    N = cat["n"] + cat["m"] if mode == W.AS else cat["m"]
    assert sy["N"] == N
    # the structure is exact for the combined pattern, and no supernode mixes systems
    Lp = _brute_structure(cat, sy["perm"])
    assert sy["nnz_l"] == Lp.sum()

    def system_of(v):
        if mode == W.AS:
            return int(np.searchsorted(co, v, "right") - 1) if v < cat["n"] else \
                int(np.searchsorted(ro, v - cat["n"], "right") - 1)
        return int(np.searchsorted(ro, v, "right") - 1)

    perm = sy["perm"]
    for s_ in range(sy["nsuper"]):
        cols = perm[sy["sn_ptr"][s_]:sy["sn_ptr"][s_ + 1]]
        assert len({system_of(v) for v in cols}) == 1
    Q.qdmf_destroy(h)


def test_batch_orders_each_system_as_alone():
    """Each system is ordered on its own: the batch's factor has exactly the sum of the
    systems' nnz(L) and flops, and a plain analyse of the concatenated pattern with the
    batch's permutation gives the same structure."""
    lps = small_batch(4)
    h = analysed(lps)
    a = Q.qdmf_symbolic(h)
    alone = [Q.Solver(lp, device=-1) for lp in lps]
    assert a["nnz_l"] == sum(s.sym["nnz_l"] for s in alone)
    assert a["flops_fact"] == sum(s.sym["flops_fact"] for s in alone)
    for s in alone:
        s.close()
    cat = W.concat_systems(lps)
    s = Q.Solver(cat, device=-1, perm=a["perm"])
    for k in ("N", "nsuper", "nnz_l", "flops_fact"):
        assert a[k] == s.sym[k], k
    s.close()
    Q.qdmf_destroy(h)


def test_batch_rejects_user_and_grid_orderings():
    lps = small_batch(2)
    for o in (Q.QDMF_ORDER_USER, Q.QDMF_ORDER_GRID_ND):
        h = Q.qdmf_create(-1, None, Q.qdmf_default_options(ordering=o))
        with pytest.raises(Q.QdmfError) as ei:
            Q.qdmf_batch_analyse(h, lps, W.AS)
        assert ei.value.code == Q.QDMF_ERR_INVALID_ARG
        Q.qdmf_destroy(h)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [W.AS, W.NE])
def test_batch_gpu_per_system_parity(mode):
    """Every system of a batch, with its own Theta, rho and delta, is solved to the FP64
    backward-error target against its own K_static (the oracle's residual), with its own
    inertia, and agrees with the oracle's solution of that system alone."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lps = small_batch(6, seed=43, mode=mode)
    cnt = len(lps)
    print(f"[gpu case] batch of {cnt} mode={mode}", flush=True)
    for q, lp in enumerate(lps):  # per-system shifts
        if mode == W.AS:
            lp["rho"], lp["delta"] = 1e-10 * (q + 1), 1e-9 * (q + 1)
        else:
            lp["rho"], lp["delta"] = 1e-6 * q, 1e-8 * (q + 1)
    thetas = [W.as_batch_theta(lp, q, 0, seed=43) for q, lp in enumerate(lps)]
    rhs = [W.as_batch_rhs(lp, q, 0, 0, seed=43) for q, lp in enumerate(lps)]
    cat = W.concat_systems(lps)
    dev = "cuda:0"
    h = Q.qdmf_create(0, torch.cuda.current_stream().cuda_stream, Q.qdmf_default_options())
    Q.qdmf_batch_analyse(h, lps, mode)
    Q.qdmf_set_matrix(h, cat["val"])
    th = torch.from_numpy(np.concatenate(thetas)).to(dev)
    Q.qdmf_batch_factorise(h, th, [lp["rho"] for lp in lps], [lp["delta"] for lp in lps])
    r7 = torch.from_numpy(np.concatenate([r[0] for r in rhs])).to(dev).reshape(-1, 1)
    r1 = torch.from_numpy(np.concatenate([r[1] for r in rhs])).to(dev).reshape(-1, 1)
    dx = torch.empty((cat["n"], 1), dtype=torch.float64, device=dev)
    dy = torch.empty((cat["m"], 1), dtype=torch.float64, device=dev)
    Q.qdmf_solve(h, 1, r7 if mode == W.AS else r7, r1, dx, dy)
    bs = Q.qdmf_batch_stats(h, cnt, nrhs=1)
    dxh, dyh = dx.cpu().numpy()[:, 0], dy.cpu().numpy()[:, 0]
    for q, lp in enumerate(lps):
        c0, c1 = cat["col_off"][q], cat["col_off"][q + 1]
        r0_, r1_ = cat["row_off"][q], cat["row_off"][q + 1]
        x = np.concatenate([dxh[c0:c1], dyh[r0_:r1_]]) if mode == W.AS else dyh[r0_:r1_]
        b = O.system_rhs(lp, rhs[q][0], rhs[q][1], thetas[q])
        _, nw, _, _ = O.residual(lp, thetas[q], lp["rho"], lp["delta"], x, b)
        S = O.Sym(lp)
        F = O.Num(S, lp["val"], thetas[q], lp["rho"], lp["delta"])
        ro = F.solve(rhs[q][0], rhs[q][1])
        xo = np.concatenate([ro["dx"][:, 0], ro["dy"][:, 0]]) if mode == W.AS else ro["dy"][:, 0]
        rel = np.abs(x - xo).max() / max(np.abs(xo).max(), 1e-300)
        K = PB.dense_k_static(lp, thetas[q], lp["rho"], lp["delta"])
        gap, bound = PB.solution_gap_bound(K, b, x, xo)
        print(f"  system {q}: m={lp['m']} berr_nw={nw:.2e} reported={bs['berr_nw'][0, q]:.2e} rel={rel:.2e} "
              f"bound {bound / max(np.abs(xo).max(), 1e-300):.2e}")
        assert gap <= bound
        assert nw <= 1e-12
        assert bs["berr_nw"][0, q] <= 1e-12
        st = F.stats()
        assert tuple(bs["inertia"][q]) == (st["nneg"], st["npos"], st["nzero"])
        assert tuple(bs["inertia"][q][:2]) == ((lp["n"], lp["m"]) if mode == W.AS else (0, lp["m"]))
    Q.qdmf_destroy(h)
