"""Pins of the GPU-vs-oracle tolerances in parity_bounds.py (CPU only).

The bounds come from perturbation theory, so they are checked against perturbations whose
size is known: two solutions of one system with known residuals, and two oracle
factorisations of matrices that differ by a known diagonal perturbation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

import parity_bounds as PB

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


@pytest.mark.parametrize("cond", [1e2, 1e10])
def test_solution_gap_bound_holds_and_is_tight(cond):
    """x_g - x_o = K^-1 (r_o - r_g): for a perturbation of b along the direction K^-1 amplifies
    most, the gap reaches the bound to within a small factor; for any it stays below."""
    g = W.rng(900, int(np.log10(cond)))
    N = 60
    Q1, _ = np.linalg.qr(g.standard_normal((N, N)))
    Q2, _ = np.linalg.qr(g.standard_normal((N, N)))
    s = np.logspace(0, -np.log10(cond), N)
    K = Q1 @ np.diag(s) @ Q2.T
    x = g.standard_normal(N)
    b = K @ x
    xo = np.linalg.solve(K, b)
    for direction in ("worst", "random"):
        e = Q1[:, -1] if direction == "worst" else g.standard_normal(N)
        e = 1e-9 * e / np.abs(e).max()
        xg = np.linalg.solve(K, b + e)  # residual b - K xg = -e (plus rounding)
        gap, bound = PB.solution_gap_bound(K, b, xg, xo)
        assert gap <= bound
        if direction == "worst":
            assert gap >= bound / (10 * N)


def _oracle_pair(lp, perm, theta2, presort=1):
    S = O.Sym(lp, perm)
    opts = O.default_opts(presort=presort)
    F1 = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"], opts=opts)
    F2 = O.Num(S, lp["val"], theta2, lp["rho"], lp["delta"], opts=opts)
    return S, F1, F2


@pytest.mark.parametrize("case", sorted(PB.MATCHED_CASES))
def test_matched_cases_exercise_every_pivot_rule_in_large_fronts(case):
    """The GPU's matched-mode cases: in the oracle, fronts above 64 rows (the pivot-window
    kernel's at the default small-front cutoff) hold 2x2 pivots, Proposition 3 and sign-rule
    events, and without the presort Bunch-Kaufman branch (d) swaps; the largest front has
    129..300 rows.  Lifts occur in fronts of about 60 rows, which the GPU test also sends
    through the window kernel (small_front = 1)."""
    lp, perm, presort = PB.matched_case(case)
    S = O.Sym(lp, perm)
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"], opts=O.default_opts(presort=presort))
    ex, st = F.export(dense=False), F.stats()
    rp, _ = S.front_rows()
    front = np.diff(rp)
    snp = S.snptr()
    big = np.repeat(front > 64, np.diff(snp))  # per position: in a front of more than 64 rows
    assert 129 <= front.max() <= 300
    assert ((ex["ptype"] == 1) & big).sum() > 0
    for bit in (PB.EF_PROP3, PB.EF_SIGN):
        assert (((ex["eflag"] & bit) != 0) & big).sum() > 0, bit
    assert ((ex["eflag"] & PB.EF_LIFT) != 0).sum() > 0
    if presort == 0:
        assert st["nbkd"] > 0
    print(case, {k: st[k] for k in ("n2x2", "nbkd", "nprop3", "nsign", "nlift")})


@pytest.mark.parametrize("case", sorted(PB.MATCHED_CASES))
def test_pivot_bounds_cover_a_known_perturbation(case):
    """Theta perturbed by a relative 1e-10 moves M = P (K + E) P^T by a known diagonal dM;
    with gamma = max |dM_ll| / (|L||D||L^T|)_ll (plus both factorisations' rounding), the
    first-order bounds contain every change of D, of the 2x2 off-diagonals and of E_dyn
    between the two oracle factorisations, which take the same decisions.  On the wide-Theta
    case the naive bound gamma (|L||D||L^T|)_kk, without the amplification through the
    eliminated rows, does not: its pivots are far more sensitive than their own entries."""
    lp, perm, presort = PB.matched_case(case)
    g = W.rng(901)
    theta2 = lp["theta"] * (1.0 + 1e-10 * g.uniform(-1, 1, lp["n"]))
    S, F1, F2 = _oracle_pair(lp, perm, theta2, presort)
    e1, e2 = F1.export(), F2.export()
    assert np.array_equal(e1["fperm"], e2["fperm"]) and np.array_equal(e1["ptype"], e2["ptype"])
    assert np.array_equal(e1["eflag"], e2["eflag"])
    K1 = PB.dense_k_static(lp, lp["theta"], lp["rho"], lp["delta"])
    K2 = PB.dense_k_static(lp, theta2, lp["rho"], lp["delta"])
    fp = e1["fperm"]
    dM = np.abs(np.diag(K2 - K1))[fp]
    D1 = PB._block_d(e1["d"], e1["doff"], e1["ptype"])
    G = np.abs(e1["L"]) @ np.abs(D1) @ np.abs(e1["L"]).T
    gamma = (dM / np.diag(G)).max() + 4 * (S.N + 16) * U
    sigma, shift = PB.signs_shifts(lp, fp)
    dE = e2["edyn"] - e1["edyn"]
    kn_rtol = abs(F2.knorm() - F1.knorm()) / F1.knorm() + 4 * U
    bd, bo, be, _ = PB.pivot_bounds(K1, e1, sigma, shift, S.snptr(), F1.knorm(), dE, gamma=gamma,
                                    knorm_rtol=kn_rtol)
    diff_d = np.abs(e2["d"] - e1["d"])
    print(f"{case}: max |dd|/bound {np.max(diff_d / bd):.3e}, 2x2 {int((e1['ptype'] == 1).sum())}, "
          f"flags {np.bincount(e1['eflag'].astype(np.int64), minlength=8)}")
    assert np.all(diff_d <= bd)
    two = e1["ptype"] == 1
    assert np.all(np.abs(e2["doff"] - e1["doff"])[two] <= bo[two])
    fl = e1["eflag"] != 0
    assert np.all(np.abs(dE)[fl] <= be[fl])
    # the bound is not vacuous; on wide Theta the naive one (no amplification) fails somewhere
    assert np.max(diff_d / bd) >= 1e-4
    naive = gamma * np.diag(G) + 2 * U * np.abs(e1["d"])
    if not PB.MATCHED_CASES[case]["full"]:
        assert np.any(diff_d > naive)
