"""Decision-by-decision parity of the pivot-window kernel with the oracle (needs an MI355X).

The library takes the oracle's ordering and fundamental supernodes (amalgamation off), so both
sides see the same fronts and the same 64-column windows (Section 4.4).  The cases
(tests/parity_bounds.py) have a largest front of order 129..300 that holds 2x2 pivots,
Proposition 3 and sign-rule events (Section 4.6), with the presort on, and off (Bunch-Kaufman
branch (d)); with small_front = 1 every front, also those with the lifts, goes through the
window kernel.  Decisions must be equal; D, the 2x2 off-diagonals and E_dyn within the derived
rounding bounds."""
import numpy as np
import pytest

from oracle import oracle as O

import parity_bounds as PB
from test_gpu_parity import check_pivot_values, gpu_solve, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("small_front", [64, 1])
@pytest.mark.parametrize("case", sorted(PB.MATCHED_CASES))
def test_window_kernel_decisions_match_oracle(torch_dev, case, small_front):
    lp, perm, presort = PB.matched_case(case)
    S = O.Sym(lp, perm)
    F = O.Num(S, lp["val"], lp["theta"], lp["rho"], lp["delta"], opts=O.default_opts(presort=presort))
    ex = F.export()
    st = F.stats()
    g = gpu_solve(torch_dev, lp, perm=S.perm(), amalgamate=0, presort=presort, small_front=small_front)
    s = g["solver"]
    assert np.array_equal(s.sym["sn_ptr"], S.snptr())
    front = np.asarray(s.sym["sn_front"])
    assert 129 <= front.max() <= 300
    gd = s.export_d()
    gf = s.export_flags()
    N = len(ex["fperm"])
    bad = np.nonzero((gd["pivot_order"] != ex["fperm"]) | (gd["ptype"] != ex["ptype"]) |
                     (gf != ex["eflag"].astype(np.uint8)))[0]
    u = int(bad[0]) if len(bad) else N
    print(f"  decisions agree on {u} of {N} positions; events "
          f"{dict((k, st[k]) for k in ('n2x2', 'nbkd', 'nlift', 'nprop3', 'nsign'))}")
    if u < N:
        k = u - 1 if ex["ptype"][u] == 2 else u  # the step that placed position u
        K = PB.dense_k_static(lp, lp["theta"], lp["rho"], lp["delta"])
        sigma, shift = PB.signs_shifts(lp, ex["fperm"])
        m = PB.decision_margins(K, ex, sigma, shift, S.snptr(), F.knorm(), presort)
        print(f"  first disagreement at {u}: gpu ({gd['pivot_order'][u]}, {gd['ptype'][u]}, {gf[u]}) "
              f"oracle ({ex['fperm'][u]}, {ex['ptype'][u]}, {ex['eflag'][u]}); margin/bound {m[k]:.3e}")
        assert not PB.MATCHED_CASES[case]["full"]
        assert m[k] < 1.0  # only where the input does not fix the decision at working precision
        assert u >= 64  # the first window at least
        check_pivot_values(lp, S, F, ex, gd, upto=k)
    else:
        fs = g["fstats"]
        for key in ("n2x2", "nlift", "nprop3", "nsign"):
            assert fs[key] == st[key], key
        assert (fs["nneg"], fs["npos"], fs["nzero"]) == (st["nneg"], st["npos"], st["nzero"])
        check_pivot_values(lp, S, F, ex, gd)
    s.close()
