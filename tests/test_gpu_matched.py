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
    # first disagreement, if any, for the report
    bad = np.nonzero((gd["pivot_order"] != ex["fperm"]) | (gd["ptype"] != ex["ptype"]) |
                     (gf != ex["eflag"].astype(np.uint8)))[0]
    if len(bad):
        k = int(bad[0])
        print(f"  first disagreement at position {k}: gpu ({gd['pivot_order'][k]}, {gd['ptype'][k]}, {gf[k]}) "
              f"oracle ({ex['fperm'][k]}, {ex['ptype'][k]}, {ex['eflag'][k]})")
    assert np.array_equal(gd["pivot_order"], ex["fperm"])
    assert np.array_equal(gd["ptype"], ex["ptype"])
    assert np.array_equal(gf, ex["eflag"].astype(np.uint8))
    fs = g["fstats"]
    for key in ("n2x2", "nlift", "nprop3", "nsign"):
        assert fs[key] == st[key], key
    assert (fs["nneg"], fs["npos"], fs["nzero"]) == (st["nneg"], st["npos"], st["nzero"])
    print(f"  events: {dict((k, st[k]) for k in ('n2x2', 'nbkd', 'nlift', 'nprop3', 'nsign'))}")
    check_pivot_values(lp, S, F, ex, gd)
    s.close()
