"""Grouped trailing updates (the syrk_group_front / syrk_group options) on the GPU path,
through the C ABI (needs an MI355X): a front applies the Schur update of several consecutive
pivot windows to its trailing matrix at once, and only the next window's columns are brought
up to date inside a group.  Checked against the oracle, by the factor's reconstruction, and
with a group of one window against the ungrouped path bit for bit."""
import numpy as np
import pytest

from paper_2508_04370_amd import workloads as W

from test_gpu_edge import dense_as
from test_gpu_parity import U, _dense_factor, check_against_oracle, gpu_solve, system_x, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def case(name):
    if name == "dense_ne":  # one front of order ~200 with four windows
        return W.ne_random(m=200, n=400, density=0.08, seed=21)
    if name == "ne_front_300":  # a dense front of order 300: five windows, the last partial
        return W.ne_dense_front(300, seed=3, nrhs=2)
    if name == "staircase":  # fronts of order up to ~300 beside many small ones
        return W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24)
    raise KeyError(name)


@pytest.mark.parametrize("group", [2, 3, 4])
@pytest.mark.parametrize("name", ["dense_ne", "ne_front_300", "staircase"])
def test_grouped_updates_match_oracle(torch_dev, name, group):
    lp = case(name)
    g = gpu_solve(torch_dev, lp, syrk_group_front=64, syrk_group=group)
    check_against_oracle(lp, g)


@pytest.mark.parametrize("group", [2, 3])
def test_grouped_updates_reconstruct_K(torch_dev, group):
    """A dense augmented system whose largest front has order 129 (windows of 64, 64 and 1
    pivots): ||P K P^T + E - L D L^T|| within the factorisation's error bound, and the solve
    (no refinement) backward stable for that factor."""
    from test_oracle import dense_K
    lp = dense_as(62, 67)
    g = gpu_solve(torch_dev, lp, max_refine=0, syrk_group_front=64, syrk_group=group)
    s = g["solver"]
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    po, L, D, ed = _dense_factor(s, s.N)
    R = K[np.ix_(po, po)] + np.diag(ed) - L @ D @ L.T
    scale = np.abs(L) @ np.abs(D) @ np.abs(L).T
    print("reconstruction error / (|L||D||L^T|)_max:", np.abs(R).max() / scale.max())
    assert np.abs(R).max() <= 100 * s.sym["max_front"] * U * scale.max()
    b = np.concatenate([lp["r7"][:, 0], lp["r1"][:, 0]])[po]
    x = system_x(lp, g["dx"][:, 0], g["dy"][:, 0])[po]
    r = b - L @ (D @ (L.T @ x))
    bound = np.abs(scale).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()
    assert np.abs(r).max() <= 100 * s.sym["max_front"] * U * bound


def test_group_of_one_window_is_the_ungrouped_path(torch_dev):
    lp = case("ne_front_300")
    a = gpu_solve(torch_dev, lp, syrk_group_front=0)
    b = gpu_solve(torch_dev, lp, syrk_group_front=64, syrk_group=1)
    assert np.array_equal(a["dy"], b["dy"])
    assert np.array_equal(a["solver"].export_d()["d"], b["solver"].export_d()["d"])


@pytest.mark.parametrize("group", [2, 4])
def test_grouped_mixed_precision_refines_to_target(torch_dev, group):
    """FP32 matrix-core Schur updates (f_mix lowered) with grouped windows: the refinement in
    FP64 still reaches a normwise backward error <= 1e-10 against the oracle's residual."""
    from test_gpu_parity import oracle_berr
    lp = W.ne_random(m=300, n=600, density=0.08, seed=22)
    g = gpu_solve(torch_dev, lp, prec=1, f_mix=65, syrk_group_front=64, syrk_group=group)
    assert g["solver"].sym["max_front"] >= 129
    ss = g["sstats"]
    print(f"  mixed grouped: initial berr {ss['berr_nw_initial']:.2e} final {ss['berr_nw']:.2e} "
          f"steps {ss['max_steps']}")
    x = g["dy"][:, 0]
    nw, _ = oracle_berr(lp, lp["theta"], x, None, lp["r1"][:, 0])
    assert nw <= 1e-10, nw


@pytest.mark.parametrize("group", [1, 4])
@pytest.mark.parametrize("name", ["dense_ne", "ne_front_300", "staircase"])
def test_wide_tiles_match_oracle(torch_dev, name, group):
    """Full trailing updates in 128 x 128 tiles (syrk_tile_front lowered so that they apply
    here, with ragged last tiles and diagonal tiles whose upper quarter is skipped): FP64
    against the oracle, ungrouped and in groups of four windows."""
    lp = case(name)
    g = gpu_solve(torch_dev, lp, syrk_group_front=64 if group > 1 else 0, syrk_group=group, syrk_tile_front=65)
    check_against_oracle(lp, g)


def test_wide_tiles_reconstruct_K(torch_dev):
    """The factor made with 128 x 128 trailing tiles reconstructs K within the factorisation's
    error bound (dense augmented system, largest front of order 129: trailing matrices of 65
    and 1 rows)."""
    from test_oracle import dense_K
    lp = dense_as(62, 67)
    g = gpu_solve(torch_dev, lp, max_refine=0, syrk_tile_front=1)
    s = g["solver"]
    K = dense_K(lp, lp["theta"], lp["rho"], lp["delta"])
    po, L, D, ed = _dense_factor(s, s.N)
    R = K[np.ix_(po, po)] + np.diag(ed) - L @ D @ L.T
    scale = np.abs(L) @ np.abs(D) @ np.abs(L).T
    print("reconstruction error / (|L||D||L^T|)_max:", np.abs(R).max() / scale.max())
    assert np.abs(R).max() <= 100 * s.sym["max_front"] * U * scale.max()


@pytest.mark.parametrize("group", [1, 4])
def test_wide_tiles_mixed_precision_refines_to_target(torch_dev, group):
    """FP32 products in 128 x 128 tiles (f_mix and syrk_tile_front lowered): the FP64
    refinement reaches a normwise backward error <= 1e-10 against the oracle's residual, and
    the unrefined error shows that the FP32 products ran."""
    from test_gpu_parity import oracle_berr
    lp = W.ne_random(m=300, n=600, density=0.08, seed=22)
    g64 = gpu_solve(torch_dev, lp, prec=0, syrk_group_front=64 if group > 1 else 0, syrk_group=group,
                    syrk_tile_front=65)
    g = gpu_solve(torch_dev, lp, prec=1, f_mix=65, syrk_group_front=64 if group > 1 else 0, syrk_group=group,
                  syrk_tile_front=65)
    ss = g["sstats"]
    print(f"  mixed wide tiles: initial berr {ss['berr_nw_initial']:.2e} final {ss['berr_nw']:.2e} "
          f"steps {ss['max_steps']}; fp64 initial {g64['sstats']['berr_nw_initial']:.2e}")
    nw, _ = oracle_berr(lp, lp["theta"], g["dy"][:, 0], None, lp["r1"][:, 0])
    assert nw <= 1e-10, nw
    assert ss["berr_nw_initial"] > g64["sstats"]["berr_nw_initial"]
