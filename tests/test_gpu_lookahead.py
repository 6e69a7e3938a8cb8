"""Factorisation lookahead (the lookahead_front option) on the GPU path, through the C ABI
(needs an MI355X): the tiles of a full trailing update beyond the next group's pivot columns
run on a second stream while the next pivot windows run on the first.  Every entry still
receives the same products summed in the same order, so the factor, D and the solution must
be bitwise those of the path without lookahead, in FP64 and with FP32 products; and the
result still meets the oracle's bounds."""
import numpy as np
import pytest

from paper_2508_04370_amd import workloads as W

from test_gpu_parity import check_against_oracle, gpu_solve, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def case(name):
    if name == "dense_ne":  # one front of order ~200 with four windows
        return W.ne_random(m=200, n=400, density=0.08, seed=21)
    if name == "ne_front_300":  # a dense front of order 300: five windows, the last partial
        return W.ne_dense_front(300, seed=3, nrhs=2)
    if name == "ne_front_700":  # eleven windows, several groups of four, ragged last tile
        return W.ne_dense_front(700, seed=5, nrhs=1)
    if name == "staircase":  # fronts of order up to ~300 beside many small ones, several per level
        return W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24)
    raise KeyError(name)


SHAPES = {  # (syrk_group_front, syrk_group, syrk_tile_front)
    "ungrouped": (0, 1, 0),
    "groups_of_3": (64, 3, 0),
    "groups_of_4": (64, 4, 0),
    "wide_tiles": (0, 1, 65),
    "groups_wide_tiles": (64, 4, 65),
}


def _factor_bits(g):
    """D and the pivot data, and the factor columns (the lower part, diagonal included, of
    the f x p panel: its strict upper triangle is work space, not part of L) of the three
    largest fronts."""
    s = g["solver"]
    d = s.export_d()
    fronts = []
    for q in np.argsort(s.sym["sn_front"])[-3:]:
        panel, rows = s.export_front(q)
        fronts.append((np.tril(panel), rows))
    return d, fronts


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("name", ["dense_ne", "ne_front_300", "ne_front_700", "staircase"])
def test_lookahead_is_bitwise_the_plain_path(torch_dev, name, shape, prec):
    lp = case(name)
    gf, gs, tf = SHAPES[shape]
    opts = dict(syrk_group_front=gf, syrk_group=gs, syrk_tile_front=tf, max_refine=0)
    if prec == 1:
        opts["f_mix"] = 65
    a = gpu_solve(torch_dev, lp, prec=prec, lookahead_front=0, **opts)
    b = gpu_solve(torch_dev, lp, prec=prec, lookahead_front=64, **opts)
    da, fa = _factor_bits(a)
    db, fb = _factor_bits(b)
    for k in da:
        assert np.array_equal(da[k], db[k]), k
    for (pa, ra), (pb, rb) in zip(fa, fb):
        assert np.array_equal(ra, rb)
        assert np.array_equal(pa, pb, equal_nan=True)
    assert np.array_equal(a["dy"], b["dy"]) and np.array_equal(a["dx"], b["dx"])
    assert a["fstats"] == b["fstats"]


@pytest.mark.parametrize("shape", ["groups_of_4", "groups_wide_tiles"])
@pytest.mark.parametrize("name", ["ne_front_700", "staircase"])
def test_lookahead_matches_oracle(torch_dev, name, shape):
    lp = case(name)
    gf, gs, tf = SHAPES[shape]
    g = gpu_solve(torch_dev, lp, syrk_group_front=gf, syrk_group=gs, syrk_tile_front=tf, lookahead_front=64)
    check_against_oracle(lp, g)


def test_lookahead_splits_the_updates(torch_dev):
    """The option changes the launch plan: a full update of a lookahead front becomes two
    launches (its columns for the next group, and the rest on the second stream), so the
    trailing-update launches of one factorisation grow in number while their work stays."""
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    lp = case("ne_front_700")
    counts = {}
    for la in (0, 64):
        s = Q.Solver(lp, device=0, syrk_group_front=64, syrk_group=4, lookahead_front=la)
        th = torch.from_numpy(lp["theta"]).to(dev)
        Q.qdmf_profile_kind(s.h, Q.QDMF_K_SYRK)
        s.factorise(th, lp["rho"], lp["delta"], 0)
        torch.cuda.synchronize()
        counts[la] = Q.qdmf_profile_read(s.h)
        Q.qdmf_profile_kind(s.h, -1)
        s.close()
    print("k_syrk launches, flops:", counts)
    assert counts[64]["launches"] > counts[0]["launches"]
    assert counts[64]["flops"] == pytest.approx(counts[0]["flops"], rel=1e-12)

