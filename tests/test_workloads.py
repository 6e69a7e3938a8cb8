"""Seeded generators: reproducibility and the structure each workload promises."""
import numpy as np

from paper_2508_04370_amd import workloads as W


def _check_csc(lp):
    cp, ri = lp["colptr"], lp["rowidx"]
    assert cp.dtype == np.int64 and ri.dtype == np.int32
    assert cp[0] == 0 and np.all(np.diff(cp) >= 0) and cp[-1] == len(ri) == len(lp["val"])
    for j in range(lp["n"]):
        r = ri[cp[j]:cp[j + 1]]
        assert np.all(np.diff(r) > 0) and (len(r) == 0 or (r[0] >= 0 and r[-1] < lp["m"]))


def test_ne_random_shape_and_seed():
    a, b = W.ne_random(), W.ne_random()
    assert np.array_equal(a["rowidx"], b["rowidx"]) and np.array_equal(a["val"], b["val"])
    assert a["m"] == 300 and a["n"] == 600
    _check_csc(a)
    assert np.all(np.diff(a["colptr"]) >= 1)
    rows = np.bincount(a["rowidx"], minlength=a["m"])
    assert rows.min() >= 2
    assert 2000 < a.nnz < 3000
    assert a["theta"].min() >= 1e-6 and a["theta"].max() <= 1e6
    c = W.ne_random(seed=5)
    assert not np.array_equal(a["val"][:10], c["val"][:10])


def test_staircase_structure():
    lp = W.as_staircase(periods=5, rows=40, cols=80, link_cols=10)
    _check_csc(lp)
    cp, ri = lp["colptr"], lp["rowidx"]
    for j in range(lp["n"]):
        t = j // 80
        r = ri[cp[j]:cp[j + 1]]
        own = r[(r >= 40 * t) & (r < 40 * (t + 1))]
        assert len(own) >= 5
        other = r[(r < 40 * t) | (r >= 40 * (t + 1))]
        if len(other):
            assert j % 80 < 10 and np.all(other // 40 == t + 1)
    assert np.bincount(ri, minlength=lp["m"]).min() >= 1
    assert lp["theta"].min() >= 1e-10 and lp["theta"].max() <= 1e10


def test_full_staircase_size():
    lp = W.as_staircase()
    assert (lp["m"], lp["n"]) == (20000, 40000)
    assert 200000 < lp.nnz < 206000


def test_grid_and_dense_columns_small():
    g = W.ne_grid(6, 5, 4, nrhs=2)
    _check_csc(g)
    assert g["m"] == 120 and g["n"] == 240 and g["r1"].shape == (120, 2)
    d = W.as_dense_cols(8, 5, 5, ndense=3)
    _check_csc(d)
    cnt = np.diff(d["colptr"])
    assert cnt[-3:].min() > 0.3 * d["m"] and cnt[:-3].max() <= 4


def test_batch_system_ranges():
    for s in range(5):
        lp = W.as_batch_system(s)
        _check_csc(lp)
        assert 50 <= lp["m"] <= 2000 and lp["n"] == 2 * lp["m"]
        th = W.as_batch_theta(lp, s, 3)
        assert th.min() >= 1e-8 and th.max() <= 1e8


def test_dense_front_signs():
    F, s = W.dense_front(64, 32, seed=1)
    assert np.allclose(F, F.T)
    assert np.all(np.sign(np.diag(F)) == s)
