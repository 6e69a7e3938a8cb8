"""The allocation-free solve (qdmf_solve_noalloc) through the C ABI (needs an MI355X), against
qdmf_solve on the same factorisation and right-hand sides.  Both run the same kernels, and the
enqueue that reads no flags from the host computes what the eager one does, so the solutions
and the refinement statistics must agree bit for bit.  Two calls in a row share the GPU's one
work space, the second on a smaller system; device memory in use does not change across
them; a work space above the fixed size is refused before anything runs."""
import numpy as np
import pytest

from paper_2508_04370_amd import workloads as W

from test_gpu_parity import torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _system(torch, dev, lp, nrhs, seed):
    g = W.rng(88, seed)
    th = torch.from_numpy(W.log_uniform(g, 1e-10, 1e10, lp["n"])).to(dev)
    r7 = torch.from_numpy(g.standard_normal((nrhs, lp["n"]))).to(dev).T
    r1 = torch.from_numpy(g.standard_normal((nrhs, lp["m"]))).to(dev).T
    return th, r7, r1


def _outputs(torch, dev, lp, nrhs, fill=np.nan):
    dx = torch.full((nrhs, lp["n"]), fill, dtype=torch.float64, device=dev).T
    dy = torch.full((nrhs, lp["m"]), fill, dtype=torch.float64, device=dev).T
    return dx, dy


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_matches_solve_two_calls(torch_dev, prec):
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    big = W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24)
    small = W.ne_grid(10, 8, 6, nrhs=1)
    cases = []
    for lp, nrhs, seed in ((big, 3, 1), (small, 2, 2)):
        s = Q.Solver(lp, device=0, f_mix=65)
        th, r7, r1 = _system(torch, dev, lp, nrhs, seed)
        s.factorise(th, lp["rho"], lp["delta"], prec)
        cases.append((lp, nrhs, s, th, r7, r1))
    assert cases[1][0]["n"] + cases[1][0]["m"] < cases[0][0]["n"] + cases[0][0]["m"]
    # the existing entry point first (it allocates its own work space)
    ref = []
    for lp, nrhs, s, th, r7, r1 in cases:
        ex, ey = s.solve(r7, r1)
        torch.cuda.synchronize()
        st = s.solve_stats(nrhs)
        ref.append((ex.cpu().numpy(), ey.cpu().numpy(), st))
    outs = [_outputs(torch, dev, lp, nrhs) for lp, nrhs, *_ in cases]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    for (lp, nrhs, s, th, r7, r1), (dx, dy) in zip(cases, outs):
        s.solve_noalloc(r7, r1, dx, dy)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(0)[0] == free0
    for (lp, nrhs, s, *_), (dx, dy), (ex, ey, st) in zip(cases, outs, ref):
        assert np.array_equal(dx.cpu().numpy(), ex) and np.array_equal(dy.cpu().numpy(), ey), lp["name"]
        sn = s.solve_stats(nrhs)
        assert np.array_equal(sn["berr_nw_per_rhs"], st["berr_nw_per_rhs"]), lp["name"]
        assert np.array_equal(sn["steps_per_rhs"], st["steps_per_rhs"]), lp["name"]
        assert sn["berr_nw"] <= (1e-10 if prec else 1e-12), (lp["name"], sn["berr_nw"])
        print(f"  {lp['name']} nrhs {nrhs}: berr {sn['berr_nw']:.2e} steps {sn['max_steps']}")
    # after the allocation-free calls the handles' own solves still give the same results
    for (lp, nrhs, s, th, r7, r1), (ex, ey, st) in zip(cases, ref):
        fx, fy = s.solve(r7, r1)
        torch.cuda.synchronize()
        assert np.array_equal(fx.cpu().numpy(), ex) and np.array_equal(fy.cpu().numpy(), ey)
    for c in cases:
        c[2].close()


def test_noalloc_on_a_handle_that_never_solved(torch_dev):
    """Mixed factorisation, then the allocation-free solve before any qdmf_solve (the handle has
    no work space of its own yet), then qdmf_solve: equal."""
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_staircase(periods=3, rows=200, cols=400, link_cols=40, seed=25)
    s = Q.Solver(lp, device=0, f_mix=65)
    th, r7, r1 = _system(torch, dev, lp, 2, 3)
    s.factorise(th, lp["rho"], lp["delta"], Q.QDMF_MIXED)
    dx, dy = _outputs(torch, dev, lp, 2)
    s.solve_noalloc(r7, r1, dx, dy)
    torch.cuda.synchronize()
    nx, ny = dx.cpu().numpy(), dy.cpu().numpy()
    sn = s.solve_stats(2)
    ex, ey = s.solve(r7, r1)
    torch.cuda.synchronize()
    se = s.solve_stats(2)
    assert np.array_equal(nx, ex.cpu().numpy()) and np.array_equal(ny, ey.cpu().numpy())
    assert np.array_equal(sn["berr_nw_per_rhs"], se["berr_nw_per_rhs"])
    s.close()


def test_noalloc_rejects_work_space_above_the_limit(torch_dev):
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_staircase(periods=3, rows=200, cols=400, link_cols=40, seed=25)
    N = lp["n"] + lp["m"]
    nrhs = Q.NOALLOC_SCRATCH_BYTES // (6 * 8 * N) + 1  # the six N x nrhs solve vectors alone exceed it
    s = Q.Solver(lp, device=0)
    th, r7, r1 = _system(torch, dev, lp, nrhs, 4)
    s.factorise(th, lp["rho"], lp["delta"], Q.QDMF_FP64)
    dx, dy = _outputs(torch, dev, lp, nrhs, fill=7.0)
    torch.cuda.synchronize()
    with pytest.raises(Q.QdmfError) as ei:
        s.solve_noalloc(r7, r1, dx, dy)
    assert ei.value.code == Q.QDMF_ERR_OOM
    torch.cuda.synchronize()
    assert bool((dx == 7.0).all()) and bool((dy == 7.0).all())  # nothing launched
    s.close()
