"""Mixed precision (FP32 matrix-core Schur updates, FP64 refinement with a device GMRES
correction, Section 4.5) under HIP graph capture, through the C ABI (needs an MI355X): every
replay on refreshed Theta equals an eager factorise + solve of the same inputs bit for bit (the
eager solve stops launching finished steps, the graph's kernels return at once for them) and
meets the 1e-10 backward-error target against the oracle's residual."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import workloads as W

from test_gpu_parity import oracle_berr, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _buffers(torch, dev, n, m, nrhs=1):
    th = torch.empty(n, dtype=torch.float64, device=dev)
    r7 = torch.empty((nrhs, n), dtype=torch.float64, device=dev).T
    r1 = torch.empty((nrhs, m), dtype=torch.float64, device=dev).T
    dx = torch.empty((nrhs, n), dtype=torch.float64, device=dev).T
    dy = torch.empty((nrhs, m), dtype=torch.float64, device=dev).T
    return th, r7, r1, dx, dy


def test_mixed_graph_matches_eager_small(torch_dev):
    """A staircase whose fronts of order >= 65 take FP32 updates (f_mix lowered), Theta over
    [1e-10, 1e10] refreshed per replay: three replays of factorise + 2 solves."""
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    lp = W.as_staircase(periods=4, rows=300, cols=600, link_cols=60, seed=24)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = Q.Solver(lp, device=0, stream=stream.cuda_stream, f_mix=65)
        assert s.sym["max_front"] >= 65
        th, r7, r1, dx, dy = _buffers(torch, dev, lp["n"], lp["m"])

        def refresh(k):
            g = W.rng(56, k)
            th.copy_(torch.from_numpy(W.log_uniform(g, 1e-10, 1e10, lp["n"])))
            r7.copy_(torch.from_numpy(g.standard_normal((lp["n"], 1))))
            r1.copy_(torch.from_numpy(g.standard_normal((lp["m"], 1))))

        refresh(0)
        Q.qdmf_graph_capture(s.h, th, lp["rho"], lp["delta"], Q.QDMF_MIXED, 2, 1, r7, r1, dx, dy)
        for k in range(3):
            refresh(k)
            stream.synchronize()
            Q.qdmf_graph_launch(s.h)
            stream.synchronize()
            gx, gy = dx.cpu().numpy().copy(), dy.cpu().numpy().copy()
            gst = s.solve_stats(1)
            s.factorise(th, lp["rho"], lp["delta"], Q.QDMF_MIXED)
            ex, ey = s.solve(r7, r1)
            s.solve(r7, r1, ex, ey)
            stream.synchronize()
            est = s.solve_stats(1)
            print(f"  replay {k}: berr graph {gst['berr_nw']:.2e} eager {est['berr_nw']:.2e} "
                  f"steps {gst['max_steps']} initial {gst['berr_nw_initial']:.2e}")
            assert np.array_equal(gx, ex.cpu().numpy()) and np.array_equal(gy, ey.cpu().numpy()), k
            x = np.concatenate([gx[:, 0], gy[:, 0]])
            nw, _ = oracle_berr(lp, th.cpu().numpy(), x, r7.cpu().numpy()[:, 0], r1.cpu().numpy()[:, 0])
            assert nw <= 1e-10, (k, nw)
            assert gst["berr_nw"] == est["berr_nw"]
        s.close()


def test_batch_full_mixed_graph_replays(torch_dev):
    """All 512 systems of the batched workload in mixed precision, factorise + predictor +
    corrector captured once and replayed for three IPM-like iterations (Theta redrawn per
    system and iteration, seed [4, s, k]; right-hand sides seed [4, s, k, j]): every replay
    equals eager bit for bit, and every system of every replay meets 1e-10 against its own
    K_static (the oracle's residual)."""
    torch, dev = torch_dev
    from paper_2508_04370_amd import qdmf as Q
    lps = W.as_batch(512)
    cat = W.concat_systems(lps)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = Q.Solver(cat, device=0, stream=stream.cuda_stream, systems=lps, ordering=0)
        th, r7, r1, dx, dy = _buffers(torch, dev, cat["n"], cat["m"])
        cpu = {}

        def refresh(k, j):
            t = np.concatenate([W.as_batch_theta(q, si, k) for si, q in enumerate(lps)])
            rs = [W.as_batch_rhs(q, si, k, j) for si, q in enumerate(lps)]
            a7, a1 = np.concatenate([r[0] for r in rs]), np.concatenate([r[1] for r in rs])
            th.copy_(torch.from_numpy(t))
            r7.copy_(torch.from_numpy(a7.reshape(-1, 1)))
            r1.copy_(torch.from_numpy(a1.reshape(-1, 1)))
            cpu.update(theta=t, r7=a7, r1=a1)

        refresh(0, 0)
        rho, delta = lps[0]["rho"], lps[0]["delta"]
        Q.qdmf_graph_capture(s.h, th, rho, delta, Q.QDMF_MIXED, 1, 1, r7, r1, dx, dy)
        for k in range(3):
            refresh(k, 0)
            stream.synchronize()
            Q.qdmf_graph_launch(s.h)
            stream.synchronize()
            gx, gy = dx.cpu().numpy()[:, 0].copy(), dy.cpu().numpy()[:, 0].copy()
            s.factorise(th, rho, delta, Q.QDMF_MIXED)
            ex, ey = s.solve(r7, r1)
            stream.synchronize()
            assert np.array_equal(gx, ex.cpu().numpy()[:, 0]) and np.array_equal(gy, ey.cpu().numpy()[:, 0]), k
            worst = 0.0
            for q, lp in enumerate(lps):
                c0, c1 = cat["col_off"][q], cat["col_off"][q + 1]
                q0, q1 = cat["row_off"][q], cat["row_off"][q + 1]
                x = np.concatenate([gx[c0:c1], gy[q0:q1]])
                b = O.system_rhs(lp, cpu["r7"][c0:c1], cpu["r1"][q0:q1], cpu["theta"][c0:c1])
                _, nw, _, _ = O.residual(lp, cpu["theta"][c0:c1], lp["rho"], lp["delta"], x, b)
                worst = max(worst, nw)
                assert nw <= 1e-10, (k, q, nw)
            print(f"  batch mixed replay {k}: worst system berr {worst:.2e}")
        s.close()
