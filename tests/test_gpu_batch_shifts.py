"""Per-system rho and delta read from device memory (qdmf_batch_factorise_dev and
qdmf_batch_graph_capture), through the C ABI (needs an MI355X): the factorisation equals the one
with the same shifts given on the host bit for bit; a captured batch replays with Theta and the
shifts refreshed in place, equal to the eager calls bit for bit and every system at the FP64
target against its own K_static (the oracle's residual); an invalid shift is reported."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_04370_amd import qdmf as Q
from paper_2508_04370_amd import workloads as W

from test_batch import small_batch
from test_gpu_parity import torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _setup(torch, lps, stream):
    cat = W.concat_systems(lps)
    h = Q.qdmf_create(0, stream.cuda_stream, Q.qdmf_default_options())
    Q.qdmf_batch_analyse(h, lps, lps[0]["mode"])
    Q.qdmf_set_matrix(h, cat["val"])
    return h, cat


def _draw(lps, k):
    """Theta, per-system shifts and right-hand sides of iteration k."""
    g = W.rng(61, k)
    rho = 1e-10 * (1.0 + 9.0 * g.random(len(lps)))
    delta = 1e-10 * (1.0 + 9.0 * g.random(len(lps)))
    th = np.concatenate([W.as_batch_theta(lp, q, k, seed=61) for q, lp in enumerate(lps)])
    rhs = [W.as_batch_rhs(lp, q, k, 0, seed=61) for q, lp in enumerate(lps)]
    return th, rho, delta, rhs


def _per_system_berr(lps, cat, th, rho, delta, rhs, dx, dy):
    out = []
    for q, lp in enumerate(lps):
        c0, c1 = cat["col_off"][q], cat["col_off"][q + 1]
        r0, r1 = cat["row_off"][q], cat["row_off"][q + 1]
        x = np.concatenate([dx[c0:c1], dy[r0:r1]])
        thq = th[c0:c1]
        b = O.system_rhs(lp, rhs[q][0], rhs[q][1], thq)
        lq = W.LP(dict(lp, rho=float(rho[q]), delta=float(delta[q])))
        _, nw, _, _ = O.residual(lq, thq, float(rho[q]), float(delta[q]), x, b)
        out.append(nw)
    return np.array(out)


def test_device_shifts_equal_host_shifts(torch_dev):
    torch, dev = torch_dev
    lps = small_batch(6, seed=47)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        print(f"[gpu case] batch of {len(lps)}: device shifts against host shifts", flush=True)
        h, cat = _setup(torch, lps, stream)
        th, rho, delta, rhs = _draw(lps, 0)
        thd = torch.from_numpy(th).to(dev)
        r7 = torch.from_numpy(np.concatenate([r[0] for r in rhs])).to(dev).reshape(-1, 1)
        r1 = torch.from_numpy(np.concatenate([r[1] for r in rhs])).to(dev).reshape(-1, 1)
        out = []
        for use_dev in (False, True):
            dx = torch.empty((cat["n"], 1), dtype=torch.float64, device=dev)
            dy = torch.empty((cat["m"], 1), dtype=torch.float64, device=dev)
            if use_dev:
                rd = torch.from_numpy(rho).to(dev)
                dd = torch.from_numpy(delta).to(dev)
                Q.qdmf_batch_factorise_dev(h, thd, rd, dd)
            else:
                Q.qdmf_batch_factorise(h, thd, rho, delta)
            Q.qdmf_solve(h, 1, r7, r1, dx, dy)
            stream.synchronize()
            out.append((dx.cpu().numpy()[:, 0], dy.cpu().numpy()[:, 0], Q.qdmf_batch_stats(h, len(lps), 1)))
        (ax, ay, sa), (bx, by, sb) = out
        assert np.array_equal(ax, bx) and np.array_equal(ay, by)
        assert np.array_equal(sa["inertia"], sb["inertia"]) and np.array_equal(sa["berr_nw"], sb["berr_nw"])
        nw = _per_system_berr(lps, cat, th, rho, delta, rhs, bx, by)
        print("  per-system berr (oracle residual):", nw.max())
        assert nw.max() <= 1e-12
        Q.qdmf_destroy(h)


def test_batch_graph_with_device_shifts_matches_eager(torch_dev):
    torch, dev = torch_dev
    lps = small_batch(6, seed=48)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        print(f"[gpu case] batch of {len(lps)}: graph with device shifts, 3 replays", flush=True)
        h, cat = _setup(torch, lps, stream)
        e, _ = _setup(torch, lps, stream)
        n, m, ns = cat["n"], cat["m"], len(lps)
        thd = torch.empty(n, dtype=torch.float64, device=dev)
        rd = torch.empty(ns, dtype=torch.float64, device=dev)
        dd = torch.empty(ns, dtype=torch.float64, device=dev)
        r7 = torch.empty((1, n), dtype=torch.float64, device=dev).T
        r1 = torch.empty((1, m), dtype=torch.float64, device=dev).T
        dx = torch.empty((1, n), dtype=torch.float64, device=dev).T
        dy = torch.empty((1, m), dtype=torch.float64, device=dev).T

        def refresh(k):
            th, rho, delta, rhs = _draw(lps, k)
            thd.copy_(torch.from_numpy(th))
            rd.copy_(torch.from_numpy(rho))
            dd.copy_(torch.from_numpy(delta))
            r7.copy_(torch.from_numpy(np.concatenate([r[0] for r in rhs])).reshape(-1, 1))
            r1.copy_(torch.from_numpy(np.concatenate([r[1] for r in rhs])).reshape(-1, 1))
            return th, rho, delta, rhs

        refresh(0)
        Q.qdmf_batch_graph_capture(h, thd, rd, dd, 0, 2, 1, r7, r1, dx, dy)
        for k in range(3):
            th, rho, delta, rhs = refresh(k + 1)
            stream.synchronize()
            Q.qdmf_graph_launch(h)
            stream.synchronize()
            gx, gy = dx.cpu().numpy()[:, 0].copy(), dy.cpu().numpy()[:, 0].copy()
            gs = Q.qdmf_batch_stats(h, ns, 1)
            Q.qdmf_batch_factorise_dev(e, thd, rd, dd)
            ex = torch.empty_like(dx)
            ey = torch.empty_like(dy)
            Q.qdmf_solve(e, 1, r7, r1, ex, ey)
            Q.qdmf_solve(e, 1, r7, r1, ex, ey)
            stream.synchronize()
            es = Q.qdmf_batch_stats(e, ns, 1)
            assert np.array_equal(gx, ex.cpu().numpy()[:, 0]) and np.array_equal(gy, ey.cpu().numpy()[:, 0]), k
            assert np.array_equal(gs["berr_nw"], es["berr_nw"]) and np.array_equal(gs["inertia"], es["inertia"])
            nw = _per_system_berr(lps, cat, th, rho, delta, rhs, gx, gy)
            print(f"  replay {k}: worst system berr {nw.max():.2e}")
            assert nw.max() <= 1e-12
            for q, lp in enumerate(lps):
                assert tuple(gs["inertia"][q][:2]) == (lp["n"], lp["m"])
        Q.qdmf_destroy(e)
        Q.qdmf_destroy(h)


def test_invalid_device_shift_is_reported(torch_dev):
    torch, dev = torch_dev
    lps = small_batch(4, seed=49)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, cat = _setup(torch, lps, stream)
        th, rho, delta, _ = _draw(lps, 0)
        rho[2] = -1e-8
        Q.qdmf_batch_factorise_dev(h, torch.from_numpy(th).to(dev), torch.from_numpy(rho).to(dev),
                                   torch.from_numpy(delta).to(dev))
        with pytest.raises(Q.QdmfError) as ei:
            Q.qdmf_factor_stats(h)
        assert ei.value.code == Q.QDMF_ERR_INVALID_ARG
        Q.qdmf_destroy(h)
