"""Seeded synthetic inputs for the regularised Newton systems of an LP interior point method.

This module only draws random numbers and lays them out (a sparse constraint matrix in CSC
form, the diagonal Theta, the right-hand sides and the regularisation scalars).  It holds none
of the method's arithmetic, so the factorisation library, its tests and the CPU reference
implementation can all draw from it without sharing computation.

The paper measures on LP collections that are not available here; every workload below is a
synthetic stand-in with the shape of the systems the paper factorises (Sections 3 and 5):

* ``ne_random``      -- small random LP, normal-equations form (300 x 600, ~1 % density).
* ``as_staircase``   -- multi-period staircase LP, augmented-system form (40 periods of
                        500 x 1000, ~5 nonzeros per column, links between consecutive periods).
* ``ne_grid``        -- LP coupled on a 3-D 7-point grid, normal-equations form.
* ``as_batch``       -- many independent small random LPs, augmented-system form.
* ``as_dense_cols``  -- grid-coupled LP with a few dense columns, augmented-system form.
* ``dense_front``    -- a single dense symmetric front with quasi-definite diagonal signs.
* ``feasible_lp``, ``bounded_lp`` -- b, c (and bounds l, u) making an LP over a workload's A
                        primal and dual feasible, for the interior point driver.
* ``with_hessian``   -- a sparse positive semidefinite Q on a workload's columns (quadratic
                        programs).

All randomness comes from ``numpy.random.Generator(PCG64(SeedSequence(seed_list)))``.
"""
from __future__ import annotations

import numpy as np

NE = 0
AS = 1


def rng(*seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(s) for s in seed])))


def log_uniform(g, lo, hi, size):
    """Theta_j = 10**U(log10 lo, log10 hi)."""
    return 10.0 ** g.uniform(np.log10(lo), np.log10(hi), size)


class LP(dict):
    """A sparse matrix A (m x n, CSC with sorted row indices) plus the scalars of one system."""

    __getattr__ = dict.__getitem__

    @property
    def nnz(self):
        return int(self["colptr"][-1])


def _csc_from_columns(m, cols, g_vals):
    """cols: list of sorted unique int arrays (row indices of each column)."""
    n = len(cols)
    colptr = np.zeros(n + 1, dtype=np.int64)
    for j, c in enumerate(cols):
        colptr[j + 1] = colptr[j] + len(c)
    rowidx = np.concatenate(cols).astype(np.int32) if n else np.zeros(0, np.int32)
    val = g_vals.standard_normal(int(colptr[-1]))
    return colptr, rowidx, val


def _csc_from_pairs(m, n, rows, cols, g_vals):
    """Build CSC from (row, col) pairs; duplicates merged; rows sorted within a column."""
    key = np.unique(cols.astype(np.int64) * m + rows.astype(np.int64))
    c = (key // m).astype(np.int64)
    r = (key % m).astype(np.int32)
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    val = g_vals.standard_normal(len(r))
    return colptr, r, val


def random_lp_pattern(g, m, n, density):
    """Bernoulli(density) pattern plus one forced entry (pi[j mod m], j) per column."""
    mask = g.random((m, n)) < density
    pi = g.permutation(m)
    mask[pi[np.arange(n) % m], np.arange(n)] = True
    r, c = np.nonzero(mask)
    return r, c


def ne_random(m=300, n=600, density=0.01, seed=1, theta_range=(1e-6, 1e6), rho=0.0,
              delta=1e-8, nrhs=1):
    """Small random LP in normal-equations form (one forced nonzero per column)."""
    g = rng(seed)
    r, c = random_lp_pattern(g, m, n, density)
    colptr, rowidx, val = _csc_from_pairs(m, n, r, c, g)
    theta = log_uniform(g, *theta_range, n)
    gr = rng(seed, 1)
    r1 = gr.standard_normal((nrhs, m)).T.copy(order="F")
    r7 = np.zeros((n, nrhs), order="F")
    return LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=rho,
              delta=delta, mode=NE, r1=r1, r7=r7, name=f"ne_random_{m}x{n}")


def as_staircase(periods=40, rows=500, cols=1000, per_col=5, link_cols=100, seed=2,
                 theta_range=(1e-10, 1e10), rho=1e-10, delta=1e-10, nrhs=1):
    """Multi-period staircase LP (energy-model-like) in augmented-system form.

    Period t owns rows [rows*t, rows*(t+1)) and columns [cols*t, cols*(t+1)); each column
    has ``per_col`` distinct rows of its own period; the first ``link_cols`` columns of
    period t also touch one row of period t+1; empty rows get one entry in their period.
    """
    g = rng(seed)
    m, n = periods * rows, periods * cols
    rr = []
    cc = []
    for t in range(periods):
        base_r, base_c = rows * t, cols * t
        picks = np.argsort(g.random((cols, rows)), axis=1)[:, :per_col]
        rr.append((picks + base_r).ravel())
        cc.append(np.repeat(np.arange(cols) + base_c, per_col))
        if t < periods - 1:
            lr = g.integers(0, rows, link_cols) + rows * (t + 1)
            rr.append(lr)
            cc.append(np.arange(link_cols) + base_c)
    rr = np.concatenate(rr)
    cc = np.concatenate(cc)
    present = np.zeros(m, bool)
    present[rr] = True
    empty = np.nonzero(~present)[0]
    if len(empty):
        per = empty // rows
        ec = g.integers(0, cols, len(empty)) + per * cols
        rr = np.concatenate([rr, empty])
        cc = np.concatenate([cc, ec])
    colptr, rowidx, val = _csc_from_pairs(m, n, rr, cc, g)
    theta = log_uniform(g, *theta_range, n)
    gr = rng(seed, 1)
    r7 = gr.standard_normal((nrhs, n)).T.copy(order="F")
    r1 = gr.standard_normal((nrhs, m)).T.copy(order="F")
    return LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=rho,
              delta=delta, mode=AS, r1=r1, r7=r7, name=f"as_staircase_{periods}x{rows}x{cols}")


def _grid_neighbours(nx, ny, nz):
    """For every node r = x + nx*y + nx*ny*z: array (m, 6) of 6-neighbours, -1 if outside."""
    m = nx * ny * nz
    r = np.arange(m)
    x, y, z = r % nx, (r // nx) % ny, r // (nx * ny)
    nb = np.full((m, 6), -1, np.int64)
    nb[:, 0] = np.where(x > 0, r - 1, -1)
    nb[:, 1] = np.where(x < nx - 1, r + 1, -1)
    nb[:, 2] = np.where(y > 0, r - nx, -1)
    nb[:, 3] = np.where(y < ny - 1, r + nx, -1)
    nb[:, 4] = np.where(z > 0, r - nx * ny, -1)
    nb[:, 5] = np.where(z < nz - 1, r + nx * ny, -1)
    return nb


def ne_grid(nx=50, ny=50, nz=40, seed=3, theta_range=(1e-6, 1e6), rho=0.0, delta=1e-8,
            nrhs=8):
    """LP coupled on a 3-D grid: columns 2r and 2r+1 touch row r and its 6 grid neighbours."""
    g = rng(seed)
    m = nx * ny * nz
    n = 2 * m
    nb = _grid_neighbours(nx, ny, nz)
    sup = np.concatenate([np.arange(m)[:, None], nb], axis=1)
    sup.sort(axis=1)
    cols = []
    for r in range(m):
        s = sup[r][sup[r] >= 0]
        cols.append(s)
        cols.append(s)
    colptr, rowidx, val = _csc_from_columns(m, cols, g)
    theta = log_uniform(g, *theta_range, n)
    gr = rng(seed, 1)
    r1 = gr.standard_normal((nrhs, m)).T.copy(order="F")
    r7 = np.zeros((n, nrhs), order="F")
    return LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=rho,
              delta=delta, mode=NE, r1=r1, r7=r7, grid=(nx, ny, nz),
              name=f"ne_grid_{nx}x{ny}x{nz}")


def as_batch_system(s, seed=4, mrange=(50, 2000), drange=(0.005, 0.02), rho=1e-10,
                    delta=1e-10):
    """System s of the batched workload: random LP with m ~ U{mlo..mhi}, n = 2m."""
    g = rng(seed, s)
    m = int(g.integers(mrange[0], mrange[1] + 1))
    n = 2 * m
    d = float(g.uniform(*drange))
    r, c = random_lp_pattern(g, m, n, d)
    colptr, rowidx, val = _csc_from_pairs(m, n, r, c, g)
    return LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, rho=rho, delta=delta, mode=AS,
              name=f"as_batch_{s}")


def as_batch_theta(lp, s, k, seed=4, theta_range=(1e-8, 1e8)):
    return log_uniform(rng(seed, s, k), *theta_range, lp["n"])


def as_batch_rhs(lp, s, k, j, seed=4):
    g = rng(seed, s, k, j)
    return g.standard_normal(lp["n"]), g.standard_normal(lp["m"])


def ne_dense_front(f=4096, q=4, seed=0, theta_range=(1e-2, 1e2), delta=1e-8, nrhs=1):
    """Normal equations whose K is one dense f x f front: A = [I | G] (f x (f + q)), G dense
    N(0,1)/sqrt(f); K = diag(theta_I) + G diag(theta_G) G^T + delta I, so the single
    supernode has p = f (the dense-front measurement of the Schur updates)."""
    g = rng(0, f, q, seed)
    n = f + q
    cols = [np.array([j]) for j in range(f)] + [np.arange(f) for _ in range(q)]
    colptr = np.zeros(n + 1, np.int64)
    colptr[1:] = np.cumsum([len(c) for c in cols])
    rowidx = np.concatenate(cols).astype(np.int32)
    val = np.concatenate([np.ones(f), g.standard_normal(q * f) / np.sqrt(f)])
    theta = log_uniform(g, *theta_range, n)
    gr = rng(0, f, q, seed, 1)
    r1 = gr.standard_normal((nrhs, f)).T.copy(order="F")
    r7 = np.zeros((n, nrhs), order="F")
    return LP(m=f, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=0.0, delta=delta, mode=NE,
              r1=r1, r7=r7, name=f"ne_dense_front_{f}")


def dense_front_system(f, p, q=4, seed=0, delta=1e-8):
    """Normal equations whose elimination in the natural order gives one dense front of order f
    with p pivots (the dense-front measurement of the Schur updates) and, when p < f, its dense
    parent of order f - p + 1.  A has m = f (+1 when p < f) rows: the identity on rows 0..f-1
    (Theta log-uniform in [1, 10]), q dense columns over rows 0..f-1 with N(0,1)/sqrt(f) values
    (Theta 1), and for p < f one column over rows p..f-1 and an extra last row z, so that the
    pattern of K separates the first p columns from the rest.  Returns (lp, perm) with perm the
    natural order (new -> old)."""
    g = rng(0, f, p, seed)
    split = p < f
    m = f + (1 if split else 0)
    cols = [np.array([j]) for j in range(f)] + [np.arange(f) for _ in range(q)]
    if split:
        cols.append(np.arange(p, f + 1))
    n = len(cols)
    colptr = np.zeros(n + 1, np.int64)
    colptr[1:] = np.cumsum([len(c) for c in cols])
    rowidx = np.concatenate(cols).astype(np.int32)
    val = np.concatenate([np.ones(f), g.standard_normal(int(colptr[-1]) - f) / np.sqrt(f)])
    theta = np.concatenate([log_uniform(g, 1.0, 10.0, f), np.ones(n - f)])
    gr = rng(0, f, p, seed, 1)
    r1 = gr.standard_normal((1, m)).T.copy(order="F")
    r7 = np.zeros((n, 1), order="F")
    lp = LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=0.0, delta=delta, mode=NE,
            r1=r1, r7=r7, name=f"dense_front_{f}_{p}")
    return lp, np.arange(m, dtype=np.int32)


def as_batch(count, seed=4, mrange=(50, 2000), drange=(0.005, 0.02), rho=1e-10, delta=1e-10):
    """The first count systems of the batched workload (system s from seed [seed, s])."""
    return [as_batch_system(s, seed, mrange, drange, rho, delta) for s in range(count)]


def concat_systems(lps):
    """Block-diagonal concatenation of several systems (data layout only): system q's column
    j becomes column col_off[q] + j and its row i row row_off[q] + i; values and per-system
    vectors are concatenated in system order."""
    col_off = np.concatenate([[0], np.cumsum([lp["n"] for lp in lps])]).astype(np.int64)
    row_off = np.concatenate([[0], np.cumsum([lp["m"] for lp in lps])]).astype(np.int64)
    cps, ris = [np.zeros(1, np.int64)], []
    base = 0
    for q, lp in enumerate(lps):
        cps.append(np.asarray(lp["colptr"][1:], np.int64) - lp["colptr"][0] + base)
        ris.append(np.asarray(lp["rowidx"], np.int64) + row_off[q])
        base += int(lp["colptr"][-1] - lp["colptr"][0])
    val = np.concatenate([np.asarray(lp["val"], np.float64) for lp in lps])
    return LP(m=int(row_off[-1]), n=int(col_off[-1]), colptr=np.concatenate(cps),
              rowidx=np.concatenate(ris).astype(np.int32), val=val, mode=lps[0]["mode"],
              rho=lps[0]["rho"], delta=lps[0]["delta"], col_off=col_off, row_off=row_off,
              name=f"batch_{len(lps)}")


def as_dense_cols(nx=80, ny=50, nz=50, ndense=20, dense_p=0.5, seed=5,
                  theta_range=(1e-10, 1e10), rho=1e-9, delta=1e-9, nrhs=1):
    """Grid-coupled sparse columns (anchor + 3 grid neighbours) plus a few dense columns."""
    g = rng(seed)
    m = nx * ny * nz
    n = 2 * m
    nb = _grid_neighbours(nx, ny, nz)
    cols = []
    for j in range(n - ndense):
        a = j % m
        cand = nb[a][nb[a] >= 0]
        pick = cand if len(cand) <= 3 else g.choice(cand, 3, replace=False)
        cols.append(np.unique(np.concatenate([[a], pick])))
    for _ in range(ndense):
        cols.append(np.nonzero(g.random(m) < dense_p)[0])
    colptr, rowidx, val = _csc_from_columns(m, cols, g)
    theta = log_uniform(g, *theta_range, n)
    gr = rng(seed, 1)
    r7 = gr.standard_normal((nrhs, n)).T.copy(order="F")
    r1 = gr.standard_normal((nrhs, m)).T.copy(order="F")
    return LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=rho,
              delta=delta, mode=AS, r1=r1, r7=r7, grid=(nx, ny, nz), ndense=ndense,
              name=f"as_dense_cols_{nx}x{ny}x{nz}")


def dense_front(f, p, seed=0, dmin=1.0, dmax=10.0):
    """One dense symmetric front (column-major, full) with a quasi-definite sign pattern.

    sigma_i = -1 for a primal row, +1 for a dual row (random); |F_ii| in [dmin, dmax] with
    sign sigma_i; off-diagonal N(0,1)/sqrt(f).
    """
    g = rng(0, f, p, seed)
    sigma = np.where(g.random(f) < 0.5, -1, 1).astype(np.int8)
    F = g.standard_normal((f, f)) / np.sqrt(f)
    F = np.tril(F, -1)
    F = F + F.T
    F[np.arange(f), np.arange(f)] = sigma * g.uniform(dmin, dmax, f)
    return np.asfortranarray(F), sigma


def feasible_lp(lp, seed=7):
    """An LP min c^T x, A x = b, x >= 0 on the pattern and values of `lp`, primal and dual
    feasible by construction (so with a finite optimum): b = A x0 and c = A^T y0 + z0 for
    x0, z0 uniform in [0.5, 1.5] and y0 standard normal.  Returns (A as a LP dict with mode AS,
    b, c)."""
    g = rng(seed, 71)
    m, n = lp["m"], lp["n"]
    x0 = g.uniform(0.5, 1.5, n)
    z0 = g.uniform(0.5, 1.5, n)
    y0 = g.standard_normal(m)
    cp, ri, v = lp["colptr"], lp["rowidx"], lp["val"]
    b = np.zeros(m)
    c = z0.copy()
    for j in range(n):
        rows, vals = ri[cp[j]:cp[j + 1]], v[cp[j]:cp[j + 1]]
        b[rows] += vals * x0[j]
        c[j] += float(vals @ y0[rows])
    out = LP(dict(lp, mode=AS))
    return out, b, c


def bounded_lp(lp, seed=7, upper=0.5):
    """An LP min c^T x, A x = b, l <= x <= u on the pattern and values of `lp`, primal and dual
    feasible by construction: l uniform in [-1, 1]; a fraction `upper` of the columns (chosen at
    random) gets u = l + w with w uniform in [1, 3], the rest u = +inf; x0 strictly inside the
    bounds; b = A x0 and c = A^T y0 + z^l0 - z^u0 with z^l0 uniform in [0.5, 1.5], z^u0 uniform
    in [0, 1] where u is finite.  For a quadratic program (`lp` with Q, see with_hessian) c is
    lowered by Q x0, so that (x0, y0, z0) is feasible for the dual of min c^T x + x^T Q x / 2.
    Returns (A as a LP dict with mode AS, b, c, l, u)."""
    g = rng(seed, 72)
    m, n = lp["m"], lp["n"]
    l = g.uniform(-1.0, 1.0, n)
    hasu = g.random(n) < upper
    w = g.uniform(1.0, 3.0, n)
    u = np.where(hasu, l + w, np.inf)
    x0 = l + np.where(hasu, w * g.uniform(0.2, 0.8, n), g.uniform(0.5, 1.5, n))
    zl0 = g.uniform(0.5, 1.5, n)
    zu0 = np.where(hasu, g.uniform(0.0, 1.0, n), 0.0)
    y0 = g.standard_normal(m)
    cp, ri, v = lp["colptr"], lp["rowidx"], lp["val"]
    b = np.zeros(m)
    c = zl0 - zu0
    for j in range(n):
        rows, vals = ri[cp[j]:cp[j + 1]], v[cp[j]:cp[j + 1]]
        b[rows] += vals * x0[j]
        c[j] += float(vals @ y0[rows])
    if lp.get("q_colptr") is not None:
        qcp, qri, qv = lp["q_colptr"], lp["q_rowidx"], lp["q_val"]
        for j in range(n):
            for e in range(qcp[j], qcp[j + 1]):
                i = qri[e]
                c[i] -= qv[e] * x0[j]
                if i != j:
                    c[j] -= qv[e] * x0[i]
    out = LP(dict(lp, mode=AS))
    return out, b, c, l, u


def with_hessian(lp, seed=7, frac=0.5, per_row=3, window=50, ridge=0.1):
    """A quadratic program on the pattern and values of `lp` (mode AS): Q = G^T G + R, positive
    semidefinite by construction.  G has one row per column c of a random subset (a fraction
    `frac` of the columns); the row touches c and per_row - 1 other columns within `window`
    positions of c (local couplings, as in a staircase model's periods), values standard
    normal.  R is diagonal, ridge * U[0.5, 1.5] on the subset.  Adds q_colptr, q_rowidx, q_val:
    Q's lower triangle in CSC, rows ascending."""
    g = rng(seed, 73)
    n = lp["n"]
    sel = np.flatnonzero(g.random(n) < frac)
    ii, jj, vv = [], [], []
    for c in sel:
        lo, hi = max(0, c - window), min(n, c + window + 1)
        others = g.choice(np.setdiff1d(np.arange(lo, hi), [c]), size=min(per_row - 1, hi - lo - 1), replace=False)
        cols = np.concatenate([[c], others]).astype(np.int64)
        vals = g.standard_normal(len(cols))
        for a in range(len(cols)):
            for b in range(len(cols)):
                if cols[a] >= cols[b]:
                    ii.append(cols[a])
                    jj.append(cols[b])
                    vv.append(vals[a] * vals[b])
    ii.extend(sel.tolist())
    jj.extend(sel.tolist())
    vv.extend((ridge * g.uniform(0.5, 1.5, len(sel))).tolist())
    ii, jj, vv = np.asarray(ii, np.int64), np.asarray(jj, np.int64), np.asarray(vv, float)
    key, inv = np.unique(jj * n + ii, return_inverse=True)
    val = np.zeros(len(key))
    np.add.at(val, inv, vv)
    c = key // n
    colptr = np.zeros(n + 1, np.int64)
    np.add.at(colptr, c + 1, 1)
    out = LP(dict(lp, mode=AS, name=lp.get("name", "lp") + "_qp"))
    out["q_colptr"] = np.cumsum(colptr)
    out["q_rowidx"] = (key % n).astype(np.int32)
    out["q_val"] = val
    return out


def as_dense_interleaved(m=100, n=200, density=0.3, seed=0, theta_range=(1e2, 1e6), rho=1e-10,
                         delta=1e-10, nrhs=1, scale=1.0):
    """A dense-ish random LP (Bernoulli(density) pattern, N(0,1) values, no empty row or
    column) in augmented-system form, and an elimination order that interleaves primal and
    dual variables (x_0, then y_0, x_1, x_2, y_1, ...), so that after x_0 the rest of K forms
    one front of mixed-sign pivots of order ~ n + m - 1.  Returns (lp, perm), perm new -> old
    in the augmented numbering (x first, then y)."""
    g = rng(300, seed)
    A = np.where(g.random((m, n)) < density, scale * g.standard_normal((m, n)), 0.0)
    for j in np.flatnonzero(~A.any(axis=0)):
        A[g.integers(m), j] = scale * g.standard_normal()
    for i in np.flatnonzero(~A.any(axis=1)):
        A[i, g.integers(n)] = scale * g.standard_normal()
    cols = [np.flatnonzero(A[:, j]) for j in range(n)]
    colptr = np.zeros(n + 1, np.int64)
    for j, c in enumerate(cols):
        colptr[j + 1] = colptr[j] + len(c)
    rowidx = np.concatenate(cols).astype(np.int32)
    val = np.concatenate([A[c, j] for j, c in enumerate(cols)])
    theta = log_uniform(g, *theta_range, n)
    gr = rng(300, seed, 1)
    r7 = gr.standard_normal((nrhs, n)).T.copy(order="F")
    r1 = gr.standard_normal((nrhs, m)).T.copy(order="F")
    lp = LP(m=m, n=n, colptr=colptr, rowidx=rowidx, val=val, theta=theta, rho=rho, delta=delta,
            mode=AS, r1=r1, r7=r7, name=f"as_dense_interleaved_{m}x{n}")
    xs, ys = list(range(n)), list(range(n, n + m))
    perm = [xs.pop(0)]
    while xs or ys:
        if ys:
            perm.append(ys.pop(0))
        if xs:
            perm.append(xs.pop(0))
        if xs and len(xs) > len(ys):
            perm.append(xs.pop(0))
    return lp, np.asarray(perm, np.int32)


def indefinite_hessian(lp, seed=0, per_row=3, window=30, diag_scale=1.0):
    """A symmetric Q on the columns of `lp` that is NOT positive semidefinite: every column c
    is coupled to per_row others within `window` positions (N(0,1) values, each pair drawn
    once per direction and summed) and has an N(0, diag_scale^2) diagonal of either sign.
    With it the (1,1) block -(Q + Theta^-1 + rho I) is indefinite, so the augmented system
    is no longer quasidefinite.  Adds q_colptr, q_rowidx, q_val (lower triangle, CSC)."""
    g = rng(310, seed)
    n = lp["n"]
    Q = np.zeros((n, n))
    for c in range(n):
        lo, hi = max(0, c - window), min(n, c + window + 1)
        others = g.choice(np.setdiff1d(np.arange(lo, hi), [c]), size=per_row, replace=False)
        for o in others:
            v = g.standard_normal()
            Q[c, o] += v
            Q[o, c] += v
        Q[c, c] = diag_scale * g.standard_normal()
    lower = np.tril(Q)
    cols = [np.flatnonzero(lower[:, j]) for j in range(n)]
    qcp = np.zeros(n + 1, np.int64)
    for j in range(n):
        qcp[j + 1] = qcp[j] + len(cols[j])
    out = LP(dict(lp, mode=AS, name=lp.get("name", "lp") + "_indefinite_qp"))
    out["q_colptr"] = qcp
    out["q_rowidx"] = np.concatenate(cols).astype(np.int32)
    out["q_val"] = np.concatenate([lower[c, j] for j, c in enumerate(cols)])
    return out


def planted_hessian(lp, perm, seed=0, npairs=2, coupling=0.01):
    """A Hessian that is indefinite on `npairs` planted pairs of primal columns (k, j), moved to
    the end of the elimination order `perm` (new -> old, augmented numbering) so that they are
    the last pivots of the last front.  On a pair, Theta is 1, the A column is scaled by
    `coupling`, and Q_kk = a - 1, Q_jj = -b - 1, Q_kj = -c with a ~ U[2, 3], b ~ U[0.5, 1],
    c = sqrt(a b) U[1.2, 1.4]; Q is zero elsewhere.  The (1,1) block of K_static then holds
    [[-a, c], [c, +b]] (up to rho) on each pair: a diagonal of the expected sign next to a
    partner of the wrong sign whose coupling exceeds sqrt(a b) by at least 20 %.  Returns
    (lp with q_colptr, q_rowidx, q_val (lower triangle, CSC), the new order)."""
    g = rng(311, seed)
    n = lp["n"]
    pairs = [(n - 2 * npairs + 2 * i, n - 2 * npairs + 2 * i + 1) for i in range(npairs)]
    out = LP(dict(lp, mode=AS, name=lp.get("name", "lp") + "_planted_qp"))
    theta = np.array(lp["theta"], float)
    val = np.array(lp["val"], float)
    cols, vals = [[] for _ in range(n)], [[] for _ in range(n)]
    for k, j in pairs:
        a, b = g.uniform(2.0, 3.0), g.uniform(0.5, 1.0)
        c = np.sqrt(a * b) * g.uniform(1.2, 1.4)
        cols[k] += [k, j]
        vals[k] += [a - 1.0, -c]
        cols[j] += [j]
        vals[j] += [-b - 1.0]
        for q in (k, j):
            theta[q] = 1.0
            val[lp["colptr"][q]:lp["colptr"][q + 1]] *= coupling
    qcp = np.zeros(n + 1, np.int64)
    for q in range(n):
        qcp[q + 1] = qcp[q] + len(cols[q])
    out["theta"], out["val"] = theta, val
    out["q_colptr"] = qcp
    out["q_rowidx"] = np.asarray([r for c in cols for r in c], np.int32)
    out["q_val"] = np.asarray([v for c in vals for v in c], float)
    planted = [q for pr in pairs for q in pr]
    rest = [int(v) for v in perm if int(v) not in set(planted)]
    return out, np.asarray(rest + planted, np.int32)


def q_dense(lp):
    """Q of a quadratic program's dict as a dense symmetric array."""
    n = lp["n"]
    Q = np.zeros((n, n))
    cp, ri, v = lp["q_colptr"], lp["q_rowidx"], lp["q_val"]
    for j in range(n):
        for e in range(cp[j], cp[j + 1]):
            Q[ri[e], j] = Q[j, ri[e]] = v[e]
    return Q


def lp_dense(lp):
    """A of an LP dict as a dense array."""
    A = np.zeros((lp["m"], lp["n"]))
    cp, ri, v = lp["colptr"], lp["rowidx"], lp["val"]
    for j in range(lp["n"]):
        A[ri[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
    return A


def small_config():
    """The small correctness workload: random 300 x 600 LP, normal equations, FP64."""
    return ne_random()


def main_config():
    """The 20000 x 40000 staircase LP, augmented system, FP64."""
    return as_staircase()


# ------------------------------------------------------------------ measured workloads

def named_workload(name):
    """The measured workloads by name: (system, analyse options).  Batches carry their systems
    under "systems"."""
    if name == "as_staircase":
        return as_staircase(), dict()
    if name == "ne_random":
        return ne_random(), dict()
    if name == "ne_grid":
        lp = ne_grid(nrhs=8)
        return lp, dict(ordering=2, grid=lp["grid"])
    if name == "ne_grid_small":
        lp = ne_grid(24, 24, 20, nrhs=8)
        return lp, dict(ordering=2, grid=lp["grid"])
    if name.startswith("ne_dense_front"):  # ne_dense_front or ne_dense_front_<f>
        f = int(name.split("_")[-1]) if name[-1].isdigit() else 4096
        return ne_dense_front(f), dict(ordering=0)
    if name in ("as_batch", "as_batch_small"):
        lps = as_batch(512 if name == "as_batch" else 32)
        cat = concat_systems(lps)
        cat["systems"] = lps
        return cat, dict(systems=lps, ordering=0)
    if name == "as_dense_cols":
        lp = as_dense_cols()
        return lp, dict(ordering=2, grid=lp["grid"])
    if name == "as_staircase_qp":  # the staircase with a Hessian on half of its columns
        return with_hessian(as_staircase(), seed=1, frac=0.5, per_row=3, window=50), dict()
    raise ValueError(f"unknown workload {name}")


def iteration_theta(lp, k, seed):
    """Theta of iteration k of a measured workload (batches: system s draws from seed [4, s, k])."""
    if "systems" in lp:  # batch: system s, iteration k draws from seed [4, s, k]
        return np.concatenate([as_batch_theta(q, s, k) for s, q in enumerate(lp["systems"])])
    if lp["name"].startswith("ne_dense_front"):
        return log_uniform(rng(seed, 1000 + k), 1e-2, 1e2, lp["n"])
    g = rng(seed, 1000 + k)
    lo, hi = (1e-10, 1e10) if lp["mode"] == AS else (1e-6, 1e6)
    return log_uniform(g, lo, hi, lp["n"])
