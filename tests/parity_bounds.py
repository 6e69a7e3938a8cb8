"""Tolerances of the GPU-vs-oracle comparisons, derived from perturbation theory (no GPU here).

Two functions, both used by the GPU tests and pinned on the CPU in test_parity_bounds.py:

* ``solution_gap_bound``: two approximate solutions x_g, x_o of K x = b with residuals r_g, r_o
  satisfy x_g - x_o = K^-1 (r_o - r_g), so ||x_g - x_o||_inf <= ||K^-1||_inf (||r_g|| + ||r_o||).
  The residuals are formed in FP64 from K itself, with an error of at most (w + 1) u (|K||x| +
  |b|) per row (w: the most nonzeros in a row), which is added.  This is the kappa-times-
  backward-error bound in its exact form.

* ``pivot_bounds``: the factor of one pivot sequence is unique, so the GPU's and the oracle's
  D differ only by rounding.  Each computed factor is the exact factor of P (K_static + E) P^T
  + dM with |dM| <= gamma |L||D||L^T| (backward stability of LDL^T with 1x1 and 2x2 pivots,
  gamma = (N + 16) u per side).  After k pivots the remaining Schur complement is
  S = W M W^T restricted to rows and columns >= k, where row i of W is [-L[i, :k] L11^-1, e_i]
  (L11 = L[:k, :k]).  To first order dS_ij = w_i^T dM w_j, so
      |dS_ij| <= 2 gamma |w_i|^T |L||D||L^T| |w_j| + sum_{l<k} |w_i[l]| |w_j[l]| |dE_l|,
  the last term for the dynamic regularisation of earlier pivots, which enters M on its
  diagonal and may differ between the two sides.  Every pivot value is a function of such
  entries at its step: an unmodified 1x1 pivot and the entries of a 2x2 block are S entries
  plus a static shift; a lift is sigma eps ||K||_1 + s (equal up to ||K||_1's agreement);
  Proposition 3 sets sigma beta with beta = max_j S_jk^2 / |S_jj + s_j| over the window's
  same-sign columns (its first-order change is bounded through dS_jk and dS_jj, and a
  maximum moves by at most the largest change of its arguments); the sign rule takes
  sigma max(|S_kk + s_k|, beta, eps ||K||_1).  E_dyn = d - (S_kk + s_k) then moves by at most
  |dd| + |dS_kk|.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from paper_2508_04370_amd import workloads as W

U = 2.0 ** -53
EF_LIFT, EF_PROP3, EF_SIGN = 1, 2, 4


# Matched cases whose biggest front (order ~270) goes through the pivot-window kernel: a dense
# interleaved augmented system (2x2 pivots and lifts) with indefinite Hessian pairs planted as
# its last pivots (Proposition 3 and the sign rule), with the presort on, and off (Bunch-Kaufman
# branch (d), which the presort makes unreachable).  "full" cases have a moderate Theta range;
# the GPU must take every decision the oracle takes.  The wide-Theta case (Theta up to 1e6)
# has pivots computed through heavy cancellation; there the two sides may part at a decision
# that the input does not fix at working precision (decision_margins below 1), and agree up to
# it.  All have decisions that do not move under a 1e-10 relative perturbation of Theta
# (test_parity_bounds.py).
MATCHED_CASES = {
    "presort": dict(seed=4, theta_range=(1e-1, 1e1), presort=1, full=True),
    "no_presort": dict(seed=2, theta_range=(1e-2, 1e2), presort=0, full=True),
    "presort_wide_theta": dict(seed=0, theta_range=(1e2, 1e6), presort=1, full=False),
}


def matched_case(name):
    """(lp, perm, presort) of one matched case; perm new -> old for the oracle's analyse."""
    c = MATCHED_CASES[name]
    lp, perm = W.as_dense_interleaved(100, 200, 0.3, seed=c["seed"], theta_range=c["theta_range"],
                                      rho=1e-10, delta=1e-10)
    lp, perm = W.planted_hessian(lp, perm, seed=c["seed"], npairs=3)
    return lp, perm, c["presort"]


def signs_shifts(lp, fperm):
    """Expected pivot sign and static shift of every position (Section 4.5)."""
    primal = fperm < lp["n"] if lp["mode"] == W.AS else np.zeros(len(fperm), bool)
    return np.where(primal, -1, 1), np.where(primal, -lp["rho"], lp["delta"])


def dense_k_static(lp, theta, rho, delta):
    """K_static of Section 3.2 written out densely (and the QP's -(Q + Theta^-1 + rho I))."""
    A = W.lp_dense(lp)
    m, n = A.shape
    if lp["mode"] == W.AS:
        H = np.diag(1.0 / np.asarray(theta) + rho)
        if lp.get("q_colptr") is not None:
            H = H + W.q_dense(lp)
        return np.block([[-H, A.T], [A, delta * np.eye(m)]])
    tt = 1.0 / (1.0 / np.asarray(theta) + rho)
    return (A * tt) @ A.T + delta * np.eye(m)


def solution_gap_bound(K, b, xg, xo):
    """(||x_g - x_o||_inf, the bound on it from K^-1 and both residuals)."""
    Kinv_norm = np.abs(np.linalg.inv(K)).sum(axis=1).max()
    w = int((K != 0).sum(axis=1).max())
    bound = 0.0
    for x in (xg, xo):
        r = b - K @ x
        err = (w + 1) * U * (np.abs(K) @ np.abs(x) + np.abs(b))
        bound += np.abs(r).max() + err.max()
    # the computed inverse's norm is relatively accurate to about kappa u; 10 % margin
    return np.abs(xg - xo).max(), 1.1 * Kinv_norm * bound


def _block_d(d, doff, ptype):
    D = np.diag(d)
    for k in np.nonzero(ptype == 1)[0]:
        D[k, k + 1] = D[k + 1, k] = doff[k]
    return D


def windows_of(sn_ptr, nb=64):
    """(start, end) of the pivot window of every position."""
    N = int(sn_ptr[-1])
    ws, we = np.zeros(N, np.int64), np.zeros(N, np.int64)
    for s in range(len(sn_ptr) - 1):
        c0, c1 = int(sn_ptr[s]), int(sn_ptr[s + 1])
        for a in range(c0, c1, nb):
            ws[a:min(a + nb, c1)] = a
            we[a:min(a + nb, c1)] = min(a + nb, c1)
    return ws, we


def pivot_bounds(K, ex, sigma, shift, sn_ptr, knorm, dE, eps_lift=2.0 ** -52, nb=64, gamma=None,
                 knorm_rtol=1e-13):
    """Per-position bounds on |d_gpu - d_oracle|, |doff_gpu - doff_oracle| and
    |E_gpu - E_oracle| for one pivot sequence (the oracle's export ``ex``: fperm, dense L by
    position, d, doff, ptype, edyn, eflag).  sigma, shift: per position.  dE: E_gpu - E_oracle
    by position.  knorm_rtol: how closely the two sides' ||K_static||_1 agree (the lift value
    sigma eps ||K||_1 inherits it).  Also returns the step-k Schur complement diagonal (before
    E) for reports."""
    fperm = ex["fperm"]
    N = len(fperm)
    L = np.asarray(ex["L"])
    D = _block_d(ex["d"], ex["doff"], ex["ptype"])
    M0 = K[np.ix_(fperm, fperm)]
    G = np.abs(L) @ np.abs(D) @ np.abs(L).T
    if gamma is None:
        gamma = 2.0 * (N + 16) * U  # both sides
    ws, we = windows_of(sn_ptr, nb)
    bd, bo, be = np.zeros(N), np.zeros(N), np.zeros(N)
    skk = np.zeros(N)
    adE = np.abs(np.asarray(dE, float))
    tiny = eps_lift * knorm
    pt = ex["ptype"]
    for k in range(N):
        if pt[k] == 2:
            continue
        e = int(we[k])
        idx = np.arange(k, e)
        L11 = L[:k, :k]
        X = solve_triangular(L11, L[k:e, :k].T, lower=True, unit_diagonal=True, trans="T").T if k else \
            np.zeros((e - k, 0))  # rows L[i, :k] L11^-1
        A = np.abs(X)
        T = gamma * (A @ G[:k, :k] @ A.T + A @ G[:k, idx] + G[np.ix_(idx, np.arange(k))] @ A.T + G[np.ix_(idx, idx)])
        if k:
            T += (A * adE[:k]) @ A.T
        # Schur complement entries of the window at step k (oracle's values, before E_k)
        Lk = L[idx, :k]
        S = M0[np.ix_(idx, idx)] - Lk @ D[:k, :k] @ Lk.T
        skk[k] = S[0, 0]
        if pt[k] == 1:  # 2x2 block: three Schur complement entries plus shifts
            bd[k] = T[0, 0] + 2 * U * abs(ex["d"][k])
            bd[k + 1] = T[1, 1] + 2 * U * abs(ex["d"][k + 1])
            bo[k] = T[1, 0] + 2 * U * abs(ex["doff"][k])
            continue
        fl = int(ex["eflag"][k])
        dbeta = 0.0
        same = [j for j in range(1, e - k) if sigma[k + j] == sigma[k]]
        for j in same:
            den = abs(S[j, j] + shift[k + j])
            if den == 0.0:
                continue
            q = (2.0 * abs(S[j, 0]) * T[j, 0] + S[j, 0] ** 2 * T[j, j] / den) / den
            dbeta = max(dbeta, q)
        kn_err = knorm_rtol * tiny
        if fl == 0:
            bd[k] = T[0, 0]
        elif fl & EF_SIGN:
            bd[k] = max(T[0, 0], dbeta) + kn_err
        elif fl & EF_PROP3:
            bd[k] = dbeta
        else:  # a lift alone
            bd[k] = kn_err
        be[k] = bd[k] + T[0, 0] + kn_err if fl else 0.0
        # one rounding of the stored value itself
        bd[k] += 2 * U * abs(ex["d"][k])
    return bd, bo, be, skk


def decision_margins(K, ex, sigma, shift, sn_ptr, knorm, presort, alpha=(1 + 17 ** 0.5) / 8,
                     eps_lift=2.0 ** -52, nb=64, gamma=None):
    """Per pivot step k: how far the oracle's decisions are from their thresholds, over the
    first-order rounding bound of the values compared (>= 1: the input fixes the decision at
    working precision; < 1: another correct rounding of the same algorithm may decide the
    other way).  Checked: the presort's argmax of |S_jj| over the window (gap between the two
    largest against both bounds), the lift test max(|S_kk|, gamma_p) <= eps ||K||_1 and the
    Bunch-Kaufman test |S_kk| >= alpha gamma_p.  Returns the ratio per step start (inf where
    nothing is compared)."""
    fperm = ex["fperm"]
    N = len(fperm)
    L = np.asarray(ex["L"])
    D = _block_d(ex["d"], ex["doff"], ex["ptype"])
    M0 = K[np.ix_(fperm, fperm)]
    G = np.abs(L) @ np.abs(D) @ np.abs(L).T
    if gamma is None:
        gamma = 2.0 * (N + 16) * U
    ws, we = windows_of(sn_ptr, nb)
    tiny = eps_lift * knorm
    out = np.full(N, np.inf)
    for k in range(N):
        if ex["ptype"][k] == 2:
            continue
        e = int(we[k])
        idx = np.arange(k, e)
        X = solve_triangular(L[:k, :k], L[k:e, :k].T, lower=True, unit_diagonal=True, trans="T").T if k else \
            np.zeros((e - k, 0))
        A = np.abs(X)
        T = gamma * (A @ G[:k, :k] @ A.T + A @ G[:k, idx] + G[np.ix_(idx, np.arange(k))] @ A.T + G[np.ix_(idx, idx)])
        Lk = L[idx, :k]
        S = M0[np.ix_(idx, idx)] - Lk @ D[:k, :k] @ Lk.T
        S[np.arange(e - k), np.arange(e - k)] -= shift[idx]  # the tests read unregularised values
        r = np.inf
        dg = np.abs(np.diag(S))
        if presort and e - k > 1:
            o = np.argsort(-dg, kind="stable")
            r = min(r, (dg[o[0]] - dg[o[1]]) / max(T[o[0], o[0]] + T[o[1], o[1]], 1e-300))
        # the pivot at k after the step's swaps: its column in the window
        if e - k > 1:
            col = np.abs(S[1:, 0])
            q = int(np.argmax(col))
            gp, tg = col[q], T[1 + q, 0]
        else:
            gp, tg = 0.0, 0.0
        a, ta = dg[0], T[0, 0]
        big = max(a, gp)
        r = min(r, abs(big - tiny) / max(ta + tg, 1e-300))
        if big > tiny and gp > 0:
            r = min(r, abs(a - alpha * gp) / max(ta + alpha * tg, 1e-300))
        out[k] = r
    return out
