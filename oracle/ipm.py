"""Plain reference interior point method for linear programs, written from the paper's
Section 2 (formulation with bounds), Section 3 (Newton system, its reduction to the augmented
system, recovery, termination, regularisation) and Section 4.7 (number of correctors):

    min c^T x (+ x^T Q x / 2)  subject to  A x = b,  x - x^l = l,  x + x^u = u,  x^l, x^u >= 0,

with every lower bound finite (no free variables, as the paper assumes) and upper bounds
finite or +inf (then x^u and z^u are absent: zero in every formula).  The optional Q (dense,
symmetric positive semidefinite) gives the quadratic-programming variant: the dual residual
gains +Q x, the (1,1) block of the augmented system becomes -(Q + Theta^-1 + rho I), and both
objectives carry x^T Q x / 2.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product library.  Dense
NumPy linear algebra; every step in the order the paper gives it.  The readings of what the
paper leaves open (starting point, centring parameter, corrector targets and acceptance, step
factor) are the ones the device driver takes as well and are listed with it.
"""
from __future__ import annotations

import numpy as np

# Readings (shared with the device driver; the paper leaves these open)
STEP_FACTOR = 0.995      # fraction of the step to the boundary that is taken
ALPHA_PLUS = 0.1         # a centrality corrector aims at steps enlarged by this much
BETA_MIN, BETA_MAX = 0.1, 10.0   # target band of the complementarity products, times sigma*mu
ACCEPT_GAIN = 0.01       # a further corrector must raise alpha_p + alpha_d by this fraction


class State:
    """x, x^l, x^u, y, z^l, z^u; hasu marks the finite upper bounds (x^u = z^u = 0 elsewhere)."""

    def __init__(self, x, xl, xu, y, zl, zu):
        self.x, self.xl, self.xu, self.y, self.zl, self.zu = x, xl, xu, y, zl, zu


def start(l, u, m):
    """x = l + 1, or the midpoint where u - l < 2; x^l = x - l, x^u = u - x; z = 1; y = 0."""
    hasu = np.isfinite(u)
    x = l + 1.0
    narrow = hasu & (u - l < 2.0)
    x[narrow] = 0.5 * (l[narrow] + u[narrow])
    xl = x - l
    xu = np.where(hasu, u - x, 0.0)
    zl = np.ones_like(x)
    zu = np.where(hasu, 1.0, 0.0)
    return State(x, xl, xu, np.zeros(m), zl, zu)


def residuals(A, b, c, l, u, s, Q=None):
    """Section 3: r1 = b - A x, r2 = l - x + x^l, r3 = u - x - x^u (finite u only),
    r4 = c - A^T y - z^l + z^u (+ Q x for a quadratic program)."""
    hasu = np.isfinite(u)
    r1 = b - A @ s.x
    r2 = l - s.x + s.xl
    r3 = np.where(hasu, u - s.x - s.xu, 0.0)
    r4 = c - A.T @ s.y - s.zl + s.zu
    if Q is not None:
        r4 = r4 + Q @ s.x
    return r1, r2, r3, r4


def mu_of(s, hasu):
    return float(s.xl @ s.zl + s.xu[hasu] @ s.zu[hasu]) / (len(s.x) + int(hasu.sum()))


def newton_direction(A, s, hasu, tinv_reg, delta, r1, r2, r3, r4, r5, r6, Q=None):
    """Section 3: the Newton system reduced to [[-(Theta^-1 + rho I), A^T], [A, delta I]]
    [dx; dy] = [r7; r1] (the (1,1) block -(Q + Theta^-1 + rho I) for a quadratic program)
    with Theta^-1 = z^l/x^l + z^u/x^u and
    r7 = r4 - (X^l)^-1 (r5 + Z^l r2) + (X^u)^-1 (r6 - Z^u r3); then
    dx^l = dx - r2, dx^u = r3 - dx, dz^l = (X^l)^-1 (r5 - Z^l dx^l),
    dz^u = (X^u)^-1 (r6 - Z^u dx^u)."""
    m, n = A.shape
    K = np.zeros((n + m, n + m))
    K[:n, :n] = -np.diag(tinv_reg) if Q is None else -(Q + np.diag(tinv_reg))
    K[:n, n:] = A.T
    K[n:, :n] = A
    K[n:, n:] = delta * np.eye(m)
    xu_safe = np.where(hasu, s.xu, 1.0)
    r7 = r4 - (r5 + s.zl * r2) / s.xl + np.where(hasu, (r6 - s.zu * r3) / xu_safe, 0.0)
    sol = np.linalg.solve(K, np.concatenate([r7, r1]))
    dx, dy = sol[:n], sol[n:]
    dxl = dx - r2
    dxu = np.where(hasu, r3 - dx, 0.0)
    dzl = (r5 - s.zl * dxl) / s.xl
    dzu = np.where(hasu, (r6 - s.zu * dxu) / xu_safe, 0.0)
    return State(dx, dxl, dxu, dy, dzl, dzu)


def max_step(v, dv, mask=None):
    """Largest alpha in (0, 1] with v + alpha dv >= 0 (over mask)."""
    neg = dv < 0
    if mask is not None:
        neg &= mask
    if not neg.any():
        return 1.0
    return float(min(1.0, np.min(-v[neg] / dv[neg])))


def steps(s, d, hasu):
    ap = min(max_step(s.xl, d.xl), max_step(s.xu, d.xu, hasu))
    ad = min(max_step(s.zl, d.zl), max_step(s.zu, d.zu, hasu))
    return ap, ad


def add(d, e):
    return State(d.x + e.x, d.xl + e.xl, d.xu + e.xu, d.y + e.y, d.zl + e.zl, d.zu + e.zu)


def corrector_count(nnz_l, flops_fact, f, alpha_f, kmax):
    """Section 4.7: (1 + k)(1 + f/2) E_s ~ E_f alpha_F with E_s = 2 nnz(L) and E_f the
    factorisation flops; k at least 1 (the first corrector always pays) and at most kmax."""
    es = 2.0 * nnz_l
    k = int(np.floor(alpha_f * flops_fact / ((1.0 + f / 2.0) * es) - 1.0))
    return max(1, min(kmax, k))


def converged(A, b, c, l, u, s, tau, Q=None):
    """Section 3.1, without scaling: primal and dual feasibility and the relative gap, with
    f_p = c^T x (+ x^T Q x / 2) and f_d = b^T y + l^T z^l - u^T z^u (- x^T Q x / 2)."""
    hasu = np.isfinite(u)
    r1, r2, r3, r4 = residuals(A, b, c, l, u, s, Q)
    half_xqx = 0.0 if Q is None else 0.5 * float(s.x @ (Q @ s.x))
    fp = float(c @ s.x) + half_xqx
    fd = float(b @ s.y + l @ s.zl - u[hasu] @ s.zu[hasu]) - half_xqx
    pinf = max(np.max(np.abs(r1), initial=0.0), np.max(np.abs(r2), initial=0.0), np.max(np.abs(r3), initial=0.0))
    pscale = max(np.max(np.abs(b), initial=0.0), np.max(np.abs(l), initial=0.0),
                 np.max(np.abs(u[hasu]), initial=0.0))
    ok = (pinf <= tau * (1.0 + pscale)
          and np.max(np.abs(r4), initial=0.0) <= tau * (1.0 + np.max(np.abs(c), initial=0.0))
          and abs(fp - fd) <= tau * (1.0 + 0.5 * abs(fp + fd)))
    return ok, fp, fd


def ipm(A, b, c, l=None, u=None, rho=1e-10, delta=1e-10, k=1, tau=1e-8, max_iter=100, Q=None):
    """Returns dict(x, y, zl, zu, state, iters, status ('optimal' | 'max_iter'), history, fp, fd)
    where history holds per iteration (mu, alpha_p, alpha_d, correctors used).  l defaults to
    0 and u to +inf; Q (dense) makes it a quadratic program."""
    A = np.asarray(A, dtype=float)
    m, n = A.shape
    l = np.zeros(n) if l is None else np.asarray(l, dtype=float)
    u = np.full(n, np.inf) if u is None else np.asarray(u, dtype=float)
    hasu = np.isfinite(u)
    s = start(l, u, m)
    history = []
    it = 0
    for it in range(max_iter + 1):
        ok, fp, fd = converged(A, b, c, l, u, s, tau, Q)
        if ok or it == max_iter:
            break
        r1, r2, r3, r4 = residuals(A, b, c, l, u, s, Q)
        mu = mu_of(s, hasu)
        xu_safe = np.where(hasu, s.xu, 1.0)
        tinv = s.zl / s.xl + np.where(hasu, s.zu / xu_safe, 0.0) + rho  # plus the primal regularisation
        # predictor: sigma = 0
        r5, r6 = -s.xl * s.zl, np.where(hasu, -s.xu * s.zu, 0.0)
        da = newton_direction(A, s, hasu, tinv, delta, r1, r2, r3, r4, r5, r6, Q)
        apa, ada = steps(s, da, hasu)
        nc = n + int(hasu.sum())
        comp = float((s.xl + apa * da.xl) @ (s.zl + ada * da.zl)
                     + ((s.xu + apa * da.xu) @ (s.zu + ada * da.zu) if hasu.any() else 0.0))
        mu_aff = comp / nc
        sigma = (mu_aff / mu) ** 3
        smu = sigma * mu
        # correctors from the complementarity products at the trial point (Section 3):
        # r1 = r2 = r3 = r4 = 0; r5, r6 move the products into [BETA_MIN, BETA_MAX] * sigma * mu
        d, ap, ad = da, apa, ada
        zero_m, zero_n = np.zeros(m), np.zeros(n)
        used = 0
        for j in range(k):
            tp, td = min(1.0, ap + ALPHA_PLUS), min(1.0, ad + ALPHA_PLUS)

            def target(xv, dxv, zv, dzv):
                v = (xv + tp * dxv) * (zv + td * dzv)
                t = np.clip(v, BETA_MIN * smu, BETA_MAX * smu) - v
                return np.maximum(t, -BETA_MAX * smu)

            t5 = target(s.xl, d.xl, s.zl, d.zl)
            t6 = np.where(hasu, target(s.xu, d.xu, s.zu, d.zu), 0.0)
            e = newton_direction(A, s, hasu, tinv, delta, zero_m, zero_n, zero_n, zero_n, t5, t6, Q)
            nd = add(d, e)
            nap, nad = steps(s, nd, hasu)
            if j > 0 and nap + nad < (1.0 + ACCEPT_GAIN) * (ap + ad):
                break
            d, ap, ad = nd, nap, nad
            used += 1
        history.append((mu, ap, ad, used))
        sp, sd = STEP_FACTOR * ap, STEP_FACTOR * ad
        s = State(s.x + sp * d.x, s.xl + sp * d.xl, s.xu + sp * d.xu, s.y + sd * d.y, s.zl + sd * d.zl,
                  s.zu + sd * d.zu)
    return dict(x=s.x, y=s.y, zl=s.zl, zu=s.zu, z=s.zl - s.zu, state=s, iters=it,
                status="optimal" if ok else "max_iter", history=history, fp=fp, fd=fd)
