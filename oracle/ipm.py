"""Plain reference interior point method for linear programs, written from the paper's
Section 3 (Newton system, its reduction to the augmented system, termination, regularisation)
and Section 4.7 (number of correctors), for the LP of Section 2 with every variable bounded
below by zero and none bounded above (l = 0, U empty): min c^T x, A x = b, x >= 0.

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


def newton_direction(A, x, z, theta_inv_reg, delta, r1, r4, r5):
    """Section 3: the Newton system with r2 = r3 = 0 (lower bounds at zero, x^l = x) reduced to
    the augmented system [[-(Theta^-1 + rho I), A^T], [A, delta I]] [dx; dy] = [r7; r1] with
    r7 = r4 - X^-1 r5, and dz = X^-1 (r5 - Z dx)."""
    m, n = A.shape
    K = np.zeros((n + m, n + m))
    K[:n, :n] = -np.diag(theta_inv_reg)
    K[:n, n:] = A.T
    K[n:, :n] = A
    K[n:, n:] = delta * np.eye(m)
    r7 = r4 - r5 / x
    sol = np.linalg.solve(K, np.concatenate([r7, r1]))
    dx, dy = sol[:n], sol[n:]
    dz = (r5 - z * dx) / x
    return dx, dy, dz


def max_step(v, dv):
    """Largest alpha in (0, 1] with v + alpha dv >= 0."""
    neg = dv < 0
    if not neg.any():
        return 1.0
    return float(min(1.0, np.min(-v[neg] / dv[neg])))


def corrector_count(nnz_l, flops_fact, f, alpha_f, kmax):
    """Section 4.7: (1 + k)(1 + f/2) E_s ~ E_f alpha_F with E_s = 2 nnz(L) and E_f the
    factorisation flops; k at least 1 (the first corrector always pays) and at most kmax."""
    es = 2.0 * nnz_l
    k = int(np.floor(alpha_f * flops_fact / ((1.0 + f / 2.0) * es) - 1.0))
    return max(1, min(kmax, k))


def converged(A, b, c, x, y, z, tau):
    """Section 3.1, without scaling: primal and dual feasibility and the relative gap."""
    r1 = b - A @ x
    r4 = c - A.T @ y - z
    fp, fd = float(c @ x), float(b @ y)
    ok = (np.max(np.abs(r1), initial=0.0) <= tau * (1.0 + np.max(np.abs(b), initial=0.0))
          and np.max(np.abs(r4), initial=0.0) <= tau * (1.0 + np.max(np.abs(c), initial=0.0))
          and abs(fp - fd) <= tau * (1.0 + 0.5 * abs(fp + fd)))
    return ok, fp, fd


def ipm(A, b, c, rho=1e-10, delta=1e-10, k=1, tau=1e-8, max_iter=100):
    """Returns dict(x, y, z, iters, status ('optimal' | 'max_iter'), history) where history
    holds per iteration (mu, alpha_p, alpha_d, correctors used)."""
    A = np.asarray(A, dtype=float)
    m, n = A.shape
    x = np.ones(n)
    z = np.ones(n)
    y = np.zeros(m)
    history = []
    for it in range(max_iter):
        ok, fp, fd = converged(A, b, c, x, y, z, tau)
        if ok:
            return dict(x=x, y=y, z=z, iters=it, status="optimal", history=history, fp=fp, fd=fd)
        r1 = b - A @ x
        r4 = c - A.T @ y - z
        mu = float(x @ z) / n
        tinv = z / x + rho  # Theta^-1 plus the primal regularisation
        # predictor: sigma = 0
        r5 = -x * z
        dxa, dya, dza = newton_direction(A, x, z, tinv, delta, r1, r4, r5)
        apa, ada = max_step(x, dxa), max_step(z, dza)
        mu_aff = float((x + apa * dxa) @ (z + ada * dza)) / n
        sigma = (mu_aff / mu) ** 3
        smu = sigma * mu
        # correctors from the complementarity products at the trial point (Section 3):
        # r1 = r4 = 0, r5 moves the products into [BETA_MIN, BETA_MAX] * sigma * mu
        dx, dy, dz = dxa, dya, dza
        ap, ad = apa, ada
        used = 0
        for j in range(k):
            tp, td = min(1.0, ap + ALPHA_PLUS), min(1.0, ad + ALPHA_PLUS)
            v = (x + tp * dx) * (z + td * dz)
            t = np.clip(v, BETA_MIN * smu, BETA_MAX * smu) - v
            t = np.maximum(t, -BETA_MAX * smu)
            cx, cy, cz = newton_direction(A, x, z, tinv, delta, np.zeros(m), np.zeros(n), t)
            nx, ny, nz = dx + cx, dy + cy, dz + cz
            nap, nad = max_step(x, nx), max_step(z, nz)
            if j > 0 and nap + nad < (1.0 + ACCEPT_GAIN) * (ap + ad):
                break
            dx, dy, dz, ap, ad = nx, ny, nz, nap, nad
            used += 1
        history.append((mu, ap, ad, used))
        x = x + STEP_FACTOR * ap * dx
        y = y + STEP_FACTOR * ad * dy
        z = z + STEP_FACTOR * ad * dz
    ok, fp, fd = converged(A, b, c, x, y, z, tau)
    return dict(x=x, y=y, z=z, iters=max_iter, status="optimal" if ok else "max_iter", history=history,
                fp=fp, fd=fd)
