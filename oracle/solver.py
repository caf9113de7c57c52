"""Ring filter and SPGL1-style basis-pursuit denoising (oracle, test
infrastructure).

The paper reconstructs a slice by solving

    min ||x||_1  subject to  ||filter(Radon{x} - data)||_2 < epsilon

with the SPGL1 software of van den Berg and Friedlander, where filter is a
3rd-order polynomial operator that suppresses ring artifacts and epsilon is
fixed in advance (introduction, problem statement and the paragraphs on ring
artifacts before it). Neither the filter nor the solver settings are given.

Readings:

  * ring filter F: ring artifacts are detector-dependent and angle-independent,
    so F removes, from every view, the part of the per-detector angle mean that
    a least-squares cubic in the detector coordinate does not explain:
        m[d] = mean_a y[a, d],   F y = y - 1 (x) (I - P3) m,
    P3 the orthogonal projection onto cubic polynomials in s_d. F is a
    symmetric projection (F = F^T = F^2).
  * solver: SPGL1 (van den Berg & Friedlander, SIAM J. Sci. Comput. 31(2), 2008)
    as published: root finding on the Pareto curve phi(tau) = min ||r|| subject
    to ||x||_1 <= tau by Newton steps tau += (phi - sigma) phi / ||A^T r||_inf,
    each LASSO(tau) subproblem by spectral projected gradient (Barzilai-Borwein
    step, non-monotone Grippo-Lampariello-Lucidi line search, Euclidean
    projection onto the l1 ball). The operator is A~ = F A, the data b~ = F b.
"""
from __future__ import annotations

import numpy as np

__all__ = ["cubic_basis", "ring_filter", "project_l1", "spgl1_bpdn"]


def cubic_basis(n_det: int) -> np.ndarray:
    """Orthonormal basis (n_det x 4) of cubic polynomials in s_d = d - N/2."""
    s = np.arange(n_det, dtype=np.float64) - n_det / 2
    V = np.vander(s / (n_det / 2), 4, increasing=True)
    Q, _ = np.linalg.qr(V)
    return Q


def ring_filter(y) -> np.ndarray:
    """F y = y - 1 (x) (I - P3) m, m the per-detector mean over views."""
    y = np.asarray(y, dtype=np.float64)
    m = y.mean(axis=0)
    Q = cubic_basis(y.shape[1])
    ring = m - Q @ (Q.T @ m)
    return y - ring[None, :]


def project_l1(x, tau: float) -> np.ndarray:
    """Euclidean projection onto {||x||_1 <= tau} (soft threshold at the
    level lambda that makes the l1 norm equal tau; sort-based)."""
    x = np.asarray(x, dtype=np.float64)
    if tau <= 0:
        return np.zeros_like(x)
    a = np.abs(x).ravel()
    if a.sum() <= tau:
        return x.copy()
    u = np.sort(a)[::-1]
    cs = np.cumsum(u)
    k = np.arange(1, u.size + 1)
    idx = np.nonzero(u * k > (cs - tau))[0]
    rho = idx[-1] if idx.size else 0
    lam = (cs[rho] - tau) / (rho + 1.0)
    return np.sign(x) * np.maximum(np.abs(x) - lam, 0.0)


def spgl1_bpdn(A, At, b, sigma: float, x0=None, tau0: float | None = None, opt_tol: float = 1e-4,
               bp_tol: float = 1e-6, dec_tol: float = 1e-4, max_iter: int = 5000, bb_min: float = 1e-16,
               bb_max: float = 1e5, n_mem: int = 3):
    """min ||x||_1 s.t. ||A x - b||_2 <= sigma by SPGL1 root finding.

    A, At: callables for the operator and its adjoint (float64 arrays).
    Per iteration, with f = ||r||^2/2, r = b - A x, g = -A^T r:
      * relative LASSO duality gap rgap = |r.(r - b) + tau ||g||_inf| / max(1, f);
      * exit when rgap <= max(opt_tol, |f - sigma^2/2|/max(1, f)) or the
        residual error | ||r|| - sigma | / max(1, ||r||) <= opt_tol, and then
        either ||r|| <= bp_tol ||b|| (basis pursuit) or that residual error is
        below opt_tol (root of the Pareto curve found);
      * Newton step tau += ||r|| (||r|| - sigma) / ||g||_inf once the projected
        gradient iterations stall: |f - f_old| <= dec_tol f while
        ||r|| > 2 sigma, or |f - f_old| <= 0.1 f | ||r|| - sigma | nearer the root.
    Returns (x, info): residual norm, tau, iterations, A and At applications.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(At(b).shape) if x0 is None else np.array(x0, dtype=np.float64)
    tau = float(np.abs(x).sum()) if tau0 is None else float(tau0)
    x = project_l1(x, tau)
    n_a = n_at = 0

    def resid(xx):
        nonlocal n_a
        n_a += 1
        return b - A(xx)

    def grad(rr):
        nonlocal n_at
        n_at += 1
        return -At(rr)

    r = resid(x)
    f = 0.5 * float(np.vdot(r, r))
    f_old = np.inf
    g = grad(r)
    fs = [f] * n_mem
    gn = float(np.abs(g).max())
    alpha = min(max(1.0 / gn if gn > 0 else 1.0, bb_min), bb_max)
    it = 0
    status = "max_iter"
    for it in range(1, max_iter + 1):
        rnorm = float(np.sqrt(2 * f))
        gnorm = float(np.abs(g).max())
        gap = float(np.vdot(r, r - b)) + tau * gnorm
        rgap = abs(gap) / max(1.0, f)
        aerr1 = rnorm - sigma
        rerr1 = abs(aerr1) / max(1.0, rnorm)
        rerr2 = abs(f - 0.5 * sigma * sigma) / max(1.0, f)
        if rgap <= max(opt_tol, rerr2) or rerr1 <= opt_tol:
            if rnorm <= bp_tol * bnorm:
                status = "bp"
                break
            if rerr1 <= opt_tol:
                status = "root"
                break
        change = abs(f - f_old)
        stalled = (change <= dec_tol * f and rnorm > 2 * sigma) or \
                  (change <= 0.1 * f * abs(rnorm - sigma) and rnorm <= 2 * sigma)
        if stalled and gnorm > 0:
            tau_old = tau
            tau = max(0.0, tau + rnorm * aerr1 / gnorm)   # Newton step on the Pareto curve
            if tau < tau_old:
                # the ball shrank: restart the subproblem from the projected
                # (feasible) iterate with its own residual and gradient
                x = project_l1(x, tau)
                r = resid(x)
                f = 0.5 * float(np.vdot(r, r))
                g = grad(r)
            fs = [f] * n_mem
        # spectral projected gradient step, non-monotone (GLL) backtracking
        fmax = max(fs)
        step = 1.0
        while True:
            xn = project_l1(x - step * alpha * g, tau)
            dx = xn - x
            rn = resid(xn)
            fn = 0.5 * float(np.vdot(rn, rn))
            if fn <= fmax + 1e-4 * float(np.vdot(g, dx)) or step < 1e-10:
                break
            step *= 0.5
        gn_ = grad(rn)
        s = (xn - x).ravel()
        yv = (gn_ - g).ravel()
        sts, sty = float(s @ s), float(s @ yv)
        alpha = bb_max if sty <= 0 else min(max(sts / sty, bb_min), bb_max)
        f_old = f
        x, r, f, g = xn, rn, fn, gn_
        fs = fs[1:] + [f]
    info = {"rnorm": float(np.sqrt(2 * f)), "tau": tau, "iterations": it, "n_A": n_a, "n_At": n_at,
            "status": status}
    return x, info
