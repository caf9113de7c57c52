"""Pins for the oracle's ring filter, l1-ball projection and SPGL1 solver.

The ring filter is pinned by its algebra (symmetric projection that removes
angle-independent non-cubic detector patterns and keeps cubic ones), the
projection by an independent bisection on the threshold, and the solver by
a linear-programming solution of basis pursuit (scipy's HiGHS) and by the
optimality conditions of basis-pursuit denoising.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle.solver import cubic_basis, project_l1, ring_filter, spgl1_bpdn


def test_cubic_basis_spans_cubics():
    N = 40
    Q = cubic_basis(N)
    assert np.allclose(Q.T @ Q, np.eye(4), atol=1e-12)
    s = np.arange(N) - N / 2
    cubic = 0.3 - 0.02 * s + 1e-3 * s ** 2 + 2e-5 * s ** 3
    assert np.allclose(Q @ (Q.T @ cubic), cubic, atol=1e-12)
    # a non-polynomial profile is not in the span; its residual matches polyfit
    g = np.cos(0.9 * s)
    res = g - Q @ (Q.T @ g)
    fit = np.polyval(np.polyfit(s, g, 3), s)
    assert np.allclose(res, g - fit, atol=1e-10)


def test_ring_filter_algebra():
    rng = np.random.default_rng(0)
    nv, N = 17, 32
    y, z = rng.standard_normal((nv, N)), rng.standard_normal((nv, N))
    Fy = ring_filter(y)
    assert abs(np.sum(Fy * z) - np.sum(y * ring_filter(z))) < 1e-12      # symmetric
    assert np.allclose(ring_filter(Fy), Fy, atol=1e-12)                  # idempotent
    s = np.arange(N) - N / 2
    g = rng.standard_normal(N)
    Q = cubic_basis(N)
    ring = g - Q @ (Q.T @ g)                                             # non-cubic stripe profile
    assert np.allclose(ring_filter(np.tile(ring, (nv, 1))), 0.0, atol=1e-12)
    smooth = np.tile(1.0 + 0.01 * s - 1e-4 * s ** 3, (nv, 1))
    assert np.allclose(ring_filter(smooth), smooth, atol=1e-12)
    zero_mean = y - y.mean(axis=0)
    assert np.allclose(ring_filter(zero_mean), zero_mean, atol=1e-12)


def _proj_bisect(x, tau):
    lo, hi = 0.0, np.abs(x).max()
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        if np.maximum(np.abs(x) - lam, 0).sum() > tau:
            lo = lam
        else:
            hi = lam
    return np.sign(x) * np.maximum(np.abs(x) - 0.5 * (lo + hi), 0)


@pytest.mark.parametrize("tau", [0.0, 0.3, 2.0, 7.5, 100.0])
def test_project_l1(tau):
    x = np.random.default_rng(1).standard_normal(50)
    p = project_l1(x, tau)
    if np.abs(x).sum() <= tau:
        assert np.array_equal(p, x)
    else:
        assert abs(np.abs(p).sum() - tau) <= 1e-12 * max(1, tau)
        assert np.allclose(p, _proj_bisect(x, tau), atol=1e-12)


def _random_cs(seed, m=60, n=200, k=8):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    x0 = np.zeros(n)
    x0[rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    return A, x0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_basis_pursuit_matches_linear_program(seed):
    A, x0 = _random_cs(seed)
    b = A @ x0
    bp_tol = 1e-6
    x, info = spgl1_bpdn(lambda v: A @ v, lambda r: A.T @ r, b, 0.0, opt_tol=1e-6, bp_tol=bp_tol, max_iter=20000)
    assert info["status"] == "bp"
    r = A @ x - b
    assert np.linalg.norm(r) <= bp_tol * np.linalg.norm(b)
    n = A.shape[1]
    lp = linprog(np.ones(2 * n), A_eq=np.hstack([A, -A]), b_eq=b, bounds=(0, None), method="highs")
    assert lp.status == 0
    # The basis-pursuit exit leaves A x = b satisfied only to bp_tol, so x may
    # undercut the LP optimum; weak duality bounds by how much. The LP dual y
    # (|A^T y|_inf <= 1) gives ||x||_1 >= y.(A x) = LP* + y.(A x - b)
    # >= LP* - ||y|| ||A x - b||. From above, the root of the Pareto curve is
    # approached from below, so ||x||_1 <= LP* up to the subproblem tolerance.
    y = lp.eqlin.marginals
    assert np.abs(A.T @ y).max() <= 1 + 1e-9
    err = np.abs(x).sum() - lp.fun
    assert err >= -(np.linalg.norm(y) * np.linalg.norm(r) + 1e-12 * lp.fun)
    assert err <= 1e-6 * lp.fun
    assert np.linalg.norm(x - x0) <= 1e-4 * np.linalg.norm(x0)     # exact sparse recovery


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_basis_pursuit_tight_tolerance_matches_linear_program(seed):
    """With the basis-pursuit exit out of reach (bp_tol below what a root exit
    leaves) the solve ends at the root sigma = 0 to opt_tol, and the l1 norm
    meets the LP optimum to within the same dual bound."""
    A, x0 = _random_cs(seed)
    b = A @ x0
    x, info = spgl1_bpdn(lambda v: A @ v, lambda r: A.T @ r, b, 0.0, opt_tol=1e-8, bp_tol=1e-12, max_iter=20000)
    n = A.shape[1]
    lp = linprog(np.ones(2 * n), A_eq=np.hstack([A, -A]), b_eq=b, bounds=(0, None), method="highs")
    y = lp.eqlin.marginals
    r = A @ x - b
    err = np.abs(x).sum() - lp.fun
    assert err >= -(np.linalg.norm(y) * np.linalg.norm(r) + 1e-12 * lp.fun)
    assert abs(err) <= 1e-6 * lp.fun


def test_bpdn_optimality_conditions():
    A, x0 = _random_cs(3)
    rng = np.random.default_rng(4)
    e = 0.01 * rng.standard_normal(A.shape[0])
    b = A @ x0 + e
    sigma = float(np.linalg.norm(e))
    x, info = spgl1_bpdn(lambda v: A @ v, lambda r: A.T @ r, b, sigma, opt_tol=1e-9, max_iter=20000)
    assert info["status"] == "root"
    r = b - A @ x
    assert abs(np.linalg.norm(r) - sigma) <= 1e-8 * sigma
    g = A.T @ r
    lam = np.abs(g).max()
    tau = np.abs(x).sum()
    sup = np.abs(x) > 1e-9
    # Dual conditions to the accuracy the duality gap allows. For LASSO(tau)
    # at a point of the ball's surface, the gap delta = tau lam - x.g equals
    # sum_i |x_i| (lam - sign(x_i) g_i), a sum of non-negative terms, so on
    # the support lam - sign(x_i) g_i <= delta / |x_i|. The root exit does not
    # drive delta to zero, so delta is required small first.
    assert abs(tau - info["tau"]) <= 1e-9 * tau
    delta = tau * lam - float(x @ g)
    assert -1e-12 * tau * lam <= delta <= 1e-2 * float(r @ r)
    assert np.all(lam - np.sign(x[sup]) * g[sup] <= delta / np.abs(x[sup]) * (1 + 1e-9) + 1e-12 * lam)
    # the optimal l1 norm is the root tau* of phi(tau) = sigma on the Pareto
    # curve; phi is evaluated independently by accelerated projected gradient
    # (FISTA, fixed step 1/||A||^2) and the root bracketed by bisection
    L = np.linalg.norm(A, 2) ** 2

    def phi(tau, its=2000):
        z = y = np.zeros(A.shape[1])
        t = 1.0
        for _ in range(its):
            zn = project_l1(y - A.T @ (A @ y - b) / L, tau)
            tn = 0.5 * (1 + np.sqrt(1 + 4 * t * t))
            y, z, t = zn + (t - 1) / tn * (zn - z), zn, tn
        return np.linalg.norm(b - A @ z)

    lo, hi = 0.0, 2 * np.abs(x0).sum()
    for _ in range(36):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if phi(mid) > sigma else (lo, mid)
    assert abs(np.abs(x).sum() - 0.5 * (lo + hi)) <= 1e-5 * hi
