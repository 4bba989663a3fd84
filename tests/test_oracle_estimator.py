"""Pins of the oracle's range-only estimator (CPU only).

The linearised least-squares solve (Sec. III-A) is pinned to: exact recovery
from noise-free ranges, numpy's SVD least squares on the same linear system,
a brute-force grid search of the linearised objective, the invariances of the
geometry, and (for the Gauss-Newton refinement) a brute-force grid search of
the range-residual objective.
"""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st


def _track(rng, n, start=(0.0, 0.0), step=1.0, turn=0.3):
    """A vehicle path of n positions: unit steps with random heading changes."""
    psi = rng.uniform(-np.pi, np.pi)
    p = np.array(start, float)
    out = []
    for _ in range(n):
        psi += rng.uniform(-turn, turn)
        p = p + step * np.array([np.cos(psi), np.sin(psi)])
        out.append(p.copy())
    return np.array(out)


@pytest.mark.parametrize("seed", range(20))
def test_exact_recovery_noise_free(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 17))
    a = rng.uniform(-50, 50, size=(n, 2)) + rng.uniform(-1000, 1000, size=2)
    tgt = rng.uniform(-1500, 1500, size=2)
    r = np.hypot(a[:, 0] - tgt[0], a[:, 1] - tgt[1])
    ok, x, y = orc.ls_estimate(a[:, 0], a[:, 1], r)
    assert ok
    assert np.hypot(x - tgt[0], y - tgt[1]) <= 1e-9 * max(1.0, np.abs(tgt).max())
    ok, x, y = orc.ls_estimate(a[:, 0], a[:, 1], r, gn_iters=5)
    assert ok and np.hypot(x - tgt[0], y - tgt[1]) <= 1e-8 * max(1.0, np.abs(tgt).max())


@pytest.mark.parametrize("seed", range(20))
def test_matches_numpy_lstsq(orc, seed):
    """Rows [2 u_k, -1] [q; rho] = |u_k|^2 - r_k^2, solved by numpy's SVD."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 17))
    a = _track(rng, n, start=rng.uniform(-200, 200, 2))
    tgt = rng.uniform(-2000, 2000, size=2)
    r = np.hypot(*(a - tgt).T) + rng.normal(0, 2.0, n)
    ok, x, y = orc.ls_estimate(a[:, 0], a[:, 1], r)
    abar = a.mean(axis=0)
    u = a - abar
    M = np.column_stack([2 * u, -np.ones(n)])
    rhs = (u**2).sum(1) - r**2
    sol, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    want = abar + sol[:2]
    cond = np.linalg.cond(u.T @ u)
    if not ok:
        assert cond > 1e3  # only the guard may reject a solvable window
        return
    scale = max(1.0, np.abs(want).max())
    assert np.hypot(x - want[0], y - want[1]) <= 1e-9 * scale * max(1.0, cond)


def test_grid_search_linearised_objective(orc):
    """The minimiser of sum_k (2 u_k.q - rho - c_k)^2 found by brute force."""
    rng = np.random.default_rng(42)
    a = np.array([[0.0, 0.0], [8.0, 1.0], [3.0, 9.0], [-4.0, 6.0], [2.0, -5.0]])
    tgt = np.array([37.0, -21.0])
    r = np.hypot(*(a - tgt).T) + rng.normal(0, 0.5, len(a))
    ok, x, y = orc.ls_estimate(a[:, 0], a[:, 1], r)
    assert ok
    abar = a.mean(0)
    u = a - abar
    c = (u**2).sum(1) - r**2
    h = 0.05
    gx = np.arange(x - abar[0] - 3, x - abar[0] + 3, h)
    gy = np.arange(y - abar[1] - 3, y - abar[1] + 3, h)
    QX, QY = np.meshgrid(gx, gy, indexing="ij")
    lin = 2 * (QX[..., None] * u[:, 0] + QY[..., None] * u[:, 1]) - c  # [gx, gy, n]
    rho = lin.mean(-1, keepdims=True)  # best free rho for each q
    J = ((lin - rho) ** 2).sum(-1)
    i, j = np.unravel_index(np.argmin(J), J.shape)
    best = abar + np.array([gx[i], gy[j]])
    assert abs(best[0] - x) <= h and abs(best[1] - y) <= h


def test_grid_search_gauss_newton(orc):
    """With refinement, the estimate minimises sum (|p - a_k| - r_k)^2 on a
    well-conditioned scene (agents around the target)."""
    rng = np.random.default_rng(9)
    ang = np.linspace(0, 2 * np.pi, 8, endpoint=False) + rng.uniform(0, 0.3, 8)
    tgt = np.array([120.0, -40.0])
    a = tgt + 60 * np.column_stack([np.cos(ang), np.sin(ang)])
    r = np.hypot(*(a - tgt).T) + rng.normal(0, 3.0, len(a))
    ok, x, y = orc.ls_estimate(a[:, 0], a[:, 1], r, gn_iters=10)
    assert ok
    h = 0.02
    gx = np.arange(x - 2, x + 2, h)
    gy = np.arange(y - 2, y + 2, h)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    D = np.hypot(X[..., None] - a[:, 0], Y[..., None] - a[:, 1])
    J = ((D - r) ** 2).sum(-1)
    i, j = np.unravel_index(np.argmin(J), J.shape)
    assert abs(gx[i] - x) <= h and abs(gy[j] - y) <= h
    # the refinement does not increase the range-residual cost
    ok0, x0, y0 = orc.ls_estimate(a[:, 0], a[:, 1], r, gn_iters=0)
    cost = lambda px, py: ((np.hypot(px - a[:, 0], py - a[:, 1]) - r) ** 2).sum()
    assert cost(x, y) <= cost(x0, y0) + 1e-12


def test_guards(orc):
    # fewer than three entries
    assert not orc.ls_estimate([0.0, 1.0], [0.0, 0.0], [5.0, 5.0])[0]
    # collinear agents: S is singular
    xs = np.arange(6.0)
    assert not orc.ls_estimate(xs, 2 * xs + 1, np.hypot(xs - 50, 2 * xs + 1 - 20))[0]
    # a single repeated position
    assert not orc.ls_estimate([1.0] * 5, [2.0] * 5, [10.0] * 5)[0]


def test_batch_skips_missing_entries(orc):
    rng = np.random.default_rng(3)
    N, W = 50, 10
    win = np.zeros((N, W, 3))
    for i in range(N):
        a = _track(rng, W, start=rng.uniform(-100, 100, 2))
        tgt = rng.uniform(-500, 500, 2)
        win[i, :, :2] = a
        win[i, :, 2] = np.hypot(*(a - tgt).T) + rng.normal(0, 1, W)
        drop = rng.random(W) < 0.3
        win[i, drop, 2] = np.nan
    out, valid = orc.ls_batch(win)
    for i in range(N):
        keep = ~np.isnan(win[i, :, 2])
        ok, x, y = orc.ls_estimate(win[i, keep, 0], win[i, keep, 1], win[i, keep, 2])
        assert bool(valid[i]) == ok
        if ok:
            assert out[i, 0] == x and out[i, 1] == y


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 2**31), theta=st.floats(-np.pi, np.pi),
       shift=st.tuples(st.floats(-3000, 3000), st.floats(-3000, 3000)))
def test_equivariance(orc, seed, theta, shift):
    """Rotating and translating the scene moves the estimate the same way;
    permuting the window entries changes nothing."""
    rng = np.random.default_rng(seed)
    n = 10
    a = rng.uniform(-30, 30, size=(n, 2))
    tgt = rng.uniform(-300, 300, 2)
    r = np.hypot(*(a - tgt).T) + rng.normal(0, 1.0, n)
    ok, x, y = orc.ls_estimate(a[:, 0], a[:, 1], r)
    if not ok:
        return
    R = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
    b = a @ R.T + np.array(shift)
    ok2, x2, y2 = orc.ls_estimate(b[:, 0], b[:, 1], r)
    assert ok2
    want = R @ np.array([x, y]) + np.array(shift)
    cond = np.linalg.cond(np.cov(a.T))
    tol = 1e-9 * (1 + np.abs(want).max()) * max(1.0, cond) * (1 + np.abs(r).max())
    assert np.hypot(x2 - want[0], y2 - want[1]) <= tol
    perm = rng.permutation(n)
    ok3, x3, y3 = orc.ls_estimate(a[perm, 0], a[perm, 1], r[perm])
    assert ok3 and np.hypot(x3 - x, y3 - y) <= 1e-9 * (1 + abs(x) + abs(y)) * max(1.0, cond)


def test_sensitivity_is_derivative_bound(orc):
    """The reported sensitivity bounds the estimate's response to a small
    perturbation of every window input."""
    rng = np.random.default_rng(21)
    a = _track(rng, 10)
    tgt = np.array([400.0, 250.0])
    r = np.hypot(*(a - tgt).T) + rng.normal(0, 1, 10)
    ok, x, y, s = orc.ls_estimate(a[:, 0], a[:, 1], r, with_sens=True)
    assert ok and np.isfinite(s) and s > 0
    for _ in range(20):
        d = 1e-6
        da = rng.uniform(-d, d, size=a.shape)
        dr = rng.uniform(-d, d, size=r.shape)
        ok2, x2, y2 = orc.ls_estimate(a[:, 0] + da[:, 0], a[:, 1] + da[:, 1], r + dr)
        assert ok2 and np.hypot(x2 - x, y2 - y) <= 1.05 * s * d
