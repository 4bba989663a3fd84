"""Pins of the oracle's particle-filter tracker (bootstrap filter: seed on the
first range's ring, random-walk move, Gaussian range likelihood, systematic
resampling; Sec. II names the method, the reading is the oracle's).

Each check rests on something other than the oracle's own code: a closed
form of the resampling decision with two particles, the offspring-count
property and unbiasedness of systematic resampling (Kitagawa 1996; Douc and
Cappe 2005), the geometry of the seeding ring, translation equivariance, and
convergence on a static target from exact ranges.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_08222_amd import configs


def words_with_u(n, u3=None, seed=5):
    """Random inputs of one update for n particles; the resampling offset's
    word set so that U = u3 (the grid point nearest to it)."""
    rng = np.random.default_rng(seed)
    zw = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    uw = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    uoff = int(rng.integers(0, 2**32, dtype=np.uint64))
    if u3 is not None:
        uoff = min(int(u3 * 2**23), 2**23 - 1) << 9
    return orc.PfWords(zw, uw, uoff)


@pytest.mark.parametrize("delta,sigma", [(3.0, 2.0), (1.0, 1.5), (6.0, 5.0)])
def test_two_particle_resampling_closed_form(delta, sigma):
    """Two particles, one range: particle a on the measured ring, particle b
    off it by delta. With weights 1 and w = exp(-delta^2 / (2 sigma^2)) and
    offset U, systematic resampling gives output 0 <- a always and output
    1 <- a exactly when (1 + U)(1 + w) / 2 < 1, i.e. U < (1 - w) / (1 + w)."""
    w = math.exp(-delta * delta / (2 * sigma * sigma))
    thr = (1 - w) / (1 + w)
    rows = [[0.0, 0.0, 100.0]]
    for U in (0.5 * thr, min(0.999, thr + 0.5 * (1 - thr)), 0.02, 0.98):
        if abs(U - thr) < 1e-3:
            continue
        wd = words_with_u(2, U)
        Ue = orc.u01(wd.uoff)
        ok, px, py, est, src = orc.pf_update([100.0, 100.0 + delta], [0.0, 0.0], True, rows,
                                             sigma, 0.0, wd)
        assert ok
        assert src[0] == 0
        assert src[1] == (0 if Ue < thr else 1), (U, thr)
        # the same with the particles swapped: a is now index 1
        ok, px, py, est, src = orc.pf_update([100.0 + delta, 100.0], [0.0, 0.0], True, rows,
                                             sigma, 0.0, wd)
        # output 0 <- b iff U (1 + w) / 2 < w; output 1 <- a always
        assert src[0] == (0 if Ue * (1 + w) / 2 < w else 1)
        assert src[1] == 1


def test_likelihood_uses_sigma_squared_over_two():
    """A factor-2 slip in the exponent would move the decision threshold; the
    two sides of the true threshold are resolved exactly."""
    sigma, delta = 2.0, 2.0
    w = math.exp(-0.5)
    thr = (1 - w) / (1 + w)  # 0.2449
    wrong = (1 - math.exp(-1.0)) / (1 + math.exp(-1.0))  # 0.4621
    rows = [[0.0, 0.0, 50.0]]
    U = 0.5 * (thr + wrong)  # between the two readings
    wd = words_with_u(2, U)
    _, _, _, _, src = orc.pf_update([50.0, 50.0 + delta], [0.0, 0.0], True, rows, sigma, 0.0, wd)
    assert src[1] == 1  # U > true threshold: the off-ring particle survives


def test_offspring_counts_bracket_expected_and_are_unbiased():
    """Systematic resampling copies particle m either floor(n p_m) or
    ceil(n p_m) times (p_m its normalised weight), in index order, and the
    copies average exactly n p_m over a uniform offset."""
    rng = np.random.default_rng(11)
    n = 64
    px = rng.normal(0.0, 30.0, n) + 80.0
    py = rng.normal(0.0, 30.0, n)
    rows = [[0.0, 0.0, 90.0], [20.0, -10.0, 75.0]]
    sig = 12.0
    # normalised weights from the Gaussian range likelihood (brute force)
    lw = np.zeros(n)
    for ax, ay, r in rows:
        lw -= (np.hypot(px - ax, py - ay) - r) ** 2 / (2 * sig * sig)
    p = np.exp(lw - lw.max())
    p /= p.sum()
    G = 512
    mean_counts = np.zeros(n)
    for g in range(G):
        wd = words_with_u(n, (g + 0.5) / G, seed=g)
        ok, qx, qy, est, src = orc.pf_update(px, py, True, rows, sig, 0.0, wd)
        assert ok
        assert np.all(np.diff(src) >= 0)
        counts = np.bincount(src, minlength=n)
        assert counts.sum() == n
        lo = np.floor(n * p - 1e-9)
        hi = np.ceil(n * p + 1e-9)
        assert np.all(counts >= lo) and np.all(counts <= hi)
        np.testing.assert_array_equal(qx, px[src])
        np.testing.assert_array_equal(qy, py[src])
        assert est[0] == pytest.approx(qx.mean(), abs=1e-12)
        mean_counts += counts
    mean_counts /= G
    # midpoint rule over U: exact up to the grid's resolution
    np.testing.assert_allclose(mean_counts, n * p, atol=2.0 / G + 1e-9)


def test_seed_ring_geometry():
    """No belief and one range: particle k sits on the ring about the agent at
    radius r + sigma z_k, inside the k-th of n equal sectors, and no
    resampling happens."""
    n = 64
    wd = words_with_u(n, seed=3)
    a = (120.0, -40.0)
    r, sig = 150.0, 4.0
    ok, px, py, est, src = orc.pf_update(np.zeros(n), np.zeros(n), False, [[a[0], a[1], r]], sig,
                                         7.0, wd)
    assert ok and np.all(src == -1)
    ang = np.mod(np.arctan2(py - a[1], px - a[0]), 2 * np.pi)
    k = np.arange(n)
    assert np.all(ang >= 2 * np.pi * k / n - 1e-12) and np.all(ang < 2 * np.pi * (k + 1) / n + 1e-12)
    for kk in range(n):
        z0, _ = orc.normal2(int(wd.zw[kk, 0]), int(wd.zw[kk, 1]))
        assert math.hypot(px[kk] - a[0], py[kk] - a[1]) == pytest.approx(abs(r + sig * z0), rel=1e-12)
    # a ring's mean is near its centre
    assert math.hypot(est[0] - a[0], est[1] - a[1]) < 0.2 * r


def test_no_belief_no_row_and_predict_only():
    n = 8
    wd = words_with_u(n, 0.3)
    px0 = np.arange(n, dtype=float)
    py0 = -np.arange(n, dtype=float)
    ok, px, py, est, src = orc.pf_update(px0, py0, False, np.zeros((0, 3)), 2.0, 1.0, wd)
    assert not ok
    np.testing.assert_array_equal(px, px0)
    # belief held, no row: the random walk only, q (z0, z1) per particle
    q = 2.5
    ok, px, py, est, src = orc.pf_update(px0, py0, True, np.zeros((0, 3)), 2.0, q, wd)
    assert ok and np.all(src == -1)
    for k in range(n):
        z0, z1 = orc.normal2(int(wd.zw[k, 0]), int(wd.zw[k, 1]))
        assert px[k] == pytest.approx(px0[k] + q * z0, abs=1e-12)
        assert py[k] == pytest.approx(py0[k] + q * z1, abs=1e-12)
    assert est == pytest.approx((px.mean(), py.mean()), abs=1e-12)


def test_translation_equivariance():
    rng = np.random.default_rng(2)
    n = 64
    px = rng.normal(200.0, 40.0, n)
    py = rng.normal(-100.0, 40.0, n)
    rows = np.array([[10.0, 5.0, 230.0], [-30.0, 12.0, 260.0]])
    wd = words_with_u(n, 0.61)
    sh = np.array([1234.5, -678.25])
    r0 = orc.pf_update(px, py, True, rows, 6.0, 3.0, wd)
    rows2 = rows.copy()
    rows2[:, :2] += sh
    r1 = orc.pf_update(px + sh[0], py + sh[1], True, rows2, 6.0, 3.0, wd)
    np.testing.assert_array_equal(r0[4], r1[4])
    np.testing.assert_allclose(r1[1], r0[1] + sh[0], atol=1e-9)
    np.testing.assert_allclose(r1[2], r0[2] + sh[1], atol=1e-9)


@pytest.mark.parametrize("n_agents", [1, 3])
def test_converges_on_static_target(n_agents):
    """Exact ranges from agents circling a point 60 m from a static target:
    the filter's mean settles within 2 m of the target."""
    n = 64
    target = np.array([40.0, -25.0])
    px, py = np.zeros(n), np.zeros(n)
    init = False
    for t in range(150):
        rows = []
        for a in range(n_agents):
            ang = 0.1 * t + 2 * np.pi * a / n_agents
            ax, ay = target[0] + 60.0 + 50.0 * np.cos(ang), target[1] + 50.0 * np.sin(ang)
            rows.append([ax, ay, math.hypot(ax - target[0], ay - target[1])])
        wd = orc.pf_words(9, 0, t, 4, 1, 2)
        ok, px, py, est, _ = orc.pf_update(px, py, init, rows, 2.0, 0.5, wd)
        init = init or ok
    assert math.hypot(est[0] - target[0], est[1] - target[1]) < 2.0


def test_rollout_words_and_rows():
    """The rollout's filter equals orc_pf_update driven by the documented
    counter words and rows (one agent: the own range of each step)."""
    cfg = configs.env_config("plain", est_kind=1, pf_q=1.0, pf_lik_sigma=2.0, episode_len=30)
    seed, T = 3, 30
    ids = np.array([7])
    r = orc.rollout(cfg, ids, [1], [1], seed, T, records=("agent", "ranges", "est", "est_valid",
                                                          "sigma_r"))
    sl = math.sqrt(r["sigma_r"][0] ** 2 + 4.0)
    px, py = np.zeros(64), np.zeros(64)
    init = False
    for t in range(T):
        a = r["agent"][t, 0]
        rows = [[a[0], a[1], r["ranges"][t, 0]]]
        wd = orc.pf_words(seed, 0, t, 7, 0, 0)
        ok, px, py, est, _ = orc.pf_update(px, py, init, rows, sl, 1.0, wd)
        init = init or ok
        assert r["est_valid"][t, 0] == 1
        np.testing.assert_allclose(r["est"][t, 0], est, rtol=0, atol=1e-9)


def test_pf_tracks_moving_targets_better_than_window_ls():
    """The paper's motivation for the filter: least squares over a window
    assumes a still target and degrades when targets move, the filter keeps
    tracking. Agents circle (rudder held at its largest angle) among targets
    moving at half their speed, 30 s steps."""
    T, E = 40, 64
    out = {}
    for kind in (0, 1):
        cfg = configs.env_config("paper", est_kind=kind, episode_len=T, pf_q=15.0,
                                 pf_lik_sigma=5.0, det_range=math.inf)
        ids = np.arange(E)
        na, nt = orc.env_counts(cfg, 0, ids)
        acts = np.full((T, int(na.sum())), 2, np.int32)
        r = orc.rollout(cfg, ids, na, nt, 0, T, actions=acts, records=("err",), n_threads=4)
        e = r["err"][10:]
        out[kind] = np.median(e[np.isfinite(e)])
    assert out[1] < 0.7 * out[0], out
