"""Pins of the survey-geometry power-spectrum oracle (Sec. 2 general estimator
with the binned kernels of Sec. 3; no periodicity, observer at the origin,
pair-midpoint line of sight).  Each test fixes the oracle against something
other than itself: the periodic oracle (pinned in test_oracle_pk.py) in cases
where the two estimators reduce to the same pair sum, exact identities of the
DD - 2DR + RR combination, and invariances."""
import numpy as np
import pytest

import oracle

K = np.linspace(0.2, 2.0, 7)


def _rel(a, b, scale):
    return np.max(np.abs(a - b) / np.maximum(scale, 1e-300))


def _ring(n, rho, plane, seed, z0=0.0):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2 * np.pi, n)
    c, s = rho * np.cos(t), rho * np.sin(t)
    if plane == "xy":
        return np.stack([c, s, np.full(n, z0)], axis=1)
    return np.stack([c, np.full(n, z0), s], axis=1)  # "xz"


@pytest.mark.parametrize("plane,los", [("xy", 2), ("xz", 1)])
def test_ring_about_observer_has_zero_mu_like_fixed_los(plane, los):
    # Points on a circle centred on the observer are equidistant from it, so
    # every pair's separation is perpendicular to its midpoint: mu = 0.  The
    # periodic estimator with the line of sight normal to the circle's plane
    # also has mu = 0 for every pair, and sums the same pairs (the box is far
    # larger than the ring, so the minimum image is the plain difference).
    # An endpoint line of sight (mu = r / 2 rho) or a fixed axis inside the
    # plane would break the equality for l = 2, 4.
    pos = _ring(240, 30.0, plane, 1)
    rnd = _ring(5, 30.0, plane, 2)
    s = oracle.pk_survey(pos, None, rnd, None, 1e6, 15.0, K, 4)
    L = 1000.0
    per = oracle.pk_ell(pos + L / 2, None, L, 15.0, K, 4, los_axis=los)
    assert s["n_dd"] == per["n_pairs"]
    assert _rel(s["raw_dd"], per["raw"], per["l1"]) < 1e-13


def test_far_observer_limit_is_fixed_line_of_sight():
    # As the observer recedes along z the midpoint direction tends to z and
    # the estimator's DD sum tends to the periodic one with a z line of sight;
    # at distance 1e12 the difference is O(extent / distance) ~ 1e-10.
    rng = np.random.default_rng(3)
    D = 1.0e12
    local = rng.uniform(-40.0, 40.0, (400, 3))
    pos = local + np.array([0.0, 0.0, D])
    rnd = rng.uniform(-40.0, 40.0, (10, 3)) + np.array([0.0, 0.0, D])
    s = oracle.pk_survey(pos, None, rnd, None, 1e6, 20.0, K, 4)
    L = 1000.0
    back = (pos - np.array([0.0, 0.0, D])) + L / 2  # exact: recovers the local offsets
    per = oracle.pk_ell(back, None, L, 20.0, K, 4, los_axis=2)
    assert s["n_dd"] == per["n_pairs"]
    assert _rel(s["raw_dd"], per["raw"], per["l1"]) < 1e-8


def test_monopole_does_not_see_the_line_of_sight():
    # L_0 = 1: the l = 0 DD sum is the periodic pair sum of the same pairs for
    # any observer position.
    rng = np.random.default_rng(4)
    pos = rng.uniform(0.0, 120.0, (500, 3)) + np.array([10.0, -30.0, 60.0])
    rnd = rng.uniform(0.0, 120.0, (10, 3))
    w = rng.uniform(0.5, 1.5, 500)
    s = oracle.pk_survey(pos, w, rnd, None, 1e6, 25.0, K, 4)
    L = 2000.0
    per = oracle.pk_ell(pos + L / 2, w, L, 25.0, K, 4, los_axis=0)
    assert _rel(s["raw_dd"][0], per["raw"][0], per["l1"][0]) < 1e-13


def test_rotation_about_observer():
    rng = np.random.default_rng(5)
    pos = rng.uniform(-60.0, 60.0, (400, 3)) + np.array([0.0, 80.0, 40.0])
    rnd = rng.uniform(-60.0, 60.0, (1200, 3)) + np.array([0.0, 80.0, 40.0])
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    a = oracle.pk_survey(pos, None, rnd, None, 1e6, 20.0, K, 4)
    b = oracle.pk_survey(pos @ q.T, None, rnd @ q.T, None, 1e6, 20.0, K, 4)
    assert (a["n_dd"], a["n_dr"], a["n_rr"]) == (b["n_dd"], b["n_dr"], b["n_rr"])
    assert _rel(a["raw_dd"] - a["raw_dr"] + a["raw_rr"], b["raw_dd"] - b["raw_dr"] + b["raw_rr"], a["l1"]) < 1e-12


@pytest.mark.parametrize("masked", [False, True])
def test_randoms_equal_to_data_leave_only_the_coincident_terms(masked):
    # With the randoms a copy of the data (s_R = 1): RR = DD, and DR + RD =
    # 2 DD + 2 sum_i w_i^2 K(0), the i = j pairs at r = 0 that DR (distinct
    # catalogues) includes.  K^a_0(0) = 1 in every bin and K^a_{l>0}(0) = 0,
    # so DD - (DR + RD) + RR = -2 sum w^2 for l = 0 and 0 for l > 0.  With the
    # same mask on both, the sum runs over the masked points.
    rng = np.random.default_rng(6)
    pos = rng.uniform(-50.0, 50.0, (300, 3)) + np.array([0.0, 0.0, 150.0])
    w = rng.uniform(0.5, 1.5, 300)
    mask = (np.arange(300) % 3 == 0).astype(np.uint8) if masked else None
    s = oracle.pk_survey(pos, w, pos.copy(), w.copy(), 1e6, 20.0, K, 4, mask_d=mask, mask_r=mask)
    combo = s["raw_dd"] - s["raw_dr"] + s["raw_rr"]
    sw2 = np.sum(w ** 2 if mask is None else w[mask == 1] ** 2)
    expect = np.zeros_like(combo)
    expect[0, :] = -2.0 * sw2
    assert np.max(np.abs(combo - expect)) <= 1e-12 * np.max(s["l1"])


def test_masks_partition_the_ordered_pairs():
    # The subset hook: complementary masks split every ordered pair sum.
    rng = np.random.default_rng(7)
    pos = rng.uniform(-40.0, 40.0, (250, 3)) + np.array([20.0, 0.0, 100.0])
    rnd = rng.uniform(-40.0, 40.0, (750, 3)) + np.array([20.0, 0.0, 100.0])
    md = (rng.uniform(size=250) < 0.4).astype(np.uint8)
    mr = (rng.uniform(size=750) < 0.6).astype(np.uint8)
    full = oracle.pk_survey(pos, None, rnd, None, 1e6, 20.0, K, 4)
    a = oracle.pk_survey(pos, None, rnd, None, 1e6, 20.0, K, 4, mask_d=md, mask_r=mr)
    b = oracle.pk_survey(pos, None, rnd, None, 1e6, 20.0, K, 4, mask_d=1 - md, mask_r=1 - mr)
    for key in ("n_dd", "n_dr", "n_rr"):
        assert a[key] + b[key] == full[key]
    for key in ("raw_dd", "raw_dr", "raw_rr"):
        assert _rel(a[key] + b[key], full[key], full["l1"]) < 1e-13
