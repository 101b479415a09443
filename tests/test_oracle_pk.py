"""Pins for the oracle's power-spectrum estimator (Sec. 3, binned P^a_ell):
explicit all-images sums, exact expectations and variance for uniform
catalogues, the Thomas-process expectation, lattice shell sums, and
invariances."""
import itertools

import numpy as np
import pytest
from scipy import integrate
from scipy.special import eval_legendre

import oracle
import synthetic
from oracle import reference


def test_min_image_equals_all_images_sum():
    # (a) Tiny N: the minimum-image sum equals the explicit sum over every
    # periodic image inside R0 (R0 <= L/2 makes them the same set).
    L, r0 = 10.0, 5.0
    pos = synthetic.poisson(14, L, 11)
    w = synthetic.uniform_weights(14, 12, np.float64)
    k = np.array([0.3, 0.8, 1.5, 2.2])
    out = oracle.pk_ell(pos, w, L, r0, k, 4)
    S, npairs = reference.pk_all_images(pos, w, L, r0, k, 4)
    assert out["n_pairs"] == npairs
    assert np.allclose(out["raw"], S, rtol=1e-13, atol=1e-13 * np.abs(S).max())


def _moments(w):
    return [float(np.sum(w ** p)) for p in range(5)]


def _zeta2(ell, r0, k1, k2, V, wt):
    f = lambda r: r * r * oracle.window(r / r0) ** 2 * oracle.jbar(ell, r, k1, k2) ** 2
    pts = np.linspace(0, r0, 41)
    val = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11)[0] for a, b in zip(pts[:-1], pts[1:]))
    z = (2 * ell + 1) * 4 * np.pi * val / V
    if ell == 0:
        z -= (wt / V) ** 2
    return z


def test_poisson_null_mean_and_variance():
    # (b) Uniform points, fixed N and weights: E[P^a_0] = -(p2/p1^2) W~^a,
    # E[P^a_{l>0}] = 0, Var = 2 (p2^2 - p4) zeta2 / (n_w^2 V)^2 (a degenerate
    # U-statistic; no shot-noise term survives).  z-scores over 400 seeds.
    L, r0, N, T = 100.0, 30.0, 30, 400
    k = np.array([0.1, 0.2])
    w = synthetic.uniform_weights(N, 99, np.float64)
    p = _moments(w)
    V = L ** 3
    vals = []
    for t in range(T):
        pos = synthetic.poisson(N, L, 1000 + t)
        vals.append(oracle.pk_ell(pos, w, L, r0, k, 4, nthreads=1)["pk"][:, 0])
    vals = np.array(vals)
    wt = oracle.wtilde(r0, k[0], k[1])
    nw = p[1] / V
    for li, ell in enumerate((0, 2, 4)):
        mean_ex = -(p[2] / p[1] ** 2) * wt if ell == 0 else 0.0
        var_ex = 2 * (p[2] ** 2 - p[4]) * _zeta2(ell, r0, k[0], k[1], V, wt) / (nw ** 2 * V) ** 2
        m = vals[:, li].mean()
        z = (m - mean_ex) / np.sqrt(var_ex / T)
        assert abs(z) < 4.0, (ell, m, mean_ex, z)
        # sample variance within its own sampling error (chi-square, ~5 sigma)
        s2 = vals[:, li].var(ddof=1)
        assert abs(s2 / var_ex - 1) < 5 * np.sqrt(2.0 / (T - 1)) * 1.5, (ell, s2, var_ex)


def _thomas_expectation(ell, r0, k1, k2, sig, sigz, c, N, L):
    # E[P^a_ell] = (-i)^ell (c-1)/n (2 ell+1) int d^3r G(r) W jbar L_ell(mu) - (c/N) delta_l0 W~^a,
    # G = N(0, diag(2s^2, 2s^2, 2s^2 + 2 sz^2)) density (finite-N form of the
    # windowed-theory relation of Sec. 5 for this process).
    sx2, sz2 = 2 * sig ** 2, 2 * sig ** 2 + 2 * sigz ** 2
    norm = 1.0 / ((2 * np.pi) ** 1.5 * np.sqrt(sx2 * sx2 * sz2))

    def inner(r):
        g = lambda mu: np.exp(-r * r * (1 - mu * mu) / (2 * sx2) - r * r * mu * mu / (2 * sz2)) * eval_legendre(ell, mu)
        return 2 * np.pi * integrate.quad(g, -1, 1, epsabs=0, epsrel=1e-12)[0]

    f = lambda r: norm * r * r * oracle.window(r / r0) * oracle.jbar(ell, r, k1, k2) * inner(r)
    pts = np.linspace(0, r0, 31)
    I = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-10)[0] for a, b in zip(pts[:-1], pts[1:]))
    n = N / L ** 3
    ph = (-1) ** (ell // 2)
    val = ph * (c - 1) / n * (2 * ell + 1) * I
    if ell == 0:
        val -= c / N * oracle.wtilde(r0, k1, k2)
    return val


def test_thomas_expectation():
    # (c) Thomas cluster process with z displacement: the mean over seeds
    # converges to the closed-form expectation for ell = 0, 2, 4.
    L, r0, Np, c, sig, sigz, T = 100.0, 30.0, 20, 5, 2.0, 4.0, 600
    N = Np * c
    k = np.array([0.3, 0.5])
    vals = np.array([oracle.pk_ell(synthetic.thomas(N, L, c, sig, sigz, 5000 + t, np.float64),
                                   None, L, r0, k, 4, nthreads=1)["pk"][:, 0] for t in range(T)])
    for li, ell in enumerate((0, 2, 4)):
        ex = _thomas_expectation(ell, r0, k[0], k[1], sig, sigz, c, N, L)
        m, se = vals[:, li].mean(), vals[:, li].std(ddof=1) / np.sqrt(T)
        assert abs(m - ex) < 4 * se, (ell, m, ex, se)
        # and the signal is resolved: the expectation is many standard errors from 0
        assert abs(ex) > 10 * se


def test_translation_invariance_bitwise_on_dyadic_grid():
    # (d) Coordinates and shift on a common dyadic grid: every difference is
    # exact, so the result is bit-identical.
    L, r0 = 64.0, 16.0
    rng = np.random.default_rng(3)
    pos = rng.integers(0, 64 * 256, size=(300, 3)) / 256.0
    shift = np.array([5.25, 60.5, 33.125])
    k = np.linspace(0.2, 1.0, 6)
    a = oracle.pk_ell(pos, None, L, r0, k, 4, nthreads=1)
    b = oracle.pk_ell(np.mod(pos + shift, L), None, L, r0, k, 4, nthreads=1)
    assert a["n_pairs"] == b["n_pairs"]
    assert np.array_equal(a["raw"], b["raw"])


def test_translation_permutation_axis_invariance():
    L, r0 = 100.0, 25.0
    pos = synthetic.thomas(400, L, 10, 2.0, 3.0, 21, np.float64)
    w = synthetic.uniform_weights(400, 22, np.float64)
    k = np.geomspace(0.3, 3.0, 7)
    ref = oracle.pk_ell(pos, w, L, r0, k, 4)
    tol = dict(rtol=1e-12, atol=1e-12 * np.abs(ref["raw"]).max())
    moved = oracle.pk_ell(np.mod(pos + np.array([17.3, 81.1, 49.9]), L), w, L, r0, k, 4)
    assert np.allclose(moved["raw"], ref["raw"], **tol)
    perm = np.random.default_rng(1).permutation(400)
    permuted = oracle.pk_ell(pos[perm], w[perm], L, r0, k, 4)
    assert permuted["n_pairs"] == ref["n_pairs"]
    assert np.allclose(permuted["raw"], ref["raw"], **tol)
    # cyclic axis permutation with the line of sight carried along
    rolled = oracle.pk_ell(pos[:, [1, 2, 0]], w, L, r0, k, 4, los_axis=1)
    assert np.allclose(rolled["raw"], ref["raw"], **tol)


def test_lattice_shell_sums():
    # Cubic lattice, spacing a, M^3 points: every point sees the same shells,
    # so S = N sum_{0<|v|<R0} (2l+1)(-i)^l W jbar L_l(v_z/|v|), enumerated here
    # over integer vectors; P_2 vanishes by cubic symmetry.  R0/a = 4 puts
    # shells exactly on the window breakpoints r = R0/2 and 3R0/4.
    M, a = 10, 1.0
    L, r0 = M * a, 4.0
    g = np.arange(M) * a
    pos = np.array(list(itertools.product(g, g, g)), dtype=np.float64)
    N = len(pos)
    k = np.array([0.5, 1.0, 2.0, 3.5])
    out = oracle.pk_ell(pos, None, L, r0, k, 4)
    S = np.zeros((3, 3))
    cnt = 0
    R = int(np.ceil(r0 / a))
    for v in itertools.product(range(-R, R + 1), repeat=3):
        v = np.array(v, dtype=np.float64) * a
        r = np.sqrt(v @ v)
        if r == 0 or r >= r0:
            continue
        cnt += 1
        for li, ell in enumerate((0, 2, 4)):
            jb = np.array([oracle.jbar(ell, r, k[b], k[b + 1]) for b in range(3)])
            S[li] += (-1) ** li * (2 * ell + 1) * oracle.window(r / r0) * eval_legendre(ell, v[2] / r) * jb
    assert out["n_pairs"] == N * cnt
    assert np.allclose(out["raw"], N * S, rtol=1e-12, atol=1e-12 * np.abs(S).max() * N)
    assert np.all(np.abs(out["raw"][1]) < 1e-9 * np.abs(out["raw"][0]).max())


def test_primary_mask_is_additive():
    L, r0 = 100.0, 25.0
    pos = synthetic.thomas(300, L, 10, 2.0, 0.0, 31, np.float64)
    k = np.geomspace(0.5, 4.0, 6)
    full = oracle.pk_ell(pos, None, L, r0, k, 2)
    m = np.zeros(300, np.uint8)
    m[::3] = 1
    a = oracle.pk_ell(pos, None, L, r0, k, 2, primary_mask=m)
    b = oracle.pk_ell(pos, None, L, r0, k, 2, primary_mask=1 - m)
    assert a["n_pairs"] + b["n_pairs"] == full["n_pairs"]
    assert np.allclose(a["raw"] + b["raw"], full["raw"], rtol=1e-12, atol=1e-12 * np.abs(full["raw"]).max())


def test_coincident_points_and_empty():
    # Two distinct particles at one position: r = 0 enters with jbar_0(0) = 1,
    # W(0) = 1 and nothing for ell > 0; far-apart particles give nothing.
    L, r0 = 100.0, 20.0
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0], [60.0, 60.0, 60.0]])
    out = oracle.pk_ell(pos, None, L, r0, np.array([0.5, 1.0]), 4)
    assert out["n_pairs"] == 2
    assert out["raw"][0, 0] == pytest.approx(2.0, rel=1e-15)
    assert out["raw"][1, 0] == 0.0 and out["raw"][2, 0] == 0.0
