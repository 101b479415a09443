"""Pins for the oracle's theory side (Secs. 5 and 6): the spherical Bessel
function and Wigner 3j symbols against scipy and sympy; omega^a_l(p; R0)
against scipy's adaptive quadrature of its definition, its p -> 0 limit
(W~^a for l = 0) and Parseval's relation with the analytic-DDR^II kernel at
zero separation, int p^2 dp/(2 pi^2) omega^a omega^b = E^{II,ab}(0)
(Appendix A); the Gaussian covariance through that relation for a constant
power spectrum and through Q_ll' as a direct angular integral; the windowed
theory power spectrum against an independent evaluation."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import eval_legendre, spherical_jn
from sympy.physics.wigner import wigner_3j

import oracle

R0 = 20.0
K = np.linspace(0.1, 0.5, 4)


def test_spherical_bessel_and_wigner3j():
    for ell in range(7):
        for x in (1e-6, 0.1, 1.0, 3.0, 4.99, 5.0, 7.3, 20.0):
            ref = spherical_jn(ell, x)
            assert abs(oracle.sph_jl(ell, x) - ref) <= 1e-13 * max(abs(ref), 1e-300)
    for a in range(0, 8):
        for b in range(0, 8):
            for c in range(0, 15):
                assert abs(oracle.wigner3j_000(a, b, c) - float(wigner_3j(a, b, c, 0, 0, 0))) < 1e-14


@pytest.mark.parametrize("p,ell", [(0.05, 0), (0.33, 2), (0.9, 4), (2.5, 2)])
def test_omega_matches_adaptive_quadrature(p, ell):
    got = oracle.omega(p, R0, ell, K)
    for a in range(3):
        f = lambda r: r * r * spherical_jn(ell, p * r) * oracle.jbar(ell, r, K[a], K[a + 1]) * oracle.window(r / R0)
        ref = 4 * np.pi * integrate.quad(f, 0.0, R0, points=[0.5 * R0, 0.75 * R0], epsabs=0, epsrel=1e-12,
                                         limit=400)[0]
        assert abs(got[a] - ref) <= 1e-10 * np.abs(got).max()


def test_omega_at_zero_momentum():
    wt = np.array([oracle.wtilde(R0, K[a], K[a + 1]) for a in range(3)])
    assert np.allclose(oracle.omega(0.0, R0, 0, K), wt, rtol=1e-11, atol=0)
    for ell in (2, 4):
        assert np.all(oracle.omega(0.0, R0, ell, K) == 0.0)


def _p_quadrature(pmax, panels=150, n=16):
    gx, gw = np.polynomial.legendre.leggauss(n)
    e = np.linspace(0.0, pmax, panels + 1)
    mid, half = 0.5 * (e[:-1] + e[1:]), 0.5 * (e[1:] - e[:-1])
    return (mid[:, None] + half[:, None] * gx).ravel(), (half[:, None] * gw).ravel()


@pytest.mark.parametrize("ell", [0, 2])
def test_parseval_with_eii_at_zero(ell):
    # int_0^inf p^2 dp/(2 pi^2) omega^a omega^b = 4 pi int r^2 g^a g^b dr = E^{II,ab}(0)
    p, w = _p_quadrature(12.0)
    om = np.array([oracle.omega(pi, R0, ell, K) for pi in p])
    lhs = np.einsum("i,ia,ib->ab", w * p * p / (2 * np.pi ** 2), om, om)
    ref = oracle.eii(0.0, R0, ell, K)
    assert np.abs(lhs - ref).max() <= 1e-7 * np.abs(ref).max()


def test_covariance_constant_power_and_Q():
    V, ell_max = 1e6, 4
    # constant monopole P0, no higher multipoles: C = 2 (2l+1) P0^2 / V delta_ll' E^{II,ab}_l(0)
    p, w = _p_quadrature(12.0)
    P0 = 250.0
    pk = np.zeros((3, p.size))
    pk[0] = P0
    C = oracle.cov_gauss(R0, V, K, ell_max, p, w, pk)
    for li in range(3):
        ref = 2 * (4 * li + 1) * P0 ** 2 / V * oracle.eii(0.0, R0, 2 * li, K)
        assert np.abs(C[li, :, li, :] - ref).max() <= 1e-7 * np.abs(ref).max()
        for lj in range(3):
            if lj != li:
                assert np.abs(C[li, :, lj, :]).max() <= 1e-9 * np.abs(ref).max()
    # one p node: Q_ll'(p) = (1/2) int dmu L_l L_l' (sum_l1 P_l1 L_l1)^2
    pk1 = np.array([[300.0], [-80.0], [25.0]])
    p1 = 0.37
    C1 = oracle.cov_gauss(R0, V, K, ell_max, [p1], [1.0], pk1)
    om = [oracle.omega(p1, R0, 2 * li, K) for li in range(3)]
    mu, wmu = np.polynomial.legendre.leggauss(24)
    Pmu = sum(pk1[m, 0] * eval_legendre(2 * m, mu) for m in range(3))
    for li in range(3):
        for lj in range(3):
            Q = 0.5 * np.sum(wmu * eval_legendre(2 * li, mu) * eval_legendre(2 * lj, mu) * Pmu ** 2)
            ref = 2 * (4 * li + 1) * (4 * lj + 1) / V * p1 ** 2 / (2 * np.pi ** 2) * Q * np.outer(om[li], om[lj])
            assert np.allclose(C1[li, :, lj, :], ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_window_theory_independent_sum():
    # P^a_l = 4 pi (-i)^l sum_m w_m r_m^2 xi_l(r_m) W(r_m/R0) jbar^a_l(r_m), with
    # jbar and W from the pinned special functions, in plain numpy
    gx, gw = np.polynomial.legendre.leggauss(40)
    r, wr = 0.5 * R0 * (gx + 1), 0.5 * R0 * gw
    xi = np.array([5.0 * np.exp(-r / 7.0), -1.0 * np.exp(-r / 5.0) * r / 10.0, 0.1 * np.exp(-r / 9.0)])
    got = oracle.pk_window_theory(R0, K, 4, r, wr, xi)
    for li in range(3):
        ell = 2 * li
        for a in range(3):
            s = sum(wr[m] * r[m] ** 2 * xi[li, m] * oracle.window(r[m] / R0) * oracle.jbar(ell, r[m], K[a], K[a + 1])
                    for m in range(r.size))
            ref = 4 * np.pi * (-1) ** li * s
            assert abs(got[li, a] - ref) <= 1e-12 * abs(ref)


def _x_quadrature(r0, panels=24, n=16):
    gx, gw = np.polynomial.legendre.leggauss(n)
    cuts = [0.0, 0.5 * r0, 0.75 * r0, r0]
    xs, ws = [], []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        e = np.linspace(lo, hi, panels + 1)
        mid, half = 0.5 * (e[:-1] + e[1:]), 0.5 * (e[1:] - e[:-1])
        xs.append((mid[:, None] + half[:, None] * gx).ravel())
        ws.append((half[:, None] * gw).ravel())
    return np.concatenate(xs), np.concatenate(ws)


def test_poisson2_equals_exact_fixed_n_covariance():
    # xi = 0: for N unit-weight uniform points the estimator's exact covariance is
    #   2 (N^2 - N) / (n^2 V)^2 [delta_ll' (2l+1) 4 pi int r^2 W^2 jbar^a jbar^b dr / V
    #                            - delta_l0 delta_l'0 W~^a W~^b / V^2]
    # (the degenerate U-statistic whose variance the Poisson-null simulation pins),
    # so C2 = exact / (1 - 1/N) + 2 delta delta W~^a W~^b / (n^2 V^2)
    N, L = 500, 200.0
    V, nbar = L ** 3, 500 / 200.0 ** 3
    x, w = _x_quadrature(R0)
    C2 = oracle.cov_poisson2(R0, nbar, V, K, 4, x, w, np.zeros((3, x.size)))
    wt = np.array([oracle.wtilde(R0, K[a], K[a + 1]) for a in range(3)])
    for li in range(3):
        ell = 2 * li
        I = np.array([[np.sum(w * x * x * np.array([oracle.window(xx / R0) ** 2 * oracle.jbar(ell, xx, K[a], K[a + 1])
                                                      * oracle.jbar(ell, xx, K[b], K[b + 1]) for xx in x]))
                       for b in range(3)] for a in range(3)])
        zeta = (2 * ell + 1) * 4 * np.pi * I / V
        if ell == 0:
            zeta = zeta - np.outer(wt, wt) / V ** 2
        exact = 2 * (N * N - N) / (nbar * nbar * V) ** 2 * zeta
        ref = exact / (1 - 1 / N) + (2 * np.outer(wt, wt) / (nbar ** 2 * V ** 2) if ell == 0 else 0.0)
        assert np.allclose(C2[li, :, li, :], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
        for lj in range(3):
            if lj != li:
                assert np.all(C2[li, :, lj, :] == 0.0)


def test_poisson2_xi_term_is_the_angular_average():
    # the xi part: (1/2) int dmu L_l L_l' xi(x, mu) = sum_L (L l l'; 000)^2 xi_L(x)
    x, w = _x_quadrature(R0, panels=4)
    xi = np.array([3.0 * np.exp(-x / 6.0), -0.8 * np.exp(-x / 4.0), 0.2 * np.exp(-x / 3.0)])
    nbar, V = 1e-3, 1e6
    C0 = oracle.cov_poisson2(R0, nbar, V, K, 4, x, w, np.zeros_like(xi))
    C = oracle.cov_poisson2(R0, nbar, V, K, 4, x, w, xi) - C0
    mu, wmu = np.polynomial.legendre.leggauss(24)
    for li in range(3):
        for lj in range(3):
            ang = np.array([0.5 * np.sum(wmu * eval_legendre(2 * li, mu) * eval_legendre(2 * lj, mu)
                                         * sum(xi[L, m] * eval_legendre(2 * L, mu) for L in range(3)))
                            for m in range(x.size)])
            g = lambda ell: np.array([[oracle.window(xx / R0) * oracle.jbar(ell, xx, K[a], K[a + 1]) for a in range(3)]
                                      for xx in x])
            ga, gb = g(2 * li), g(2 * lj)
            ref = (2 / (nbar ** 2 * V) * (4 * li + 1) * (4 * lj + 1) * (-1) ** (li + lj) * 4 * np.pi
                   * np.einsum("m,ma,mb->ab", w * x * x * ang, ga, gb))
            assert np.allclose(C[li, :, lj, :], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def _poisson_moments(lam):
    # E[N(N-1)] and Var[N(N-1)] summed from the Poisson distribution itself
    from scipy.stats import poisson
    n = np.arange(0, int(lam + 40 * np.sqrt(lam) + 50))
    pmf = poisson.pmf(n, lam)
    pmf = pmf / np.sum(pmf)
    f = n * (n - 1.0)
    m1 = np.sum(pmf * f)
    return m1, np.sum(pmf * (f - m1) ** 2)


def test_poisson_terms_give_exact_variance_of_poisson_catalogue():
    # xi = 0, N ~ Poisson(nV): by the law of total covariance the estimator's
    # covariance is E_N[2 N(N-1)] zeta / (n^2 V)^2 + Var_N[N(N-1)] W~^a W~^b
    # d_l0 d_l'0 / (n^2 V^2)^2, with zeta the per-pair covariance of the
    # fixed-N U-statistic; 2C + 3C must equal it exactly
    L, nbar = 150.0, 0.1
    V = L ** 3
    lam = nbar * V
    x, w = _x_quadrature(R0)
    p, wp = _p_quadrature(12.0, panels=40)
    C2 = oracle.cov_poisson2(R0, nbar, V, K, 4, x, w, np.zeros((3, x.size)))
    C3 = oracle.cov_poisson3(R0, nbar, V, K, 4, p, wp, np.zeros((3, p.size)))
    m1, var = _poisson_moments(lam)
    wt = np.array([oracle.wtilde(R0, K[a], K[a + 1]) for a in range(3)])
    for li in range(3):
        ell = 2 * li
        I = np.array([[np.sum(w * x * x * np.array([oracle.window(xx / R0) ** 2 * oracle.jbar(ell, xx, K[a], K[a + 1])
                                                      * oracle.jbar(ell, xx, K[b], K[b + 1]) for xx in x]))
                       for b in range(3)] for a in range(3)])
        zeta = (2 * ell + 1) * 4 * np.pi * I / V
        if ell == 0:
            zeta = zeta - np.outer(wt, wt) / V ** 2
        ref = 2 * m1 * zeta / (nbar * nbar * V) ** 2
        if ell == 0:
            ref = ref + var * np.outer(wt, wt) / (nbar * nbar * V * V) ** 2
        got = C2[li, :, li, :] + C3[li, :, li, :]
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
        for lj in range(3):
            if lj != li:
                assert np.all(C2[li, :, lj, :] + C3[li, :, lj, :] == 0.0)


def test_poisson3_constant_power_and_single_node():
    V, nbar = 1e6, 2e-3
    f0 = 4 / (nbar * V)
    wt = np.array([oracle.wtilde(R0, K[a], K[a + 1]) for a in range(3)])
    # constant monopole P0: the P_L part is f0 (2l+1) P0 E^{II,ab}_l(0) delta_ll' (Parseval)
    p, w = _p_quadrature(12.0)
    P0 = 250.0
    pk = np.zeros((3, p.size))
    pk[0] = P0
    C = oracle.cov_poisson3(R0, nbar, V, K, 4, p, w, pk)
    for li in range(3):
        ref = f0 * (4 * li + 1) * P0 * oracle.eii(0.0, R0, 2 * li, K)
        if li == 0:
            ref = ref + f0 * np.outer(wt, wt)
        assert np.abs(C[li, :, li, :] - ref).max() <= 1e-7 * np.abs(ref).max()
        for lj in range(3):
            if lj != li:
                assert np.abs(C[li, :, lj, :]).max() <= 1e-9 * np.abs(ref).max()
    # one p node: (1/2) int dmu L_l L_l' P(p, mu) by direct angular quadrature
    pk1 = np.array([[300.0], [-80.0], [25.0]])
    p1 = 0.37
    C1 = oracle.cov_poisson3(R0, nbar, V, K, 4, [p1], [1.0], pk1)
    om = [oracle.omega(p1, R0, 2 * li, K) for li in range(3)]
    mu, wmu = np.polynomial.legendre.leggauss(24)
    Pmu = sum(pk1[m, 0] * eval_legendre(2 * m, mu) for m in range(3))
    for li in range(3):
        for lj in range(3):
            ang = 0.5 * np.sum(wmu * eval_legendre(2 * li, mu) * eval_legendre(2 * lj, mu) * Pmu)
            ref = f0 * (4 * li + 1) * (4 * lj + 1) * p1 ** 2 / (2 * np.pi ** 2) * ang * np.outer(om[li], om[lj])
            if li == 0 and lj == 0:
                ref = ref + f0 * np.outer(wt, wt)
            assert np.allclose(C1[li, :, lj, :], ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_poisson3_mean_fluctuation_terms():
    # a catalogue whose conditional mean given N is N(N-1)/(nV)^2 (P^a_l + W~^a
    # d_l0) - W~^a d_l0 gets, from Poisson fluctuations of N, the covariance
    # Var_N[N(N-1)]/(nV)^4 (P^a_l + W~^a d_l0)(P^b_l' + W~^b d_l'0), whose
    # 1/(nV) part is 4/(nV) times that product less P^a P^b: the first three
    # 3C terms.  The B term only enters symmetrically.
    V, nbar = 1e5, 1e-2
    lam = nbar * V
    rng = np.random.default_rng(3)
    pbin = rng.normal(size=(3, 3)) * 50.0
    B = rng.normal(size=(3, 3, 3)) * 1e3
    B = B + B.transpose(0, 2, 1)
    p, w = np.array([0.2]), np.array([0.0])  # the P_L part is zero here
    C = oracle.cov_poisson3(R0, nbar, V, K, 4, p, w, np.zeros((3, 1)), pbin=pbin)
    wt = np.array([oracle.wtilde(R0, K[a], K[a + 1]) for a in range(3)])
    m = pbin.copy()
    m[0] += wt
    _, var = _poisson_moments(lam)
    lead = (var / lam ** 4 - 2 / lam ** 2)  # the 1/(nV) coefficient times 1/(nV)
    assert abs(lead * lam - 4.0) < 1e-8
    for li in range(3):
        for lj in range(3):
            ref = lead * (np.outer(m[li], m[lj]) - np.outer(pbin[li], pbin[lj]))
            assert np.allclose(C[li, :, lj, :], ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max() + 1e-300)
    CB = oracle.cov_poisson3(R0, nbar, V, K, 4, p, w, np.zeros((3, 1)), pbin=pbin, bk=B)
    T = CB.transpose(2, 3, 0, 1)
    assert np.allclose(CB, T, rtol=1e-14, atol=0)
    assert not np.allclose(CB, C)


def test_nongauss_reduces_to_gaussian_for_diagonal_trispectrum():
    # with T_ll'(p_i, p_j) = delta_ij 2 Q_ll'(p_i) / u_i, u_i = w_i p_i^2/(2 pi^2),
    # the double sum collapses onto the single sum of the Gaussian term:
    # 4C^NG = 2 (2l+1)(2l'+1)/V sum_i u_i Q_ll'(p_i) omega omega = 4C^G, with
    # Q_ll' the direct angular integral (1/2) int dmu L_l L_l' P(p, mu)^2
    V = 1e6
    p, w = _p_quadrature(4.0, panels=6, n=8)
    pk = np.array([300.0 / (1 + (p / 0.2) ** 2), -80.0 / (1 + (p / 0.3) ** 2), 25.0 / (1 + (p / 0.4) ** 2)])
    mu, wmu = np.polynomial.legendre.leggauss(24)
    Pmu = sum(pk[m][:, None] * eval_legendre(2 * m, mu)[None, :] for m in range(3))  # [n_p, n_mu]
    u = w * p * p / (2 * np.pi ** 2)
    T = np.zeros((3, 3, p.size, p.size))
    for li in range(3):
        for lj in range(3):
            Q = 0.5 * np.sum(wmu * eval_legendre(2 * li, mu) * eval_legendre(2 * lj, mu) * Pmu ** 2, axis=1)
            T[li, lj] = np.diag(2.0 * Q / u)
    ng = oracle.cov_nongauss(R0, V, K, 4, p, w, T)
    g = oracle.cov_gauss(R0, V, K, 4, p, w, pk)
    assert np.allclose(ng, g, rtol=1e-11, atol=1e-13 * np.abs(g).max())


def test_nongauss_symmetry_and_separable_trispectrum():
    # T_ll'(p1, p2) = T_l'l(p2, p1) makes C^ab_ll' = C^ba_l'l; a separable
    # T_ll' = f_l(p1) f_l'(p2) factorises the double sum into two single sums
    V = 5e5
    p, w = _p_quadrature(3.0, panels=4, n=8)
    f = np.array([np.exp(-p), 0.5 * p * np.exp(-p / 2), 0.1 / (1 + p * p)])
    T = np.einsum("li,mj->lmij", f, f)
    C = oracle.cov_nongauss(R0, V, K, 4, p, w, T)
    assert np.allclose(C, C.transpose(2, 3, 0, 1), rtol=1e-12, atol=0)
    u = w * p * p / (2 * np.pi ** 2)
    om = np.array([[oracle.omega(pi, R0, 2 * li, K) for pi in p] for li in range(3)])  # [l, i, a]
    v = np.einsum("i,li,lia->la", u, f, om)
    for li in range(3):
        for lj in range(3):
            ref = (4 * li + 1) * (4 * lj + 1) / V * np.outer(v[li], v[lj])
            assert np.allclose(C[li, :, lj, :], ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())
