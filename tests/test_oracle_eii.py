"""Pins for the oracle's analytic DDR^II term (Sec. 4, eq. EII-intro;
Appendices A and B): the kernel E^{II,ab}_l(x) from the 2-D band integral is
checked against (a) the 3-D definition integrated in cylindrical coordinates
by scipy's adaptive quadrature (no use of the triple-Bessel identity), (b) its
exact volume integral, 4 pi int x^2 E dx = delta_l0 W~^a W~^b (the x3 and x_j
integrals of the two windows factorise), (c) its x -> 0 limit, (d) symmetry
and support; the pair sum over the interpolated table is checked against the
random-primary DDR^II of the bispectrum oracle with the randoms on a fine
lattice (a Riemann sum of the same x3 integral), against per-pair kernel
values, and through the exact expectation of the assembled estimator for
uniform catalogues."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import eval_legendre

import oracle
import synthetic

R0 = 20.0
K = np.linspace(0.1, 0.5, 4)


def _g(ell, r, a, k=K, r0=R0):
    return oracle.jbar(ell, r, k[a], k[a + 1]) * oracle.window(r / r0)


def _cylindrical(x, ell, a, b):
    """E^{II,ab}_l(x) = int d^3x3 g^a(|x_i - x3|) g^b(|x_j - x3|) L_l(cos gamma)
    with x_i at the origin and x_j at (0, 0, x), in (rho, z) coordinates."""
    def f(rho, z):
        r1, r2 = np.hypot(rho, z), np.hypot(rho, z - x)
        if r1 >= R0 or r2 >= R0:
            return 0.0
        c = (rho * rho + z * z - x * z) / (r1 * r2) if r1 > 0 and r2 > 0 else 1.0
        return 2 * np.pi * rho * _g(ell, r1, a) * _g(ell, r2, b) * eval_legendre(ell, min(1.0, max(-1.0, c)))

    top = lambda z: np.sqrt(max(0.0, min(R0 * R0 - z * z, R0 * R0 - (z - x) ** 2)))
    v, err = integrate.dblquad(f, x - R0, R0, lambda z: 0.0, top, epsabs=1e-9, epsrel=1e-10)
    return v, err


@pytest.mark.parametrize("x,ell,a,b", [(7.0, 0, 0, 1), (7.0, 2, 1, 2), (27.0, 1, 2, 0), (13.0, 3, 1, 1)])
def test_kernel_matches_cylindrical_definition(x, ell, a, b):
    ref, err = _cylindrical(x, ell, a, b)
    got = oracle.eii(x, R0, ell, K)[a, b]
    assert abs(got - ref) <= 1e-8 * abs(ref) + 10 * err


@pytest.mark.parametrize("ell", [0, 1, 2, 3])
def test_kernel_volume_integral(ell):
    # int d^3x E^{II,ab}_l(|x|) = [int d^3r g^a_l Y] [int d^3r g^b_l Y] -> W~^a W~^b for l = 0, else 0
    gx, gw = np.polynomial.legendre.leggauss(12)
    edges = np.linspace(0.0, 2 * R0, 17)
    tot = np.zeros((3, 3))
    for lo, hi in zip(edges[:-1], edges[1:]):
        for xq, wq in zip(gx, gw):
            x = 0.5 * (lo + hi) + 0.5 * (hi - lo) * xq
            tot += 0.5 * (hi - lo) * wq * 4 * np.pi * x * x * oracle.eii(x, R0, ell, K)
    wt = np.array([oracle.wtilde(R0, K[i], K[i + 1]) for i in range(3)])
    ref = np.outer(wt, wt) if ell == 0 else np.zeros((3, 3))
    assert np.abs(tot - ref).max() <= 1e-12 * np.abs(np.outer(wt, wt)).max()


def test_kernel_limit_at_zero():
    for ell in (0, 2):
        lim = oracle.eii(0.0, R0, ell, K)
        for a in range(3):
            for b in range(3):
                ref = 4 * np.pi * integrate.quad(lambda r: r * r * _g(ell, r, a) * _g(ell, r, b), 0.0, R0,
                                                 points=[0.5 * R0, 0.75 * R0], epsabs=0, epsrel=1e-12, limit=200)[0]
                assert abs(lim[a, b] - ref) <= 1e-11 * np.abs(lim).max()
        # the band integral runs continuously into the limit (E is even in x: O(x^2))
        near = oracle.eii(1e-4, R0, ell, K)
        assert np.abs(near - lim).max() <= 1e-8 * np.abs(lim).max()


def test_kernel_symmetry_and_support():
    for x in (3.0, 19.0, 33.0):
        for ell in (0, 1, 4):
            e = oracle.eii(x, R0, ell, K)
            assert np.allclose(e, e.T, rtol=1e-12, atol=1e-14 * np.abs(e).max())
    assert np.all(oracle.eii(2 * R0, R0, 0, K) == 0.0)
    assert np.all(oracle.eii(2.5 * R0, R0, 2, K) == 0.0)
    # W vanishes to third order at R0, so E fades smoothly at 2 R0
    assert np.abs(oracle.eii(2 * R0 - 0.05, R0, 0, K)).max() < 1e-9 * np.abs(oracle.eii(0.0, R0, 0, K)).max()


def test_pair_sum_matches_lattice_randoms():
    # DDR^II from random primaries on an M^3 lattice (the bispectrum oracle's
    # A_lm / C_l route) converges to n_w T; 2 R0 > L/2 exercises several images
    L, r0, ell_max = 60.0, 20.0, 3
    k = np.linspace(0.1, 0.4, 4)
    pos = np.random.default_rng(5).uniform(0, L, (8, 3))
    d = oracle.ddr2(pos, None, L, r0, k, ell_max, 256)
    nw = len(pos) / L ** 3
    M = 48
    g = (np.arange(M) + 0.5) * L / M
    R = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    b = oracle.bk_ell(pos, None, R, None, L, r0, k, ell_max)
    est = len(pos) / len(R) * (b["gr"] - b["cr"])
    ref = nw * d["t2"]
    assert np.abs(est - ref).max() <= 1e-6 * np.abs(ref).max()


def test_pair_sum_interpolation_converges():
    # T from the n_x-interval table against per-pair kernel values: sixth-order convergence
    L, r0, ell_max = 50.0, 12.0, 2
    k = np.array([0.2, 0.35, 0.5])
    pos = np.random.default_rng(9).uniform(0, L, (10, 3))
    exact = np.zeros((ell_max + 1, 2, 2))
    for i in range(len(pos)):
        for j in range(len(pos)):
            if i == j:
                continue
            for s in np.ndindex(3, 3, 3):
                dv = pos[i] - pos[j] + (np.array(s) - 1) * L
                r = float(np.sqrt(dv @ dv))
                if r < 2 * r0:
                    for ell in range(ell_max + 1):
                        exact[ell] += oracle.eii(r, r0, ell, k)
    errs = []
    for n_x in (16, 128):
        t = oracle.ddr2(pos, None, L, r0, k, ell_max, n_x)
        errs.append(np.abs(t["t2"] - exact).max() / np.abs(exact).max())
    # an 8x finer table: 8^6 = 262144 for a sixth-order rule (a fifth-order one gives 32768)
    assert errs[1] < 1e-9
    assert errs[0] / errs[1] > 60000


def test_interpolated_kernel_exact_at_nodes():
    # two points whose separation is exactly a table node: the pair sum is that node value
    L, r0, n_x = 64.0, 16.0, 32
    k = np.array([0.1, 0.3])
    h = 2 * r0 / n_x
    tab = oracle.eii_table(r0, k, 2, n_x)
    for m in (0, 1, 7, 20, 31):
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + m * h, 10.0, 10.0]])
        t = oracle.ddr2(pos, None, L, r0, k, 2, n_x, table=tab)
        if m == 0:
            assert t["n_pairs"] == 2  # coincident points: one (pair, image) term each way
        assert np.allclose(t["t2"][:, 0, 0], 2 * tab[:, 0, 0, m], rtol=1e-14, atol=1e-300)


def test_uniform_null_expectation_analytic():
    # uniform data: E[T] = (p1^2 - p2)/V int d^3x E, so with the exact volume
    # integral the DDR^II part has mean -(p1^2 - p2)/p1^2 W~aW~b (l = 0) and 0
    # (l > 0), and the estimator 2 p3/p1^3 W~aW~b
    L, r0, N, T, n_x = 100.0, 30.0, 30, 300, 64
    k = np.array([0.1, 0.2, 0.3])
    w = synthetic.uniform_weights(N, 7, np.float64)
    p1, p2, p3 = (float(np.sum(w ** q)) for q in (1, 2, 3))
    V = L ** 3
    nw = p1 / V
    tab = oracle.eii_table(r0, k, 2, n_x)
    d2, tot = [], []
    for t in range(T):
        pos = synthetic.poisson(N, L, 20000 + t)
        o = oracle.bk_ell_analytic(pos, w, L, r0, k, 2, n_x, table=tab, nthreads=1)
        d2.append(-nw * o["t2"] / (V * nw ** 3) * np.array([1, -3, 5])[:, None, None])
        tot.append(o["bk"])
    wt = np.array([oracle.wtilde(r0, k[0], k[1]), oracle.wtilde(r0, k[1], k[2])])
    WW = np.outer(wt, wt)
    for arr, ex in ((np.array(d2), -(p1 ** 2 - p2) / p1 ** 2 * WW), (np.array(tot), 2 * p3 / p1 ** 3 * WW)):
        m, se = arr.mean(0), arr.std(0, ddof=1) / np.sqrt(T)
        assert np.all(np.abs((m[0] - ex) / se[0]) < 4.0), (m[0], ex)
        for l in (1, 2):
            assert np.all(np.abs(m[l] / se[l]) < 4.0)
