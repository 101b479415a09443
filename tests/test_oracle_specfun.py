"""Pins for the oracle's special functions against values fixed by the
mathematics: exact window breakpoints, mpmath quadrature of the defining
integrals, and library special cases (scipy)."""
import mpmath as mp
import numpy as np
import pytest
import scipy.special as sps

import oracle

mp.mp.dps = 30


def test_window_breakpoints_and_continuity():
    # W(x) (Sec. 2, eq. window_defn): W(1/2)=1, W(3/4)=1/2, W(1)=0, W=1 below 1/2.
    assert oracle.window(0.0) == 1.0
    assert oracle.window(0.49) == 1.0
    assert oracle.window(0.5) == 1.0
    assert oracle.window(0.75) == 0.5
    assert oracle.window(1.0) == 0.0
    assert oracle.window(1.3) == 0.0
    for x0 in (0.5, 0.75, 1.0):
        assert abs(oracle.window(x0 - 1e-9) - oracle.window(x0 + 1e-9)) < 1e-7
    # derivative continuous too: the pieces join smoothly
    h = 1e-6
    for x0 in (0.5, 0.75):
        dl = (oracle.window(x0 - h) - oracle.window(x0 - 2 * h)) / h
        dr = (oracle.window(x0 + 2 * h) - oracle.window(x0 + h)) / h
        assert abs(dl - dr) < 1e-4
    # a plain interior value, by hand: x = 0.6 -> t = 0.2, 1 - 8 t^3 + 8 t^4
    assert oracle.window(0.6) == pytest.approx(1 - 8 * 0.008 + 8 * 0.0016, rel=1e-15)
    # x = 0.9 -> t = -0.1: -64 t^3 - 128 t^4
    assert oracle.window(0.9) == pytest.approx(0.064 - 0.0128, rel=1e-14)


def test_legendre_matches_scipy():
    for ell in range(7):
        for mu in np.linspace(-1, 1, 17):
            assert oracle.legendre(ell, mu) == pytest.approx(sps.eval_legendre(ell, mu), abs=1e-15)


def test_sine_integral_matches_scipy_both_branches():
    for u in np.concatenate([np.linspace(1e-3, 4, 40), np.linspace(4.0001, 400, 200)]):
        assert oracle.si(u) == pytest.approx(sps.sici(u)[0], rel=2e-15, abs=2e-15)


def test_spherical_bessel_upward_matches_scipy_where_used():
    for u in np.linspace(5.0, 200.0, 60):
        j = oracle.sph_bessel_up(7, u)
        ref = sps.spherical_jn(np.arange(8), u)
        assert np.allclose(j, ref, rtol=1e-12, atol=1e-15)


def _Dtilde_exact(ell, u):
    f = lambda t: t ** 2 * mp.sqrt(mp.pi / (2 * t)) * mp.besselj(ell + mp.mpf(1) / 2, t) if t > 0 else mp.mpf(0)
    return mp.quad(f, mp.linspace(0, u, int(float(u) // 3) + 2))


@pytest.mark.parametrize("ell", range(7))
def test_D_ell_against_quadrature(ell):
    # D_ell(u) - D_ell(0) = int_0^u t^2 j_ell(t) dt (Appendix C definition)
    rng = np.random.default_rng(100 + ell)
    us = np.concatenate([rng.uniform(0.01, 5, 8), [4.999, 5.0, 5.001], rng.uniform(5, 120, 10)])
    for u in us:
        ex = float(_Dtilde_exact(ell, mp.mpf(u)))
        got = oracle.D(ell, u) - oracle.D_at_zero(ell)
        # odd ell carry the constant D_ell(0) in D_ell itself, so their error is
        # measured against that size too
        scale = max(abs(ex), abs(oracle.D_at_zero(ell)), 1e-3 * u ** 2)
        assert abs(got - ex) <= 2e-13 * scale, (ell, u, got, ex)


def test_D_at_zero_values():
    # The recursion's constant: D_ell(0) = ell(ell+1) I_ell(0), I_0(0)=0, I_1(0)=-1.
    assert [oracle.D_at_zero(l) for l in range(7)] == [0.0, -2.0, 0.0, -8.0, 0.0, -16.0, 0.0]


def _jbar_exact(ell, x, k1, k2):
    f = lambda kk: kk ** 2 * mp.sqrt(mp.pi / (2 * kk * x)) * mp.besselj(ell + mp.mpf(1) / 2, kk * x)
    nseg = int(float((k2 - k1) * x) // 2) + 2
    return 3 * mp.quad(f, mp.linspace(k1, k2, nseg)) / (mp.mpf(k2) ** 3 - mp.mpf(k1) ** 3)


@pytest.mark.parametrize("ell", range(7))
def test_jbar_against_bin_average_quadrature(ell):
    # jbar^a_ell(x) = (4 pi / v_a) int k^2 dk Theta^a(k) j_ell(k x)  (Sec. 3, eq. jla-def)
    rng = np.random.default_rng(200 + ell)
    bins = [(0.2, 0.29), (1.0, 1.06), (2.0, 2.1), (0.0, 0.05), (0.5, 0.71)]
    for (k1, k2) in bins:
        xs = np.concatenate([rng.uniform(0.01, 5 / k2, 4), rng.uniform(5 / k2, 5 / k2 + 60, 6)])
        vals = []
        for x in xs:
            ex = float(_jbar_exact(ell, mp.mpf(x), mp.mpf(k1), mp.mpf(k2)))
            vals.append((x, ex, oracle.jbar(ell, x, k1, k2)))
        peak = max(abs(v[1]) for v in vals)
        for x, ex, got in vals:
            assert abs(got - ex) <= 1e-12 * max(abs(ex), 1e-2 * peak), (ell, k1, k2, x, got, ex)


def test_jbar_at_zero_and_branch_overlap():
    for ell in range(7):
        assert oracle.jbar(ell, 0.0, 0.5, 0.6) == (1.0 if ell == 0 else 0.0)
    # The series and the closed-form difference agree where both are valid.
    for ell in range(7):
        for x in (5.2, 6.0, 8.0):
            k1, k2 = 0.9, 1.0
            closed = 3 * (oracle.D(ell, x * k2) - oracle.D(ell, x * k1)) / (x ** 3 * (k2 ** 3 - k1 ** 3))
            ser = oracle.jbar_series(ell, x, k1, k2)
            assert closed == pytest.approx(ser, rel=1e-11, abs=1e-14)


def test_ylm_matches_scipy():
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.normal(size=3)
        y = oracle.ylm(6, v)
        th = np.arccos(v[2] / np.linalg.norm(v))
        ph = np.arctan2(v[1], v[0])
        for l in range(7):
            for m in range(-l, l + 1):
                ref = sps.sph_harm_y(l, m, th, ph)
                assert abs(y[l * l + l + m] - ref) < 1e-13


def test_ylm_addition_theorem():
    # L_l(a.b) = 4 pi/(2l+1) sum_m Y_lm(a) Y*_lm(b)  (Sec. 4)
    rng = np.random.default_rng(6)
    for _ in range(10):
        a, b = rng.normal(size=3), rng.normal(size=3)
        ya, yb = oracle.ylm(6, a), oracle.ylm(6, b)
        c = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
        for l in range(7):
            s = sum(ya[l * l + l + m] * np.conj(yb[l * l + l + m]) for m in range(-l, l + 1))
            assert abs(4 * np.pi / (2 * l + 1) * s - sps.eval_legendre(l, c)) < 1e-13


def _wtilde_exact(r0, k1, k2):
    # 4 pi int_0^R0 r^2 jbar_0 W dr with jbar_0 from D_0(u) = sin u - u cos u, in mpmath.
    D0 = lambda u: mp.sin(u) - u * mp.cos(u)
    dk3 = mp.mpf(k2) ** 3 - mp.mpf(k1) ** 3

    def W(x):
        if x < 0.5:
            return mp.mpf(1)
        if x < 0.75:
            t = 2 * x - 1
            return 1 - 8 * t ** 3 + 8 * t ** 4
        t = x - 1
        return -64 * t ** 3 - 128 * t ** 4

    f = lambda r: 3 * (D0(k2 * r) - D0(k1 * r)) / (r * dk3) * W(r / r0) if r > 0 else mp.mpf(0)
    pts = sorted(set([mp.mpf(0), r0 / 2, 3 * mp.mpf(r0) / 4, mp.mpf(r0)] + list(mp.linspace(0, r0, 40))))
    return 4 * mp.pi * mp.quad(f, pts)


@pytest.mark.parametrize("r0,k1,k2", [(50.0, 0.2, 0.29), (25.0, 1.0, 1.06), (30.0, 0.5, 0.7083), (15.0, 19.0, 20.0), (50.0, 0.0, 0.05)])
def test_wtilde_quadrature(r0, k1, k2):
    a = oracle.wtilde(r0, k1, k2, 4.0)
    b = oracle.wtilde(r0, k1, k2, 8.0)
    ex = float(_wtilde_exact(mp.mpf(r0), mp.mpf(k1), mp.mpf(k2)))
    # The two resolutions agree, and both agree with mpmath.  W~ is small
    # where kR0 >> 1, so the scale is the integrand's L1 size ~ 4 pi R0^3/3.
    scale = max(abs(ex), 1e-6 * 4 * np.pi * r0 ** 3 / 3)
    assert abs(a - b) <= 1e-13 * scale
    assert abs(a - ex) <= 1e-12 * scale, (a, ex)
