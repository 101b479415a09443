"""GPU parity of the theory side (hipster_omega, hipster_pk_window_theory,
hipster_cov_gauss, hipster_cov_nongauss, hipster_cov_poisson2,
hipster_cov_poisson3) against the FP64 oracle.  Both sides are double-precision
quadratures of the same integrals with different rules (omega) or the same
caller quadrature (the windowed P, the covariance's p sum), so:
* omega agrees to 1e-10 of the largest |omega| of its multipole;
* the windowed P to 1e-11 relative per bin (only the bin averages differ in
  how they are evaluated);
* the covariance, its non-Gaussian term and the Poisson three-point term
  to 1e-9 of the largest entry, the Poisson two-point term (same caller quadrature, no omega) to
  1e-11.
At the 40-bin size of the headline power spectrum, where the oracle's omega
quadrature is too slow, the covariance is checked through an identity that
holds at any size: for a constant monopole power P0 (higher multipoles
zero), C^ab_ll' = 2 (2l+1) P0^2 / V delta_ll' E^{II,ab}_l(0), with
E^{II,ab}_l(0) = 4 pi int r^2 g^a g^b dr from the oracle (Parseval)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

R0 = 20.0
K = np.linspace(0.1, 0.5, 4)


def _p_quadrature(pmax, panels=150, n=16):
    gx, gw = np.polynomial.legendre.leggauss(n)
    e = np.linspace(0.0, pmax, panels + 1)
    mid, half = 0.5 * (e[:-1] + e[1:]), 0.5 * (e[1:] - e[:-1])
    return (mid[:, None] + half[:, None] * gx).ravel(), (half[:, None] * gw).ravel()


def test_omega_parity():
    import paper_2005_01739_amd as hp
    p = np.array([0.0, 1e-3, 0.05, 0.2, 0.33, 0.9, 2.5, 7.0])
    got = hp.omega(p, R0, K, 6)
    for ell in range(7):
        ref = np.array([oracle.omega(pi, R0, ell, K) for pi in p])
        assert np.abs(got[ell] - ref).max() <= 1e-10 * np.abs(ref).max(), ell


def test_window_theory_parity():
    import paper_2005_01739_amd as hp
    gx, gw = np.polynomial.legendre.leggauss(48)
    r, wr = 0.5 * R0 * (gx + 1), 0.5 * R0 * gw
    xi = np.array([5.0 * np.exp(-r / 7.0), -1.0 * np.exp(-r / 5.0) * r / 10.0, 0.1 * np.exp(-r / 9.0),
                   0.02 * np.exp(-r / 4.0)])
    k = np.geomspace(0.05, 2.0, 9)
    got = hp.pk_window_theory(R0, k, 6, r, wr, xi)
    ref = oracle.pk_window_theory(R0, k, 6, r, wr, xi)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_covariance_parity():
    import paper_2005_01739_amd as hp
    p, w = _p_quadrature(6.0, panels=60)
    pk = np.array([800.0 / (1 + (p / 0.2) ** 2), -200.0 / (1 + (p / 0.3) ** 2), 40.0 / (1 + (p / 0.5) ** 2)])
    got = hp.cov_gauss(R0, 1e6, K, 4, p, w, pk)
    ref = oracle.cov_gauss(R0, 1e6, K, 4, p, w, pk)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_covariance_identity_at_headline_bins():
    # 40 log bins over 1-10 h/Mpc, R0 = 25, l = 0, 2, 4
    import paper_2005_01739_amd as hp
    r0, k, V, P0 = 25.0, np.geomspace(1.0, 10.0, 41), 1e9, 400.0
    p, w = _p_quadrature(40.0, panels=600)
    pk = np.zeros((3, p.size))
    pk[0] = P0
    C = hp.cov_gauss(r0, V, k, 4, p, w, pk)
    scale = np.abs(C).max()
    for li in range(3):
        ref = 2 * (4 * li + 1) * P0 ** 2 / V * oracle.eii(0.0, r0, 2 * li, k)
        assert np.abs(C[li, :, li, :] - ref).max() <= 1e-6 * np.abs(ref).max(), li
        for lj in range(3):
            if lj != li:
                assert np.abs(C[li, :, lj, :]).max() <= 1e-9 * scale


def test_theory_errors():
    import paper_2005_01739_amd as hp
    with pytest.raises(hp.HipsterError) as e:
        hp.omega([0.1, -1.0], R0, K, 2)
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError) as e:
        hp.pk_window_theory(R0, K, 3, [1.0], [1.0], np.zeros((2, 1)))
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError) as e:
        hp.pk_window_theory(R0, K, 2, [1.0, 30.0], [1.0, 1.0], np.zeros((2, 2)))
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError) as e:
        hp.cov_gauss(R0, 0.0, K, 2, [0.1], [1.0], np.zeros((2, 1)))
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError) as e:
        hp.omega([1e6], R0, K, 2)
    assert e.value.name == "HIPSTER_EUNSUPPORTED"


def test_poisson2_parity():
    import paper_2005_01739_amd as hp
    gx, gw = np.polynomial.legendre.leggauss(16)
    cuts = [0.0, 0.5 * R0, 0.75 * R0, R0]
    x = np.concatenate([0.5 * (hi - lo) * gx + 0.5 * (hi + lo) for lo, hi in zip(cuts[:-1], cuts[1:])])
    w = np.concatenate([0.5 * (hi - lo) * gw for lo, hi in zip(cuts[:-1], cuts[1:])])
    xi = np.array([3.0 * np.exp(-x / 6.0), -0.8 * np.exp(-x / 4.0), 0.2 * np.exp(-x / 3.0)])
    k = np.geomspace(0.05, 2.0, 9)
    got = hp.cov_poisson2(R0, 1e-3, 1e6, k, 4, x, w, xi)
    ref = oracle.cov_poisson2(R0, 1e-3, 1e6, k, 4, x, w, xi)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_poisson3_parity():
    import paper_2005_01739_amd as hp
    p, w = _p_quadrature(6.0, panels=60)
    pk = np.array([800.0 / (1 + (p / 0.2) ** 2), -200.0 / (1 + (p / 0.3) ** 2), 40.0 / (1 + (p / 0.5) ** 2)])
    rng = np.random.default_rng(11)
    pbin = rng.normal(size=(3, 3)) * 30.0
    B = rng.normal(size=(3, 3, 3)) * 500.0
    for pb, bk in ((None, None), (pbin, B)):
        got = hp.cov_poisson3(R0, 1e-3, 1e6, K, 4, p, w, pk, pb, bk)
        ref = oracle.cov_poisson3(R0, 1e-3, 1e6, K, 4, p, w, pk, pbin=pb, bk=bk)
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    with pytest.raises(hp.HipsterError) as e:
        hp.cov_poisson3(R0, 0.0, 1e6, K, 2, [0.1], [1.0], np.zeros((2, 1)))
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError) as e:
        hp.cov_poisson2(R0, -1.0, 1e6, K, 2, [1.0], [1.0], np.zeros((2, 1)))
    assert e.value.name == "HIPSTER_EDOMAIN"


def test_nongauss_parity():
    import paper_2005_01739_amd as hp
    p, w = _p_quadrature(4.0, panels=10, n=8)
    f = np.array([400.0 * np.exp(-p), 60.0 * p * np.exp(-p / 2), 10.0 / (1 + p * p)])
    rng = np.random.default_rng(5)
    T = np.einsum("li,mj->lmij", f, f) * (1.0 + 0.1 * rng.standard_normal((3, 3, p.size, p.size)))
    got = hp.cov_nongauss(R0, 1e6, K, 4, p, w, T)
    ref = oracle.cov_nongauss(R0, 1e6, K, 4, p, w, T)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    with pytest.raises(hp.HipsterError) as e:
        hp.cov_nongauss(R0, -1.0, K, 2, [0.1], [1.0], np.zeros((2, 2, 1, 1)))
    assert e.value.name == "HIPSTER_EDOMAIN"
