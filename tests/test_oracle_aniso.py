"""Pins of the anisotropic-bispectrum oracle (the Sec. 10 reading in
oracle.c): literal triple and pair sums over tiny catalogues with scipy's
spherical harmonics, and the identity that its m-sum at l1 = l2 is the
(separately pinned) isotropic estimator of Sec. 4."""
import numpy as np
import pytest
from scipy import special

import oracle
import synthetic


def _ylm(l, m, d):
    r = np.linalg.norm(d)
    theta = np.arccos(np.clip(d[2] / r, -1.0, 1.0))
    phi = np.arctan2(d[1], d[0])
    return special.sph_harm_y(l, m, theta, phi)


def _g(l, r, r0, k):
    return np.array([oracle.jbar(l, r, k[a], k[a + 1]) for a in range(len(k) - 1)]) * oracle.window(r / r0)


def _min_image(d, L):
    return d - L * np.round(d / L)


def _neighbours(p, pos, L, r0, exclude):
    out = []
    for j in range(len(pos)):
        if exclude is not None and j == exclude:
            continue
        d = _min_image(p - pos[j], L)
        r = np.linalg.norm(d)
        if r < r0:
            out.append((j, d, r))
    return out


def _triple(prim, pos, w, L, r0, k, combos, self_set, wp=None):
    """sum_p w_p sum_{j != k, both neighbours of p} w_j w_k g^a_{l1}(r_pj)
    g^b_{l2}(r_pk) sum_{mu in M(m)} Y_{l1 mu}(xhat_pj) Y*_{l2 mu}(xhat_pk)."""
    n_k = len(k) - 1
    out = np.zeros((len(combos), n_k, n_k))
    for ip, p in enumerate(prim):
        nb = _neighbours(p, pos, L, r0, ip if self_set else None)
        for c, (l1, l2, m) in enumerate(combos):
            mus = [0] if m == 0 else [m, -m]
            for (j, dj, rj) in nb:
                gj = _g(l1, rj, r0, k)
                for (kk, dk, rk) in nb:
                    if kk == j:
                        continue
                    gk = _g(l2, rk, r0, k)
                    q = sum((_ylm(l1, mu, dj) * np.conj(_ylm(l2, mu, dk))).real for mu in mus)
                    out[c] += (1.0 if wp is None else wp[ip]) * w[j] * w[kk] * q * np.outer(gj, gk)
    return out


@pytest.fixture(scope="module")
def tiny():
    L, r0 = 20.0, 7.0
    pos = synthetic.thomas(16, L, 8, 1.5, 0.0, 21, np.float64)
    w = synthetic.uniform_weights(16, 22, np.float64)
    rpos = synthetic.poisson(6, L, 23, np.float64)
    k = np.array([0.4, 0.9, 1.6])
    return L, r0, pos, w, rpos, k


def test_pair_form_equals_triple_sum(tiny):
    L, r0, pos, w, rpos, k = tiny
    ell_max = 2
    res = oracle.bk_aniso(pos, w, rpos, None, L, r0, k, ell_max)
    combos = res["combos"]
    td = _triple(pos, pos, w, L, r0, k, combos, True, wp=w)
    tr = _triple(rpos, pos, w, L, r0, k, combos, False)
    scale = np.abs(res["gd"]).max() + np.abs(res["cd"]).max()
    assert np.allclose(res["gd"] - res["cd"], td, rtol=1e-11, atol=1e-12 * scale)
    scale_r = np.abs(res["gr"]).max() + np.abs(res["cr"]).max()
    assert np.allclose(res["gr"] - res["cr"], tr, rtol=1e-11, atol=1e-12 * scale_r)
    assert np.abs(td).max() > 0 and np.abs(tr).max() > 0


def test_t_is_the_pair_sum_of_y_l0(tiny):
    L, r0, pos, w, rpos, k = tiny
    ell_max = 3
    res = oracle.bk_aniso(pos, w, None, None, L, r0, k, ell_max)
    for l in range(ell_max + 1):
        ref, mass = np.zeros(len(k) - 1), np.zeros(len(k) - 1)
        for i in range(len(pos)):
            for (j, d, r) in _neighbours(pos[i], pos, L, r0, i):
                term = w[i] * w[j] * _g(l, r, r0, k) * _ylm(l, 0, d).real
                ref += term
                mass += np.abs(term)
        # odd l cancel between the two orientations of each pair
        assert np.allclose(res["t"][l], ref, rtol=1e-11, atol=1e-13 * mass.max())
        if l % 2:
            assert np.abs(res["t"][l]).max() < 1e-13 * mass.max()


@pytest.mark.parametrize("weighted", [False, True])
def test_m_sum_is_the_isotropic_estimator(weighted):
    L, r0 = 60.0, 12.0
    pos = synthetic.thomas(300, L, 10, 2.0, 0.0, 3, np.float64)
    w = synthetic.uniform_weights(300, 5, np.float64) if weighted else None
    rpos = synthetic.poisson(600, L, 4, np.float64)
    k = np.linspace(0.3, 1.5, 5)
    ell_max = 4
    iso = oracle.bk_ell(pos, w, rpos, None, L, r0, k, ell_max)
    an = oracle.bk_aniso(pos, w, rpos, None, L, r0, k, ell_max)
    assert an["n_pairs_dd"] == iso["n_pairs_dd"] and an["n_pairs_rd"] == iso["n_pairs_rd"]
    for l in range(ell_max + 1):
        s = sum(an["bk"][i] for i, (l1, l2, m) in enumerate(an["combos"]) if l1 == l2 == l)
        assert np.allclose(s, iso["bk"][l], rtol=1e-10, atol=1e-12 * np.abs(iso["bk"][l]).max())
    # the m = 0, l1 = l2 = 0 entry is the isotropic monopole itself
    assert np.allclose(an["bk"][0], iso["bk"][0], rtol=1e-12, atol=0)


def test_combination_order():
    assert oracle.aniso_combos(2) == [(0, 0, 0), (0, 1, 0), (0, 2, 0), (1, 1, 0), (1, 1, 1), (1, 2, 0), (1, 2, 1),
                                      (2, 2, 0), (2, 2, 1), (2, 2, 2)]
    assert len(oracle.aniso_combos(4)) == oracle.lib().oracle_aniso_count(4) == 35
