"""Pins for the oracle's bispectrum estimator (Sec. 4): the spherical-harmonic
pair form against a literal triple sum and Cartesian identities, exact
expectations for uniform catalogues, symmetries and invariances.  A closed
form for clustered catalogues is not derived: for those the pins are the
triple sum and the invariances only."""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import reference


def _setup(n=18, nr=20, seed=41, L=20.0):
    pos = synthetic.thomas(n, L, 3, 1.5, 0.0, seed, np.float64)
    w = synthetic.uniform_weights(n, seed + 1, np.float64)
    rp = synthetic.poisson(nr, L, seed + 2)
    rw = synthetic.uniform_weights(nr, seed + 3, np.float64)
    return pos, w, rp, rw, L


def test_pair_form_equals_triple_sum():
    # DDD and DDR^II via A_lm and C (Sec. 4, eq. AC-def) equal the literal sum
    # over distinct triples with L_l of the opening angle (Legendre addition).
    pos, w, rp, rw, L = _setup()
    r0, lmax = 8.0, 4
    k = np.array([0.3, 0.7, 1.2])
    out = oracle.bk_ell(pos, w, rp, rw, L, r0, k, lmax)
    tD = reference.bk_triple_sum(pos, w, pos, w, L, r0, k, lmax, True)
    tR = reference.bk_triple_sum(rp, rw, pos, w, L, r0, k, lmax, False)
    for l in range(lmax + 1):
        sc = np.abs(out["gd"][l]).max() + np.abs(out["cd"][l]).max()
        assert np.allclose(out["gd"][l] - out["cd"][l], tD[l], rtol=1e-12, atol=1e-12 * sc)
        sc = np.abs(out["gr"][l]).max() + np.abs(out["cr"][l]).max()
        assert np.allclose(out["gr"][l] - out["cr"][l], tR[l], rtol=1e-12, atol=1e-12 * sc)


def test_cartesian_identities_l012():
    pos, w, rp, rw, L = _setup(24, 10, 51)
    r0 = 8.0
    k = np.array([0.2, 0.6, 1.1, 1.9])
    out = oracle.bk_ell(pos, w, rp, rw, L, r0, k, 2)
    G = reference.bk_cartesian(pos, w, pos, w, L, r0, k, True)
    GR = reference.bk_cartesian(rp, rw, pos, w, L, r0, k, False)
    for l in range(3):
        assert np.allclose(out["gd"][l], G[l], rtol=1e-12, atol=1e-12 * np.abs(G[l]).max())
        assert np.allclose(out["gr"][l], GR[l], rtol=1e-12, atol=1e-12 * np.abs(GR[l]).max())


def test_s0_equals_power_spectrum_monopole_pair_sum():
    # S0^b = sum_{i!=j} w_i w_j jbar^b_0 W is the ell = 0 power-spectrum pair sum.
    pos, w, rp, rw, L = _setup(30, 5, 61)
    r0 = 8.0
    k = np.array([0.2, 0.6, 1.1])
    b = oracle.bk_ell(pos, w, rp, rw, L, r0, k, 0)
    p = oracle.pk_ell(pos, w, L, r0, k, 0)
    assert np.allclose(b["s0"], p["raw"][0], rtol=1e-13)
    assert b["n_pairs_dd"] == p["n_pairs"]


def test_symmetry_and_assembly():
    pos, w, rp, rw, L = _setup(21, 30, 71)
    r0, lmax = 8.0, 3
    k = np.array([0.2, 0.5, 0.9, 1.4])
    o = oracle.bk_ell(pos, w, rp, rw, L, r0, k, lmax)
    for name in ("bk", "gd", "cd", "gr", "cr"):
        assert np.allclose(o[name], np.transpose(o[name], (0, 2, 1)), rtol=1e-13, atol=1e-13 * np.abs(o[name]).max())
    # re-assemble from the parts (Sec. 4 summary) with weights read as n -> n_w
    V = L ** 3
    p1, pr = w.sum(), rw.sum()
    nw, sR = p1 / V, p1 / pr
    wt = o["wtilde"]
    for l in range(lmax + 1):
        v = (-1) ** l * (2 * l + 1) / (V * nw ** 3) * ((o["gd"][l] - o["cd"][l]) - sR * (o["gr"][l] - o["cr"][l]))
        if l == 0:
            v = v - (np.outer(wt, o["s0"]) + np.outer(o["s0"], wt)) / (V * nw ** 2) + 2 * np.outer(wt, wt)
        assert np.allclose(o["bk"][l], v, rtol=1e-12, atol=1e-12 * np.abs(v).max())


def test_cube_symmetry_invariance():
    # The isotropic bispectrum is invariant under the 48 symmetries of the
    # cube (axis permutations and reflections x -> L - x).
    pos, w, rp, rw, L = _setup(24, 24, 81)
    r0 = 8.0
    k = np.array([0.3, 0.8, 1.4])
    ref = oracle.bk_ell(pos, w, rp, rw, L, r0, k, 3)
    rng = np.random.default_rng(2)
    for _ in range(4):
        perm = rng.permutation(3)
        flip = rng.integers(0, 2, 3).astype(bool)

        def tf(x):
            y = x[:, perm].copy()
            y[:, flip] = np.mod(L - y[:, flip], L)
            return y

        o = oracle.bk_ell(tf(pos), w, tf(rp), rw, L, r0, k, 3)
        assert o["n_pairs_dd"] == ref["n_pairs_dd"]
        assert np.allclose(o["bk"], ref["bk"], rtol=1e-9, atol=1e-9 * np.abs(ref["bk"]).max())


def test_uniform_null_expectations_per_term():
    # Uniform data and randoms: E[DDD part] = (p1^3 - 3 p1 p2 + 2 p3)/p1^3 W~aW~b,
    # E[DDR^II part] = -(p1^2 - p2)/p1^2 W~aW~b, E[DDR^I part] = -2 (p1^2 - p2)/p1^2
    # W~aW~b, RRR = +2 W~aW~b; ell > 0 vanish; total 2 p3/p1^3 W~aW~b.
    L, r0, N, NR, T = 100.0, 30.0, 30, 90, 400
    k = np.array([0.1, 0.2, 0.3])
    w = synthetic.uniform_weights(N, 7, np.float64)
    p1, p2, p3 = (float(np.sum(w ** q)) for q in (1, 2, 3))
    V = L ** 3
    nw = p1 / V
    parts = []
    for t in range(T):
        pos = synthetic.poisson(N, L, 20000 + t)
        rp = synthetic.poisson(NR, L, 30000 + t)
        o = oracle.bk_ell(pos, w, rp, None, L, r0, k, 2, nthreads=1)
        sR = p1 / NR
        ddd = (o["gd"] - o["cd"]) / (V * nw ** 3) * np.array([1, -3, 5])[:, None, None]
        ddr2 = -sR * (o["gr"] - o["cr"]) / (V * nw ** 3) * np.array([1, -3, 5])[:, None, None]
        wt = o["wtilde"]
        ddr1 = -(np.outer(wt, o["s0"]) + np.outer(o["s0"], wt)) / (V * nw ** 2)
        parts.append((ddd, ddr2, ddr1, o["bk"]))
    wt = oracle.wtilde(r0, k[0], k[1]), oracle.wtilde(r0, k[1], k[2])
    WW = np.outer(wt, wt)
    ex_ddd = (p1 ** 3 - 3 * p1 * p2 + 2 * p3) / p1 ** 3 * WW
    ex_ddr2 = -(p1 ** 2 - p2) / p1 ** 2 * WW
    ex_ddr1 = -2 * (p1 ** 2 - p2) / p1 ** 2 * WW
    ex_tot = 2 * p3 / p1 ** 3 * WW
    arr = [np.array([p[i] for p in parts]) for i in range(4)]
    for a, ex in ((arr[0][:, 0], ex_ddd), (arr[1][:, 0], ex_ddr2), (arr[2], ex_ddr1), (arr[3][:, 0], ex_tot)):
        m, se = a.mean(0), a.std(0, ddof=1) / np.sqrt(T)
        z = (m - ex) / se
        assert np.all(np.abs(z) < 4.0), (m, ex, z)
    for l in (1, 2):
        for a in (arr[0][:, l], arr[1][:, l], arr[3][:, l]):
            m, se = a.mean(0), a.std(0, ddof=1) / np.sqrt(T)
            assert np.all(np.abs(m / se) < 4.0)


def _sphere_grid(nt=24, nph=48):
    x, wx = np.polynomial.legendre.leggauss(nt)
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    ct, P = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    n = np.stack([st * np.cos(P), st * np.sin(P), ct], -1).reshape(-1, 3)
    wq = (wx[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).reshape(-1)
    return n, wq


def test_multipole_factor_from_angular_quadrature():
    # The estimator's factor (-1)^l (2l+1) comes from the definition of B_l as
    # (2l+1) times the angular average of B(k1, k2) L_l(k1hat.k2hat) with
    # Fourier weights e^{-i k.x} (Sec. 2).  Measure that factor by direct
    # quadrature over both k directions for one triangle, then check the
    # oracle's ell > 0 output (no randoms, so only the DDD term is present)
    # against the brute-force triple sum times the measured factor.
    from scipy.special import eval_legendre, spherical_jn
    n, wq = _sphere_grid()
    r1, r2 = np.array([1.1, -0.4, 0.7]), np.array([-0.3, 0.9, 0.5])
    k1, k2 = 1.7, 2.3
    e1 = np.exp(-1j * k1 * n @ r1)
    e2 = np.exp(-1j * k2 * n @ r2)
    c12 = n @ n.T
    factors = []
    for l in range(5):
        avg = (wq * e1) @ eval_legendre(l, c12) @ (wq * e2) / (4 * np.pi) ** 2
        val = (2 * l + 1) * avg
        base = spherical_jn(l, k1 * np.linalg.norm(r1)) * spherical_jn(l, k2 * np.linalg.norm(r2)) * \
            eval_legendre(l, r1 @ r2 / np.linalg.norm(r1) / np.linalg.norm(r2))
        assert abs(val.imag) < 1e-10
        factors.append(val.real / base)
    pos, w, rp, rw, L = _setup(18, 1, 91)
    r0, lmax = 8.0, 4
    k = np.array([0.3, 0.7, 1.2])
    out = oracle.bk_ell(pos, w, None, None, L, r0, k, lmax)
    t = reference.bk_triple_sum(pos, w, pos, w, L, r0, k, lmax, True)
    V, nw = L ** 3, w.sum() / L ** 3
    for l in range(1, lmax + 1):
        ex = factors[l] * t[l] / (V * nw ** 3)
        assert np.allclose(out["bk"][l], ex, rtol=1e-8, atol=1e-8 * np.abs(ex).max()), l
