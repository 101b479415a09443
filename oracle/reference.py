"""Tiny-N independent references for pinning the oracle (TEST INFRASTRUCTURE).

These are deliberately different computations of the same quantities:

* ``pk_all_images`` sums every periodic image explicitly instead of taking
  the minimum image;
* ``bk_triple_sum`` evaluates the isotropic triple count of Sec. 4 (the
  DDD kernel, and the random-primary DDR^II kernel) as a literal O(N^3) sum
  over distinct triples with the Legendre polynomial of the opening angle,
  instead of the spherical-harmonic pair form;
* ``bk_cartesian`` evaluates (4 pi/(2l+1)) sum_m A^a_lm A^b*_lm for l <= 2 by
  Cartesian tensor identities instead of spherical harmonics.

The per-pair radial factors W and jbar come from the oracle's special
functions, which are pinned separately against mpmath.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.special import eval_legendre

from . import jbar, window


def _g(ell, r, r0, k):
    """g^a_ell(r) = jbar^a_ell(r) W(r/R0) for all bins a."""
    return np.array([jbar(ell, r, k[a], k[a + 1]) for a in range(len(k) - 1)]) * window(r / r0)


def pk_all_images(pos, w, box, r0, k, ell_max, los_axis=2):
    """S^a_ell = sum over ordered pairs i != j and over every periodic image
    n in {-2..2}^3 with |x_i - x_j + n L| < R0 (tiny N only)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    n_ell = ell_max // 2 + 1
    S = np.zeros((n_ell, len(k) - 1))
    shifts = np.array(list(itertools.product(range(-2, 3), repeat=3)), dtype=np.float64) * box
    npairs = 0
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            for s in shifts:
                d = pos[i] - pos[j] + s
                r = float(np.sqrt(d @ d))
                if r >= r0:
                    continue
                npairs += 1
                mu = d[los_axis] / r if r > 0 else 0.0
                for li in range(n_ell):
                    ell = 2 * li
                    ph = -1.0 if li % 2 else 1.0
                    S[li] += w[i] * w[j] * (2 * ell + 1) * ph * eval_legendre(ell, mu) * _g(ell, r, r0, k)
    return S, npairs


def _min_image(d, box):
    return d - box * np.round(d / box)


def bk_triple_sum(ppos, pw, pos, w, box, r0, k, lmax, self_exclude):
    """sum_p w_p sum_{j != k} w_j w_k g^a_l(r_pj) g^b_l(r_pk) L_l(xhat_pj . xhat_pk)
    over primaries p and distinct data secondaries j, k (both != p when the
    primaries are the data themselves).  Returns [lmax+1, n_k, n_k]."""
    ppos = np.asarray(ppos, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    n_k = len(k) - 1
    pw = np.ones(len(ppos)) if pw is None else np.asarray(pw, dtype=np.float64)
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    out = np.zeros((lmax + 1, n_k, n_k))
    for p in range(len(ppos)):
        d = _min_image(ppos[p][None, :] - pos, box)
        r = np.sqrt((d * d).sum(1))
        sel = [j for j in range(len(pos)) if r[j] < r0 and not (self_exclude and j == p)]
        if not sel:
            continue
        g = {l: {j: _g(l, r[j], r0, k) for j in sel} for l in range(lmax + 1)}
        u = {j: d[j] / r[j] if r[j] > 0 else np.array([0.0, 0.0, 1.0]) for j in sel}
        for j in sel:
            for kk in sel:
                if j == kk:
                    continue
                c = float(u[j] @ u[kk])
                for l in range(lmax + 1):
                    out[l] += pw[p] * w[j] * w[kk] * eval_legendre(l, c) * np.outer(g[l][j], g[l][kk])
    return out


def bk_cartesian(ppos, pw, pos, w, box, r0, k, self_exclude):
    """G^ab_l = sum_p w_p (4 pi/(2l+1)) sum_m A^a_lm A^b*_lm for l = 0, 1, 2 from
    Cartesian moments: l=0: F^a F^b; l=1: V^a . V^b; l=2: 3/2 T^a:T^b - 1/2 F^a F^b,
    with F = sum_j w_j g_l, V = sum_j w_j g_1 rhat, T = sum_j w_j g_2 rhat rhat^T."""
    ppos = np.asarray(ppos, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    n_k = len(k) - 1
    pw = np.ones(len(ppos)) if pw is None else np.asarray(pw, dtype=np.float64)
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    G = np.zeros((3, n_k, n_k))
    for p in range(len(ppos)):
        d = _min_image(ppos[p][None, :] - pos, box)
        r = np.sqrt((d * d).sum(1))
        F0 = np.zeros(n_k)
        V1 = np.zeros((n_k, 3))
        F2 = np.zeros(n_k)
        T2 = np.zeros((n_k, 3, 3))
        for j in range(len(pos)):
            if r[j] >= r0 or (self_exclude and j == p):
                continue
            u = d[j] / r[j] if r[j] > 0 else np.array([0.0, 0.0, 1.0])
            F0 += w[j] * _g(0, r[j], r0, k)
            g1 = w[j] * _g(1, r[j], r0, k)
            V1 += g1[:, None] * u[None, :]
            g2 = w[j] * _g(2, r[j], r0, k)
            F2 += g2
            T2 += g2[:, None, None] * np.outer(u, u)[None]
        G[0] += pw[p] * np.outer(F0, F0)
        G[1] += pw[p] * V1 @ V1.T
        G[2] += pw[p] * (1.5 * np.einsum("aij,bij->ab", T2, T2) - 0.5 * np.outer(F2, F2))
    return G
