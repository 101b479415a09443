"""FP64 brute-force CPU oracle (TEST INFRASTRUCTURE ONLY).

A plain, slow, independent implementation of the periodic-box power-spectrum
and bispectrum estimators of arXiv:2005.01739, used to check the GPU library.
Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this module; the library never does.  See oracle.c for the
definitions and the readings of the paper they follow.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_dp = ct.POINTER(ct.c_double)
_u8p = ct.POINTER(ct.c_uint8)
_u64p = ct.POINTER(ct.c_uint64)


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        src = os.path.join(_HERE, "oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = ct.CDLL(path)
        L.oracle_window.restype = ct.c_double
        L.oracle_window.argtypes = [ct.c_double]
        L.oracle_si.restype = ct.c_double
        L.oracle_si.argtypes = [ct.c_double]
        L.oracle_legendre.restype = ct.c_double
        L.oracle_legendre.argtypes = [ct.c_int, ct.c_double]
        L.oracle_D.restype = ct.c_double
        L.oracle_D.argtypes = [ct.c_int, ct.c_double]
        L.oracle_D_at_zero.restype = ct.c_double
        L.oracle_D_at_zero.argtypes = [ct.c_int]
        L.oracle_jbar.restype = ct.c_double
        L.oracle_jbar.argtypes = [ct.c_int, ct.c_double, ct.c_double, ct.c_double]
        L.oracle_jbar_series.restype = ct.c_double
        L.oracle_jbar_series.argtypes = [ct.c_int, ct.c_double, ct.c_double, ct.c_double]
        L.oracle_wtilde.restype = ct.c_double
        L.oracle_wtilde.argtypes = [ct.c_double, ct.c_double, ct.c_double, ct.c_double]
        L.oracle_ylm.restype = None
        L.oracle_ylm.argtypes = [ct.c_int, ct.c_double, ct.c_double, ct.c_double, _dp, _dp]
        L.oracle_sph_bessel_up.restype = None
        L.oracle_sph_bessel_up.argtypes = [ct.c_int, ct.c_double, _dp]
        L.oracle_pk_ell.restype = ct.c_int
        L.oracle_pk_ell.argtypes = [ct.c_int64, _dp, _dp, ct.c_double, ct.c_double, ct.c_int, _dp,
                                    ct.c_int, ct.c_int, _u8p, _dp, _dp, _dp, _dp, _u64p, ct.c_int]
        L.oracle_pk_survey.restype = ct.c_int
        L.oracle_pk_survey.argtypes = [ct.c_int64, _dp, _dp, _u8p, ct.c_int64, _dp, _dp, _u8p,
                                       ct.c_double, ct.c_double, ct.c_int, _dp, ct.c_int,
                                       _dp, _dp, _dp, _dp, _dp, _u64p, ct.c_int]
        L.oracle_bk_ell.restype = ct.c_int
        L.oracle_bk_ell.argtypes = [ct.c_int64, _dp, _dp, ct.c_int64, _dp, _dp, ct.c_double,
                                    ct.c_double, ct.c_int, _dp, ct.c_int, _u8p, _u8p, _dp, _dp,
                                    _dp, _dp, _dp, _dp, _dp, _u64p, _u64p, ct.c_int]
        L.oracle_aniso_count.restype = ct.c_int
        L.oracle_aniso_count.argtypes = [ct.c_int]
        L.oracle_bk_aniso.restype = ct.c_int
        L.oracle_bk_aniso.argtypes = [ct.c_int64, _dp, _dp, ct.c_int64, _dp, _dp, ct.c_double, ct.c_double, ct.c_int,
                                      _dp, ct.c_int, _u8p, _u8p, _dp, _dp, _dp, _dp, _dp, _dp, _u64p, _u64p,
                                      ct.c_int]
        L.oracle_eii.restype = ct.c_int
        L.oracle_eii.argtypes = [ct.c_double, ct.c_double, ct.c_int, ct.c_int, _dp, _dp]
        L.oracle_eii_table.restype = ct.c_int
        L.oracle_eii_table.argtypes = [ct.c_double, ct.c_int, _dp, ct.c_int, ct.c_int, _dp, ct.c_int]
        L.oracle_ddr2.restype = ct.c_int
        L.oracle_ddr2.argtypes = [ct.c_int64, _dp, _dp, ct.c_double, ct.c_double, ct.c_int, _dp, ct.c_int,
                                  ct.c_int, _dp, _u8p, _dp, _dp, _u64p, ct.c_int]
        L.oracle_bk_ell_analytic.restype = ct.c_int
        L.oracle_bk_ell_analytic.argtypes = [ct.c_int64, _dp, _dp, ct.c_double, ct.c_double, ct.c_int, _dp,
                                             ct.c_int, ct.c_int, _dp, _u8p, _dp, _dp, _dp, _dp, _dp, _dp,
                                             _dp, _u64p, _u64p, ct.c_int]
        L.oracle_sph_jl.restype = ct.c_double
        L.oracle_sph_jl.argtypes = [ct.c_int, ct.c_double]
        L.oracle_wigner3j_000.restype = ct.c_double
        L.oracle_wigner3j_000.argtypes = [ct.c_int, ct.c_int, ct.c_int]
        L.oracle_omega.restype = ct.c_int
        L.oracle_omega.argtypes = [ct.c_double, ct.c_double, ct.c_int, ct.c_int, _dp, _dp]
        L.oracle_pk_window_theory.restype = ct.c_int
        L.oracle_pk_window_theory.argtypes = [ct.c_double, ct.c_int, _dp, ct.c_int, ct.c_int, _dp, _dp, _dp, _dp]
        L.oracle_cov_gauss.restype = ct.c_int
        L.oracle_cov_gauss.argtypes = [ct.c_double, ct.c_double, ct.c_int, _dp, ct.c_int, ct.c_int, _dp, _dp, _dp,
                                       _dp, ct.c_int]
        L.oracle_cov_poisson2.restype = ct.c_int
        L.oracle_cov_poisson2.argtypes = [ct.c_double, ct.c_double, ct.c_double, ct.c_int, _dp, ct.c_int, ct.c_int,
                                          _dp, _dp, _dp, _dp]
        L.oracle_cov_nongauss.restype = ct.c_int
        L.oracle_cov_nongauss.argtypes = [ct.c_double, ct.c_double, ct.c_int, _dp, ct.c_int, ct.c_int, _dp, _dp, _dp,
                                          _dp, ct.c_int]
        L.oracle_cov_poisson3.restype = ct.c_int
        L.oracle_cov_poisson3.argtypes = [ct.c_double, ct.c_double, ct.c_double, ct.c_int, _dp, ct.c_int, ct.c_int,
                                          _dp, _dp, _dp, _dp, _dp, _dp, ct.c_int]
        _lib = L
    return _lib


def philox_randoms(n: int, box: float, seed: int) -> np.ndarray:
    """The uniform random catalogue that hipster_bk_ell draws when it is given
    none, restated here independently of the library: point i takes block
    i + 1 of the Philox4x64-10 counter-based generator (Salmon, Moraes, Dror
    and Shaw 2011) keyed by (seed, 0), and x_d = box * (word_d >> 11) * 2^-53
    for d = 0, 1, 2, a coordinate that rounds to box set to 0.  numpy's Philox
    bit generator is that generator (its counter is incremented before each
    block); the tests pin it to the published round function and its
    known-answer vectors.  Returns float64 (n, 3)."""
    raw = np.random.Philox(key=np.array([int(seed) & (2 ** 64 - 1), 0], dtype=np.uint64)).random_raw(4 * int(n)).reshape(int(n), 4)[:, :3]
    x = float(box) * ((raw >> np.uint64(11)).astype(np.float64) * 2.0 ** -53)
    x[x >= box] = 0.0
    return np.ascontiguousarray(x)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def window(x: float) -> float:
    return lib().oracle_window(float(x))


def si(u: float) -> float:
    return lib().oracle_si(float(u))


def legendre(ell: int, mu: float) -> float:
    return lib().oracle_legendre(int(ell), float(mu))


def D(ell: int, u: float) -> float:
    return lib().oracle_D(int(ell), float(u))


def D_at_zero(ell: int) -> float:
    return lib().oracle_D_at_zero(int(ell))


def jbar(ell: int, x: float, k1: float, k2: float) -> float:
    return lib().oracle_jbar(int(ell), float(x), float(k1), float(k2))


def jbar_series(ell: int, x: float, k1: float, k2: float) -> float:
    return lib().oracle_jbar_series(int(ell), float(x), float(k1), float(k2))


def wtilde(r0: float, k1: float, k2: float, resolution: float = 4.0) -> float:
    return lib().oracle_wtilde(float(r0), float(k1), float(k2), float(resolution))


def sph_bessel_up(nmax: int, u: float) -> np.ndarray:
    out = np.zeros(nmax + 1)
    lib().oracle_sph_bessel_up(int(nmax), float(u), _ptr(out))
    return out


def ylm(lmax: int, v) -> np.ndarray:
    """Complex Y_lm(v/|v|) at index l*l + l + m."""
    re = np.zeros((lmax + 1) ** 2)
    im = np.zeros((lmax + 1) ** 2)
    lib().oracle_ylm(int(lmax), float(v[0]), float(v[1]), float(v[2]), _ptr(re), _ptr(im))
    return re + 1j * im


def pk_ell(pos, w, box, r0, k_edges, ell_max=4, los_axis=2, primary_mask=None, nthreads=0):
    """Brute-force P^a_ell (even ell <= ell_max).  Returns a dict with pk, raw,
    l1 ([n_ell, n_k]), wtilde [n_k] and n_pairs (ordered pairs inside R0)."""
    pos = _f64(pos).reshape(-1, 3)
    w = _f64(w)
    k = _f64(k_edges)
    n_k = k.size - 1
    n_ell = ell_max // 2 + 1
    pk = np.zeros((n_ell, n_k))
    raw = np.zeros_like(pk)
    l1 = np.zeros_like(pk)
    wt = np.zeros(n_k)
    npairs = ct.c_uint64(0)
    mask = None if primary_mask is None else np.ascontiguousarray(primary_mask, dtype=np.uint8)
    rc = lib().oracle_pk_ell(pos.shape[0], _ptr(pos), _ptr(w), float(box), float(r0), n_k, _ptr(k),
                             int(ell_max), int(los_axis), _ptr(mask, _u8p), _ptr(pk), _ptr(raw),
                             _ptr(l1), _ptr(wt), ct.byref(npairs), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_pk_ell: argument outside the oracle's range")
    return {"pk": pk, "raw": raw, "l1": l1, "wtilde": wt, "n_pairs": int(npairs.value)}


def pk_survey(pos, w, rpos, rw, volume, r0, k_edges, ell_max=4, mask_d=None, mask_r=None, nthreads=0):
    """Brute-force survey-geometry P^a_ell (no periodicity, observer at the
    origin, pair-midpoint line of sight; even ell <= ell_max).  Returns a dict
    with pk, raw_dd, raw_dr (DR + RD), raw_rr, l1 ([n_ell, n_k]) and the
    contributing ordered pair counts n_dd, n_dr, n_rr."""
    pos = _f64(pos).reshape(-1, 3)
    w = _f64(w)
    rpos = _f64(rpos).reshape(-1, 3)
    rw = _f64(rw)
    k = _f64(k_edges)
    n_k = k.size - 1
    shp = (ell_max // 2 + 1, n_k)
    out = {name: np.zeros(shp) for name in ("pk", "raw_dd", "raw_dr", "raw_rr", "l1")}
    counts = (ct.c_uint64 * 3)()
    md = None if mask_d is None else np.ascontiguousarray(mask_d, dtype=np.uint8)
    mr = None if mask_r is None else np.ascontiguousarray(mask_r, dtype=np.uint8)
    rc = lib().oracle_pk_survey(pos.shape[0], _ptr(pos), _ptr(w), _ptr(md, _u8p), rpos.shape[0], _ptr(rpos),
                                _ptr(rw), _ptr(mr, _u8p), float(volume), float(r0), n_k, _ptr(k), int(ell_max),
                                _ptr(out["pk"]), _ptr(out["raw_dd"]), _ptr(out["raw_dr"]), _ptr(out["raw_rr"]),
                                _ptr(out["l1"]), ct.cast(counts, _u64p), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_pk_survey: argument outside the oracle's range")
    out["n_dd"], out["n_dr"], out["n_rr"] = int(counts[0]), int(counts[1]), int(counts[2])
    return out


def bk_ell(pos, w, rpos, rw, box, r0, k_edges, ell_max, mask_d=None, mask_r=None, nthreads=0):
    """Brute-force B^ab_ell, ell = 0..ell_max.  Returns a dict with bk, gd, cd,
    gr, cr ([ell_max+1, n_k, n_k]), s0, wtilde [n_k], n_pairs_dd, n_pairs_rd."""
    pos = _f64(pos).reshape(-1, 3)
    w = _f64(w)
    rpos = np.zeros((0, 3)) if rpos is None else _f64(rpos).reshape(-1, 3)
    rw = _f64(rw)
    k = _f64(k_edges)
    n_k = k.size - 1
    shp = (ell_max + 1, n_k, n_k)
    out = {name: np.zeros(shp) for name in ("bk", "gd", "cd", "gr", "cr")}
    s0 = np.zeros(n_k)
    wt = np.zeros(n_k)
    ndd = ct.c_uint64(0)
    nrd = ct.c_uint64(0)
    md = None if mask_d is None else np.ascontiguousarray(mask_d, dtype=np.uint8)
    mr = None if mask_r is None else np.ascontiguousarray(mask_r, dtype=np.uint8)
    rc = lib().oracle_bk_ell(pos.shape[0], _ptr(pos), _ptr(w), rpos.shape[0],
                             _ptr(rpos) if rpos.shape[0] else None, _ptr(rw), float(box),
                             float(r0), n_k, _ptr(k), int(ell_max), _ptr(md, _u8p),
                             _ptr(mr, _u8p), _ptr(out["bk"]), _ptr(out["gd"]), _ptr(out["cd"]),
                             _ptr(out["gr"]), _ptr(out["cr"]), _ptr(s0), _ptr(wt),
                             ct.byref(ndd), ct.byref(nrd), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_bk_ell: argument outside the oracle's range")
    out.update(s0=s0, wtilde=wt, n_pairs_dd=int(ndd.value), n_pairs_rd=int(nrd.value))
    return out


def aniso_combos(ell_max):
    """(l1, l2, m) of the anisotropic bispectrum, l1 <= l2 <= ell_max, m = 0..l1."""
    return [(l1, l2, m) for l1 in range(ell_max + 1) for l2 in range(l1, ell_max + 1) for m in range(l1 + 1)]


def bk_aniso(pos, w, rpos, rw, box, r0, k_edges, ell_max, mask_d=None, mask_r=None, nthreads=0):
    """Brute-force anisotropic B^{ab}_{l1 l2 m} (the reading of Sec. 10 in
    oracle.c).  Returns a dict with combos, bk, gd, cd, gr, cr ([n_c, n_k,
    n_k]), t [ell_max+1, n_k], n_pairs_dd, n_pairs_rd."""
    pos = _f64(pos).reshape(-1, 3)
    w = _f64(w)
    rpos = np.zeros((0, 3)) if rpos is None else _f64(rpos).reshape(-1, 3)
    rw = _f64(rw)
    k = _f64(k_edges)
    n_k = k.size - 1
    nc = lib().oracle_aniso_count(int(ell_max))
    out = {name: np.zeros((nc, n_k, n_k)) for name in ("bk", "gd", "cd", "gr", "cr")}
    t = np.zeros((ell_max + 1, n_k))
    ndd, nrd = ct.c_uint64(0), ct.c_uint64(0)
    md = None if mask_d is None else np.ascontiguousarray(mask_d, dtype=np.uint8)
    mr = None if mask_r is None else np.ascontiguousarray(mask_r, dtype=np.uint8)
    st = lib().oracle_bk_aniso(pos.shape[0], _ptr(pos), _ptr(w), rpos.shape[0], _ptr(rpos), _ptr(rw), float(box),
                               float(r0), n_k, _ptr(k), int(ell_max), _ptr(md, _u8p), _ptr(mr, _u8p),
                               _ptr(out["bk"]), _ptr(out["gd"]), _ptr(out["cd"]), _ptr(out["gr"]), _ptr(out["cr"]),
                               _ptr(t), ct.byref(ndd), ct.byref(nrd), int(nthreads))
    if st != 0:
        raise ValueError("oracle_bk_aniso: bad arguments")
    out.update(combos=aniso_combos(ell_max), t=t, n_pairs_dd=int(ndd.value), n_pairs_rd=int(nrd.value))
    return out


def eii(x, r0, ell, k_edges):
    """E^{II,ab}_ell(x) of the analytic DDR^II term, [n_k, n_k]."""
    k = _f64(k_edges)
    n_k = k.size - 1
    out = np.zeros((n_k, n_k))
    if lib().oracle_eii(float(x), float(r0), int(ell), n_k, _ptr(k), _ptr(out)) != 0:
        raise ValueError("oracle_eii: argument outside the oracle's range")
    return out


def eii_table(r0, k_edges, ell_max, n_x, nthreads=0):
    """E^{II,ab}_ell on the nodes m 2 R0 / n_x, m = 0..n_x:
    [ell_max+1, n_k, n_k, n_x+1]."""
    k = _f64(k_edges)
    n_k = k.size - 1
    out = np.zeros((ell_max + 1, n_k, n_k, n_x + 1))
    if lib().oracle_eii_table(float(r0), n_k, _ptr(k), int(ell_max), int(n_x), _ptr(out), int(nthreads)) != 0:
        raise ValueError("oracle_eii_table: argument outside the oracle's range")
    return out


def ddr2(pos, w, box, r0, k_edges, ell_max, n_x, table=None, mask=None, nthreads=0):
    """T^ab_ell = sum over ordered pairs i != j and periodic images inside 2 R0
    of w_i w_j E^{II,ab}_ell (interpolated table).  Returns a dict with t2,
    l1 ([ell_max+1, n_k, n_k]), n_pairs and the table used."""
    pos = _f64(pos).reshape(-1, 3)
    w = _f64(w)
    k = _f64(k_edges)
    n_k = k.size - 1
    tab = eii_table(r0, k, ell_max, n_x, nthreads) if table is None else _f64(table)
    shp = (ell_max + 1, n_k, n_k)
    T = np.zeros(shp)
    l1 = np.zeros(shp)
    npairs = ct.c_uint64(0)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().oracle_ddr2(pos.shape[0], _ptr(pos), _ptr(w), float(box), float(r0), n_k, _ptr(k),
                           int(ell_max), int(n_x), _ptr(tab), _ptr(m, _u8p), _ptr(T), _ptr(l1),
                           ct.byref(npairs), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_ddr2: argument outside the oracle's range")
    return {"t2": T, "l1": l1, "n_pairs": int(npairs.value), "table": tab}


def bk_ell_analytic(pos, w, box, r0, k_edges, ell_max, n_x, table=None, mask_d=None, nthreads=0):
    """B^ab_ell with the DDR^II term from the E^II kernel (no randoms).
    Returns a dict with bk, gd, cd, t2, t2_l1 ([ell_max+1, n_k, n_k]), s0,
    wtilde [n_k], n_pairs_dd (inside R0), n_pairs_2r0 and the table."""
    pos = _f64(pos).reshape(-1, 3)
    w = _f64(w)
    k = _f64(k_edges)
    n_k = k.size - 1
    tab = eii_table(r0, k, ell_max, n_x, nthreads) if table is None else _f64(table)
    shp = (ell_max + 1, n_k, n_k)
    out = {name: np.zeros(shp) for name in ("bk", "gd", "cd", "t2", "t2_l1")}
    s0 = np.zeros(n_k)
    wt = np.zeros(n_k)
    ndd = ct.c_uint64(0)
    n2 = ct.c_uint64(0)
    md = None if mask_d is None else np.ascontiguousarray(mask_d, dtype=np.uint8)
    rc = lib().oracle_bk_ell_analytic(pos.shape[0], _ptr(pos), _ptr(w), float(box), float(r0), n_k, _ptr(k),
                                      int(ell_max), int(n_x), _ptr(tab), _ptr(md, _u8p), _ptr(out["bk"]),
                                      _ptr(out["gd"]), _ptr(out["cd"]), _ptr(out["t2"]), _ptr(out["t2_l1"]),
                                      _ptr(s0), _ptr(wt), ct.byref(ndd), ct.byref(n2), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_bk_ell_analytic: argument outside the oracle's range")
    out.update(s0=s0, wtilde=wt, n_pairs_dd=int(ndd.value), n_pairs_2r0=int(n2.value), table=tab)
    return out


def sph_jl(ell, x):
    return lib().oracle_sph_jl(int(ell), float(x))


def wigner3j_000(l1, l2, l3):
    return lib().oracle_wigner3j_000(int(l1), int(l2), int(l3))


def omega(p, r0, ell, k_edges):
    """omega^a_ell(p; R0) for all bins, [n_k]."""
    k = _f64(k_edges)
    out = np.zeros(k.size - 1)
    if lib().oracle_omega(float(p), float(r0), int(ell), k.size - 1, _ptr(k), _ptr(out)) != 0:
        raise ValueError("oracle_omega: argument outside the oracle's range")
    return out


def pk_window_theory(r0, k_edges, ell_max, r, wr, xi):
    """Windowed P^a_ell(R0) of model multipoles xi [ell_max/2+1, n_r] on the
    quadrature (r, wr): [ell_max/2+1, n_k]."""
    k = _f64(k_edges)
    r, wr = _f64(r), _f64(wr)
    xi = _f64(xi).reshape(ell_max // 2 + 1, r.size)
    out = np.zeros((ell_max // 2 + 1, k.size - 1))
    if lib().oracle_pk_window_theory(float(r0), k.size - 1, _ptr(k), int(ell_max), r.size, _ptr(r), _ptr(wr),
                                     _ptr(xi), _ptr(out)) != 0:
        raise ValueError("oracle_pk_window_theory: argument outside the oracle's range")
    return out


def cov_gauss(r0, volume, k_edges, ell_max, p, wp, pk, nthreads=0):
    """Gaussian covariance of the binned windowed multipoles on the p
    quadrature (p, wp) with model P_ell(p) [ell_max/2+1, n_p]:
    [n_ell, n_k, n_ell, n_k]."""
    k = _f64(k_edges)
    p, wp = _f64(p), _f64(wp)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    pk = _f64(pk).reshape(n_ell, p.size)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    if lib().oracle_cov_gauss(float(r0), float(volume), n_k, _ptr(k), int(ell_max), p.size, _ptr(p), _ptr(wp),
                              _ptr(pk), _ptr(out), int(nthreads)) != 0:
        raise ValueError("oracle_cov_gauss: argument outside the oracle's range")
    return out


def cov_nongauss(r0, volume, k_edges, ell_max, p, wp, tbar, nthreads=0):
    """Non-Gaussian intrinsic covariance term on the p quadrature (p, wp) with
    collapsed-trispectrum multipoles tbar [n_ell, n_ell, n_p, n_p]:
    [n_ell, n_k, n_ell, n_k]."""
    k = _f64(k_edges)
    p, wp = _f64(p), _f64(wp)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    tb = _f64(tbar).reshape(n_ell, n_ell, p.size, p.size)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    if lib().oracle_cov_nongauss(float(r0), float(volume), n_k, _ptr(k), int(ell_max), p.size, _ptr(p), _ptr(wp),
                                 _ptr(tb), _ptr(out), int(nthreads)) != 0:
        raise ValueError("oracle_cov_nongauss: argument outside the oracle's range")
    return out


def cov_poisson3(r0, nbar, volume, k_edges, ell_max, p, wp, pk, pbin=None, bk=None, nthreads=0):
    """Poisson three-point covariance term on the p quadrature (p, wp) with
    model P_L(p) [ell_max/2+1, n_p], windowed binned multipoles pbin
    [ell_max/2+1, n_k] and bispectrum bk [ell_max/2+1, n_k, n_k] (either
    None: zero): [n_ell, n_k, n_ell, n_k]."""
    k = _f64(k_edges)
    p, wp = _f64(p), _f64(wp)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    pk = _f64(pk).reshape(n_ell, p.size)
    pb = None if pbin is None else _f64(pbin).reshape(n_ell, n_k)
    bb = None if bk is None else _f64(bk).reshape(n_ell, n_k, n_k)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    if lib().oracle_cov_poisson3(float(r0), float(nbar), float(volume), n_k, _ptr(k), int(ell_max), p.size, _ptr(p),
                                 _ptr(wp), _ptr(pk), None if pb is None else _ptr(pb),
                                 None if bb is None else _ptr(bb), _ptr(out), int(nthreads)) != 0:
        raise ValueError("oracle_cov_poisson3: argument outside the oracle's range")
    return out


def cov_poisson2(r0, nbar, volume, k_edges, ell_max, r, wr, xi):
    """Poisson two-point covariance term on the x quadrature (r, wr) with model
    multipoles xi [ell_max/2+1, n_r]: [n_ell, n_k, n_ell, n_k]."""
    k = _f64(k_edges)
    r, wr = _f64(r), _f64(wr)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    xi = _f64(xi).reshape(n_ell, r.size)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    if lib().oracle_cov_poisson2(float(r0), float(nbar), float(volume), n_k, _ptr(k), int(ell_max), r.size,
                                 _ptr(r), _ptr(wr), _ptr(xi), _ptr(out)) != 0:
        raise ValueError("oracle_cov_poisson2: argument outside the oracle's range")
    return out
