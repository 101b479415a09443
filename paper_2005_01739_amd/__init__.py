"""Python binding of libhipster, the MI355X pair-sweep library for the
periodic-box small-scale power spectrum and bispectrum of Philcox (2020),
arXiv:2005.01739.

Argument marshalling only: every step of the estimators runs in the HIP
library (include/hipster.h).  PyTorch is used, when present, for device
memory and streams: a CUDA (HIP) tensor is passed to the library as a device
pointer on torch's current stream.  NumPy arrays are passed as host memory.
There is no fallback: if the shared library is missing the import of this
module's functions raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Any

import numpy as np

__all__ = ["Context", "wtilde", "pk_ell", "pk_ell_noalloc", "bk_ell", "bk_aniso", "aniso_combos", "batch", "HipsterError", "library_path", "load_library",
           "EXPORTED_SYMBOLS", "MIXED", "FP64", "TABLE", "pk_survey", "bk_ell_analytic", "eii_table",
           "omega", "pk_window_theory", "cov_gauss", "cov_poisson2", "cov_poisson3", "cov_nongauss"]

_HERE = os.path.dirname(os.path.abspath(__file__))
MIXED, FP64, TABLE = 0, 1, 2
_F32, _F64 = 0, 1

EXPORTED_SYMBOLS = ("hipster_create", "hipster_destroy", "hipster_pk_ell", "hipster_bk_ell",
                    "hipster_batch", "hipster_last_error", "hipster_status_string",
                    "hipster_set_memory_cap", "hipster_wtilde", "hipster_pk_survey",
                    "hipster_bk_ell_analytic", "hipster_eii_table", "hipster_omega",
                    "hipster_pk_window_theory", "hipster_cov_gauss", "hipster_cov_poisson2",
                    "hipster_cov_poisson3", "hipster_cov_nongauss", "hipster_pk_ell_noalloc", "hipster_bk_aniso")


class HipsterError(RuntimeError):
    def __init__(self, status: int, name: str, message: str):
        super().__init__(f"{name}: {message}")
        self.status = status
        self.name = name


class _Points(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("dtype", ct.c_int32), ("on_device", ct.c_int32),
                ("pos", ct.c_void_p), ("w", ct.c_void_p)]


class _Params(ct.Structure):
    _fields_ = [("box", ct.c_double), ("r0", ct.c_double), ("n_k", ct.c_int32), ("ell_max", ct.c_int32),
                ("k_edges", ct.POINTER(ct.c_double)), ("los_axis", ct.c_int32), ("precision", ct.c_int32),
                ("primary_mask", ct.POINTER(ct.c_uint8)), ("random_mask", ct.POINTER(ct.c_uint8))]


_dp = ct.POINTER(ct.c_double)


class _Diag(ct.Structure):
    _fields_ = [("n_pairs", ct.c_uint64), ("n_pairs_rand", ct.c_uint64), ("raw", _dp), ("gd", _dp),
                ("cd", _dp), ("gr", _dp), ("cr", _dp), ("s0", _dp), ("wtilde", _dp),
                ("ms_build", ct.c_double), ("ms_pairs", ct.c_double), ("ms_sweep", ct.c_double),
                ("ms_total", ct.c_double), ("sweep_launches", ct.c_uint64), ("n_pairs_rr", ct.c_uint64),
                ("ms_sweep_far", ct.c_double), ("n_pairs_far", ct.c_uint64), ("ms_eii_table", ct.c_double),
                ("ms_ddr2", ct.c_double), ("n_pairs_2r0", ct.c_uint64), ("eii_nodes", ct.c_int64),
                ("ms_cterm", ct.c_double), ("l1_mass", _dp), ("n_rand", ct.c_uint64)]


class _SurveyParams(ct.Structure):
    _fields_ = [("volume", ct.c_double), ("r0", ct.c_double), ("n_k", ct.c_int32), ("ell_max", ct.c_int32),
                ("k_edges", _dp), ("precision", ct.c_int32), ("reserved", ct.c_int32),
                ("primary_mask", ct.POINTER(ct.c_uint8)), ("random_mask", ct.POINTER(ct.c_uint8))]


class _BoxJob(ct.Structure):
    _fields_ = [("data", _Points), ("randoms", _Points), ("pk_params", _Params), ("bk_params", _Params),
                ("pk", _dp), ("bk", _dp), ("n_pairs", ct.c_uint64), ("bk_eii_nodes", ct.c_int32),
                ("reserved", ct.c_int32), ("f_rand", ct.c_double), ("seed", ct.c_uint64)]


_lib = None


def library_path() -> str:
    """The in-tree build, or the file named by HIPSTER_LIBRARY (an alternative
    build of the same sources, e.g. with different compile-time tuning)."""
    return os.environ.get("HIPSTER_LIBRARY") or os.path.join(_HERE, "libhipster.so")


def load_library():
    """Load libhipster.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2005_01739_amd.build`")
    L = ct.CDLL(path)
    L.hipster_create.restype = ct.c_int
    L.hipster_create.argtypes = [ct.POINTER(ct.c_void_p), ct.c_int, ct.c_void_p]
    L.hipster_destroy.restype = None
    L.hipster_destroy.argtypes = [ct.c_void_p]
    L.hipster_pk_ell.restype = ct.c_int
    L.hipster_pk_ell.argtypes = [ct.c_void_p, ct.POINTER(_Points), ct.POINTER(_Params), _dp, ct.POINTER(_Diag)]
    L.hipster_bk_aniso.restype = ct.c_int
    L.hipster_bk_aniso.argtypes = [ct.c_void_p, ct.POINTER(_Points), ct.POINTER(_Points), ct.c_double, ct.c_uint64,
                                   ct.POINTER(_Params), _dp, ct.POINTER(_Diag)]
    L.hipster_pk_ell_noalloc.restype = ct.c_int
    L.hipster_pk_ell_noalloc.argtypes = [ct.c_void_p, ct.POINTER(_Points), ct.POINTER(_Params), _dp,
                                         ct.POINTER(_Diag)]
    L.hipster_pk_survey.restype = ct.c_int
    L.hipster_pk_survey.argtypes = [ct.c_void_p, ct.POINTER(_Points), ct.POINTER(_Points), ct.POINTER(_SurveyParams),
                                    _dp, ct.POINTER(_Diag)]
    L.hipster_bk_ell.restype = ct.c_int
    L.hipster_bk_ell.argtypes = [ct.c_void_p, ct.POINTER(_Points), ct.POINTER(_Points), ct.c_double, ct.c_uint64,
                                 ct.POINTER(_Params), _dp, ct.POINTER(_Diag)]
    L.hipster_bk_ell_analytic.restype = ct.c_int
    L.hipster_bk_ell_analytic.argtypes = [ct.c_void_p, ct.POINTER(_Points), ct.POINTER(_Params), ct.c_int32, _dp,
                                          ct.POINTER(_Diag)]
    L.hipster_eii_table.restype = ct.c_int
    L.hipster_eii_table.argtypes = [ct.c_void_p, ct.c_double, ct.c_int32, _dp, ct.c_int32, ct.c_int32, _dp]
    L.hipster_omega.restype = ct.c_int
    L.hipster_omega.argtypes = [ct.c_void_p, ct.c_double, ct.c_int32, _dp, ct.c_int32, ct.c_int32, _dp, _dp]
    L.hipster_pk_window_theory.restype = ct.c_int
    L.hipster_pk_window_theory.argtypes = [ct.c_void_p, ct.c_double, ct.c_int32, _dp, ct.c_int32, ct.c_int32, _dp,
                                           _dp, _dp, _dp]
    L.hipster_cov_gauss.restype = ct.c_int
    L.hipster_cov_gauss.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_int32, _dp, ct.c_int32, ct.c_int32,
                                    _dp, _dp, _dp, _dp]
    L.hipster_cov_poisson2.restype = ct.c_int
    L.hipster_cov_poisson2.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_double, ct.c_int32, _dp, ct.c_int32,
                                       ct.c_int32, _dp, _dp, _dp, _dp]
    L.hipster_cov_poisson3.restype = ct.c_int
    L.hipster_cov_poisson3.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_double, ct.c_int32, _dp, ct.c_int32,
                                       ct.c_int32, _dp, _dp, _dp, _dp, _dp, _dp]
    L.hipster_cov_nongauss.restype = ct.c_int
    L.hipster_cov_nongauss.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_int32, _dp, ct.c_int32, ct.c_int32,
                                       _dp, _dp, _dp, _dp]
    L.hipster_batch.restype = ct.c_int
    L.hipster_batch.argtypes = [ct.c_void_p, ct.c_int, ct.POINTER(_BoxJob), ct.POINTER(_Diag)]
    L.hipster_last_error.restype = ct.c_char_p
    L.hipster_last_error.argtypes = [ct.c_void_p]
    L.hipster_status_string.restype = ct.c_char_p
    L.hipster_status_string.argtypes = [ct.c_int]
    L.hipster_wtilde.restype = ct.c_int
    L.hipster_wtilde.argtypes = [ct.c_double, ct.c_int32, _dp, _dp]
    L.hipster_set_memory_cap.restype = ct.c_int
    L.hipster_set_memory_cap.argtypes = [ct.c_void_p, ct.c_uint64]
    _lib = L
    return L


def _torch():
    try:
        import torch
        return torch
    except Exception:  # pragma: no cover
        return None


def _is_device_tensor(x) -> bool:
    t = _torch()
    return t is not None and isinstance(x, t.Tensor) and x.is_cuda


class Context:
    """A library context bound to one HIP device and stream."""

    def __init__(self, device: int = 0, stream: int | None = None):
        L = load_library()
        h = ct.c_void_p()
        st = L.hipster_create(ct.byref(h), int(device), ct.c_void_p(stream) if stream else None)
        if st != 0:
            raise HipsterError(st, L.hipster_status_string(st).decode(), "hipster_create failed")
        self._h = h
        self.device = device
        self.stream = stream

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().hipster_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != 0:
            L = load_library()
            raise HipsterError(st, L.hipster_status_string(st).decode(),
                               L.hipster_last_error(self._h).decode())

    def set_memory_cap(self, nbytes: int):
        self.check(load_library().hipster_set_memory_cap(self._h, int(nbytes)))


_default_ctx: dict = {}


def _context_for(x) -> Context:
    t = _torch()
    if _is_device_tensor(x):
        dev = x.device.index or 0
        stream = t.cuda.current_stream(dev).cuda_stream
    else:
        dev, stream = 0, None
    key = (dev, stream)
    if key not in _default_ctx:
        _default_ctx[key] = Context(dev, stream)
    return _default_ctx[key]


def _points(pos, w, keep: list) -> _Points:
    """Describe a catalogue; `keep` holds references for the call's duration."""
    if pos is None:
        return _Points(0, _F32, 0, None, None)
    if _is_device_tensor(pos):
        if pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
            raise ValueError("positions must be a contiguous (N, 3) tensor")
        t = _torch()
        dt = {t.float32: _F32, t.float64: _F64}.get(pos.dtype)
        if dt is None:
            raise ValueError("positions must be float32 or float64")
        if w is not None:
            if not _is_device_tensor(w) or w.dtype != pos.dtype or w.numel() != pos.shape[0] or not w.is_contiguous():
                raise ValueError("weights must be a contiguous device tensor of the positions' dtype and length")
        keep += [pos, w]
        return _Points(int(pos.shape[0]), dt, 1, pos.data_ptr(), None if w is None else w.data_ptr())
    a = np.ascontiguousarray(pos)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("positions must have shape (N, 3)")
    if a.dtype not in (np.float32, np.float64):
        raise ValueError("positions must be float32 or float64")
    dt = _F32 if a.dtype == np.float32 else _F64
    wa = None
    if w is not None:
        wa = np.ascontiguousarray(np.asarray(w), dtype=a.dtype)
        if wa.shape != (a.shape[0],):
            raise ValueError("weights must have shape (N,)")
    keep += [a, wa]
    return _Points(int(a.shape[0]), dt, 0, a.ctypes.data, None if wa is None else wa.ctypes.data)


def _params(box, r0, k_edges, ell_max, los_axis, precision, mask, rmask, keep) -> _Params:
    k = np.ascontiguousarray(k_edges, dtype=np.float64)
    if k.ndim != 1 or k.size < 2:
        raise ValueError("k_edges must be 1-D with at least two entries")
    prec = {"mixed": MIXED, "fp64": FP64, "table": TABLE, MIXED: MIXED, FP64: FP64, TABLE: TABLE}[precision]
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rm = None if rmask is None else np.ascontiguousarray(rmask, dtype=np.uint8)
    keep += [k, m, rm]
    u8 = ct.POINTER(ct.c_uint8)
    return _Params(float(box), float(r0), int(k.size - 1), int(ell_max), k.ctypes.data_as(_dp), int(los_axis), prec,
                   None if m is None else m.ctypes.data_as(u8), None if rm is None else rm.ctypes.data_as(u8))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def wtilde(r0: float, k_edges) -> np.ndarray:
    """W~^a(R0) for each bin (host computation in the library)."""
    L = load_library()
    k = np.ascontiguousarray(k_edges, dtype=np.float64)
    out = np.zeros(k.size - 1)
    st = L.hipster_wtilde(float(r0), int(k.size - 1), k.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    if st != 0:
        raise HipsterError(st, L.hipster_status_string(st).decode(), "hipster_wtilde: bad arguments")
    return out


def pk_ell(pos, w=None, *, box: float, r0: float, k_edges, ell_max: int = 4, los_axis: int = 2,
           precision: str = "mixed", primary_mask=None, ctx: Context | None = None,
           return_diag: bool = False, l1_mass: bool = False) -> Any:
    """Power-spectrum multipoles P^a_ell, ell = 0, 2, .., ell_max: float64 array
    of shape (ell_max/2 + 1, n_k).  precision: "mixed", "fp64" or "table"
    (jbar from a quintic table, fixed-point histograms; see HIPSTER_TABLE).
    With return_diag, also a dict of the raw pair sums, W~^a, the ordered pair
    count and device timings (and "table_nodes", the table's interval count,
    in the table form); with l1_mass as well, "l1_mass", the L1 mass of the
    raw sums per bin (an extra double-precision pass of the library)."""
    return _pk_ell_call("hipster_pk_ell", pos, w, box, r0, k_edges, ell_max, los_axis, precision, primary_mask,
                        ctx, return_diag, l1_mass)


def pk_ell_noalloc(pos, w=None, *, box: float, r0: float, k_edges, ell_max: int = 4, los_axis: int = 2,
                   precision: str = "mixed", primary_mask=None, ctx: Context | None = None,
                   return_diag: bool = False) -> Any:
    """pk_ell through hipster_pk_ell_noalloc: the same result, with the
    library's device scratch taken from its static per-device workspace
    instead of allocations (timings in the diag read 0; no l1_mass)."""
    return _pk_ell_call("hipster_pk_ell_noalloc", pos, w, box, r0, k_edges, ell_max, los_axis, precision,
                        primary_mask, ctx, return_diag, False)


def _pk_ell_call(entry, pos, w, box, r0, k_edges, ell_max, los_axis, precision, primary_mask, ctx, return_diag,
                 l1_mass):
    L = load_library()
    keep: list = []
    pts = _points(pos, w, keep)
    prm = _params(box, r0, k_edges, ell_max, los_axis, precision, primary_mask, None, keep)
    n_ell, n_k = ell_max // 2 + 1, prm.n_k
    out = np.zeros((n_ell, n_k))
    raw = np.zeros((n_ell, n_k))
    wt = np.zeros(n_k)
    l1 = np.zeros((n_ell, n_k)) if l1_mass else None
    d = _Diag()
    d.raw, d.wtilde, d.l1_mass = _ptr(raw), _ptr(wt), _ptr(l1)
    c = ctx or _context_for(pos)
    c.check(getattr(L, entry)(c.handle, ct.byref(pts), ct.byref(prm), _ptr(out), ct.byref(d)))
    if not return_diag:
        return out
    info = {"raw": raw, "wtilde": wt, "n_pairs": int(d.n_pairs), "ms_build": d.ms_build,
            "ms_pairs": d.ms_pairs, "ms_sweep": d.ms_sweep, "ms_total": d.ms_total,
            "sweep_launches": int(d.sweep_launches), "ms_sweep_far": d.ms_sweep_far,
            "n_pairs_far": int(d.n_pairs_far), "table_nodes": int(d.eii_nodes)}
    if l1_mass:
        info["l1_mass"] = l1
    return out, info


def pk_survey(pos, w=None, randoms=None, rw=None, *, volume: float, r0: float, k_edges, ell_max: int = 4,
              precision: str = "mixed", primary_mask=None, random_mask=None, ctx: Context | None = None,
              return_diag: bool = False) -> Any:
    """Survey-geometry power-spectrum multipoles (DD - 2DR + RR, pair-midpoint
    line of sight, observer at the origin, no periodicity): float64 array of
    shape (ell_max/2 + 1, n_k).  `randoms` is required.  precision: "mixed",
    "fp64" or "table".  With return_diag, also the raw pair sums, the DD,
    DR + RD and RR pair counts and timings."""
    L = load_library()
    if randoms is None:
        raise ValueError("pk_survey needs a random catalogue")
    keep: list = []
    pts = _points(pos, w, keep)
    rpts = _points(randoms, rw, keep)
    k = np.ascontiguousarray(k_edges, dtype=np.float64)
    if k.ndim != 1 or k.size < 2:
        raise ValueError("k_edges must be 1-D with at least two entries")
    prec = {"mixed": MIXED, "fp64": FP64, "table": TABLE, MIXED: MIXED, FP64: FP64, TABLE: TABLE}[precision]
    m = None if primary_mask is None else np.ascontiguousarray(primary_mask, dtype=np.uint8)
    rm = None if random_mask is None else np.ascontiguousarray(random_mask, dtype=np.uint8)
    keep += [k, m, rm]
    u8 = ct.POINTER(ct.c_uint8)
    prm = _SurveyParams(float(volume), float(r0), int(k.size - 1), int(ell_max), k.ctypes.data_as(_dp), prec, 0,
                        None if m is None else m.ctypes.data_as(u8), None if rm is None else rm.ctypes.data_as(u8))
    n_ell, n_k = ell_max // 2 + 1, prm.n_k
    out = np.zeros((n_ell, n_k))
    raw = np.zeros((n_ell, n_k))
    d = _Diag()
    d.raw = _ptr(raw)
    c = ctx or _context_for(pos)
    c.check(L.hipster_pk_survey(c.handle, ct.byref(pts), ct.byref(rpts), ct.byref(prm), _ptr(out), ct.byref(d)))
    if not return_diag:
        return out
    return out, {"raw": raw, "n_pairs": int(d.n_pairs), "n_pairs_rand": int(d.n_pairs_rand),
                 "n_pairs_rr": int(d.n_pairs_rr), "ms_build": d.ms_build, "ms_pairs": d.ms_pairs,
                 "ms_sweep": d.ms_sweep, "ms_total": d.ms_total, "sweep_launches": int(d.sweep_launches),
                 "ms_sweep_far": d.ms_sweep_far, "n_pairs_far": int(d.n_pairs_far)}


def bk_ell(pos, w=None, randoms=None, rw=None, *, box: float, r0: float, k_edges, ell_max: int = 4,
           precision: str = "mixed", primary_mask=None, random_mask=None, f_rand: float = 0.0, seed: int = 0,
           ctx: Context | None = None, return_diag: bool = False) -> Any:
    """Bispectrum multipoles B^ab_ell, ell = 0..ell_max: float64 array of shape
    (ell_max + 1, n_k, n_k).  `randoms` are the random primaries of the DDR^II
    term; without them the library draws round(f_rand N) uniform randoms from
    `seed` (Philox4x64-10, see hipster_bk_ell), and f_rand <= 0 is an error.
    With return_diag, also the raw components (gd, cd, gr, cr, s0), W~^a,
    l1_mass, pair counts, the random count and timings."""
    L = load_library()
    keep: list = []
    pts = _points(pos, w, keep)
    rpts = _points(randoms, rw, keep)
    prm = _params(box, r0, k_edges, ell_max, 2, precision, primary_mask, random_mask, keep)
    n_k = prm.n_k
    shp = (ell_max + 1, n_k, n_k)
    out = np.zeros(shp)
    parts = {k: np.zeros(shp) for k in ("gd", "cd", "gr", "cr")}
    s0 = np.zeros(n_k)
    wt = np.zeros(n_k)
    l1 = np.zeros(shp)
    d = _Diag()
    d.gd, d.cd, d.gr, d.cr = (_ptr(parts[k]) for k in ("gd", "cd", "gr", "cr"))
    d.s0, d.wtilde, d.l1_mass = _ptr(s0), _ptr(wt), _ptr(l1)
    c = ctx or _context_for(pos)
    c.check(L.hipster_bk_ell(c.handle, ct.byref(pts), ct.byref(rpts), float(f_rand), int(seed) & (2 ** 64 - 1),
                             ct.byref(prm), _ptr(out), ct.byref(d)))
    if not return_diag:
        return out
    info = dict(parts)
    info.update(s0=s0, wtilde=wt, l1_mass=l1, n_pairs=int(d.n_pairs), n_pairs_rand=int(d.n_pairs_rand),
                n_rand=int(d.n_rand), ms_build=d.ms_build, ms_pairs=d.ms_pairs, ms_sweep=d.ms_sweep,
                ms_total=d.ms_total, sweep_launches=int(d.sweep_launches), ms_cterm=d.ms_cterm)
    return out, info


def aniso_combos(ell_max: int):
    """(l1, l2, m) of hipster_bk_aniso's output rows: l1 <= l2 <= ell_max, m = 0..l1."""
    return [(l1, l2, m) for l1 in range(ell_max + 1) for l2 in range(l1, ell_max + 1) for m in range(l1 + 1)]


def bk_aniso(pos, w=None, randoms=None, rw=None, *, box: float, r0: float, k_edges, ell_max: int = 4,
             precision: str = "mixed", primary_mask=None, random_mask=None, f_rand: float = 0.0, seed: int = 0,
             ctx: Context | None = None, return_diag: bool = False) -> Any:
    """Anisotropic bispectrum multipoles B^ab_{l1 l2 m} about the z axis:
    float64 array (n_c, n_k, n_k), rows in the order of aniso_combos(ell_max).
    Random primaries as for bk_ell.  With return_diag, also the pair counts,
    the random count, W~^a and timings."""
    L = load_library()
    keep: list = []
    pts = _points(pos, w, keep)
    rpts = _points(randoms, rw, keep)
    prm = _params(box, r0, k_edges, ell_max, 2, precision, primary_mask, random_mask, keep)
    n_k = prm.n_k
    out = np.zeros((len(aniso_combos(ell_max)), n_k, n_k))
    wt = np.zeros(n_k)
    d = _Diag()
    d.wtilde = _ptr(wt)
    c = ctx or _context_for(pos)
    c.check(L.hipster_bk_aniso(c.handle, ct.byref(pts), ct.byref(rpts), float(f_rand), int(seed) & (2 ** 64 - 1),
                               ct.byref(prm), _ptr(out), ct.byref(d)))
    if not return_diag:
        return out
    return out, dict(wtilde=wt, n_pairs=int(d.n_pairs), n_pairs_rand=int(d.n_pairs_rand), n_rand=int(d.n_rand),
                     ms_build=d.ms_build, ms_sweep=d.ms_sweep, ms_cterm=d.ms_cterm, ms_total=d.ms_total)


def bk_ell_analytic(pos, w=None, *, box: float, r0: float, k_edges, ell_max: int = 4, n_x: int = 0,
                    precision: str = "mixed", primary_mask=None, ctx: Context | None = None,
                    return_diag: bool = False) -> Any:
    """Bispectrum multipoles B^ab_ell with the DDR^II term from the E^II kernel
    (no randoms): float64 array of shape (ell_max + 1, n_k, n_k).  n_x: E^II
    table intervals over [0, 2 R0] (0: the library's default).  With
    return_diag, also gd, cd, t2 (= sum_{i!=j} w_i w_j E^II), s0, W~^a, pair
    counts and timings."""
    L = load_library()
    keep: list = []
    pts = _points(pos, w, keep)
    prm = _params(box, r0, k_edges, ell_max, 2, precision, primary_mask, None, keep)
    n_k = prm.n_k
    shp = (ell_max + 1, n_k, n_k)
    out = np.zeros(shp)
    parts = {k: np.zeros(shp) for k in ("gd", "cd", "gr", "cr")}
    s0 = np.zeros(n_k)
    wt = np.zeros(n_k)
    l1 = np.zeros(shp)
    d = _Diag()
    d.gd, d.cd, d.gr, d.cr = (_ptr(parts[k]) for k in ("gd", "cd", "gr", "cr"))
    d.s0, d.wtilde, d.l1_mass = _ptr(s0), _ptr(wt), _ptr(l1)
    c = ctx or _context_for(pos)
    c.check(L.hipster_bk_ell_analytic(c.handle, ct.byref(pts), ct.byref(prm), int(n_x), _ptr(out), ct.byref(d)))
    if not return_diag:
        return out
    info = {"gd": parts["gd"], "cd": parts["cd"], "t2": parts["gr"]}
    info.update(s0=s0, wtilde=wt, l1_mass=l1, n_pairs=int(d.n_pairs), n_pairs_2r0=int(d.n_pairs_2r0), ms_build=d.ms_build,
                ms_sweep=d.ms_sweep, ms_eii_table=d.ms_eii_table, ms_ddr2=d.ms_ddr2, ms_total=d.ms_total,
                eii_nodes=int(d.eii_nodes), ms_cterm=d.ms_cterm)
    return out, info


def eii_table(r0: float, k_edges, ell_max: int, n_x: int, *, ctx: Context | None = None):
    """The E^{II,ab}_ell table on the nodes m 2 R0 / n_x, m = 0..n_x, computed
    on the GPU: float64 array of shape (ell_max + 1, n_k, n_k, n_x + 1)."""
    L = load_library()
    k = np.ascontiguousarray(k_edges, dtype=np.float64)
    n_k = k.size - 1
    out = np.zeros((ell_max + 1, n_k, n_k, n_x + 1))
    c = ctx or _context_for(None)
    c.check(L.hipster_eii_table(c.handle, float(r0), n_k, _ptr(k), int(ell_max), int(n_x), _ptr(out)))
    return out


def _host_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def omega(p, r0: float, k_edges, ell_max: int, *, ctx: Context | None = None) -> np.ndarray:
    """omega^a_ell(p; R0) for ell = 0..ell_max at the momenta p, computed on the
    GPU: float64 array (ell_max + 1, len(p), n_k)."""
    L = load_library()
    k, p = _host_f64(k_edges), _host_f64(p)
    out = np.zeros((ell_max + 1, p.size, k.size - 1))
    c = ctx or _context_for(None)
    c.check(L.hipster_omega(c.handle, float(r0), k.size - 1, _ptr(k), int(ell_max), p.size, _ptr(p), _ptr(out)))
    return out


def pk_window_theory(r0: float, k_edges, ell_max: int, r, wr, xi, *, ctx: Context | None = None) -> np.ndarray:
    """Windowed P^a_ell(R0) (even ell) of model multipoles xi (ell_max/2 + 1, len(r))
    on the quadrature (r, wr) over [0, R0]: (ell_max/2 + 1, n_k)."""
    L = load_library()
    k, r, wr = _host_f64(k_edges), _host_f64(r), _host_f64(wr)
    xi = _host_f64(xi).reshape(ell_max // 2 + 1, r.size)
    out = np.zeros((ell_max // 2 + 1, k.size - 1))
    c = ctx or _context_for(None)
    c.check(L.hipster_pk_window_theory(c.handle, float(r0), k.size - 1, _ptr(k), int(ell_max), r.size, _ptr(r),
                                       _ptr(wr), _ptr(xi), _ptr(out)))
    return out


def cov_gauss(r0: float, volume: float, k_edges, ell_max: int, p, wp, pk, *, ctx: Context | None = None) -> np.ndarray:
    """Gaussian covariance of the binned windowed multipoles (even ell) on the p
    quadrature (p, wp) with model multipoles pk (ell_max/2 + 1, len(p)):
    (n_ell, n_k, n_ell, n_k)."""
    L = load_library()
    k, p, wp = _host_f64(k_edges), _host_f64(p), _host_f64(wp)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    pk = _host_f64(pk).reshape(n_ell, p.size)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    c = ctx or _context_for(None)
    c.check(L.hipster_cov_gauss(c.handle, float(r0), float(volume), n_k, _ptr(k), int(ell_max), p.size, _ptr(p),
                                _ptr(wp), _ptr(pk), _ptr(out)))
    return out


def cov_poisson2(r0: float, nbar: float, volume: float, k_edges, ell_max: int, r, wr, xi, *,
                 ctx: Context | None = None) -> np.ndarray:
    """Poisson two-point covariance term (even ell) on the x quadrature (r, wr)
    over [0, R0] with model multipoles xi (ell_max/2 + 1, len(r)):
    (n_ell, n_k, n_ell, n_k)."""
    L = load_library()
    k, r, wr = _host_f64(k_edges), _host_f64(r), _host_f64(wr)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    xi = _host_f64(xi).reshape(n_ell, r.size)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    c = ctx or _context_for(None)
    c.check(L.hipster_cov_poisson2(c.handle, float(r0), float(nbar), float(volume), n_k, _ptr(k), int(ell_max),
                                   r.size, _ptr(r), _ptr(wr), _ptr(xi), _ptr(out)))
    return out


def cov_poisson3(r0: float, nbar: float, volume: float, k_edges, ell_max: int, p, wp, pk, pbin=None, bk=None, *,
                 ctx: Context | None = None) -> np.ndarray:
    """Poisson three-point covariance term (even ell) on the p quadrature
    (p, wp) with model P_L(p) (ell_max/2 + 1, len(p)), windowed binned
    multipoles pbin (ell_max/2 + 1, n_k) and bispectrum bk (ell_max/2 + 1,
    n_k, n_k), either None for zero: (n_ell, n_k, n_ell, n_k)."""
    L = load_library()
    k, p, wp = _host_f64(k_edges), _host_f64(p), _host_f64(wp)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    pk = _host_f64(pk).reshape(n_ell, p.size)
    pb = None if pbin is None else _host_f64(pbin).reshape(n_ell, n_k)
    bb = None if bk is None else _host_f64(bk).reshape(n_ell, n_k, n_k)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    c = ctx or _context_for(None)
    c.check(L.hipster_cov_poisson3(c.handle, float(r0), float(nbar), float(volume), n_k, _ptr(k), int(ell_max),
                                   p.size, _ptr(p), _ptr(wp), _ptr(pk), None if pb is None else _ptr(pb),
                                   None if bb is None else _ptr(bb), _ptr(out)))
    return out


def cov_nongauss(r0: float, volume: float, k_edges, ell_max: int, p, wp, tbar, *,
                 ctx: Context | None = None) -> np.ndarray:
    """Non-Gaussian intrinsic covariance term (even ell) on the p quadrature
    (p, wp) with collapsed-trispectrum multipoles tbar (n_ell, n_ell, len(p),
    len(p)): (n_ell, n_k, n_ell, n_k)."""
    L = load_library()
    k, p, wp = _host_f64(k_edges), _host_f64(p), _host_f64(wp)
    n_ell, n_k = ell_max // 2 + 1, k.size - 1
    tb = _host_f64(tbar).reshape(n_ell, n_ell, p.size, p.size)
    out = np.zeros((n_ell, n_k, n_ell, n_k))
    c = ctx or _context_for(None)
    c.check(L.hipster_cov_nongauss(c.handle, float(r0), float(volume), n_k, _ptr(k), int(ell_max), p.size, _ptr(p),
                                   _ptr(wp), _ptr(tb), _ptr(out)))
    return out


def batch(boxes, *, precision: str = "mixed", ctx: Context | None = None, return_diag: bool = False):
    """Many boxes in one pass.  `boxes` is a sequence of dicts with keys pos,
    w (optional), randoms (optional), box, r0, pk_edges / pk_ell_max (optional),
    bk_edges / bk_ell_max (optional), mask / rmask (optional primary masks of
    the data, for P and B, and of the randoms), f_rand / seed (optional: randoms drawn by
    the library when a bispectrum box has none) and bk_eii_nodes (optional:
    >= 0 takes the bispectrum's DDR^II term from the E^II kernel with that
    table size, 0 for the default, and ignores randoms).  Returns a list of dicts with 'pk'
    and/or 'bk' arrays and 'n_pairs'."""
    L = load_library()
    keep: list = []
    jobs = (_BoxJob * len(boxes))()
    outs = []
    for b, spec in enumerate(boxes):
        j = jobs[b]
        j.data = _points(spec["pos"], spec.get("w"), keep)
        j.randoms = _points(spec.get("randoms"), spec.get("rw"), keep)
        j.bk_eii_nodes = int(spec.get("bk_eii_nodes", -1))
        j.f_rand = float(spec.get("f_rand", 0.0))
        j.seed = int(spec.get("seed", 0)) & (2 ** 64 - 1)
        res = {}
        if spec.get("pk_edges") is not None:
            lm = spec.get("pk_ell_max", 4)
            j.pk_params = _params(spec["box"], spec["r0"], spec["pk_edges"], lm, spec.get("los_axis", 2), precision,
                                  spec.get("mask"), None, keep)
            res["pk"] = np.zeros((lm // 2 + 1, j.pk_params.n_k))
            j.pk = _ptr(res["pk"])
        else:
            j.pk_params = _Params(float(spec["box"]), float(spec["r0"]), 0, 0, None, 2, 0, None, None)
        if spec.get("bk_edges") is not None:
            lm = spec.get("bk_ell_max", 4)
            j.bk_params = _params(spec["box"], spec["r0"], spec["bk_edges"], lm, 2, precision, spec.get("mask"),
                                  spec.get("rmask"), keep)
            nk = j.bk_params.n_k
            res["bk"] = np.zeros((lm + 1, nk, nk))
            j.bk = _ptr(res["bk"])
        else:
            j.bk_params = _Params(float(spec["box"]), float(spec["r0"]), 0, 0, None, 2, 0, None, None)
        outs.append(res)
    d = _Diag()
    c = ctx or _context_for(boxes[0]["pos"])
    c.check(L.hipster_batch(c.handle, len(boxes), jobs, ct.byref(d)))
    for b, res in enumerate(outs):
        res["n_pairs"] = int(jobs[b].n_pairs)
    if return_diag:
        return outs, {"ms_build": d.ms_build, "ms_pairs": d.ms_pairs, "ms_sweep": d.ms_sweep,
                      "ms_total": d.ms_total, "sweep_launches": int(d.sweep_launches)}
    return outs
