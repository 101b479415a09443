"""Seeded synthetic catalogues for the periodic-box pair-sweep estimators.

This module only draws random numbers and lays out arrays; it holds none of
the estimator's arithmetic.  Both the FP64 CPU oracle's tests and the GPU
path's tests and benchmark draw their inputs from here, so the two sides see
byte-identical catalogues.

Recipes (all FP64 internally, wrapped into [0, L) with ``np.mod`` and then cast
to the stated dtype; a coordinate that rounds up to L after the cast is set to
0 so that every coordinate satisfies 0 <= x < L):

* ``poisson(N, L)``: N points uniform in the cube.
* ``thomas(N, L, c, sigma, sigma_z)``: N/c parents uniform in the cube, each
  with exactly c children displaced by N(0, sigma^2) per axis, plus an extra
  N(0, sigma_z^2) displacement along z when sigma_z > 0 (a stand-in for
  redshift-space anisotropy).
* ``randoms(N_R, L)``: uniform random catalogue for the bispectrum's
  random-primary term, drawn from ``default_rng(seed + 1)``.
* weights, when asked for, are U[0.5, 1.5] drawn after the positions.
* ``survey(N, ...)``: a survey-like region seen by an observer at the origin:
  the cube [-h, h]^2 x [d, d + 2h] (default h = 500, d = 1000 Mpc/h), a Thomas
  catalogue wrapped into it and 3N uniform randoms over it (no periodicity is
  implied: the wrap only keeps every point inside the region).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "poisson", "thomas", "uniform_weights", "randoms", "Workload", "workload",
    "batch_boxes", "WORKLOADS", "survey", "Survey",
]


def _wrap_cast(x: np.ndarray, L: float, dtype) -> np.ndarray:
    x = np.mod(x, L)
    out = x.astype(dtype)
    out[out >= dtype(L)] = dtype(0)
    return np.ascontiguousarray(out)


def poisson(n: int, L: float, seed, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _wrap_cast(rng.uniform(0.0, L, size=(n, 3)), L, dtype)


def thomas(n: int, L: float, c: int, sigma: float, sigma_z: float, seed,
           dtype=np.float32, rng=None) -> np.ndarray:
    if n % c:
        raise ValueError("N must be a multiple of the children per parent")
    rng = np.random.default_rng(seed) if rng is None else rng
    parents = rng.uniform(0.0, L, size=(n // c, 3))
    x = np.repeat(parents, c, axis=0) + rng.normal(0.0, sigma, size=(n, 3))
    if sigma_z > 0:
        x[:, 2] += rng.normal(0.0, sigma_z, size=n)
    return _wrap_cast(x, L, dtype)


def uniform_weights(n: int, seed, dtype=np.float32, lo=0.5, hi=1.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, size=n).astype(dtype))


def randoms(n: int, L: float, seed, dtype=np.float32) -> np.ndarray:
    return poisson(n, L, seed + 1 if isinstance(seed, int) else seed, dtype)


@dataclasses.dataclass
class Workload:
    """One synthetic workload: a catalogue plus the estimator's parameters."""
    name: str
    pos: np.ndarray
    weights: np.ndarray | None
    box: float
    r0: float
    k_edges_p: np.ndarray | None      # power-spectrum bin edges (None: no P)
    ell_max_p: int
    k_edges_b: np.ndarray | None      # bispectrum bin edges (None: no B)
    ell_max_b: int
    f_rand: float = 3.0
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def randoms(self, dtype=None) -> np.ndarray:
        dt = self.pos.dtype.type if dtype is None else dtype
        return randoms(int(round(self.f_rand * self.n)), self.box, self.seed, dt)


def _w1(scale=1.0):
    return Workload(
        "pk_fp64_poisson_1e5", poisson(int(100_000 * scale), 1000.0, 1, np.float64), None,
        1000.0, 50.0, np.linspace(0.2, 2.0, 21), 4, None, 0, seed=1)


def _w2(scale=1.0):
    n = int(2_000_000 * scale) // 10 * 10
    return Workload(
        "pk_mixed_thomas_2e6", thomas(n, 1000.0, 10, 2.0, 4.0, 2, np.float32), None,
        1000.0, 25.0, np.geomspace(1.0, 10.0, 41), 4, None, 0, seed=2)


def _w3(scale=1.0):
    n = int(500_000 * scale) // 10 * 10
    return Workload(
        "bk_thomas_5e5", thomas(n, 500.0, 10, 3.0, 0.0, 3, np.float32), None,
        500.0, 30.0, None, 0, np.linspace(0.5, 3.0, 13), 5, seed=3)


def _w5(scale=1.0):
    n = int(16_777_216 * scale) // 16 * 16
    rng = np.random.default_rng(5)
    pos = thomas(n, 1000.0, 16, 1.0, 0.0, None, np.float32, rng=rng)
    w = np.ascontiguousarray(rng.uniform(0.5, 1.5, size=n).astype(np.float32))
    return Workload(
        "pk_bk_thomas_2p24_weighted", pos, w, 1000.0, 15.0,
        np.geomspace(2.0, 20.0, 61), 4, np.geomspace(2.0, 20.0, 17), 4, seed=5)


WORKLOADS = {1: _w1, 2: _w2, 3: _w3, 5: _w5}


def workload(idx: int, scale: float = 1.0) -> Workload:
    """Workload ``idx`` (1, 2, 3, 5); ``scale`` shrinks N for quick tests."""
    return WORKLOADS[idx](scale)


def batch_boxes(n_boxes: int = 64, scale: float = 1.0):
    """Many independent boxes of uneven size for the batched path.

    Box parameters are drawn from ``default_rng(4)`` in the order log10 N ~
    U(5, log10 4e6), L ~ U(250, 1500), R0 ~ U(15, 50); box b draws its points
    from ``default_rng([4, b])``, Poisson for even b and Thomas (c=10,
    sigma=2) for odd b.  Each box carries P bins geomspace(1, 10, 31) with
    ell = 0, 2, 4 and B bins linspace(0.5, 3, 11) with ell_max = 4.
    """
    rng = np.random.default_rng(4)
    logn = rng.uniform(5.0, np.log10(4e6), size=n_boxes)
    Ls = rng.uniform(250.0, 1500.0, size=n_boxes)
    r0s = rng.uniform(15.0, 50.0, size=n_boxes)
    out = []
    for b in range(n_boxes):
        n = max(20, int(10 ** logn[b] * scale) // 10 * 10)
        if b % 2 == 0:
            pos = poisson(n, Ls[b], [4, b], np.float32)
        else:
            pos = thomas(n, Ls[b], 10, 2.0, 0.0, [4, b], np.float32)
        out.append(Workload(f"box{b}", pos, None, float(Ls[b]), float(r0s[b]),
                            np.geomspace(1.0, 10.0, 31), 4,
                            np.linspace(0.5, 3.0, 11), 4, seed=4000 + b))
    return out


@dataclasses.dataclass
class Survey:
    """A survey-geometry workload: data and randoms in a region seen from the
    origin, with the power-spectrum parameters."""
    name: str
    pos: np.ndarray
    randoms: np.ndarray
    volume: float
    r0: float
    k_edges: np.ndarray
    ell_max: int

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def survey(n: int = 1_000_000, f_rand: float = 3.0, half: float = 500.0, dist: float = 1000.0,
           c: int = 10, sigma: float = 2.0, seed: int = 6, dtype=np.float32, r0: float = 25.0,
           k_edges=None, ell_max: int = 4) -> Survey:
    """Thomas catalogue (n/c parents, c children, N(0, sigma^2) offsets) and
    f_rand * n uniform randoms in [-half, half]^2 x [dist, dist + 2 half];
    default bins geomspace(1, 10, 41), ell = 0, 2, 4, R0 = 25."""
    side = 2.0 * half
    lo = np.array([-half, -half, dist])
    pos = thomas(n // c * c, side, c, sigma, 0.0, seed, np.float64)
    pos = np.ascontiguousarray((pos + lo).astype(dtype))
    rnd = poisson(int(round(f_rand * (n // c * c))), side, seed + 1, np.float64)
    rnd = np.ascontiguousarray((rnd + lo).astype(dtype))
    k = np.geomspace(1.0, 10.0, 41) if k_edges is None else np.asarray(k_edges, dtype=np.float64)
    return Survey(f"survey_thomas_{n}", pos, rnd, side ** 3, r0, k, ell_max)
