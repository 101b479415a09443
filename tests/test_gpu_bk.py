"""GPU parity of the bispectrum path (C ABI via the binding) against the FP64
oracle.  Integer pair counts (data-data and random-data) must match exactly.
Per entry, the FP64 form must agree to 1e-12 relative and the mixed form to
1e-6 relative; an entry dominated by cancellation may instead meet a scaled
bound |err| / scale <= 1e-14 (FP64) or 2^-24 (mixed), where the scale of a
Gram entry X^ab_l (X = G or C, positive semi-definite in (a, b)) is
sqrt(X^aa_l X^bb_l), and the scale of B^ab_l is the sum of its terms' scales."""
import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-14), "mixed": (1e-6, 2.0 ** -24)}


def _scale(X):
    d = np.sqrt(np.abs(np.einsum("lii->li", X)))
    return d[:, :, None] * d[:, None, :]


def check(got, ref, scale, precision, what):
    rel_tol, sc_tol = TOL[precision]
    err = np.abs(got - ref)
    rel = err / np.maximum(np.abs(ref), 1e-300)
    scn = err / np.maximum(scale, 1e-300)
    ok = (rel <= rel_tol) | (scn <= sc_tol)
    assert ok.all(), f"{what}: worst rel {rel.max():.3e}, worst scaled {scn.max():.3e}, failing {np.argwhere(~ok)[:6].tolist()}"


def run_case(pos, w, rpos, rw, L, r0, k, lmax, precision, mask=None, rmask=None, device=True):
    import torch
    import paper_2005_01739_amd as hp
    ref = oracle.bk_ell(pos, w, rpos, rw, L, r0, k, lmax, mask_d=mask, mask_r=rmask)
    if device:
        t = lambda a: None if a is None else torch.from_numpy(a).cuda()
        args = (t(pos), t(w), t(rpos), t(rw))
    else:
        args = (pos, w, rpos, rw)
    got, info = hp.bk_ell(*args, box=L, r0=r0, k_edges=k, ell_max=lmax, precision=precision,
                          primary_mask=mask, random_mask=rmask, return_diag=True)
    assert info["n_pairs"] == ref["n_pairs_dd"]
    assert info["n_pairs_rand"] == ref["n_pairs_rd"]
    scales = {}
    for name in ("gd", "cd", "gr", "cr"):
        scales[name] = _scale(ref[name])
        check(info[name], ref[name], scales[name], precision, name)
    s0_scale = np.abs(ref["s0"]) + 1e-300
    check(info["s0"], ref["s0"], np.full_like(s0_scale, np.abs(ref["s0"]).max()), precision, "s0")
    V = L ** 3
    p1 = len(pos) if w is None else float(np.sum(np.asarray(w, np.float64)))
    nw = p1 / V
    nr = 0 if rpos is None else len(rpos)
    pr = nr if rw is None else float(np.sum(np.asarray(rw, np.float64)))
    sR = p1 / pr if nr else 0.0
    fac = np.array([(2 * l + 1) for l in range(lmax + 1)])[:, None, None] / (V * nw ** 3)
    sc = fac * (scales["gd"] + scales["cd"] + sR * (scales["gr"] + scales["cr"]))
    wt = np.abs(ref["wtilde"])
    sc[0] += (np.outer(wt, np.abs(ref["s0"])) + np.outer(np.abs(ref["s0"]), wt)) / (V * nw ** 2) + 2 * np.outer(wt, wt)
    check(got, ref["bk"], sc, precision, "bk")
    return info


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_thomas_with_randoms_lmax5(precision):
    L = 200.0
    pos = synthetic.thomas(3000, L, 10, 3.0, 0.0, 3, np.float32)
    rpos = synthetic.poisson(9000, L, 4, np.float32)
    run_case(pos, None, rpos, None, L, 20.0, np.linspace(0.5, 3.0, 7), 5, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_weighted_masked_host_input(precision):
    L = 120.0
    pos = synthetic.thomas(1600, L, 16, 1.0, 0.0, 5, np.float32)
    w = synthetic.uniform_weights(1600, 6, np.float32)
    rpos = synthetic.poisson(4800, L, 7, np.float32)
    mask = (np.arange(1600) % 2 == 0).astype(np.uint8)
    rmask = (np.arange(4800) % 3 == 0).astype(np.uint8)
    run_case(pos, w, rpos, None, L, 15.0, np.geomspace(2.0, 20.0, 9), 4, precision, mask, rmask, device=False)


def test_no_randoms_and_small_grid():
    L = 30.0
    pos = synthetic.poisson(300, L, 8, np.float64)
    run_case(pos, None, None, None, L, 15.0, np.linspace(0.1, 1.5, 5), 3, "fp64")


def test_coincident_points_zero_k_edge():
    L = 40.0
    pos = synthetic.poisson(300, L, 9, np.float64)
    pos = np.concatenate([pos, pos[:30]])
    rpos = synthetic.poisson(300, L, 10, np.float64)
    run_case(pos, None, rpos, None, L, 8.0, np.linspace(0.0, 2.0, 5), 2, "fp64")
    run_case(pos, None, rpos, None, L, 8.0, np.linspace(0.0, 2.0, 5), 2, "mixed")


def test_full_size_bispectrum_workload_subset():
    # The full 5e5-point Thomas catalogue with its 1.5e6 randoms; exact
    # parity on a fixed subset of 48 data and 48 random primaries.
    wl = synthetic.workload(3)
    rpos = wl.randoms()
    rng = np.random.default_rng(1)
    mask = np.zeros(wl.n, np.uint8)
    mask[rng.choice(wl.n, 48, replace=False)] = 1
    rmask = np.zeros(len(rpos), np.uint8)
    rmask[rng.choice(len(rpos), 48, replace=False)] = 1
    run_case(wl.pos, None, rpos, None, wl.box, wl.r0, wl.k_edges_b, wl.ell_max_b, "mixed", mask, rmask)


def test_deterministic_bitwise():
    import torch
    import paper_2005_01739_amd as hp
    L = 300.0
    pos = torch.from_numpy(synthetic.thomas(20000, L, 10, 3.0, 0.0, 11, np.float32)).cuda()
    rpos = torch.from_numpy(synthetic.poisson(60000, L, 12, np.float32)).cuda()
    k = np.linspace(0.5, 3.0, 13)
    a = hp.bk_ell(pos, None, rpos, box=L, r0=30.0, k_edges=k, ell_max=5)
    b = hp.bk_ell(pos, None, rpos, box=L, r0=30.0, k_edges=k, ell_max=5)
    assert np.array_equal(a, b)
