"""GPU parity of the bispectrum path (C ABI via the binding) against the FP64
oracle.  Integer pair counts (data-data and random-data) must match exactly.
Per entry, the FP64 form must agree to 1e-12 relative and the mixed form to
1e-6 relative; an entry dominated by cancellation may instead meet a scaled
bound |err| / scale <= 1e-14 (FP64) or 2^-24 (mixed), where the scale of a
Gram entry X^ab_l (X = G or C, positive semi-definite in (a, b)) is
sqrt(X^aa_l X^bb_l), and the scale of B^ab_l is the sum of its terms' scales.
The scaled bound applies only to entries whose condition number (scale /
|value|) exceeds 1e2; better-conditioned entries must meet the relative
bound."""
import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-14), "mixed": (1e-6, 2.0 ** -24)}
KAPPA_MIN = 1e2


def _scale(X):
    d = np.sqrt(np.abs(np.einsum("lii->li", X)))
    return d[:, :, None] * d[:, None, :]


def check(got, ref, scale, precision, what):
    rel_tol, sc_tol = TOL[precision]
    err = np.abs(got - ref)
    rel = err / np.maximum(np.abs(ref), 1e-300)
    scn = err / np.maximum(scale, 1e-300)
    kappa = scale / np.maximum(np.abs(ref), 1e-300)
    ok = (rel <= rel_tol) | ((scn <= sc_tol) & (kappa > KAPPA_MIN))
    assert ok.all(), f"{what}: worst rel {rel.max():.3e}, worst scaled {scn.max():.3e}, failing {np.argwhere(~ok)[:6].tolist()}"


def run_case(pos, w, rpos, rw, L, r0, k, lmax, precision, mask=None, rmask=None, device=True, gen=None):
    """gen = (f_rand, seed): the library draws the randoms (rpos must be the
    oracle's copy of that catalogue, oracle.philox_randoms)."""
    import torch
    import paper_2005_01739_amd as hp
    ref = oracle.bk_ell(pos, w, rpos, rw, L, r0, k, lmax, mask_d=mask, mask_r=rmask)
    if device:
        t = lambda a: None if a is None else torch.from_numpy(a).cuda()
        args = (t(pos), t(w), t(rpos), t(rw))
    else:
        args = (pos, w, rpos, rw)
    extra = {}
    if gen is not None:
        args = args[:2] + (None, None)
        extra = dict(f_rand=gen[0], seed=gen[1])
    got, info = hp.bk_ell(*args, box=L, r0=r0, k_edges=k, ell_max=lmax, precision=precision,
                          primary_mask=mask, random_mask=rmask, return_diag=True, **extra)
    if gen is not None:
        assert info["n_rand"] == len(rpos)
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_generated_randoms_and_small_grid(precision):
    # no catalogue: the library draws round(f_rand N) Philox randoms from the
    # seed; the oracle uses its own copy of that catalogue
    L = 30.0
    pos = synthetic.poisson(300, L, 8, np.float64)
    rpos = oracle.philox_randoms(750, L, 123456789)
    run_case(pos, None, rpos, None, L, 15.0, np.linspace(0.1, 1.5, 5), 3, precision, gen=(2.5, 123456789))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_clump_and_sparse_primaries(precision):
    # A dense clump (700 points, sigma 0.3) among sparse background points,
    # plus a shell of primaries 5 from its centre.  Cells then hold primaries
    # with ~700 neighbours beside primaries with ~15, so quads mix very
    # different rows; a clump row's near ring and a shell row's far ring
    # (bins from k = 2: pairs beyond r = 4 are far) each take hundreds of hits
    # in a burst, which forces batches with idle rows before a ring overflows.
    L, r0 = 40.0, 8.0
    rng = np.random.default_rng(71)
    centre = np.array([20.0, 20.0, 20.0])
    clump = centre + rng.normal(scale=0.3, size=(700, 3))
    d = rng.normal(size=(60, 3))
    shell = centre + 5.0 * d / np.linalg.norm(d, axis=1)[:, None]
    background = rng.random((400, 3)) * L
    pos = np.ascontiguousarray(np.concatenate([clump, shell, background]) % L)
    rpos = rng.random((600, 3)) * L
    k = np.geomspace(2.0, 12.0, 9)
    info = run_case(pos, None, rpos, None, L, r0, k, 4, precision)
    assert info["n_pairs"] > 700 * 650


def test_generated_randoms_equal_given_catalogue():
    # the drawn catalogue is exactly the oracle's: same bits as passing it
    import paper_2005_01739_amd as hp
    L = 80.0
    pos = synthetic.thomas(2000, L, 10, 2.0, 0.0, 41, np.float32)
    seed = 2 ** 63 + 977
    rpos = oracle.philox_randoms(6000, L, seed)
    k = np.linspace(0.5, 3.0, 9)
    a = hp.bk_ell(pos, None, rpos, box=L, r0=12.0, k_edges=k, ell_max=4)
    b = hp.bk_ell(pos, box=L, r0=12.0, k_edges=k, ell_max=4, f_rand=3.0, seed=seed)
    assert np.array_equal(a, b)


def test_missing_randoms_is_an_error():
    import paper_2005_01739_amd as hp
    pos = synthetic.poisson(300, 30.0, 8, np.float64)
    for f in (0.0, -1.0, float("nan")):
        with pytest.raises(hp.HipsterError) as e:
            hp.bk_ell(pos, box=30.0, r0=10.0, k_edges=[0.1, 0.5], ell_max=2, f_rand=f)
        assert e.value.name == "HIPSTER_EINVAL"


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


@pytest.mark.parametrize("n_k,lmax", [(17, 2), (40, 6), (20, 4)])
def test_more_than_16_bins(n_k, lmax):
    # more than 16 bins: groups of 16 bins, A through a buffer and the Gram
    # as a separate matrix-core contraction (the paper's 40- and 60-bin runs)
    L = 150.0
    pos = synthetic.thomas(1500, L, 10, 2.0, 0.0, 43 + n_k, np.float32)
    rpos = synthetic.poisson(3000, L, 44 + n_k, np.float32)
    run_case(pos, None, rpos, None, L, 20.0, np.linspace(0.05, 2.5, n_k + 1), lmax, "mixed")


def test_60_bins_weighted_masked():
    L = 120.0
    pos = synthetic.thomas(1200, L, 8, 1.5, 0.0, 47, np.float32)
    w = synthetic.uniform_weights(1200, 48, np.float32)
    mask = (np.arange(1200) % 2 == 1).astype(np.uint8)
    rpos = oracle.philox_randoms(2400, L, 49)
    rmask = (np.arange(2400) % 3 == 1).astype(np.uint8)
    run_case(pos, w, rpos, None, L, 15.0, np.geomspace(0.2, 4.0, 61), 2, "mixed", mask, rmask, gen=(2.0, 49))


def test_size_limits():
    import paper_2005_01739_amd as hp
    pos = synthetic.poisson(300, 60.0, 8, np.float64)
    rpos = synthetic.poisson(300, 60.0, 9, np.float64)
    with pytest.raises(hp.HipsterError) as e:  # the FP64 form sums C per pair: at most 16 bins
        hp.bk_ell(pos, None, rpos, box=60.0, r0=10.0, k_edges=np.linspace(0.1, 2, 18), ell_max=2, precision="fp64")
    assert e.value.name == "HIPSTER_EUNSUPPORTED"
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_ell(pos, None, rpos, box=60.0, r0=10.0, k_edges=np.linspace(0.1, 2, 66), ell_max=2)
    assert e.value.name == "HIPSTER_EUNSUPPORTED"
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_ell(pos, None, rpos, box=60.0, r0=10.0, k_edges=np.linspace(0.1, 2, 5), ell_max=7)
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError) as e:  # E^II tables: at most 16 bins
        hp.bk_ell_analytic(pos, box=60.0, r0=10.0, k_edges=np.linspace(0.1, 2, 18), ell_max=2)
    assert e.value.name == "HIPSTER_EUNSUPPORTED"


def test_full_size_large_box_subset():
    # The 2^24-point weighted Thomas box with its bispectrum binning (16 log
    # bins over 2-20 h/Mpc, ell_max = 4, R0 = 15) and f_rand = 3 randoms drawn
    # by the library (5.0e7 points), exact parity on 48 data and 48 random
    # primaries against all 16.7M secondaries.
    import gc
    wl = synthetic.workload(5)
    n_r = int(round(3.0 * wl.n))
    rpos = oracle.philox_randoms(n_r, wl.box, 5)
    rng = np.random.default_rng(11)
    mask = np.zeros(wl.n, np.uint8)
    mask[rng.choice(wl.n, 48, replace=False)] = 1
    rmask = np.zeros(n_r, np.uint8)
    rmask[rng.choice(n_r, 48, replace=False)] = 1
    info = run_case(wl.pos, wl.weights, rpos, None, wl.box, wl.r0, wl.k_edges_b, wl.ell_max_b, "mixed", mask, rmask,
                    gen=(3.0, 5))
    assert info["n_pairs"] > 0 and info["n_pairs_rand"] > 0
    del rpos
    gc.collect()


def test_full_size_large_box_analytic_subset():
    # the same box through the randoms-free form: the data-primary sums at the
    # full binning, and the 2R0 pair sum T with 3 bins (the oracle's E^II
    # table is slow), on 48 primaries
    import torch
    import paper_2005_01739_amd as hp
    wl = synthetic.workload(5)
    mask = np.zeros(wl.n, np.uint8)
    mask[np.random.default_rng(12).choice(wl.n, 48, replace=False)] = 1
    pos, w = torch.from_numpy(wl.pos).cuda(), torch.from_numpy(wl.weights).cuda()
    ref = oracle.bk_ell(wl.pos, wl.weights, None, None, wl.box, wl.r0, wl.k_edges_b, wl.ell_max_b, mask_d=mask)
    got, info = hp.bk_ell_analytic(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=wl.ell_max_b,
                                   precision="mixed", primary_mask=mask, return_diag=True)
    assert info["n_pairs"] == ref["n_pairs_dd"]
    for name in ("gd", "cd"):
        check(info[name], ref[name], _scale(ref[name]), "mixed", name)
    check(info["s0"], ref["s0"], np.full(len(ref["s0"]), np.abs(ref["s0"]).max()), "mixed", "s0")
    k3 = np.geomspace(2.0, 20.0, 4)
    t_ref = oracle.ddr2(wl.pos, wl.weights, wl.box, wl.r0, k3, 1, 64, mask=mask)
    _, i3 = hp.bk_ell_analytic(pos, w, box=wl.box, r0=wl.r0, k_edges=k3, ell_max=1, n_x=64, precision="mixed",
                               primary_mask=mask, return_diag=True)
    assert i3["n_pairs_2r0"] == t_ref["n_pairs"]
    err = np.abs(i3["t2"] - t_ref["t2"])
    assert (err <= 1e-9 * t_ref["l1"]).all(), (err / t_ref["l1"]).max()


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
    k40 = np.linspace(0.5, 3.0, 41)
    a = hp.bk_ell(pos, None, rpos, box=L, r0=30.0, k_edges=k40, ell_max=2)
    b = hp.bk_ell(pos, None, rpos, box=L, r0=30.0, k_edges=k40, ell_max=2)
    assert np.array_equal(a, b)
