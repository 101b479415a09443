"""GPU parity of the batched path: many boxes of uneven size, shape and R0
in one call; every box's P_ell and B_ell checked against the FP64 oracle,
including boxes drawn from the 64-box recipe (with primary subsets)."""
import os

import numpy as np
import pytest

import oracle
import synthetic
from test_gpu_pk import TOL, check, wtilde_mass
import test_gpu_bk as tbk

pytestmark = pytest.mark.gpu


def _boxes(seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(7):
        n = int(rng.integers(300, 3000)) // 10 * 10
        L = float(rng.uniform(60, 200))
        r0 = float(rng.uniform(8, 20))
        pos = synthetic.poisson(n, L, [seed, b], np.float32) if b % 2 == 0 else \
            synthetic.thomas(n, L, 10, 2.0, 1.0, [seed, b], np.float32)
        spec = dict(pos=pos, box=L, r0=r0, pk_edges=np.geomspace(1.0, 10.0, 13), pk_ell_max=4)
        if b % 3 == 0:
            spec.update(bk_edges=np.linspace(0.5, 3.0, 6), bk_ell_max=3,
                        randoms=synthetic.poisson(2 * n, L, [seed, b, 1], np.float32))
        out.append(spec)
    return out


def bk_scale(ref, lmax, L, nw, sR):
    """Scale of each B^ab_l entry: the sum of its terms' Cauchy-Schwarz scales."""
    sc = {k: tbk._scale(ref[k]) for k in ("gd", "cd", "gr", "cr")}
    fac = np.array([(2 * l + 1) for l in range(lmax + 1)])[:, None, None] / (L ** 3 * nw ** 3)
    out = fac * (sc["gd"] + sc["cd"] + sR * (sc["gr"] + sc["cr"]))
    wt = np.abs(ref["wtilde"])
    out[0] += (np.outer(wt, np.abs(ref["s0"])) + np.outer(np.abs(ref["s0"]), wt)) / (L ** 3 * nw ** 2) + 2 * np.outer(wt, wt)
    return out


def _check_boxes(specs, outs, precision):
    for spec, res in zip(specs, outs):
        mask = spec.get("mask")
        ref = oracle.pk_ell(spec["pos"], None, spec["box"], spec["r0"], spec["pk_edges"], 4, primary_mask=mask)
        assert res["n_pairs"] == ref["n_pairs"]
        V = spec["box"] ** 3
        nw = len(spec["pos"]) / V
        l1 = ref["l1"] / (nw * nw * V)
        l1[0] += wtilde_mass(spec["r0"], spec["pk_edges"])
        check(res["pk"], ref["pk"], l1, precision, "batch pk")
        if "bk" in res:
            rpos = spec.get("randoms")
            if rpos is None:
                rpos = oracle.philox_randoms(int(round(spec["f_rand"] * len(spec["pos"]))), spec["box"], spec["seed"])
            lm = spec["bk_ell_max"]
            rb = oracle.bk_ell(spec["pos"], None, rpos, None, spec["box"], spec["r0"], spec["bk_edges"], lm,
                               mask_d=mask, mask_r=spec.get("rmask"))
            sc = bk_scale(rb, lm, spec["box"], nw, len(spec["pos"]) / len(rpos))
            tbk.check(res["bk"], rb["bk"], sc, precision, "batch bk")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_matches_oracle(precision):
    import paper_2005_01739_amd as hp
    specs = _boxes()
    outs = hp.batch(specs, precision=precision)
    _check_boxes(specs, outs, precision)


def test_batch_rejects_table_form():
    # the table form is offered by hipster_pk_ell and hipster_pk_survey only
    import paper_2005_01739_amd as hp
    with pytest.raises(hp.HipsterError) as e:
        hp.batch(_boxes(1)[:1], precision="table")
    assert e.value.name == "HIPSTER_EUNSUPPORTED"


def test_batch_split_across_stream_chunks():
    # A tiny pair-stream capacity splits boxes across several work-queue
    # launches; results must agree with the unsplit run to rounding.
    import paper_2005_01739_amd as hp
    specs = _boxes(1)
    a = hp.batch(specs, precision="mixed")
    os.environ["HIPSTER_PAIR_CHUNK"] = "5000"
    try:
        b = hp.batch(specs, precision="mixed")
    finally:
        del os.environ["HIPSTER_PAIR_CHUNK"]
    for x, y in zip(a, b):
        assert x["n_pairs"] == y["n_pairs"]
        assert np.allclose(x["pk"], y["pk"], rtol=1e-12, atol=1e-12 * np.abs(x["pk"]).max())
    _check_boxes(specs, b, "mixed")


def test_batch_generated_randoms():
    # bispectrum boxes without a catalogue draw f_rand N randoms from their seed
    import paper_2005_01739_amd as hp
    specs = _boxes(3)
    for b, spec in enumerate(specs):
        if "randoms" in spec:
            del spec["randoms"]
            spec.update(f_rand=2.0, seed=100 + b)
    outs = hp.batch(specs, precision="mixed")
    _check_boxes(specs, outs, "mixed")


def test_batch_full_and_partial_bin_groups():
    # One queued bispectrum sweep holding a box whose 16 bins fill the group
    # of edges (its steps carry the top-edge sums) beside boxes with fewer
    # bins (their top-edge sums are zero); every box against the oracle.
    import paper_2005_01739_amd as hp
    specs = []
    for b, nb in enumerate((16, 5, 11)):
        n = 800 + 200 * b
        L = 80.0 + 10.0 * b
        pos = synthetic.thomas(n, L, 10, 2.0, 1.0, [21, b], np.float32)
        specs.append(dict(pos=pos, box=L, r0=12.0, pk_edges=np.geomspace(1.0, 10.0, 13), pk_ell_max=4,
                          bk_edges=np.geomspace(0.3, 3.0, nb + 1), bk_ell_max=3,
                          randoms=synthetic.poisson(2 * n, L, [21, b, 1], np.float32)))
    outs = hp.batch(specs, precision="mixed")
    _check_boxes(specs, outs, "mixed")


def test_batch_64_box_recipe_subset():
    # The 64-box recipe (N log-uniform in [1e5, 4e6] scaled by 0.1, L in
    # [250, 1500], R0 in [15, 50], half Poisson, half Thomas; P with 30 log
    # bins, B with 10 linear bins and ell_max = 4, f_rand = 3 randoms drawn by
    # the library), every box checked against the oracle on 24 data and 24
    # random primaries.
    import paper_2005_01739_amd as hp
    specs = []
    for b, wl in enumerate(synthetic.batch_boxes(64, scale=0.1)):
        rng = np.random.default_rng([9, b])
        mask = np.zeros(wl.n, np.uint8)
        mask[rng.choice(wl.n, min(24, wl.n), replace=False)] = 1
        n_r = int(round(3.0 * wl.n))
        rmask = np.zeros(n_r, np.uint8)
        rmask[rng.choice(n_r, min(24, n_r), replace=False)] = 1
        specs.append(dict(pos=wl.pos, box=wl.box, r0=wl.r0, pk_edges=wl.k_edges_p, pk_ell_max=wl.ell_max_p,
                          bk_edges=wl.k_edges_b, bk_ell_max=wl.ell_max_b, f_rand=3.0, seed=wl.seed, mask=mask,
                          rmask=rmask))
    outs = hp.batch(specs, precision="mixed")
    _check_boxes(specs, outs, "mixed")


def test_batch_deterministic():
    import paper_2005_01739_amd as hp
    specs = _boxes(2)
    a = hp.batch(specs)
    b = hp.batch(specs)
    for x, y in zip(a, b):
        assert np.array_equal(x["pk"], y["pk"])


def test_batch_analytic_ddr2_matches_oracle():
    # the randoms-free bispectrum in a batch: each box's B against the oracle's
    # analytic estimator (its own table), and against the single call to FP64
    # rounding (the batch's queued sweep adds each box's quads in task order,
    # the single call in per-wave rows)
    import paper_2005_01739_amd as hp
    specs = []
    rng = np.random.default_rng(5)
    for b in range(4):
        n = int(rng.integers(400, 1500)) // 10 * 10
        L = float(rng.uniform(60, 120))
        r0 = float(rng.uniform(8, 15))
        pos = synthetic.thomas(n, L, 10, 2.0, 0.0, [5, b], np.float32)
        specs.append(dict(pos=pos, box=L, r0=r0, bk_edges=np.linspace(0.2, 1.0, 5), bk_ell_max=2,
                          bk_eii_nodes=64, randoms=synthetic.poisson(n, L, [5, b, 1], np.float32)))
    outs = hp.batch(specs, precision="mixed")
    for spec, res in zip(specs, outs):
        single = hp.bk_ell_analytic(spec["pos"], box=spec["box"], r0=spec["r0"], k_edges=spec["bk_edges"],
                                    ell_max=2, n_x=64, precision="mixed")
        assert np.allclose(res["bk"], single, rtol=1e-10, atol=1e-10 * np.abs(single).max())
        ref = oracle.bk_ell_analytic(spec["pos"], None, spec["box"], spec["r0"], spec["bk_edges"], 2, 64)
        scale = np.abs(ref["bk"]).max()
        assert np.allclose(res["bk"], ref["bk"], rtol=1e-6, atol=1e-7 * scale)
