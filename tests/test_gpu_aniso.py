"""GPU parity of the anisotropic bispectrum (hipster_bk_aniso, C ABI via the
binding) against the FP64 oracle's anisotropic estimator.  Pair counts must
match exactly.  Per entry, the mixed form must agree to 1e-6 relative, or,
where the entry is dominated by cancellation (condition number above 1e2),
to 2^-24 of its scale: the sum over its terms of the Cauchy-Schwarz bound
sqrt(|X^aa_{l1 l1 m}| |X^bb_{l2 l2 m}|) of the Gram-type sums X = G, C (an
inner product of the per-primary vectors A^a_{l1 mu}, A^b_{l2 mu}), plus the
sizes of the analytic terms."""
import numpy as np
import pytest

import oracle
import synthetic
from test_gpu_bk import check

pytestmark = pytest.mark.gpu


def _aniso_scale(X, combos):
    """sqrt(|X^aa_{l1 l1 m}| |X^bb_{l2 l2 m}|) for every combination."""
    idx = {c: i for i, c in enumerate(combos)}
    out = np.zeros_like(X)
    for i, (l1, l2, m) in enumerate(combos):
        d1 = np.sqrt(np.abs(np.diag(X[idx[(l1, l1, m)]])))
        d2 = np.sqrt(np.abs(np.diag(X[idx[(l2, l2, m)]])))
        out[i] = np.outer(d1, d2)
    return out


def run_case(pos, w, rpos, L, r0, k, lmax, mask=None, rmask=None, gen=None, device=True):
    import torch
    import paper_2005_01739_amd as hp
    ref = oracle.bk_aniso(pos, w, rpos, None, L, r0, k, lmax, mask_d=mask, mask_r=rmask)
    t = (lambda a: None if a is None else torch.from_numpy(a).cuda()) if device else (lambda a: a)
    extra = {}
    rarg = t(rpos)
    if gen is not None:
        rarg = None
        extra = dict(f_rand=gen[0], seed=gen[1])
    got, info = hp.bk_aniso(t(pos), t(w), rarg, box=L, r0=r0, k_edges=k, ell_max=lmax, primary_mask=mask,
                            random_mask=rmask, return_diag=True, **extra)
    assert [tuple(c) for c in ref["combos"]] == hp.aniso_combos(lmax)
    assert info["n_pairs"] == ref["n_pairs_dd"]
    assert info["n_pairs_rand"] == ref["n_pairs_rd"]
    combos = ref["combos"]
    V = L ** 3
    p1 = len(pos) if w is None else float(np.sum(w))
    nw = p1 / V
    sR = p1 / len(rpos)
    sc = 4 * np.pi / (V * nw ** 3) * (_aniso_scale(ref["gd"], combos) + _aniso_scale(ref["cd"], combos)
                                     + sR * (_aniso_scale(ref["gr"], combos) + _aniso_scale(ref["cr"], combos)))
    wt = np.abs(info["wtilde"])
    t_abs = np.abs(ref["t"])
    for i, (l1, l2, m) in enumerate(combos):
        if m == 0:
            if l2 == 0:
                sc[i] += np.sqrt(4 * np.pi) / (V * nw ** 2) * np.outer(t_abs[l1], wt)
            if l1 == 0:
                sc[i] += np.sqrt(4 * np.pi) / (V * nw ** 2) * np.outer(wt, t_abs[l2])
            if l1 == 0 and l2 == 0:
                sc[i] += 2 * np.outer(wt, wt)
    check(got, ref["bk"], sc, "mixed", "aniso bk")
    return got, ref, info


def test_thomas_with_randoms_lmax4():
    L, r0 = 80.0, 14.0
    pos = synthetic.thomas(1500, L, 10, 2.0, 1.0, 31, np.float64)
    rpos = synthetic.poisson(3000, L, 32, np.float64)
    run_case(pos, None, rpos, L, r0, np.linspace(0.3, 2.0, 9), 4)


def test_weighted_masked_float32_host_input():
    L, r0 = 100.0, 20.0
    pos = synthetic.thomas(2000, L, 10, 3.0, 0.0, 33, np.float32)
    w = synthetic.uniform_weights(2000, 34, np.float32)
    rpos = synthetic.poisson(4000, L, 35, np.float32)
    rng = np.random.default_rng(36)
    mask = (rng.random(2000) < 0.4).astype(np.uint8)
    rmask = (rng.random(4000) < 0.3).astype(np.uint8)
    run_case(pos, w, rpos, L, r0, np.geomspace(0.2, 2.5, 13), 3, mask=mask, rmask=rmask, device=False)


def test_generated_randoms_16_bins_and_m_sum():
    import torch
    import paper_2005_01739_amd as hp
    L, r0 = 90.0, 15.0
    pos = synthetic.thomas(1800, L, 10, 2.0, 0.0, 37, np.float64)
    f_rand, seed = 2.0, 38
    rpos = oracle.philox_randoms(int(round(f_rand * len(pos))), L, seed)
    k = np.geomspace(0.3, 3.0, 17)
    got, ref, info = run_case(pos, None, rpos, L, r0, k, 2, gen=(f_rand, seed))
    assert info["n_rand"] == len(rpos)
    # summed over m at l1 = l2 it is the library's own isotropic bispectrum
    iso = hp.bk_ell(torch.from_numpy(pos).cuda(), box=L, r0=r0, k_edges=k, ell_max=2, f_rand=f_rand, seed=seed)
    for l in range(3):
        s = sum(got[i] for i, (l1, l2, m) in enumerate(hp.aniso_combos(2)) if l1 == l2 == l)
        scale = np.abs(iso[l]).max()
        assert np.allclose(s, iso[l], rtol=1e-6, atol=1e-7 * scale)


def test_limits_and_forms():
    import paper_2005_01739_amd as hp
    pos = synthetic.poisson(200, 50.0, 39, np.float64)
    k = np.linspace(0.5, 1.5, 4)
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_aniso(pos, box=50.0, r0=10.0, k_edges=k, ell_max=4, precision="fp64", f_rand=2.0, seed=1)
    assert e.value.status == 6
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_aniso(pos, box=50.0, r0=10.0, k_edges=k, ell_max=5, f_rand=2.0, seed=1)
    assert e.value.status == 6
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_aniso(pos, box=50.0, r0=10.0, k_edges=np.linspace(0.5, 1.5, 18), ell_max=2, f_rand=2.0, seed=1)
    assert e.value.status == 6
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_aniso(pos, box=50.0, r0=10.0, k_edges=k, ell_max=2)  # no randoms, f_rand 0
    assert e.value.status == 1


def test_full_size_bispectrum_workload_subset():
    # the 5e5-point clustered workload (12 bins, ell_max 4 here), its 1.5e6
    # randoms, 40 data and 40 random primaries
    wl = synthetic.workload(3)
    rpos = wl.randoms(np.float32)
    rng = np.random.default_rng(40)
    mask = np.zeros(wl.n, np.uint8)
    mask[rng.choice(wl.n, 40, replace=False)] = 1
    rmask = np.zeros(len(rpos), np.uint8)
    rmask[rng.choice(len(rpos), 40, replace=False)] = 1
    run_case(wl.pos, None, rpos, wl.box, wl.r0, wl.k_edges_b, 4, mask=mask, rmask=rmask)
