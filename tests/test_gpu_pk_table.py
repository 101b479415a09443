"""GPU parity of the power spectrum's table form (precision "table": the
pair sum's jbar^a_l(r) from its quintic interpolant, each pair's exact
W L_l(mu) w_i w_j into fixed-point histograms) against the FP64 oracle, to
the mixed form's tolerance: 1e-6 relative per bin, or 2^-24 of the bin's L1
mass.  The interpolation error is ~2.4e-8 of jbar (k_max h <= 0.13) and the
fixed-point rounding below 1e-8 of the L1 mass, so the bound holds with room.
Pair counts must match exactly; results must be bitwise reproducible."""
import numpy as np
import pytest

import oracle
import synthetic
from test_gpu_pk import run_case

pytestmark = pytest.mark.gpu


def test_poisson_linear_bins():
    pos = synthetic.poisson(3000, 200.0, 1, np.float64)
    run_case(pos, None, 200.0, 25.0, np.linspace(0.2, 2.0, 21), 4, "table")


def test_thomas_log_bins_float32():
    pos = synthetic.thomas(6000, 300.0, 10, 2.0, 4.0, 2, np.float32)
    run_case(pos, None, 300.0, 25.0, np.geomspace(1.0, 10.0, 41), 4, "table")


@pytest.mark.parametrize("ell_max", [0, 2, 6])
def test_weights_mask_los_host_input(ell_max):
    # every histogram section count (1, 2, 4 multipoles), masked, weighted,
    # x line of sight, host input
    pos = synthetic.thomas(2000, 150.0, 10, 1.0, 0.0, 5, np.float32)
    w = synthetic.uniform_weights(2000, 6, np.float32)
    mask = (np.arange(2000) % 3 == 0).astype(np.uint8)
    run_case(pos, w, 150.0, 15.0, np.geomspace(2.0, 20.0, 31), ell_max, "table", los=0, mask=mask, device=False)


def test_r0_half_box_and_coincident_points():
    pos = synthetic.poisson(500, 40.0, 9, np.float64)
    run_case(pos, None, 40.0, 20.0, np.linspace(0.1, 1.5, 8), 2, "table")
    pos = synthetic.poisson(400, 50.0, 3, np.float64)
    pos = np.concatenate([pos, pos[:50]])  # r = 0 pairs
    run_case(pos, None, 50.0, 10.0, np.linspace(0.0, 3.0, 7), 4, "table", los=1)


def test_deterministic_and_table_reuse():
    import torch
    import paper_2005_01739_amd as hp
    pos = torch.from_numpy(synthetic.thomas(20000, 400.0, 10, 2.0, 4.0, 4, np.float32)).cuda()
    k = np.geomspace(1.0, 10.0, 41)
    ctx = hp.Context(0)
    a, ia = hp.pk_ell(pos, box=400.0, r0=25.0, k_edges=k, precision="table", ctx=ctx, return_diag=True)
    b = hp.pk_ell(pos, box=400.0, r0=25.0, k_edges=k, precision="table", ctx=ctx)
    assert np.array_equal(a, b)
    assert ia["table_nodes"] == max(64, int(np.ceil(10.0 * 25.0 / 0.13 / 64)) * 64)
    # a different binning rebuilds the table; the first one again gives the same bits
    hp.pk_ell(pos, box=400.0, r0=25.0, k_edges=k[:20], precision="table", ctx=ctx)
    assert np.array_equal(hp.pk_ell(pos, box=400.0, r0=25.0, k_edges=k, precision="table", ctx=ctx), a)


def test_full_size_headline_workload():
    # the 2e6-point Thomas catalogue of the bench's default workload: a
    # subset of 256 primaries against the oracle, and every bin of the whole
    # catalogue against the FP64 form of the same call
    import torch
    import paper_2005_01739_amd as hp
    wl = synthetic.workload(2)
    mask = np.zeros(wl.n, np.uint8)
    mask[np.random.default_rng(1).choice(wl.n, 256, replace=False)] = 1
    run_case(wl.pos, None, wl.box, wl.r0, wl.k_edges_p, wl.ell_max_p, "table", mask=mask)
    pos = torch.from_numpy(wl.pos).cuda()
    t, it = hp.pk_ell(pos, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_p, ell_max=wl.ell_max_p, precision="table",
                      return_diag=True)
    f, i64 = hp.pk_ell(pos, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_p, ell_max=wl.ell_max_p, precision="fp64",
                       return_diag=True)
    assert it["n_pairs"] == i64["n_pairs"]
    rel = np.abs(t - f) / np.abs(f)
    assert rel.max() <= 1e-6, rel.max()


def test_dense_box_counts_exact_on_every_call():
    # 4e5 clustered points in L = 500 (about 100 per cell of the R0 = 25 grid,
    # several home tiles per cell, runs of up to three cells): the ordered
    # pair count equals the FP64 form's on every one of several calls, and
    # the multipoles repeat bitwise (a workgroup whose waves disagreed on the
    # unit being swept would lose or repeat pairs, differently each call)
    import torch
    import paper_2005_01739_amd as hp
    pos = torch.from_numpy(synthetic.thomas(400000, 500.0, 10, 2.0, 4.0, 6, np.float64)).cuda()
    k = np.geomspace(1.0, 10.0, 41)
    _, ref = hp.pk_ell(pos, box=500.0, r0=25.0, k_edges=k, precision="fp64", return_diag=True)
    first = None
    for _ in range(4):
        got, info = hp.pk_ell(pos, box=500.0, r0=25.0, k_edges=k, precision="table", return_diag=True)
        assert info["n_pairs"] == ref["n_pairs"]
        if first is None:
            first = got
        assert np.array_equal(got, first)


def test_largest_binning_from_zero():
    # 128 bins from k = 0 (the largest binning; jbar_0(0) = 1 at every node
    # of the first bin), l <= 6 (four sections at the node count of
    # k_max R0 = 80)
    pos = synthetic.thomas(3000, 160.0, 10, 2.0, 2.0, 23, np.float32)
    run_case(pos, None, 160.0, 20.0, np.linspace(0.0, 4.0, 129), 6, "table")


def test_signed_weights():
    # weights of both signs: the fixed-point adds are signed and the scale
    # follows the largest |w|
    pos = synthetic.thomas(2500, 150.0, 10, 2.0, 0.0, 24, np.float64)
    w = np.random.default_rng(25).uniform(-1.5, 2.0, 2500)
    run_case(pos, w, 150.0, 15.0, np.geomspace(1.0, 12.0, 25), 4, "table", los=1)


def test_errors():
    import paper_2005_01739_amd as hp
    pos = synthetic.poisson(200, 100.0, 4, np.float64)
    # the histograms of k_max R0 = 50 * 40 need more LDS than a workgroup has
    with pytest.raises(hp.HipsterError) as e:
        hp.pk_ell(pos, box=100.0, r0=40.0, k_edges=[1.0, 50.0], ell_max=6, precision="table")
    assert e.value.name == "HIPSTER_EUNSUPPORTED"
    with pytest.raises(hp.HipsterError) as e:
        hp.bk_ell(pos, box=100.0, r0=20.0, k_edges=[0.1, 0.2], ell_max=2, precision="table")
    assert e.value.name == "HIPSTER_EUNSUPPORTED"
