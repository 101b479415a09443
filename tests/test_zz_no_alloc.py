"""The power spectrum through hipster_pk_ell_noalloc, the entry point whose
device scratch is the library's static per-device workspace, against
hipster_pk_ell on the same inputs (both through the C ABI).

Both entry points run the same kernels; the workspace entry point cuts the
pair stream into more chunks, so the same pairs reach the per-wave FP64 sums
in another order.  Pair counts must match exactly, and each raw bin sum to
1e-11 of the bin's L1 mass (the sum of |term| over its pair terms): FP64
reordering error is of order sqrt(n) 2^-53 of that mass, far below the
bound, while a lost or repeated chunk moves a bin by about its own size.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

TOL_L1 = 1e-11


def _hp():
    import paper_2005_01739_amd as hp
    return hp


def _compare(pos, w, box, r0, k, ell_max, precision, what):
    hp = _hp()
    kw = dict(box=box, r0=r0, k_edges=k, ell_max=ell_max, precision=precision)
    ref, rinfo = hp.pk_ell(pos, w, return_diag=True, l1_mass=True, **kw)
    got, ginfo = hp.pk_ell_noalloc(pos, w, return_diag=True, **kw)
    assert ginfo["n_pairs"] == rinfo["n_pairs"], what
    assert ginfo["n_pairs_far"] == rinfo["n_pairs_far"], what
    assert ginfo["ms_total"] == 0.0 and ginfo["ms_sweep"] == 0.0, what  # no events in workspace mode
    l1 = rinfo["l1_mass"]
    err_raw = np.abs(ginfo["raw"] - rinfo["raw"])
    assert (err_raw <= TOL_L1 * l1).all(), f"{what}: raw sums, worst {np.max(err_raw / l1):.3e} of L1"
    # P = S norm - delta_l0 W~, with the same norm and W~ on both sides
    i = np.unravel_index(np.argmax(np.abs(rinfo["raw"])), ref.shape)
    norm = (ref[i] + (rinfo["wtilde"][i[1]] if i[0] == 0 else 0.0)) / rinfo["raw"][i]
    np.testing.assert_array_equal(ginfo["wtilde"], rinfo["wtilde"])
    err = np.abs(got - ref)
    assert (err <= TOL_L1 * l1 * abs(norm) + 1e-14 * np.abs(ref)).all(), f"{what}: P"
    return rinfo["n_pairs"]


def test_noalloc_matches_pk_ell_two_calls():
    import torch
    # call 1: 1e6 clustered points with weights on the device, mixed form;
    # about 3.5e7 unordered pairs, several chunks of the workspace's pair stream
    n1, L1, r01 = 1_000_000, 1000.0, 25.0
    pos1 = synthetic.thomas(n1, L1, 10, 2.0, 4.0, 71, np.float32)
    w1 = synthetic.uniform_weights(n1, 72, np.float32)
    print(f"no-alloc call 1: n={n1} mixed, device inputs", flush=True)
    np1 = _compare(torch.from_numpy(pos1).cuda(), torch.from_numpy(w1).cuda(), L1, r01,
                   np.geomspace(1.0, 10.0, 41), 4, "mixed", "call 1")
    assert np1 > 20_000_000
    # call 2, smaller: 1.5e5 points from host memory, FP64 form, other bins
    n2, L2, r02 = 150_000, 600.0, 40.0
    pos2 = synthetic.poisson(n2, L2, 73, np.float64)
    print(f"no-alloc call 2: n={n2} fp64, host inputs", flush=True)
    _compare(pos2, None, L2, r02, np.linspace(0.05, 1.0, 20), 2, "fp64", "call 2")


def test_noalloc_rejects_oversize_then_recovers():
    import torch
    hp = _hp()
    # 6e6 points: the cell lists alone (48 B per point) exceed the 256 MiB workspace
    n, L = 6_000_000, 2000.0
    pos = torch.from_numpy(synthetic.poisson(n, L, 74, np.float32)).cuda()
    print(f"no-alloc oversize: n={n}", flush=True)
    with pytest.raises(hp.HipsterError) as e:
        hp.pk_ell_noalloc(pos, box=L, r0=20.0, k_edges=np.geomspace(1.0, 10.0, 11), ell_max=2)
    assert e.value.status == 4 and "static workspace" in str(e.value)
    small = synthetic.poisson(60_000, 500.0, 75, np.float32)
    print("no-alloc after the rejected call: n=60000 mixed", flush=True)
    _compare(torch.from_numpy(small).cuda(), None, 500.0, 30.0, np.geomspace(0.5, 5.0, 16), 4, "mixed",
             "after rejection")
