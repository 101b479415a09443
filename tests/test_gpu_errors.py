"""Error returns of the C ABI through the binding: every rejected call names
the status that include/hipster.h documents for it.  Argument checks run on
the host before any kernel; coordinates outside the box are flagged by the
cell-assignment kernel, which writes nothing for such points.  A context
needs a device, hence the gpu mark."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

K = np.linspace(0.1, 1.0, 6)


def _status(fn):
    import paper_2005_01739_amd as hp
    with pytest.raises(hp.HipsterError) as e:
        fn()
    return e.value.name


def _pts(n=200, L=100.0, seed=1):
    return np.random.default_rng(seed).uniform(0.0, L, (n, 3))


def test_power_spectrum_argument_errors():
    import paper_2005_01739_amd as hp
    x = _pts()
    pk = lambda pos=x, **kw: hp.pk_ell(pos, **{"box": 100.0, "r0": 10.0, "k_edges": K, **kw})
    assert _status(lambda: pk(r0=60.0)) == "HIPSTER_EDOMAIN"          # R0 > L/2
    assert _status(lambda: pk(r0=0.0)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: pk(box=-1.0)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: pk(k_edges=K[::-1])) == "HIPSTER_EDOMAIN"  # not increasing
    assert _status(lambda: pk(k_edges=[-0.1, 0.5])) == "HIPSTER_EDOMAIN"
    assert _status(lambda: pk(ell_max=3)) == "HIPSTER_EDOMAIN"        # odd ell_max for P
    assert _status(lambda: pk(ell_max=8)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: pk(los_axis=3)) == "HIPSTER_EINVAL"
    assert _status(lambda: pk(k_edges=np.linspace(0.1, 1.0, 130))) == "HIPSTER_EUNSUPPORTED"  # n_k > 128
    # the mixed form's table reduction covers k_max * R0 <= 1e6
    assert _status(lambda: pk(k_edges=[1.0, 2.0e5])) == "HIPSTER_EUNSUPPORTED"
    assert _status(lambda: pk(pos=x[:1])) == "HIPSTER_EINVAL"        # fewer than two points
    for v in (100.0, -1e-9, np.nan, np.inf):
        bad = x.copy()
        bad[17, 1] = v
        assert _status(lambda: pk(pos=bad)) == "HIPSTER_EOUTOFBOX"


def test_bispectrum_argument_errors():
    import paper_2005_01739_amd as hp
    x = _pts()
    bk = lambda pos=x, **kw: hp.bk_ell(pos, **{"box": 100.0, "r0": 10.0, "k_edges": K, "f_rand": 2.0, **kw})
    assert _status(lambda: bk(k_edges=np.linspace(0.1, 1.0, 66))) == "HIPSTER_EUNSUPPORTED"  # n_k > 64
    assert _status(lambda: bk(f_rand=0.0)) == "HIPSTER_EINVAL"  # no randoms, none to draw
    assert _status(lambda: bk(ell_max=7)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: bk(r0=51.0)) == "HIPSTER_EDOMAIN"
    bad = x.copy()
    bad[3, 0] = np.nan
    assert _status(lambda: bk(pos=bad)) == "HIPSTER_EOUTOFBOX"
    rbad = _pts(50, seed=2)
    rbad[0, 2] = 250.0
    assert _status(lambda: bk(randoms=rbad)) == "HIPSTER_EOUTOFBOX"


def test_survey_argument_errors():
    import paper_2005_01739_amd as hp
    x = _pts() + 1000.0
    r = _pts(600, seed=3) + 1000.0
    sv = lambda pos=x, rnd=r, **kw: hp.pk_survey(pos, None, rnd, **{"volume": 1e6, "r0": 10.0, "k_edges": K, **kw})
    assert _status(lambda: sv(rnd=r[:0])) == "HIPSTER_EINVAL"        # no randoms
    assert _status(lambda: sv(volume=0.0)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: sv(volume=np.inf)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: sv(r0=-1.0)) == "HIPSTER_EDOMAIN"
    assert _status(lambda: sv(ell_max=5)) == "HIPSTER_EDOMAIN"
    bad = x.copy()
    bad[7, 2] = np.inf
    assert _status(lambda: sv(pos=bad)) == "HIPSTER_EOUTOFBOX"


def test_context_survives_errors():
    # a rejected call leaves the context usable: the next valid call succeeds
    import paper_2005_01739_amd as hp
    x = _pts(400, seed=4)
    with pytest.raises(hp.HipsterError):
        hp.pk_ell(x, box=100.0, r0=60.0, k_edges=K)
    out = hp.pk_ell(x, box=100.0, r0=10.0, k_edges=K)
    assert np.all(np.isfinite(out))
