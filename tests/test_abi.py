"""Host-side checks of the C ABI: the library loads, exports every function
include/hipster.h declares, its host-only entry point (W~) is pinned against
mpmath, and calls fail cleanly (no device work) on bad arguments."""
import ctypes as ct
import os
import re

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hipster.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hipster_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2005_01739_amd as hp
    L = hp.load_library()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    assert sorted(hp.EXPORTED_SYMBOLS) == names


def test_status_strings():
    import paper_2005_01739_amd as hp
    L = hp.load_library()
    for code, name in enumerate(["HIPSTER_OK", "HIPSTER_EINVAL", "HIPSTER_EDOMAIN", "HIPSTER_EOUTOFBOX",
                                 "HIPSTER_ENOMEM", "HIPSTER_EHIP", "HIPSTER_EUNSUPPORTED"]):
        assert L.hipster_status_string(code).decode() == name


def _wtilde_exact(r0, k1, k2):
    mp.mp.dps = 30
    D0 = lambda u: mp.sin(u) - u * mp.cos(u)
    dk3 = mp.mpf(k2) ** 3 - mp.mpf(k1) ** 3

    def W(x):
        if x < 0.5:
            return mp.mpf(1)
        if x < 0.75:
            t = 2 * x - 1
            return 1 - 8 * t ** 3 + 8 * t ** 4
        t = x - 1
        return -64 * t ** 3 - 128 * t ** 4

    f = lambda r: 3 * (D0(k2 * r) - D0(k1 * r)) / (r * dk3) * W(r / r0) if r > 0 else mp.mpf(0)
    pts = sorted(set([mp.mpf(0), mp.mpf(r0) / 2, 3 * mp.mpf(r0) / 4, mp.mpf(r0)] + list(mp.linspace(0, r0, 40))))
    return float(4 * mp.pi * mp.quad(f, pts))


@pytest.mark.parametrize("r0,k1,k2", [(50.0, 0.2, 0.29), (50.0, 1.1, 1.19), (25.0, 5.0, 5.3), (15.0, 2.0, 2.08), (30.0, 0.0, 0.5)])
def test_library_wtilde_against_mpmath(r0, k1, k2):
    import paper_2005_01739_amd as hp
    got = hp.wtilde(r0, [k1, k2])[0]
    ex = _wtilde_exact(r0, k1, k2)
    assert abs(got - ex) <= 1e-13 * max(abs(ex), 1e-6 * 4 * np.pi * r0 ** 3 / 3), (got, ex)


def test_wtilde_rejects_bad_edges():
    import paper_2005_01739_amd as hp
    with pytest.raises(hp.HipsterError) as e:
        hp.wtilde(10.0, [0.5, 0.4])
    assert e.value.name == "HIPSTER_EDOMAIN"
    with pytest.raises(hp.HipsterError):
        hp.wtilde(-1.0, [0.1, 0.2])


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    import paper_2005_01739_amd as hp
    L = hp.load_library()
    h = ct.c_void_p()
    st = L.hipster_create(ct.byref(h), 0, None)
    assert st == 5  # HIPSTER_EHIP
    assert not h.value
    # NULL context calls are rejected without touching a device
    assert L.hipster_pk_ell(None, None, None, None, None) == 1
    assert L.hipster_bk_ell(None, None, None, 0.0, 0, None, None, None) == 1
    assert L.hipster_batch(None, 0, None, None) == 1
    L.hipster_destroy(None)


def test_binding_argument_checks():
    import paper_2005_01739_amd as hp
    keep = []
    with pytest.raises(ValueError):
        hp._points(np.zeros((10, 2)), None, keep)
    with pytest.raises(ValueError):
        hp._points(np.zeros((10, 3), np.int32), None, keep)
    with pytest.raises(ValueError):
        hp._points(np.zeros((10, 3)), np.zeros(9), keep)
    p = hp._points(np.zeros((10, 3), np.float32), np.ones(10), keep)
    assert p.n == 10 and p.dtype == 0 and p.on_device == 0
