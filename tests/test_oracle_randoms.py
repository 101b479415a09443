"""The random catalogue of the bispectrum's DDR^II term when the library
draws it (hipster_bk_ell with no catalogue, Sec. 4: f_rand times the data in
uniform randoms).  The oracle side generates it with numpy's Philox bit
generator; these tests pin that stream to the published Philox4x64-10 round
function and to its known-answer vectors (tests/golden/philox4x64_10_kat.txt),
so the oracle's catalogue is fixed by the generator's definition, not by the
library."""
import os

import numpy as np

import oracle

M64 = (1 << 64) - 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def philox4x64_10(ctr, key):
    # Philox4x64 with 10 rounds: two 64x64 -> 128-bit products per round,
    # multipliers 0xD2E7470EE14C6C93 and 0xCA5A826395121157, Weyl key
    # increments 0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B between rounds.
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B97F4A7C15) & M64
            k1 = (k1 + 0xBB67AE8584CAA73B) & M64
        p0 = 0xD2E7470EE14C6C93 * c0
        p1 = 0xCA5A826395121157 * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & M64, (p0 >> 64) ^ c3 ^ k1, p0 & M64
    return [c0, c1, c2, c3]


def _kat():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        out.append((v[0:4], v[4:6], v[6:10]))
    return out


def test_round_function_reproduces_known_answers():
    vecs = _kat()
    assert len(vecs) == 3
    for ctr, key, want in vecs:
        assert philox4x64_10(ctr, key) == want


def test_numpy_stream_is_the_published_generator():
    # numpy's Philox increments its 256-bit counter before each block: block
    # b of the stream keyed by (seed, 0) is philox4x64_10((b, 0, 0, 0), key)
    for seed in (0, 5, 2 ** 63 + 11):
        raw = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64)).random_raw(4 * 6)
        for b in range(6):
            assert [int(x) for x in raw[4 * b:4 * b + 4]] == philox4x64_10([b + 1, 0, 0, 0], [seed, 0])


def test_oracle_randoms_follow_the_definition():
    n, box, seed = 257, 123.5, 2 ** 63 + 42
    pts = oracle.philox_randoms(n, box, seed)
    assert pts.shape == (n, 3) and pts.dtype == np.float64
    assert np.all(pts >= 0.0) and np.all(pts < box)
    for i in (0, 1, 100, 256):
        words = philox4x64_10([i + 1, 0, 0, 0], [seed, 0])
        want = [box * ((w >> 11) * 2.0 ** -53) for w in words[:3]]
        assert list(pts[i]) == want


def test_oracle_randoms_are_uniform():
    pts = oracle.philox_randoms(200000, 10.0, 7)
    # each coordinate uniform on [0, 10): mean 5, variance 100/12, to 5 sigma
    m = pts.mean(axis=0)
    v = pts.var(axis=0)
    assert np.all(np.abs(m - 5.0) < 5 * np.sqrt(100 / 12 / 200000))
    assert np.all(np.abs(v - 100 / 12) < 5 * np.sqrt(100 ** 2 / 180 / 200000))
    # coordinates of one point are independent
    c = np.corrcoef(pts.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / np.sqrt(200000))
