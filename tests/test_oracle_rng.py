"""Oracle pins: Philox4x32-10 and the uniform stream."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_stream_uniforms_are_top24_bits_in_order(orc):
    seed, g = 0x1234_5678_9ABC_DEF0, 987654321012
    u = orc.stream_uniforms(seed, g, 2, 7, 12)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    exp = []
    for blk in range(3):
        out = orc.philox([blk, (2 << 16) | 7, g & 0xFFFFFFFF, g >> 32], key)
        exp += [(int(x) >> 8) / 2.0 ** 24 for x in out]
    assert np.array_equal(u, np.array(exp))
    assert np.all((u >= 0) & (u < 1))
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))


def test_stream_uniformity(orc):
    u = np.concatenate([orc.stream_uniforms(5, g, 1, 0, 64) for g in range(400)])
    hist = np.histogram(u, bins=16, range=(0, 1))[0]
    expv = len(u) / 16
    chi2 = ((hist - expv) ** 2 / expv).sum()
    assert chi2 < 40.0   # 15 dof, p ~ 5e-4
