"""Host side of the particle-file source: the record file round trip, its
size check and the alignment of the arrays in the file (the device copy is
read through pointers into it)."""
import os

import numpy as np
import pytest

from paper_1503_01725_amd import pslfile as pf


def _records(n, rng):
    rec = {f: rng.standard_normal(n).astype(np.float32) for f in pf.FLOAT_FIELDS}
    rec["hid"] = rng.integers(0, 2 ** 63, n, dtype=np.uint64)
    rec["tag"] = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    return rec


@pytest.mark.parametrize("n", [1, 7, 1000])
def test_round_trip(tmp_path, n):
    rng = np.random.default_rng(n)
    rec = _records(n, rng)
    path = str(tmp_path / "b.psl")
    size = pf.write_records(path, rec, 1)
    assert size == os.path.getsize(path) == pf.HEADER_BYTES + n * pf.RECORD_BYTES
    back, ptype = pf.read_records(path)
    assert ptype == 1
    for f in rec:
        assert np.array_equal(back[f], rec[f]), f


def test_array_alignment():
    for n in (1, 3, 5, 1 << 20):
        off = pf.offsets(n)
        assert off["hid"] % 8 == 0 and off["tag"] % 4 == 0
        assert all(off[f] % 4 == 0 for f in pf.FLOAT_FIELDS)
        assert off["end"] == pf.HEADER_BYTES + n * pf.RECORD_BYTES


def test_rejects_foreign_and_truncated_files(tmp_path):
    bad = tmp_path / "bad.psl"
    bad.write_bytes(b"NOTAPSL!" + bytes(16))
    with pytest.raises(ValueError):
        pf.read_header(str(bad))
    rng = np.random.default_rng(1)
    path = str(tmp_path / "t.psl")
    pf.write_records(path, _records(10, rng), 0)
    with open(path, "r+b") as fh:
        fh.truncate(pf.HEADER_BYTES + 5 * pf.RECORD_BYTES)
    with pytest.raises(ValueError):
        pf.read_header(path)
