"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and its host logic (channel table,
Philox) agrees with the oracle's independent implementation."""
import os
import re

import numpy as np
import pytest

from paper_1912_04457_amd import qgbe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "qgbe.h")).read()
    return sorted(set(re.findall(r"\b(qgbe_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = qgbe.lib()
    declared = _declared()
    assert set(declared) == set(qgbe.EXPORTS), declared
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("mask", [1 << 6, 0x7F, (1 << 0) | (1 << 3) | (1 << 6), 0x3F, 1 << 2])
def test_channel_table_matches_oracle(O, mask):
    rows, w = qgbe.qgbe_channel_table(mask)
    ref = O.channels(O.Grid(species_mask=mask))
    assert len(rows) == len(ref)
    for r, ww, c in zip(rows, w, ref):
        assert r[0] == c["row"] and tuple(r[1:]) == c["sp"]
        assert ww[0] == c["w"] and ww[1] == c["sigma"]


def test_row_mask(O):
    for rm in (1, 0x10, 0x40, 0x7F, 0):
        rows, _ = qgbe.qgbe_channel_table(0x7F, rm)
        assert len(rows) == len(O.channels(O.Grid(species_mask=0x7F, row_mask=rm)))


def test_philox_host_matches_oracle(O):
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(50):
        c = rng.integers(0, 2**32, 4, dtype=np.uint64).astype(np.uint32)
        k = rng.integers(0, 2**32, 2, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(qgbe.qgbe_philox4x32_10(c, k), O.philox4x32_10(c, k))


def test_invalid_descriptor_rejected_before_device_work():
    bad = qgbe.make_desc(n_p=(1, 4, 4))
    with pytest.raises(qgbe.QgbeError) as e:
        qgbe.qgbe_init_grid(bad)
    assert e.value.status in (qgbe.EINVAL, qgbe.EDEVICE)
