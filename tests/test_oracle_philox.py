"""Pins for the oracle's Philox4x32-10 generator.

The generator is not in the paper (it is silent on the random numbers); the
published definition (Salmon et al., SC'11) fixes it, so the oracle is checked
against the published known-answer vectors and against an independent
third-party implementation (PyTorch's ``at::philox_engine``) run as a black box.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split("|")
            a = [int(x, 16) for x in lhs.split()]
            b = [int(x, 16) for x in rhs.split()]
            rows.append((a[:4], a[4:], b))
    return rows


def test_known_answer_vectors(O):
    for ctr, key, out in _kat():
        assert O.philox4x32_10(ctr, key).tolist() == out


def test_against_torch_engine(O, tmp_path):
    """Black-box comparison with PyTorch's Philox4x32-10 on random blocks."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path / "philox_ref")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I" + inc, "-o", exe,
                           os.path.join(HERE, "philox_torch_ref.cpp")])
    rng = np.random.Generator(np.random.PCG64(7))
    blocks = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    blocks[:20, 1] = 0          # small counters, like the sampler's
    blocks[20:40, 0] = 0xFFFFFFFF
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in blocks) + "\n"
    res = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in line.split()] for line in res.stdout.strip().splitlines()])
    mine = np.array([O.philox4x32_10(row[:4], row[4:]) for row in blocks.astype(np.uint32)])
    assert np.array_equal(mine.astype(np.int64), ref.astype(np.int64))


def test_output_bits_uniform(O):
    """Chi-square of the 23-bit fields the sampler uses (16 bins each)."""
    n = 4000
    vals = np.array([O.philox4x32_10([s, 11, 0, 3 << 8], [0x5EED2019, 0]) for s in range(n)])
    top = (vals >> 9).astype(np.int64)          # four 23-bit fields
    counts = np.array([np.bincount(top[:, j] >> 19, minlength=16) for j in range(4)])
    exp = n / 16.0
    chi2 = ((counts - exp) ** 2 / exp).sum(axis=1)
    # 15 degrees of freedom: P(chi2 > 45) ~ 7e-5
    assert np.all(chi2 < 45.0), chi2
