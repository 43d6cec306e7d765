"""Host-side checks of bench.py (no GPU): the one-GPU refusal, how the slot
counts the roofline uses are composed, that the committed HBM-traffic figure
is only reported for the kernel sources it was measured on, and that a saved
proposal table for another grid is refused."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        spec.loader.exec_module(b)
    finally:
        sys.argv = argv
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_slot_counts_compose_from_their_parts():
    """The per-class figures the roofline uses are the Philox block, the
    uniforms and the op-count figures of tests/test_opcount.py, in that
    combination."""
    b = _bench()
    assert b.SLOTS_REJECTED == b.PHILOX_BLOCK + b.UNIFORMS_FROM_BLOCK + b.FP_OUTSIDE_BOX
    assert b.SLOTS_ACCEPTED == b.PHILOX_BLOCK + b.UNIFORMS_FROM_BLOCK + b.FP_ACCEPTED
    assert b.SLOTS_LEARNED_EXTRA == b.PHILOX_BLOCK + b.MIXTURE_INT + b.FP_MIXTURE - b.UNIFORMS_FROM_BLOCK
    assert b.SLOTS_ROOTS_SAMPLE == b.PHILOX_BLOCK + b.UNIFORMS_FROM_BLOCK + b.FP_ROOTS_SAMPLE
    assert b.SLOTS_REJECTED < b.SLOTS_ACCEPTED


def test_traffic_reported_only_for_the_measured_sources():
    b = _bench()
    digest = b.kernel_sources_digest()
    assert len(digest) == 64
    prof = open(b.traffic_profile("gg_16x16x1_20cube_f32")).read()
    recorded = [l.split(":", 1)[1].strip() for l in prof.splitlines() if l.startswith("sources_sha256:")]
    assert len(recorded) == 1
    t = b.measured_traffic("gg_16x16x1_20cube_f32")
    if recorded[0] == digest:      # counters taken on these sources: a figure of the right size
        assert t is not None and 5e7 < t < 1e9
    else:                          # sources changed since: no stale figure
        assert t is None
    assert b.measured_traffic("no_such_workload") is None


def test_load_proposal_refuses_a_table_for_another_grid(tmp_path):
    """--load-proposal checks the table's rows (channels x nodes) and the
    per-channel flags against the grid before anything reaches the device."""
    import numpy as np

    b = _bench()

    class _Solver:
        n_channels = 70
        ctx = None

    class _Wl:
        nodes = 16 ** 3

    path = str(tmp_path / "p.npz")
    rows = 70 * 20 ** 3                                   # a 20^3 table
    np.savez(path, thr=np.zeros((rows, 8), np.uint32), mu=np.zeros((rows, 8, 5), np.float32),
             sigma=np.ones((rows, 8, 5), np.float32), samplers=np.ones(70, np.uint8))
    with pytest.raises(ValueError, match="another grid"):
        b.load_proposal(_Solver(), _Wl(), path)
    rows = 70 * 16 ** 3                                   # right rows, flags for 7 channels
    np.savez(path, thr=np.zeros((rows, 8), np.uint32), mu=np.zeros((rows, 8, 5), np.float32),
             sigma=np.ones((rows, 8, 5), np.float32), samplers=np.ones(7, np.uint8))
    with pytest.raises(ValueError, match="another grid"):
        b.load_proposal(_Solver(), _Wl(), path)
