"""The roofline's work per evaluation against the op-count build of the oracle.

bench.py converts evaluations into lane-op issue slots with per-class figures;
their floating-point part must be what the oracle's own formulas cost when
every operation on a sample-dependent value is counted (oracle/opcount.cpp),
weighted 1 for full-rate and 4 for quarter-rate instructions.  A change to the
oracle's arithmetic, or a figure in bench.py edited by hand, fails here.
"""
import importlib.util
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_opc", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        spec.loader.exec_module(b)
    finally:
        sys.argv = argv
    return b


def _slots(c):
    full = c["add"] + c["mul"] - c["fma"] + c["cmp"] + c["misc"]
    return full + 4.0 * (c["div"] + c["sqrt"] + c["trans"])


@pytest.fixture(scope="module")
def counts(O):
    return O.op_counts()


def test_uniform_sampler_figures(counts):
    b = _bench()
    assert _slots(counts["uniform_outside_box"]) == pytest.approx(b.FP_OUTSIDE_BOX, abs=0.05)
    assert _slots(counts["uniform_accepted"]) == pytest.approx(b.FP_ACCEPTED, abs=0.05)
    dep = _slots(counts["uniform_accepted"]) - _slots(counts["uniform_accepted_direct"])
    assert dep == pytest.approx(b.FP_DEPOSITS, abs=0.3)


def test_mixture_and_root_figures(counts):
    b = _bench()
    assert _slots(counts["mixture_draw_and_density"]) == pytest.approx(b.FP_MIXTURE, abs=0.05)
    r0 = counts["roots_direct_0_valid"]
    assert _slots(r0) == pytest.approx(b.FP_ROOTS_SAMPLE, abs=0.05)
    # per valid root: the samples with one and two roots, weighted by roots
    r1, r2 = counts["roots_direct_1_valid"], counts["roots_direct_2_valid"]
    per = (r1["samples"] * (_slots(r1) - _slots(r0)) + r2["samples"] * (_slots(r2) - _slots(r0))) / (
        r1["samples"] + 2 * r2["samples"])
    assert per == pytest.approx(b.FP_ROOTS_PER_ROOT, abs=0.1)


def test_counts_have_the_structure_of_the_estimators(counts):
    """What the formulas fix, independent of the weights: a sample rejected at
    the threshold stops after E2, s and one comparison (one square root); a
    box-rejected one has built the CM frame and both final momenta; an accepted
    one adds t, u, |M|^2, three interpolations and the value, and the
    symmetric deposits add only multiplications (24 corner values, the
    additions being the accumulators' atomic adds); the mixture's
    transcendentals are those of three Box-Muller pairs, five logistic maps and
    an 8-component density with its Jacobian."""
    th, box, acc = counts["uniform_below_threshold"], counts["uniform_outside_box"], counts["uniform_accepted"]
    direct = counts["uniform_accepted_direct"]
    assert th["sqrt"] == 1 and th["trans"] == 0
    assert box["sqrt"] > th["sqrt"] and box["trans"] == 2      # cos and sin of the azimuth
    assert _slots(th) < _slots(box) < _slots(acc)
    for k in ("add", "div", "sqrt", "trans", "cmp"):
        assert acc[k] == pytest.approx(direct[k], abs=0.5), k
    assert 16 <= acc["mul"] - direct["mul"] <= 24
    mix = counts["mixture_draw_and_density"]
    assert mix["sqrt"] == 3                                     # Box-Muller radii
    # 3 logs + 3 cos + 3 sin (Box-Muller) + 5 exp (logistic) + 8 exp, 1 log
    # (mixture) + 5 x (2 exp + 2 log) (Jacobian), less what is shared
    assert 30 <= mix["trans"] <= 43
