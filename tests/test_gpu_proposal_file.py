"""A proposal table saved by bench.py (--save-proposal) and installed in a
fresh context (--load-proposal) gives the same learned collision term: the
table and the per-channel sampler flags are the sampler's whole state.  The
same samples are drawn; the terms agree to the rounding of the FP64 atomic
adds, whose order varies from run to run (1e-12 of the largest value), while
another sampler on the same f differs far beyond that."""
import importlib.util
import os
import sys

import numpy as np
import pytest

from paper_1912_04457_amd import qgbe
from paper_1912_04457_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SEED = 0x5EED2019


def _bench():
    spec = importlib.util.spec_from_file_location("bench_prop", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        spec.loader.exec_module(b)
    finally:
        sys.argv = argv
    return b


def test_saved_proposal_reproduces_the_learned_term(tmp_path):
    print("\n[gpu case] proposal table saved and loaded, 2 cells 5x6x4, 7 species, FP32", flush=True)
    b = _bench()
    wl = W.Workload("qg7_2cells_5x6x4", (2, 1, 1), (5, 6, 4), (3.0, 3.0, 3.0), (2.0, 2.5, 1.5),
                    0x7F, 64, "f32", 1, 0.01)
    kw = dict(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask,
              alpha_s=wl.alpha_s, seed=SEED, precision=qgbe.FP32)
    f = W.random_f(35, wl.cells, wl.nodes)
    path = str(tmp_path / "proposal.npz")
    with qgbe.Solver(**kw) as s:
        s.set_f(f)
        thr, mu, sg = W.random_mog_table(36, s.n_channels * wl.nodes, K=8, alpha=0.1, mu_scale=1.0,
                                         log_sigma=(-1.0, 0.5))
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        flags = np.ones(s.n_channels, dtype=np.uint8)
        flags[::3] = 0                                # some channels on the uniform fallback
        qgbe.qgbe_set_channel_samplers(s.ctx, flags)
        qgbe.qgbe_set_step_index(s.ctx, 3)
        A1 = s.collision(wl.n_samples, sampler=qgbe.SAMPLER_LEARNED)[0]
        b.save_proposal(s, wl, path)
    with qgbe.Solver(**kw) as s:
        s.set_f(f)
        prep = b.load_proposal(s, wl, path)
        qgbe.qgbe_set_step_index(s.ctx, 3)
        A2 = s.collision(wl.n_samples, sampler=qgbe.SAMPLER_LEARNED)[0]
        qgbe.qgbe_set_step_index(s.ctx, 3)
        A3 = s.collision(wl.n_samples, sampler=qgbe.SAMPLER_UNIFORM)[0]
    assert prep["learned_channels"] == int(flags.sum()) < prep["channels"]
    scale = np.abs(A1).max()
    assert scale > 0
    assert np.abs(A1 - A2).max() <= 1e-12 * scale
    assert np.abs(A1 - A3).max() > 1e-3 * scale
