"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The oracle cannot evaluate a whole collision term of these workloads in a
test's time, so it recomputes a seeded sample of work items one by one (their
direct sums and scales), and properties that hold at any size are checked on
the whole output: per-cell number conservation against the GPU's own scale,
and particle-number conservation over steps.
"""
import numpy as np
import pytest

from paper_1912_04457_amd import qgbe
from paper_1912_04457_amd import workloads as W

pytestmark = pytest.mark.gpu

SEED = W.PHILOX_SEED


def _case(name):
    print(f"\n[gpu case] {name}", flush=True)


def _solver(wl, **kw):
    return qgbe.Solver(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                       species_mask=wl.species_mask, alpha_s=wl.alpha_s, seed=SEED,
                       precision=qgbe.FP32, **kw)


def _sample_items(rng, cells, n_channels, nodes, k):
    return np.stack([rng.integers(0, cells, k), rng.integers(0, n_channels, k), rng.integers(0, nodes, k)], 1)


@pytest.mark.parametrize("wl", [W.C2, W.C3], ids=lambda w: w.name)
def test_full_size_items_and_conservation(O, wl):
    _case(f"full size {wl.name} N={wl.n_samples}")
    f = W.initial_f(wl)
    with _solver(wl) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 5)
        A, S, I, st = s.collision(wl.n_samples, scale=True, items=True)
        # the variant bench.py runs (no scale output): same samples, same item sums
        A2, _, I2, _ = s.collision(wl.n_samples, items=True)
        m = s.masses()
        nch = s.n_channels
    # the two variants may contract FP32 products differently: agreement at FP32 rounding
    assert np.all(np.abs(A - A2) <= 1e-5 * S + 1e-300)
    # conservation per cell, at full size
    for cell in range(wl.cells):
        assert abs(A[:, cell].sum()) <= 1e-13 * S[:, cell].sum(), cell
    # a seeded sample of items recomputed by the oracle
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
               species_mask=wl.species_mask, alpha_s=wl.alpha_s)
    m_ref = O.masses(g, f)
    assert np.allclose(m, m_ref, rtol=1e-13, atol=0)
    rng = np.random.default_rng(77)
    # half uniform over all items, half on nodes inside the occupied gluon sphere |p| < 1 GeV
    inner = np.flatnonzero(np.linalg.norm(W.node_momenta(wl.n_p, wl.p_half), axis=1) < 1.0)
    items = _sample_items(rng, wl.cells, nch, wl.nodes, 256)
    items[128:, 2] = rng.choice(inner, 128)
    ref, scale = O.item_sums(g, f, m_ref, SEED, 5, wl.n_samples, items, want_scale=True)
    for out in (I, I2):
        got = out[items[:, 0], items[:, 1], items[:, 2]]
        err = np.abs(got - ref)
        assert np.all(err <= 1e-4 * scale + 1e-300), float((err / np.maximum(scale, 1e-300)).max())
    assert np.count_nonzero(scale) > 100


def test_full_size_steps_conserve_number():
    """Three steps of the pure-gluon spatial workload as bench.py runs it."""
    _case("full size C2 steps")
    wl = W.C2
    with _solver(wl, drift=qgbe.DRIFT_UPWIND) as s:
        s.set_f(W.initial_f(wl))
        stats = s.step(wl.dt_fm, wl.n_samples, n_steps=3)
    N = np.array([st["N_total"] for st in stats])
    assert np.abs(N - N[0]).max() <= 1e-12 * N[0]
    assert all(st["flags"] & qgbe.FLAG_NONFINITE == 0 for st in stats)


def _device_items(torch, s, wl, n_samples, sampler):
    """One collision term with A, scale and item sums in device memory."""
    A = torch.zeros((7, wl.cells, wl.nodes), dtype=torch.float64, device="cuda")
    S = torch.zeros_like(A)
    I = torch.zeros((wl.cells, s.n_channels, wl.nodes), dtype=torch.float64, device="cuda")
    qgbe.qgbe_collision_term_ex(s.ctx, n_samples, sampler, A, S, I)
    torch.cuda.synchronize()
    return A, S, I


@pytest.mark.parametrize("wl", [W.C4.scaled(n_samples=256), W.C5], ids=lambda w: w.name)
def test_full_size_learned_items(O, wl):
    """The learned sampler at the benchmark sizes: the 7-species cell with the
    network's table (re-evaluated on the masses) and a few channels set back to
    the uniform sampler, and the 12^3-cell spatial grid with an installed
    table; a seeded sample of 256 work items recomputed by the oracle with the
    table the kernel used, and per-cell conservation on the whole output."""
    torch = pytest.importorskip("torch")
    _case(f"full size learned {wl.name} N={wl.n_samples}")
    f = W.initial_f(wl)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
               species_mask=wl.species_mask, alpha_s=wl.alpha_s)
    nch = len(O.channels(g))
    rows = nch * wl.nodes
    flags = None
    with _solver(wl) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 3)
        if wl.n_x == W.C4.n_x:
            qgbe.qgbe_proposal_set_weights(s.ctx, W.random_mlp_params(61, head_scale=1.0))
            qgbe.qgbe_proposal_build_table(s.ctx, 0.1)
            flags = (np.arange(nch) % 5 != 0).astype(np.uint8)
            qgbe.qgbe_set_channel_samplers(s.ctx, flags)
        else:
            thr, mu, sg = W.random_mog_table(62, rows, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
            qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, S, I = _device_items(torch, s, wl, wl.n_samples, qgbe.SAMPLER_LEARNED)
        thr, mu, sg = qgbe.qgbe_get_proposal_table(s.ctx, rows)   # the table the kernel used
        m = s.masses()
        # per-cell conservation over species and nodes, on the device
        cons = A.sum(dim=(0, 2)).abs() <= 1e-13 * S.sum(dim=(0, 2))
        assert bool(cons.all())
        rng = np.random.default_rng(63)
        items = _sample_items(rng, wl.cells, nch, wl.nodes, 256)
        inner = np.flatnonzero(np.linalg.norm(W.node_momenta(wl.n_p, wl.p_half), axis=1) < 1.0)
        items[128:, 2] = rng.choice(inner, 128)
        idx = torch.from_numpy(items).cuda()
        got = I[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    ref, scale = O.item_sums_learned(g, f, m, SEED, 3, wl.n_samples, thr, mu, sg, items, chan_learned=flags,
                                     want_scale=True)
    err = np.abs(got - ref)
    assert np.all(err <= 1e-4 * scale + 1e-300), float((err / np.maximum(scale, 1e-300)).max())
    assert np.count_nonzero(scale) > 100
