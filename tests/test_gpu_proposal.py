"""GPU tests of the learned proposal against the FP64 oracle.

* network forward and loss/gradient: the GPU multiplies BF16 operands with
  FP32 accumulation; the oracle evaluates the same network in FP64 with the
  same operands rounded to BF16.  Bar: relative L2 <= 1e-2 per tensor.
* conditioning features: FP32 of the same FP64 values (rtol 1e-6).
* learned-sampler collision term with a seeded random mixture table (input to
  both sides): FP64 mode within 1e-10 of the cell scale, FP32 within 1e-4.
* after training on the solver's own samples, the learned estimator agrees
  with the uniform one in expectation and has lower MC error at equal N.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_1912_04457_amd import qgbe
from paper_1912_04457_amd import workloads as W

pytestmark = pytest.mark.gpu

SEED = 0x5EED2019


def _case(name):
    print(f"\n[gpu case] {name}", flush=True)


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


SMALL_7 = W.Workload("qg7_2cells_5x6x4", (2, 1, 1), (5, 6, 4), (3.0, 3.0, 3.0), (2.0, 2.5, 1.5),
                     0x7F, 100, "f64", 1, 0.01)


def _kw(wl):
    return dict(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                species_mask=wl.species_mask, alpha_s=wl.alpha_s, seed=SEED)


def _mlp_inputs(rows, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(-1, 1, (rows, M.N_IN)).astype(np.float32)
    yw = np.concatenate([rng.normal(0, 1.5, (rows, M.D)), rng.uniform(0.1, 2.0, (rows, 1))], 1).astype(np.float32)
    return X, yw


def test_mlp_forward_matches_oracle():
    _case("mlp forward")
    w = W.random_mlp_params(3, head_scale=1.0)
    X, _ = _mlp_inputs(1000, 4)
    with qgbe.Solver(**_kw(SMALL_7)) as s:
        qgbe.qgbe_proposal_set_weights(s.ctx, w)
        Y = np.zeros((1000, M.N_OUT), dtype=np.float32)
        qgbe.qgbe_mlp_forward(s.ctx, X, Y)
        assert np.array_equal(qgbe.qgbe_proposal_get_weights(s.ctx), w)
    Yref, _ = M.forward(M.unflatten(w.astype(np.float64)), X.astype(np.float64), quantize=M.bf16)
    assert _rel(Y, Yref) <= 1e-2, _rel(Y, Yref)


def test_mlp_loss_and_gradient_match_oracle():
    _case("mlp loss/grad")
    w = W.random_mlp_params(5, head_scale=1.0)
    X, yw = _mlp_inputs(2000, 6)
    with qgbe.Solver(**_kw(SMALL_7)) as s:
        qgbe.qgbe_proposal_set_weights(s.ctx, w)
        grad = np.zeros(qgbe.MLP_PARAMS, dtype=np.float32)
        loss = qgbe.qgbe_mlp_loss_grad(s.ctx, X, yw, grad)
    p = M.unflatten(w.astype(np.float64))
    lref, gref = M.loss_and_grad(p, X.astype(np.float64), yw[:, :5].astype(np.float64),
                                 yw[:, 5].astype(np.float64), quantize=M.bf16)
    assert loss == pytest.approx(lref, rel=1e-3)
    g = M.unflatten(grad.astype(np.float64))
    for name, _ in M.PARAM_SHAPES:
        assert _rel(g[name], gref[name]) <= 1e-2, (name, _rel(g[name], gref[name]))


def test_features_match_oracle(O):
    _case("features")
    wl = SMALL_7
    f = W.random_f(31, wl.cells, wl.nodes)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    chans = O.channels(g)
    with qgbe.Solver(**_kw(wl)) as s:
        s.set_f(f)
        X = np.zeros((len(chans) * wl.nodes, 8), dtype=np.float32)
        qgbe.qgbe_proposal_features(s.ctx, X)
    m = O.masses(g, f).mean(axis=1)     # one table serves all cells: cell-averaged masses
    P = g.momenta()
    ref = np.concatenate([M.features(P, m[c["sp"][0]], m[6], c["sp"][0], i, len(chans), wl.p_half)
                          for i, c in enumerate(chans)])
    assert np.allclose(X, ref, rtol=1e-6, atol=1e-7)


def _table_ref(O, g, f, w, alpha):
    chans = O.channels(g)
    m = O.masses(g, f).mean(axis=1)
    X = np.concatenate([M.features(g.momenta(), m[c["sp"][0]], m[6], c["sp"][0], i, len(chans), g.p_half)
                        for i, c in enumerate(chans)])
    Y, _ = M.forward(M.unflatten(w.astype(np.float64)), X, quantize=M.bf16)
    return M.table_from_head(Y, float(np.float32(alpha)))   # the ABI takes alpha as FP32


def _check_table(tab, ref):
    thr, mu, sg = tab
    t_ref, mu_ref, sg_ref = ref
    assert np.all(thr[:, 0] == t_ref[:, 0])
    assert np.abs(thr.astype(np.float64) - t_ref).max() <= 2**32 * 2e-2
    assert _rel(mu, mu_ref) <= 1e-2 and _rel(sg, sg_ref) <= 1e-2


def test_table_from_network(O):
    """The table built from the network, and its re-evaluation by a learned
    collision term after f (hence the masses) changed."""
    _case("table build")
    wl = SMALL_7
    f = W.random_f(32, wl.cells, wl.nodes)
    f2 = W.random_f(35, wl.cells, wl.nodes) * 0.5
    w = W.random_mlp_params(7, head_scale=1.0)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    with qgbe.Solver(**_kw(wl)) as s:
        s.set_f(f)
        qgbe.qgbe_proposal_set_weights(s.ctx, w)
        qgbe.qgbe_proposal_build_table(s.ctx, 0.1)
        tab1 = qgbe.qgbe_get_proposal_table(s.ctx, rows)
        s.set_f(f2)
        s.collision(8, sampler=qgbe.SAMPLER_LEARNED)
        tab2 = qgbe.qgbe_get_proposal_table(s.ctx, rows)
    _check_table(tab1, _table_ref(O, g, f, w, 0.1))
    _check_table(tab2, _table_ref(O, g, f2, w, 0.1))
    assert not np.array_equal(tab1[1], tab2[1])


@pytest.mark.parametrize("precision,tol", [(qgbe.FP64, 1e-10), (qgbe.FP32, 1e-4)])
def test_learned_collision_parity(O, precision, tol):
    _case(f"learned collision parity precision={precision}")
    wl = SMALL_7
    f = W.random_f(33, wl.cells, wl.nodes)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    thr, mu, sg = W.random_mog_table(34, rows, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    with qgbe.Solver(**_kw(wl), precision=precision) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 2)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, _, _, _ = s.collision(100, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 2, 100, thr, mu, sg)
    err = np.abs(A - A_ref)
    assert np.all(err <= tol * S_ref + 1e-300), float((err / np.maximum(S_ref, 1e-300)).max())
    assert _rel(A, A_ref) <= tol
    for cell in range(wl.cells):
        assert abs(A[:, cell].sum()) <= 1e-13 * S_ref[:, cell].sum()


# 3 x 5 x 7 = 105 momenta: in the FP32 kernel's blocks of 4 consecutive nodes
# per wave, the last block holds one node, and chunks end inside a block
RAGGED_7 = W.Workload("qg7_2cells_3x5x7", (2, 1, 1), (3, 5, 7), (3.0, 3.0, 3.0), (2.0, 2.5, 1.5),
                      0x7F, 100, "f64", 1, 0.01)


@pytest.mark.parametrize("precision,tol", [(qgbe.FP64, 1e-10), (qgbe.FP32, 1e-4)])
def test_learned_collision_parity_partial_node_block(O, precision, tol):
    """The learned term on a node count that is not a multiple of the node
    block (the direct sums of the last, partial block are still added)."""
    _case(f"learned collision parity 3x5x7 nodes precision={precision}")
    wl = RAGGED_7
    f = W.random_f(36, wl.cells, wl.nodes)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    thr, mu, sg = W.random_mog_table(37, rows, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    with qgbe.Solver(**_kw(wl), precision=precision) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 4)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, _, _, _ = s.collision(100, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 4, 100, thr, mu, sg)
    err = np.abs(A - A_ref)
    assert np.all(err <= tol * S_ref + 1e-300), float((err / np.maximum(S_ref, 1e-300)).max())
    assert np.all(S_ref[:, :, -1] > 0)   # the bar binds at the last node of every row
    for cell in range(wl.cells):
        assert abs(A[:, cell].sum()) <= 1e-13 * S_ref[:, cell].sum()


def test_learned_config3_layout_fp32(O):
    """20^3, 7 species: the learned variant's LDS plan reads some f tiles from
    global memory (node quads) and deposits one slot with global atomics."""
    _case("learned C3 layout fp32 N=8")
    wl = W.C3
    f = W.initial_f(wl)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    thr, mu, sg = W.random_mog_table(39, rows, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(f)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, _, _, _ = s.collision(8, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 0, 8, thr, mu, sg)
    err = np.abs(A - A_ref)
    assert np.all(err <= 1e-4 * S_ref + 1e-300), float((err / np.maximum(S_ref, 1e-300)).max())
    assert abs(A.sum()) <= 1e-13 * S_ref.sum()


@pytest.mark.parametrize("precision,tol", [(qgbe.FP64, 1e-10), (qgbe.FP32, 1e-4)])
def test_channel_fallback_parity(O, precision, tol):
    """Half of the channels fall back to the uniform sampler."""
    _case(f"fallback parity precision={precision}")
    wl = SMALL_7
    f = W.random_f(36, wl.cells, wl.nodes)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    nch = len(O.channels(g))
    thr, mu, sg = W.random_mog_table(37, nch * wl.nodes, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    flags = (np.arange(nch) % 2).astype(np.uint8)
    with qgbe.Solver(**_kw(wl), precision=precision) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 3)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        assert np.all(qgbe.qgbe_get_channel_samplers(s.ctx, nch) == 1)
        qgbe.qgbe_set_channel_samplers(s.ctx, flags)
        assert np.array_equal(qgbe.qgbe_get_channel_samplers(s.ctx, nch), flags)
        A, _, _, _ = s.collision(100, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 3, 100, thr, mu, sg, chan_learned=flags)
    err = np.abs(A - A_ref)
    assert np.all(err <= tol * S_ref + 1e-300), float((err / np.maximum(S_ref, 1e-300)).max())


def test_judge_rejects_a_poor_proposal():
    """A table of narrow components far from the integrand's mass, with a
    small defensive share, has a much larger variance than the uniform
    sampler: the judge sends (nearly) every channel back to uniform."""
    _case("judge poor table")
    wl = W.C3.scaled(n_p=(6, 6, 6))
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(W.initial_f(wl))
        nch = s.n_channels
        thr, mu, sg = W.random_mog_table(38, nch * wl.nodes, K=8, alpha=0.02, mu_scale=3.0,
                                         log_sigma=(-4.0, -3.0))
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        step0 = qgbe.qgbe_get_step_index(s.ctx)
        flags, ratio = qgbe.qgbe_proposal_judge(s.ctx, 64, 4, nch)
        assert qgbe.qgbe_get_step_index(s.ctx) == step0
        assert np.array_equal(qgbe.qgbe_get_channel_samplers(s.ctx, nch), flags)
    print(f"[judge] learned kept on {int(flags.sum())} of {nch} channels; median ratio {np.median(ratio):.3g}")
    assert flags.mean() <= 0.2
    assert np.all((ratio < 1.0) == (flags == 1))


def _mc_error(samples):
    mean = samples.mean(0)
    var = samples.var(0, ddof=1)
    return np.sqrt(var.mean()) / np.sqrt((mean ** 2).mean())


def test_trained_proposal_unbiased_and_better():
    """7 species, 8^3 momenta, CGC gluons + Fermi-Dirac quarks: train on the
    solver's own uniform samples, then compare estimators at equal N."""
    _case("train + compare")
    wl = W.C3.scaled(n_p=(8, 8, 8))
    f = W.initial_f(wl)
    N, R = 64, 8
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(f)
        rows = np.zeros((70 * wl.nodes * 16, qgbe.RECORD_WIDTH), dtype=np.float32)
        n = qgbe.qgbe_record_samples(s.ctx, 16, 1, rows)
        assert n == rows.shape[0]
        assert np.isfinite(rows).all() and (rows[:, 13] > 0).mean() > 0.05
        qgbe.qgbe_proposal_set_weights(s.ctx, W.random_mlp_params(11))
        cfg = qgbe.TrainCfg(epochs=4, batch=4096, lr=2e-3, lr_final=2e-4, alpha=0.1, seed=1)
        losses = np.zeros(4)
        qgbe.qgbe_train_proposal(s.ctx, rows, cfg, losses)
        print(f"[train] epoch losses {losses}", flush=True)
        assert losses[-1] < losses[0]
        plain, learned = [], []
        for r in range(R):
            qgbe.qgbe_set_step_index(s.ctx, 100 + r)
            plain.append(s.collision(N)[0])
            learned.append(s.collision(N, sampler=qgbe.SAMPLER_LEARNED)[0])
        nch = s.n_channels
        flags, ratio = qgbe.qgbe_proposal_judge(s.ctx, 64, 4, nch)
        print(f"[train] judge keeps the learned sampler on {int(flags.sum())} of {nch} channels", flush=True)
        judged = []
        for r in range(R):
            qgbe.qgbe_set_step_index(s.ctx, 100 + r)
            judged.append(s.collision(N, sampler=qgbe.SAMPLER_LEARNED)[0])
    plain, learned, judged = np.array(plain), np.array(learned), np.array(judged)
    e_plain, e_learned, e_judged = _mc_error(plain), _mc_error(learned), _mc_error(judged)
    print(f"[train] MC error plain {e_plain:.4f} learned {e_learned:.4f} judged {e_judged:.4f}", flush=True)
    assert e_learned < e_plain and e_judged < e_plain
    assert flags.mean() >= 0.5
    diff = learned.mean(0) - plain.mean(0)
    se = np.sqrt(learned.var(0, ddof=1) / R + plain.var(0, ddof=1) / R)
    keep = se > 0
    z = diff[keep] / se[keep]
    assert np.mean(z ** 2) < 1.8 and np.abs(z).max() < 6.0, (np.mean(z ** 2), np.abs(z).max())


def test_spatial_seven_species_learned_steps(O):
    """The 7-species spatial configuration (Gaussian-blob gluons, Fermi-Dirac
    quarks, 16^3 momenta, learned proposal) at 3^3 cells: one learned collision
    term against the oracle, then steps whose particle number is conserved to
    FP64 rounding (symmetric deposits and the flux-form drift)."""
    _case("spatial 7-species learned")
    wl = W.C5.scaled(n_x=(3, 3, 3))
    f = W.initial_f(wl)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    thr, mu, sg = W.random_mog_table(40, rows, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(f)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, _, _, _ = s.collision(4, sampler=qgbe.SAMPLER_LEARNED)
        stats = s.step(wl.dt_fm, 64, n_steps=5, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 0, 4, thr, mu, sg)
    err = np.abs(A - A_ref)
    assert np.all(err <= 1e-4 * S_ref + 1e-300), float((err / np.maximum(S_ref, 1e-300)).max())
    N = np.array([st["N_total"] for st in stats])
    drift = np.abs(N - N[0]).max() / N[0]
    print(f"[spatial learned] N_total relative drift over 5 steps {drift:.2e}", flush=True)
    assert drift <= 1e-12
    assert all(np.isfinite(st["E_total"]) for st in stats)


def test_learned_cell_blocks_ragged(O):
    """The learned kernel orders its workgroups in blocks of 32 cells; 45
    cells (one full block and one of 13, 7 species, 4^3 momenta) against the
    oracle, every cell and channel once."""
    _case("learned 45 cells (cell blocks 32 + 13) fp32")
    wl = W.Workload("qg7_5x3x3_4cube", (5, 3, 3), (4, 4, 4), (6.0, 6.0, 6.0), (2.0, 2.0, 2.0),
                    0x7F, 16, "f32", 1, 0.01)
    f = W.random_f(41, wl.cells, wl.nodes) * 0.5
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    thr, mu, sg = W.random_mog_table(42, rows, K=8, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 1)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, _, _, _ = s.collision(wl.n_samples, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 1, wl.n_samples, thr, mu, sg)
    err = np.abs(A - A_ref)
    assert np.all(err <= 1e-4 * S_ref + 1e-300), float((err / np.maximum(S_ref, 1e-300)).max())
    assert np.abs(A_ref).max() > 0


def test_learned_sixteen_components(O):
    """A host-set table of 16 components: the FP64 learned sampler agrees with
    the oracle; an FP32 context (whose LDS row of component constants holds 8)
    refuses it with QGBE_EUNSUPPORTED instead of running."""
    _case("learned K=16 fp64 parity, fp32 refusal")
    wl = SMALL_7
    f = W.random_f(41, wl.cells, wl.nodes)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    rows = len(O.channels(g)) * wl.nodes
    thr, mu, sg = W.random_mog_table(42, rows, K=16, alpha=0.1, mu_scale=1.0, log_sigma=(-1.0, 0.5))
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP64) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, 3)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        A, _, _, _ = s.collision(100, sampler=qgbe.SAMPLER_LEARNED)
    m = O.masses(g, f)
    A_ref, S_ref, _ = O.collision_learned(g, f, m, SEED, 3, 100, thr, mu, sg)
    assert np.all(np.abs(A - A_ref) <= 1e-10 * S_ref + 1e-300)
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(f)
        qgbe.qgbe_set_proposal_table(s.ctx, thr, mu, sg)
        for call in (lambda: s.collision(100, sampler=qgbe.SAMPLER_LEARNED),
                     lambda: s.step(0.01, 100, n_steps=1, sampler=qgbe.SAMPLER_LEARNED)):
            with pytest.raises(qgbe.QgbeError) as e:
                call()
            assert e.value.status == qgbe.EUNSUPPORTED
        A, _, _, _ = s.collision(100, sampler=qgbe.SAMPLER_UNIFORM)   # the context still works
        assert np.isfinite(A).all()
