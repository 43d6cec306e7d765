"""GPU parity of the two pieces of proposal training that feed the network:
the recorded training rows and the Adam update.

* qgbe_record_samples writes, per recorded sample of the uniform sampler, the
  work item's eight conditioning features, the five logits y = ln(u/(1-u)) of
  the sample's unit-cube variables and |v|, the magnitude of the sample's
  value (weight x |M|^2 x bracket, Eq. ca in the CM-angle form).  The oracle
  recomputes every row: features by oracle.mlp.features with the cell's own
  thermal masses, u from the oracle's Philox stream, v by the oracle's
  evaluation of the same configuration.  The GPU computes in FP64 and stores
  FP32: features and logits within 1e-6 relative, |v| within 2^-23 of itself
  plus 1e-10 of its gain+loss scale.
* Adam (Kingma & Ba): after one and two training steps on one batch, the GPU's
  FP32 weights equal oracle.mlp.adam applied to the GPU's own gradients at the
  same weights (qgbe_mlp_loss_grad), with the learning rates of the cosine
  schedule; bound 2e-2 of the learning rate per weight (an Adam step moves a
  weight by about the learning rate; a wrong bias correction moves it by
  several times that).
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_1912_04457_amd import qgbe
from paper_1912_04457_amd import workloads as W

pytestmark = pytest.mark.gpu

SEED = 0x5EED2019
SMALL_7 = W.Workload("qg7_2cells_5x6x4", (2, 1, 1), (5, 6, 4), (3.0, 3.0, 3.0), (2.0, 2.5, 1.5),
                     0x7F, 100, "f64", 1, 0.01)


def _case(name):
    print(f"\n[gpu case] {name}", flush=True)


def _kw(wl):
    return dict(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                species_mask=wl.species_mask, alpha_s=wl.alpha_s, seed=SEED)


@pytest.mark.parametrize("step", [0, 5])
def test_recorded_rows_match_oracle(O, step):
    _case(f"record rows step={step}")
    wl = SMALL_7
    per_item, stride = 3, 7
    f = W.random_f(51, wl.cells, wl.nodes)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    chans = O.channels(g)
    nch = len(chans)
    items = wl.cells * nch * wl.nodes
    n_sel = -(-items // stride)
    rows = np.zeros((n_sel * per_item, qgbe.RECORD_WIDTH), dtype=np.float32)
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, step)
        n = qgbe.qgbe_record_samples(s.ctx, per_item, stride, rows)
    assert n == n_sel * per_item
    m = O.masses(g, f)
    P = g.momenta()
    V5 = float(np.prod(2.0 * np.asarray(wl.p_half))) * 4.0 * np.pi
    p_half = np.asarray(wl.p_half)
    n_valid = 0
    for j in range(n_sel):
        w = j * stride
        p1_lin = w % wl.nodes
        ci = (w // wl.nodes) % nch
        cell = w // (wl.nodes * nch)
        c = chans[ci]
        feat = M.features(P[p1_lin], m[c["sp"][0], cell], m[6, cell], c["sp"][0], ci, nch, wl.p_half)[0]
        for s_ in range(per_item):
            r = rows[j * per_item + s_]
            assert np.allclose(r[:8], feat, rtol=1e-6, atol=1e-7), (j, s_)
            u = O.sample_uniforms(SEED, step, s_, p1_lin, cell, c["code"])
            assert np.allclose(r[8:13], np.log(u / (1.0 - u)), rtol=1e-6, atol=1e-7), (j, s_)
            p2 = -p_half + 2.0 * p_half * u[:3]
            pt = O.eval_cm(g, c, f, m, cell, P[p1_lin], p2, 2.0 * u[3] - 1.0, 2.0 * np.pi * u[4],
                           p1_lin=p1_lin)
            v = abs(c["w"] * V5 * pt["g"] / per_item) if pt["valid"] else 0.0
            vs = abs(c["w"] * V5 * pt["gscale"] / per_item) if pt["valid"] else 0.0
            n_valid += pt["valid"]
            assert abs(float(r[13]) - v) <= 2.0 ** -23 * v + 1e-10 * vs, (j, s_, float(r[13]), v)
    assert n_valid > 0.2 * n


def test_adam_steps_match_oracle():
    _case("adam steps")
    wl = SMALL_7
    rng = np.random.Generator(np.random.PCG64(61))
    n = 3000
    X = rng.uniform(-1, 1, (n, M.N_IN)).astype(np.float32)
    yw = np.concatenate([rng.normal(0, 1.5, (n, M.D)), rng.uniform(0.1, 2.0, (n, 1))], 1).astype(np.float32)
    rows = np.ascontiguousarray(np.concatenate([X, yw], 1), dtype=np.float32)
    w0 = W.random_mlp_params(9, head_scale=1.0)
    lr0, lr1 = 2e-3, 5e-4
    cfg1 = qgbe.TrainCfg(epochs=1, batch=4096, lr=lr0, lr_final=lr0, alpha=0.1, seed=3)
    cfg2 = qgbe.TrainCfg(epochs=2, batch=4096, lr=lr0, lr_final=lr1, alpha=0.1, seed=3)
    with qgbe.Solver(**_kw(wl), precision=qgbe.FP32) as s:
        s.set_f(W.random_f(52, wl.cells, wl.nodes))

        def grad_at(w):
            qgbe.qgbe_proposal_set_weights(s.ctx, w)
            gr = np.zeros(qgbe.MLP_PARAMS, dtype=np.float32)
            qgbe.qgbe_mlp_loss_grad(s.ctx, X, yw, gr)
            return gr

        g0 = grad_at(w0)
        qgbe.qgbe_proposal_set_weights(s.ctx, w0)        # zero moments, t = 0
        qgbe.qgbe_train_proposal(s.ctx, rows, cfg1)
        w1_gpu = qgbe.qgbe_proposal_get_weights(s.ctx)
        qgbe.qgbe_proposal_set_weights(s.ctx, w0)
        qgbe.qgbe_train_proposal(s.ctx, rows, cfg2)
        w2_gpu = qgbe.qgbe_proposal_get_weights(s.ctx)
        g1 = grad_at(w1_gpu)

    p0 = M.unflatten(w0.astype(np.float64))
    state = {}
    p1 = M.adam(p0, M.unflatten(g0.astype(np.float64)), state, lr=lr0)
    w1_ref = M.flatten(p1)
    err1 = np.abs(w1_gpu - w1_ref)
    print(f"[adam] step 1: max |dw| {err1.max():.3e} (lr {lr0}), median {np.median(err1):.3e}", flush=True)
    assert err1.max() <= 2e-2 * lr0
    # the second step starts from the GPU's own first step (its gradient is
    # taken there) and the oracle's moments after the first step
    p1g = M.unflatten(w1_gpu.astype(np.float64))
    p2 = M.adam(p1g, M.unflatten(g1.astype(np.float64)), state, lr=lr1)
    w2_ref = M.flatten(p2)
    err2 = np.abs(w2_gpu - w2_ref)
    print(f"[adam] step 2: max |dw| {err2.max():.3e} (lr {lr1}), median {np.median(err2):.3e}", flush=True)
    assert err2.max() <= 2e-2 * lr0
    # the steps moved the weights by about the learning rate
    assert np.median(np.abs(w1_gpu - w0)) > 0.5 * lr0
