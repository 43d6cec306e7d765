"""Pins for the oracle of the learned proposal (MLP, mixture head, loss, Adam).

* analytic gradients equal central finite differences of the loss;
* a mixture of identical components is that single product of normals
  (scipy.stats.norm.logpdf);
* the logistic-normal density on the unit cube integrates to one (1-D quadrature
  per factor, 5-D Monte Carlo for the mixture);
* the proposal table carries the softmax weights in its thresholds;
* the first Adam step from zero moments moves every weight by -lr sign(g).
"""
import numpy as np
import pytest
from scipy import integrate, stats

from oracle import mlp as M
from paper_1912_04457_amd import workloads as W


def _data(n=64, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(0, 0.6, (n, M.N_IN))
    y = rng.normal(0, 1.5, (n, M.D))
    w = rng.uniform(0.1, 2.0, n)
    return X, y, w


def _params(seed=1, head_scale=1.0):
    return M.unflatten(W.random_mlp_params(seed, head_scale=head_scale).astype(np.float64))


def test_gradients_match_finite_differences():
    p = _params()
    X, y, w = _data()
    loss, g = M.loss_and_grad(p, X, y, w)
    rng = np.random.Generator(np.random.PCG64(5))
    h = 1e-6
    for name, shape in M.PARAM_SHAPES:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in shape)
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += h
            lp, _ = M.loss_and_grad(q, X, y, w)
            q[name][idx] -= 2 * h
            lm, _ = M.loss_and_grad(q, X, y, w)
            fd = (lp - lm) / (2 * h)
            assert g[name][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9), (name, idx)


def test_identical_components_reduce_to_normal_product():
    rng = np.random.Generator(np.random.PCG64(3))
    mu = rng.normal(0, 1, M.D)
    ls = rng.uniform(-1, 0.5, M.D)
    Y = np.concatenate([rng.normal(0, 1, M.K), np.tile(mu, M.K), np.tile(ls, M.K)])[None, :]
    y = rng.normal(0, 1, (1, M.D))
    L, _ = M.log_mixture(Y, y)
    ref = stats.norm.logpdf(y[0], loc=mu, scale=np.exp(ls)).sum()
    assert L[0] == pytest.approx(ref, rel=1e-13)


def test_logistic_normal_factor_normalised():
    for mu, s in ((0.0, 1.0), (3.0, 0.3), (-2.0, 2.0)):
        f = lambda u: stats.norm.pdf(np.log(u / (1 - u)), mu, s) / (u * (1 - u))
        val, _ = integrate.quad(f, 0, 1, limit=200, points=[1 / (1 + np.exp(-mu))])
        assert val == pytest.approx(1.0, abs=1e-9)


def test_mixture_density_integrates_to_one():
    p = _params(head_scale=3.0)
    X, _, _ = _data(1, seed=9)
    Y, _ = M.forward(p, X)
    Y[:, M.K + M.K * M.D:] = np.clip(Y[:, M.K + M.K * M.D:], -0.5, 0.5)   # moderate widths
    rng = np.random.Generator(np.random.PCG64(11))
    n = 400000
    u = rng.uniform(size=(n, M.D))
    dens = np.exp(M.log_density_unit_cube(np.repeat(Y, n, axis=0), u))
    mean, se = dens.mean(), dens.std() / np.sqrt(n)
    assert abs(mean - 1.0) < 5 * se + 1e-3, (mean, se)


def test_table_thresholds_carry_softmax():
    p = _params(head_scale=3.0)
    X, _, _ = _data(16, seed=2)
    Y, _ = M.forward(p, X)
    thr, mu, sigma = M.table_from_head(Y, alpha=0.1)
    a = Y[:, :M.K]
    pi = np.exp(a - a.max(1, keepdims=True))
    pi /= pi.sum(1, keepdims=True)
    assert np.all(thr[:, 0] == np.uint32(np.floor(0.1 * 2**32)))
    assert np.all(np.diff(thr.astype(np.int64), axis=1) >= 0)
    widths = np.diff(np.concatenate([thr.astype(np.float64), np.full((16, 1), 2.0**32)], axis=1), axis=1)
    assert np.allclose(widths / 2**32, 0.9 * pi, atol=3e-9)
    assert np.all(sigma > 0) and mu.shape == (16, M.K, M.D)


def test_first_adam_step_is_sign_step():
    p = _params()
    X, y, w = _data()
    _, g = M.loss_and_grad(p, X, y, w)
    st = {}
    q = M.adam(p, g, st, lr=1e-3)
    for name, _ in M.PARAM_SHAPES:
        nz = np.abs(g[name]) > 1e-3      # eps / |g| negligible
        assert np.allclose((q[name] - p[name])[nz], -1e-3 * np.sign(g[name][nz]), rtol=1e-4)


def test_training_reduces_loss_on_a_known_target():
    """Samples from one fixed logistic-normal: Adam steps lower the weighted NLL."""
    rng = np.random.Generator(np.random.PCG64(4))
    n = 512
    X = np.tile(rng.normal(0, 0.5, (1, M.N_IN)), (n, 1))
    y = rng.normal([1.0, -0.5, 0.0, 2.0, 0.3], 0.4, (n, M.D))
    w = np.ones(n)
    p = _params()
    st = {}
    l0, _ = M.loss_and_grad(p, X, y, w)
    for _ in range(200):
        _, g = M.loss_and_grad(p, X, y, w)
        p = M.adam(p, g, st, lr=3e-3)
    l1, _ = M.loss_and_grad(p, X, y, w)
    assert l1 < l0 - 1.0
