"""Pins for the oracle's drift operator (Eq. left handside, Eq. descrete left hand).

* A spatially homogeneous system has no drift (every difference vanishes).
* The flux form with periodic boundaries conserves the particle number exactly
  (Sec. III: the conservative rewrite is chosen for this).
* f = F(E(x, p)) with E = sqrt(p^2 + m^2(x)) is a static solution of
  p/E . grad_x f - grad_x E . grad_p f = 0 (energy is constant along the
  trajectories of a static potential), so D[F(E)] -> 0 under refinement: at
  first order for upwind, second order for the central scheme.  A wrong sign or
  factor in the force term would leave an O(1) residual.
* Constant mass: free streaming f(x - v t, p) with v = p/E; the upwind scheme
  converges at first order, which fixes the absolute advection speed.
"""
import numpy as np
import pytest

from paper_1912_04457_amd import workloads as W

G = 6


@pytest.mark.parametrize("scheme", ["upwind", "central"])
def test_homogeneous_no_drift(O, scheme):
    g = O.Grid(n_p=(6, 5, 4), species_mask=0x7F)
    f = W.random_f(1, 1, g.nodes)
    m = O.masses(g, f)
    assert np.all(O.drift(g, f, m, scheme) == 0.0)


@pytest.mark.parametrize("scheme", ["upwind", "central"])
def test_drift_conserves_number(O, scheme):
    g = O.Grid(n_x=(4, 3, 2), n_p=(5, 4, 4), x_half=(3.0, 2.0, 1.0), species_mask=0x7F)
    f = W.random_f(2, g.cells, g.nodes)
    rng = np.random.Generator(np.random.PCG64(3))
    m = rng.uniform(0.05, 0.6, (7, g.cells))
    D = O.drift(g, f, m, scheme)
    for sp in range(7):
        assert abs(D[sp].sum()) <= 1e-13 * np.abs(D[sp]).sum()
    assert np.abs(D).max() > 0


def _static_residual(O, n, scheme):
    g = O.Grid(n_x=(n, 1, 1), n_p=(n, 2, 2), x_half=(3.0, 3.0, 3.0), p_half=(3.0, 3.0, 3.0),
               species_mask=1 << G)
    x = -3 + (np.arange(n) + 0.5) * 6 / n
    m2 = np.zeros((7, n))
    m2[:] = 0.4 + 0.2 * np.sin(2 * np.pi * x / 6)
    E = np.sqrt(np.sum(g.momenta() ** 2, 1)[None, :] + m2[G][:, None])
    f = np.zeros((7, n, g.nodes))
    f[G] = np.exp(-E / 0.3)
    D = O.drift(g, f, m2, scheme)[G]
    # the same f advected without the force (constant mass) sets the scale
    D0 = O.drift(g, f, np.full_like(m2, 0.4), scheme)[G]
    return np.abs(D).max() / np.abs(D0).max()


@pytest.mark.parametrize("scheme,order", [("upwind", 1), ("central", 2)])
def test_static_solution_consistency(O, scheme, order):
    r16, r32, r64 = (_static_residual(O, n, scheme) for n in (16, 32, 64))
    assert r64 < 0.15
    rate = np.log2(r32 / r64)
    assert order - 0.3 < rate < order + 0.3, (r16, r32, r64)


def _free_stream_error(O, n, t_end=1.0):
    L = 6.0
    g = O.Grid(n_x=(n, 1, 1), n_p=(2, 1, 1), x_half=(L / 2, 1.0, 1.0), p_half=(3.0, 1.0, 1.0),
               species_mask=1 << G)
    x = -L / 2 + (np.arange(n) + 0.5) * L / n
    m2 = np.full((7, n), 0.4)
    px = g.momenta()[:, 0]
    v = px / np.sqrt(px ** 2 + 0.4)
    f = np.zeros((7, n, 2))
    f[G] = (1 + 0.5 * np.sin(2 * np.pi * x / L))[:, None] * np.ones(2)[None, :]
    dx = L / n
    steps = int(round(t_end / (0.25 * dx)))
    dt = t_end / steps
    for _ in range(steps):
        f = f - dt * O.drift(g, f, m2, "upwind")
    exact = 1 + 0.5 * np.sin(2 * np.pi * (x[:, None] - v[None, :] * t_end) / L)
    return np.abs(f[G] - exact).max()


def test_free_streaming_first_order(O):
    e32, e64 = _free_stream_error(O, 32), _free_stream_error(O, 64)
    assert e64 < 0.05
    assert 1.6 < e32 / e64 < 2.4


@pytest.mark.parametrize("scheme", ["upwind", "central"])
def test_uniform_masses_give_the_textbook_difference(O, scheme):
    """With the same masses in every cell the force vanishes, the interface
    velocity is v = p/E itself, and the operator is the textbook difference of
    v f along each spatial axis over periodic cells: first-order upwind
    v (f_i - f_{i-1}) / dx for v > 0 and v (f_{i+1} - f_i) / dx for v < 0, or
    the central v (f_{i+1} - f_{i-1}) / (2 dx), built here from array shifts
    (reading R13 on the interface average and the periodic cells)."""
    n_x = (5, 4, 3)
    g = O.Grid(n_x=n_x, n_p=(4, 3, 5), x_half=(3.0, 2.0, 1.5), p_half=(2.0, 2.5, 1.5), species_mask=0x7F)
    rng = np.random.Generator(np.random.PCG64(15))
    f = rng.uniform(0.0, 1.0, (7, g.cells, g.nodes))
    m2 = O.constant_masses(g, [0.05, 0.07, 0.09, 0.05, 0.07, 0.09, 0.3])
    D = O.drift(g, f, m2, scheme)
    q = g.momenta()
    dx = [2.0 * h / n for h, n in zip(g.x_half, n_x)]
    F = f.reshape(7, *n_x, g.nodes)
    ref = np.zeros_like(F)
    for sp in range(7):
        v = q / np.sqrt((q ** 2).sum(1) + m2[sp, 0])[:, None]
        for a in range(3):
            fs = F[sp]
            fp = np.roll(fs, -1, axis=a)      # f_{i+1}
            fm = np.roll(fs, +1, axis=a)      # f_{i-1}
            va = v[:, a]
            if scheme == "upwind":
                ref[sp] += np.where(va > 0, va * (fs - fm), va * (fp - fs)) / dx[a]
            else:
                ref[sp] += va * (fp - fm) / (2.0 * dx[a])
    assert np.allclose(D, ref.reshape(D.shape), rtol=1e-12, atol=1e-12 * np.abs(ref).max())
