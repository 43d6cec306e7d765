"""Pins for the oracle's thermal masses (Eq. mg, Eq. mq).

Textbook equilibrium values (hard-thermal-loop asymptotic masses, E = |p| as the
paper uses on the first step):
    pure glue, Bose-Einstein at T:            m_g^2 = g^2 T^2 / 2
    3 flavours of q, qbar (Fermi-Dirac) + g:  m_g^2 = (3/4) g^2 T^2
                                              m_q^2 = g^2 T^2 / 3
The grid sum is a midpoint rule with a 1/p^2 integrable singularity at the
origin, so it converges at first order; the test extrapolates (Richardson) from
n and 2n nodes per axis and checks the first-order rate.  With an odd n a node
sits at p = 0, where the Bose-Einstein f is infinite and E = 0: that node
carries no weight, and the sum must converge to the same limit.
"""
import math

import numpy as np
import pytest

ALPHA = 0.3
G2 = 4 * math.pi * ALPHA
T = 0.3


def _eq_masses(O, n, with_quarks):
    g = O.Grid(n_p=(n, n, n), p_half=(3.0, 3.0, 3.0), species_mask=0x7F)
    p = np.linalg.norm(g.momenta(), axis=1)
    f = np.zeros((7, 1, g.nodes))
    with np.errstate(divide="ignore"):
        f[6, 0] = 1.0 / np.expm1(p / T)   # inf at a node at p = 0 (odd n)
    if with_quarks:
        f[:6, 0] = 1.0 / (np.exp(p / T) + 1.0)
    return O.masses(g, f)[:, 0]


@pytest.mark.parametrize("n", [60, 61], ids=["even", "odd"])
@pytest.mark.parametrize("with_quarks", [False, True])
def test_equilibrium_masses(O, with_quarks, n):
    m_n = _eq_masses(O, n, with_quarks)
    m_2n = _eq_masses(O, 2 * n - n % 2, with_quarks)   # odd n: 2n - 1 keeps the node at p = 0
    assert np.all(np.isfinite(m_n)) and np.all(np.isfinite(m_2n))
    rich = 2.0 * m_2n - m_n
    if with_quarks:
        targets = {6: 0.75 * G2 * T * T, 0: G2 * T * T / 3, 3: G2 * T * T / 3}
    else:
        targets = {6: 0.5 * G2 * T * T}
    for sp, target in targets.items():
        e1, e2 = m_n[sp] / target - 1, m_2n[sp] / target - 1
        assert abs(rich[sp] / target - 1) < 5e-3, (sp, rich[sp], target)
        assert 1.6 < e1 / e2 < 2.4           # first-order convergence


def test_masses_linear_and_per_cell(O):
    g = O.Grid(n_x=(2, 1, 1), n_p=(6, 6, 6), p_half=(2.0, 2.0, 2.0), species_mask=0x7F)
    rng = np.random.Generator(np.random.PCG64(1))
    f = rng.uniform(0, 0.5, (7, 2, g.nodes))
    m = O.masses(g, f)
    m2 = O.masses(g, 2 * f)
    assert np.allclose(m2, 2 * m, rtol=1e-14)
    assert np.allclose(m[:3], m[3:6], rtol=0)        # m_q = m_qbar per flavour
    one = O.masses(g, np.concatenate([f[:, :1], f[:, :1]], axis=1))
    assert np.allclose(one[:, 0], one[:, 1], rtol=0)


def test_lagged_energy_lowers_masses(O):
    """Later steps use E = sqrt(p^2 + m^2_prev) >= |p|: every mass decreases."""
    g = O.Grid(n_p=(8, 8, 8), p_half=(2.0, 2.0, 2.0), species_mask=0x7F)
    rng = np.random.Generator(np.random.PCG64(2))
    f = rng.uniform(0, 0.5, (7, 1, g.nodes))
    m0 = O.masses(g, f)
    m1 = O.masses(g, f, m0)
    assert np.all(m1 < m0) and np.all(m1 > 0.5 * m0)
