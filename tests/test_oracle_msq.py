"""Pins for the oracle's Table I matrix elements.

Independent reference: the standard tree-level QCD 2->2 results, averaged over
initial and summed over final spins and colours (Combridge, Kripfganz, Ranft,
Phys. Lett. B70 (1977) 234; tabulated in Ellis, Stirling, Webber, "QCD and
collider physics", Table 7.1).  Table I sums over the initial states as well,
so in the massless, unregulated limit it must equal those forms times the
initial-state degeneracies 2*3*2*3 = 36 (qq), 2*3*2*8 = 96 (qg), 2*8*2*8 = 256
(gg).
"""
import math

import numpy as np
import pytest

ALPHA = 0.3
G4 = (4 * math.pi * ALPHA) ** 2


def textbook(row, s, t, u):
    """Spin/colour-averaged sum |M|^2 / g^4 of the textbook table, times the
    initial-state degeneracy, in Table I labelling a b -> c d."""
    if row == 1:   # q q' -> q q'
        return 36 * (4 / 9) * (s * s + u * u) / (t * t)
    if row == 2:   # q q -> q q
        return 36 * ((4 / 9) * ((s * s + u * u) / (t * t) + (s * s + t * t) / (u * u))
                     - (8 / 27) * s * s / (u * t))
    if row == 3:   # q qbar -> q qbar
        return 36 * ((4 / 9) * ((s * s + u * u) / (t * t) + (t * t + u * u) / (s * s))
                     - (8 / 27) * u * u / (s * t))
    if row == 4:   # q qbar -> q' qbar'
        return 36 * (4 / 9) * (t * t + u * u) / (s * s)
    if row == 5:   # q qbar -> g g
        return 36 * ((32 / 27) * (t * t + u * u) / (t * u) - (8 / 3) * (t * t + u * u) / (s * s))
    if row == 6:   # q g -> q g
        return 96 * (-(4 / 9) * (s * s + u * u) / (s * u) + (u * u + s * s) / (t * t))
    if row == 7:   # g g -> g g
        return 256 * (9 / 2) * (3 - t * u / (s * s) - s * u / (t * t) - s * t / (u * u))
    raise ValueError(row)


def _massless_points(n=50, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.uniform(0.2, 9.0, n)
    c = rng.uniform(-0.98, 0.98, n)
    return s, -s * (1 - c) / 2, -s * (1 + c) / 2


@pytest.mark.parametrize("row", range(1, 8))
def test_massless_limit_matches_textbook(O, row):
    for s, t, u in zip(*_massless_points()):
        got = O.msq(row, s, t, u, 0.0, ALPHA) / G4
        assert got == pytest.approx(textbook(row, s, t, u), rel=1e-12)


def test_gg_to_qqbar_is_reverse_of_qqbar_to_gg(O):
    """The textbook gg -> q qbar form times 256 equals row 5 (time reversal)."""
    for s, t, u in zip(*_massless_points(seed=5)):
        gg_qq = 256 * ((1 / 6) * (t * t + u * u) / (t * u) - (3 / 8) * (t * t + u * u) / (s * s))
        assert O.msq(5, s, t, u, 0.0, ALPHA) / G4 == pytest.approx(gg_qq, rel=1e-12)


@pytest.mark.parametrize("row", [2, 4, 5, 7])
def test_identical_final_states_symmetric_in_t_u(O, row):
    rng = np.random.Generator(np.random.PCG64(row))
    for _ in range(20):
        s, t, u, mu = rng.uniform(0.5, 5), -rng.uniform(0, 3), -rng.uniform(0, 3), rng.uniform(0.05, 1)
        assert O.msq(row, s, t, u, mu, ALPHA) == pytest.approx(O.msq(row, s, u, t, mu, ALPHA), rel=1e-13)


def test_regulator_removes_forward_pole(O):
    """With m_g^2 > 0 the t -> 0 limit is finite (every t pole regulated)."""
    for row in (1, 2, 3, 6, 7):
        v = O.msq(row, 2.0, -1e-14, -2.0 + 1e-14, 0.3, ALPHA)
        assert np.isfinite(v) and abs(v) < 1e6


def textbook_regulated(row, s, t, u, mu):
    """The textbook table with its fractions split into terms over one pole
    each (or a product of poles), and m_g^2 subtracted from t and u wherever
    they stand in a denominator: the regulator of Table I, which screens the
    t- and u-channel exchanges and leaves numerators and s poles alone.  At
    mu = 0 this is `textbook`; every coefficient is the textbook's."""
    T, U = t - mu, u - mu
    if row == 1:
        return 36 * (4 / 9) * (s * s + u * u) / (T * T)
    if row == 2:
        return 36 * ((4 / 9) * ((s * s + u * u) / (T * T) + (s * s + t * t) / (U * U))
                     - (8 / 27) * s * s / (U * T))
    if row == 3:
        return 36 * ((4 / 9) * ((s * s + u * u) / (T * T) + (t * t + u * u) / (s * s))
                     - (8 / 27) * u * u / (s * T))
    if row == 4:
        return 36 * (4 / 9) * (t * t + u * u) / (s * s)
    if row == 5:   # (t^2 + u^2) / (t u) = t / u + u / t
        return 36 * ((32 / 27) * (t / U + u / T) - (8 / 3) * (t * t + u * u) / (s * s))
    if row == 6:   # (s^2 + u^2) / (s u) = s / u + u / s
        return 96 * (-(4 / 9) * (s / U + u / s) + (u * u + s * s) / (T * T))
    if row == 7:
        return 256 * (9 / 2) * (3 - t * u / (s * s) - s * u / (T * T) - s * t / (U * U))
    raise ValueError(row)


@pytest.mark.parametrize("row", range(1, 8))
def test_regulated_rows_match_textbook_with_screened_poles(O, row):
    """Every row at m_g^2 > 0, rows 5 and 6 included (a regulator on the wrong
    pole, or on a numerator, changes the value by O(m_g^2 / t))."""
    rng = np.random.Generator(np.random.PCG64(100 + row))
    for s, t, u in zip(*_massless_points(seed=7)):
        mu = rng.uniform(0.05, 1.5)
        got = O.msq(row, s, t, u, mu, ALPHA) / G4
        assert got == pytest.approx(textbook_regulated(row, s, t, u, mu), rel=1e-12)


@pytest.mark.parametrize("row", range(1, 8))
def test_regulator_removes_both_poles(O, row):
    """With m_g^2 > 0 every row stays finite as t -> 0 and as u -> 0, and
    approaches the regulated textbook value there."""
    s, mu, eps = 2.0, 0.3, 1e-14
    for t, u in ((-eps, -s + eps), (-s + eps, -eps)):
        v = O.msq(row, s, t, u, mu, ALPHA) / G4
        assert np.isfinite(v) and abs(v) < 1e6
        assert v == pytest.approx(textbook_regulated(row, s, t, u, mu), rel=1e-9)
