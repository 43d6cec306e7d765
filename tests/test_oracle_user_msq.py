"""Pins for user-defined matrix elements in the oracle (Sec. II: an interface
for matrix elements of the user's own).

* Table I written as user terms reproduces the built-in rows (whose textbook
  forms are pinned in test_oracle_msq.py) at random Mandelstam points: the
  generic evaluator, its units (g^4) and the regulator placement;
* a user row |M|^2 = g^4 s^2/(t - mu)^2 inside the CM-angle sampler integrates
  over the angles to the closed form 4 pi g^4 s^2 / (mu (s + mu)) (massless,
  B = 1), independent of the Table I code;
* bad terms are refused.
"""
import math

import numpy as np
import pytest
from scipy import integrate

ALPHA = 0.3
G4 = (4 * math.pi * ALPHA) ** 2

TABLE_I = {
    1: [(16, (2, 0, 0, 2, 0, 0)), (16, (0, 0, 2, 2, 0, 0))],
    2: [(16, (2, 0, 0, 2, 0, 0)), (16, (0, 0, 2, 2, 0, 0)), (16, (2, 0, 0, 0, 2, 0)), (16, (0, 2, 0, 0, 2, 0)),
        (-32 / 3, (2, 0, 0, 1, 1, 0))],
    3: [(16, (2, 0, 0, 2, 0, 0)), (16, (0, 0, 2, 2, 0, 0)), (16, (0, 0, 2, 0, 0, 2)), (16, (0, 2, 0, 0, 0, 2)),
        (-32 / 3, (0, 0, 2, 1, 0, 1))],
    4: [(16, (0, 2, 0, 0, 0, 2)), (16, (0, 0, 2, 0, 0, 2))],
    5: [(128 / 3, (0, 0, 1, 1, 0, 0)), (128 / 3, (0, 1, 0, 0, 1, 0)), (-96, (0, 2, 0, 0, 0, 2)),
        (-96, (0, 0, 2, 0, 0, 2))],
    6: [(-128 / 3, (0, 0, 1, 0, 0, 1)), (-128 / 3, (1, 0, 0, 0, 1, 0)), (96, (2, 0, 0, 2, 0, 0)),
        (96, (0, 0, 2, 2, 0, 0))],
    7: [(3456, (0, 0, 0, 0, 0, 0)), (-1152, (1, 0, 1, 2, 0, 0)), (-1152, (1, 1, 0, 0, 2, 0)),
        (-1152, (0, 1, 1, 0, 0, 2))],
}


@pytest.fixture
def user(O):
    yield O
    for row in range(1, 8):
        O.set_matrix_element(row, [])


def test_table_one_as_user_terms(user):
    O = user
    rng = np.random.Generator(np.random.PCG64(3))
    pts = []
    for _ in range(40):
        s = rng.uniform(0.2, 20.0)
        t = -rng.uniform(0.0, s)
        u = -s - t + rng.uniform(-0.3, 0.3)   # off the massless shell too
        pts.append((s, t, u, rng.uniform(0.05, 1.0)))
    built_in = {row: [O.msq(row, s, t, u, mu, ALPHA) for s, t, u, mu in pts] for row in TABLE_I}
    for row, terms in TABLE_I.items():
        O.set_matrix_element(row, terms)
    for row in TABLE_I:
        got = [O.msq(row, s, t, u, mu, ALPHA) for s, t, u, mu in pts]
        assert np.allclose(got, built_in[row], rtol=1e-12, atol=0), row
    O.set_matrix_element(7, [])
    assert O.msq(7, *pts[0], ALPHA) == built_in[7][0]


@pytest.mark.parametrize("mu", [0.1, 0.6])
def test_user_row_angular_integral(user, mu):
    O = user
    O.set_matrix_element(7, [(1.0, (2, 0, 0, 2, 0, 0))])
    g = O.Grid(n_p=(4, 4, 4), p_half=(3.0, 3.0, 3.0), species_mask=1 << 6)
    ch = O.channels(g)[0]
    m2 = np.zeros((7, 1)); m2[6, 0] = mu
    f = np.zeros((7, 1, g.nodes))
    rng = np.random.Generator(np.random.PCG64(5))
    flags = O.REF_B_ONE | O.REF_NO_BOXCUT | O.REF_MASSLESS
    for _ in range(4):
        p1, p2 = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        fn = lambda c: O.eval_cm(g, ch, f, m2, 0, p1, p2, c, 0.7, flags=flags)["g"]
        ang, _ = integrate.quad(fn, -1, 1, epsabs=0, epsrel=1e-11, limit=400)
        E1, E2 = np.linalg.norm(p1), np.linalg.norm(p2)
        s = 2 * (E1 * E2 - p1 @ p2)
        pref = (math.sqrt(s) / 2) / ((2 * np.pi) ** 3 * 2 * E1 * 2 * E2 * 16 * np.pi ** 2 * math.sqrt(s))
        expect = 2 * np.pi * pref * G4 * 2 * s * s / (mu * (s + mu))
        assert 2 * np.pi * ang == pytest.approx(expect, rel=1e-9)


def test_bad_terms_refused(user):
    O = user
    with pytest.raises(ValueError):
        O.set_matrix_element(0, [(1.0, (0,) * 6)])
    with pytest.raises(ValueError):
        O.set_matrix_element(7, [(1.0, (5, 0, 0, 0, 0, 0))])
    with pytest.raises(ValueError):
        O.set_matrix_element(7, [(1.0, (0,) * 6)] * 9)
