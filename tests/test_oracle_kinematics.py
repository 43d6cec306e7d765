"""Pins for the oracle's sample kinematics and two-body phase space.

* Conservation and on-shell conditions hold per sample (Sec. III: the sampled
  configuration satisfies k1 + k2 = k3 + p exactly).
* The angular integral of the regulated gg -> gg |M|^2 over the CM solid angle,
  for massless kinematics and B = 1, has the closed form
      int_{-1}^{1} dcos [3 - su/(t-mu)^2 - st/(u-mu)^2 - tu/s^2]
        = 17/3 + 4 (s/mu - ln(1 + s/mu)),
  which fixes the two-body phase-space factor |p*|/(16 pi^2 sqrt s), the
  (2 pi)^3 2E1 2E2 measure, Table I row 7 and the regulator placement.
"""
import math

import numpy as np
import pytest
from scipy import integrate

ALPHA = 0.3
G4 = (4 * math.pi * ALPHA) ** 2


def _grid(O, **kw):
    return O.Grid(n_p=(6, 6, 6), p_half=(3.0, 3.0, 3.0), species_mask=0x7F, **kw)


def test_conservation_and_mass_shell(O):
    g = _grid(O)
    chans = O.channels(g)
    rng = np.random.Generator(np.random.PCG64(11))
    f = np.zeros((7, 1, g.nodes))
    for trial in range(300):
        ch = chans[rng.integers(len(chans))]
        m2 = np.zeros((7, 1))
        mq = rng.uniform(0.0, 0.5)
        m2[:6, 0] = mq
        m2[6, 0] = rng.uniform(0.05, 0.8)
        p1, p2 = rng.uniform(-3, 3, 3), rng.uniform(-3, 3, 3)
        r = O.eval_cm(g, ch, f, m2, 0, p1, p2, rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi),
                      flags=O.REF_NO_BOXCUT)
        if r["s"] <= (math.sqrt(m2[ch["sp"][2], 0]) + math.sqrt(m2[ch["sp"][3], 0])) ** 2:
            assert not r["valid"]
            continue
        assert r["valid"]
        k = r["k"]
        scale = np.abs(k).max()
        assert np.allclose(k[0] + k[1], k[2] + k[3], rtol=0, atol=1e-13 * scale)
        for i in range(4):
            mass2 = k[i, 0] ** 2 - k[i, 1:] @ k[i, 1:]
            assert mass2 == pytest.approx(m2[ch["sp"][i], 0], abs=1e-12 * scale ** 2)
        msum = sum(m2[ch["sp"][i], 0] for i in range(4))
        assert r["s"] + r["t"] + r["u"] == pytest.approx(msum, abs=1e-12 * scale ** 2)
        # |p*| is the final-state momentum in the CM frame
        P = k[2] + k[3]
        M = math.sqrt(P[0] ** 2 - P[1:] @ P[1:])
        e3 = (P[0] * k[2, 0] - P[1:] @ k[2, 1:]) / M
        assert math.sqrt(max(e3 ** 2 - m2[ch["sp"][2], 0], 0)) == pytest.approx(r["pstar"], rel=1e-9, abs=1e-12)


def test_polar_axis_is_observed_particle(O):
    """cos theta* = 1 sends particle 3 along particle 1 in the CM frame (t -> t_max)."""
    g = _grid(O)
    ch = [c for c in O.channels(g) if c["row"] == 7][0]
    m2 = np.zeros((7, 1)); m2[6, 0] = 0.3
    f = np.zeros((7, 1, g.nodes))
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(20):
        p1, p2 = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        r = O.eval_cm(g, ch, f, m2, 0, p1, p2, 1.0, rng.uniform(0, 6), flags=O.REF_NO_BOXCUT)
        # equal masses: forward scattering leaves k3 = k1, so t = 0
        assert abs(r["t"]) < 1e-12 * r["s"]
        assert np.allclose(r["k"][2], r["k"][0], atol=1e-12)


def _gg_closed_form(s, mu):
    return 17.0 / 3.0 + 4.0 * (s / mu - math.log1p(s / mu))


def test_closed_form_itself():
    """The closed form against direct quadrature of its integrand."""
    for s, mu in ((1.0, 0.3), (4.0, 0.2865), (0.5, 1.0), (9.0, 0.05)):
        def h(c):
            t, u = -s * (1 - c) / 2, -s * (1 + c) / 2
            return 3 - s * u / (t - mu) ** 2 - s * t / (u - mu) ** 2 - t * u / s ** 2
        val, _ = integrate.quad(h, -1, 1, epsabs=1e-13, epsrel=1e-13, limit=200)
        assert val == pytest.approx(_gg_closed_form(s, mu), rel=1e-12)


@pytest.mark.parametrize("mu", [0.05, 0.3, 1.0])
def test_gg_angular_integral_closed_form(O, mu):
    g = O.Grid(n_p=(4, 4, 4), p_half=(3.0, 3.0, 3.0), species_mask=1 << 6)
    ch = O.channels(g)[0]
    m2 = np.zeros((7, 1)); m2[6, 0] = mu
    f = np.zeros((7, 1, g.nodes))
    rng = np.random.Generator(np.random.PCG64(4))
    flags = O.REF_B_ONE | O.REF_NO_BOXCUT | O.REF_MASSLESS
    for _ in range(6):
        p1, p2 = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        phi = rng.uniform(0, 2 * np.pi)
        fn = lambda c: O.eval_cm(g, ch, f, m2, 0, p1, p2, c, phi, flags=flags)["g"]
        ang, _ = integrate.quad(fn, -1, 1, epsabs=0, epsrel=1e-11, limit=400, points=[1 - 1e-3])
        # g is independent of phi for B = 1, massless: integral over phi is 2 pi
        total = 2 * np.pi * ang
        E1, E2 = np.linalg.norm(p1), np.linalg.norm(p2)
        s = 2 * (E1 * E2 - p1 @ p2)
        pstar = math.sqrt(s) / 2
        pref = pstar / ((2 * np.pi) ** 3 * 2 * E1 * 2 * E2 * 16 * np.pi ** 2 * math.sqrt(s))
        expect = 2 * np.pi * pref * 16 * G4 * 8 * 9 * _gg_closed_form(s, mu)
        assert total == pytest.approx(expect, rel=1e-9)
        # and independent of phi indeed
        c0 = 0.37
        assert fn(c0) == pytest.approx(O.eval_cm(g, ch, f, m2, 0, p1, p2, c0, phi + 1.0, flags=flags)["g"],
                                       rel=1e-12)
