"""Pins for the oracle's thermalisation diagnostics: the Boltzmann entropy and
the diagonal of Eq. energy momentum tensor.

* on Bose-Einstein and Fermi-Dirac occupations f = 1/(e^x -+ 1), x = (E - mu)/T,
  the entropy per node equals f x + ln(1 + f) (bosons) and f x - ln(1 - f)
  (fermions): algebraic identities of the equilibrium forms;
* the trace: E_total - sum_i T_ii = sum N dV m^2 f / E, which is also four times
  E_total - E_total_mod of the modified tensor (the C observables and the numpy
  bookkeeping);
* an isotropic f on a cubic grid has T_xx = T_yy = T_zz; one stretched along z
  has T_zz > T_xx.
"""
import numpy as np
import pytest

from paper_1912_04457_amd import workloads as W


def _grid(O, n=8, mask=0x7F, cells=(1, 1, 1)):
    return O.Grid(n_x=cells, n_p=(n, n, n), p_half=(2.0, 2.0, 2.0), species_mask=mask)


def test_entropy_of_equilibrium_forms(O):
    g = _grid(O)
    m2 = O.constant_masses(g, [0.05] * 6 + [0.2])
    E = np.sqrt((g.momenta() ** 2).sum(1)[None, :] + m2[:, 0][:, None])
    T, mu = 0.35, np.array([0.1, -0.05, 0.0, -0.1, 0.05, 0.0, -0.02])
    x = (E - mu[:, None]) / T
    f = np.zeros((7, 1, g.nodes))
    per_node = np.zeros((7, g.nodes))
    for sp in range(7):
        if sp == O.GLUON:
            f[sp, 0] = 1.0 / np.expm1(x[sp])
            per_node[sp] = f[sp, 0] * x[sp] + np.log1p(f[sp, 0])
        else:
            f[sp, 0] = 1.0 / (np.exp(x[sp]) + 1.0)
            per_node[sp] = f[sp, 0] * x[sp] - np.log1p(-f[sp, 0])
    want = float((O.DEGENERACY[:, None] * per_node).sum() * O._cell_measure(g))
    assert O.thermo(g, f, m2)["entropy"] == pytest.approx(want, rel=1e-12)


def test_trace_of_the_tensor(O):
    g = _grid(O, cells=(2, 1, 1))
    f = W.smooth_f(g.cells, g.n_p, g.p_half)
    f[:, 1] *= 0.6
    m2 = O.masses(g, f)
    t = O.thermo(g, f, m2)
    E_total = O.observables(g, f, m2)["E_total"]
    mass_term = 4.0 * (E_total - O.modified_energy(g, f, m2))
    assert E_total - t["T_ii"].sum() == pytest.approx(mass_term, rel=1e-10)
    assert mass_term > 1e-3 * E_total


def test_isotropy_of_the_pressures(O):
    g = _grid(O, n=10, mask=1 << 6)
    P = g.momenta()
    f = np.zeros((7, 1, g.nodes))
    f[6, 0] = np.exp(-(P ** 2).sum(1) / 1.2)
    m2 = O.constant_masses(g, [0.0] * 6 + [0.3])
    T = O.thermo(g, f, m2)["T_ii"]
    assert T[0] == pytest.approx(T[1], rel=1e-13) and T[0] == pytest.approx(T[2], rel=1e-13)
    f[6, 0] = np.exp(-(P[:, 0] ** 2 + P[:, 1] ** 2) / 1.2 - P[:, 2] ** 2 / 2.4)
    T = O.thermo(g, f, m2)["T_ii"]
    assert T[2] > 1.3 * T[0]
