"""Pins for the oracle's time step (Sec. III, Eq. left handside with the
collision term, forward Euler), composed from the pinned primitives.

* total particle number (Eq. particle numbers, summed over species) is conserved
  to rounding with symmetric sampling and a conservative drift; per-species
  numbers change (Sec. IV B);
* without symmetric sampling the total number drifts;
* the first step evaluates the thermal masses with E = |p|, later steps with the
  lagged masses (Sec. II after Eq. mq).
"""
import numpy as np

from paper_1912_04457_amd import workloads as W


def _setup(O, n_x=(2, 2, 1)):
    g = O.Grid(n_x=n_x, n_p=(6, 6, 6), x_half=(3.0, 3.0, 3.0), p_half=(2.0, 2.0, 2.0),
               species_mask=0x7F)
    f = W.smooth_f(g.cells, g.n_p, g.p_half, amp_g=0.5)
    f[:, 1:] *= 0.7       # inhomogeneous in x
    return g, f


def test_number_conserved_over_steps(O):
    g, f = _setup(O)
    st = O.State(f=f.copy())
    N0 = O.observables(g, st.f, O.masses(g, st.f))["N_total"]
    Ns = []
    for _ in range(3):
        obs = O.step(g, st, 0.01, 16, 0x5EED2019)
        Ns.append(obs["N_total"])
    assert max(abs(n - N0) for n in Ns) <= 1e-13 * N0
    assert abs(st.history[-1]["N"][6] - O.observables(g, f, O.masses(g, f))["N"][6]) > 1e-9 * N0


def test_direct_mode_violates_number(O):
    g, f = _setup(O, n_x=(1, 1, 1))
    st = O.State(f=f.copy())
    N0 = O.observables(g, st.f, O.masses(g, st.f))["N_total"]
    obs = O.step(g, st, 0.01, 16, 0x5EED2019, symmetric=False)
    assert abs(obs["N_total"] - N0) > 1e-8 * N0


def test_lagged_masses(O):
    g, f = _setup(O, n_x=(1, 1, 1))
    st = O.State(f=f.copy())
    O.step(g, st, 0.01, 8, 1)
    assert np.allclose(st.history[0]["mass2"], O.masses(g, f))           # E = |p|
    f1 = st.f.copy()
    O.step(g, st, 0.01, 8, 1)
    assert np.allclose(st.history[1]["mass2"], O.masses(g, f1, st.history[0]["mass2"]))
