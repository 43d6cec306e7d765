"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Same seed, same step index, same f => the same Philox samples on both sides, so
the collision terms agree element by element:
  FP64 mode  |A_gpu - A_ref| <= 1e-10 * S(x,q)   and   ||dA||_2 <= 1e-10 ||A||_2
  FP32 mode  |A_gpu - A_ref| <= 1e-4  * S(x,q)   and   ||dA||_2 <= 1e-4  ||A||_2
S is the oracle's cell scale: the sum over all deposits at (x,q) of
|w V5 |M|^2 (gain + loss) ...|, the natural magnitude of the rounding error of a
gain-minus-loss difference (A itself vanishes where gain = loss).
"""
import numpy as np
import pytest

from paper_1912_04457_amd import qgbe
from paper_1912_04457_amd import workloads as W

pytestmark = pytest.mark.gpu

SEED = 0x5EED2019
TOL = {qgbe.FP64: 1e-10, qgbe.FP32: 1e-4}


def _case(name):
    print(f"\n[gpu case] {name}", flush=True)


def _grid_kw(wl):
    return dict(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
                species_mask=wl.species_mask, alpha_s=wl.alpha_s)


def _compare(A, A_ref, S_ref, tol, what=""):
    err = np.abs(A - A_ref)
    bound = tol * S_ref
    bad = err > bound + 1e-300
    assert not bad.any(), (what, int(bad.sum()), float((err / np.maximum(S_ref, 1e-300)).max()))
    l2 = np.linalg.norm((A - A_ref).ravel()) / max(np.linalg.norm(A_ref.ravel()), 1e-300)
    assert l2 <= tol, (what, l2)


def _run_pair(O, wl, f, N, precision, step=0, symmetric=True):
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half,
               species_mask=wl.species_mask, alpha_s=wl.alpha_s)
    with qgbe.Solver(**_grid_kw(wl), precision=precision, symmetric=int(symmetric), seed=SEED) as s:
        s.set_f(f)
        qgbe.qgbe_set_step_index(s.ctx, step)
        A, _, I, st = s.collision(N, items=True)
        m_gpu = s.masses()
    m_ref = O.masses(g, f)
    A_ref, S_ref, I_ref = O.collision(g, f, m_ref, SEED, step, N, symmetric=symmetric, want_items=True)
    return dict(A=A, I=I, st=st, m=m_gpu, A_ref=A_ref, S_ref=S_ref, I_ref=I_ref, m_ref=m_ref, grid=g)


def test_device_info():
    torch = pytest.importorskip("torch")
    p = torch.cuda.get_device_properties(0)
    print(f"\n[device] {p.name} CUs={p.multi_processor_count} mem={p.total_memory / 2**30:.0f} GiB "
          f"arch={getattr(p, 'gcnArchName', '?')}", flush=True)
    assert p.multi_processor_count > 0


SMALL_7 = W.Workload("qg7_2cells_5x6x4", (2, 1, 1), (5, 6, 4), (3.0, 3.0, 3.0), (2.0, 2.5, 1.5),
                     0x7F, 100, "f64", 1, 0.01)


@pytest.mark.parametrize("precision", [qgbe.FP64, qgbe.FP32])
def test_gluon_config1(O, precision):
    """1 cell, 10^3 on [-2,2]^3, gg -> gg, f = 0.5 theta(1 - |p|), N = 1000."""
    _case(f"gluon C1 precision={precision}")
    wl = W.C1
    r = _run_pair(O, wl, W.initial_f(wl), 1000, precision)
    assert np.allclose(r["m"], r["m_ref"], rtol=1e-13, atol=0)
    _compare(r["A"], r["A_ref"], r["S_ref"], TOL[precision], "A")
    scale_items = np.abs(r["I_ref"]).max()
    assert np.allclose(r["I"], r["I_ref"], rtol=TOL[precision], atol=TOL[precision] * scale_items)
    assert r["st"].n_evals == 1000 * 1000
    assert r["st"].n_collide_launches >= 1


@pytest.mark.parametrize("precision", [qgbe.FP64, qgbe.FP32])
@pytest.mark.parametrize("symmetric", [True, False])
def test_seven_species_ragged(O, precision, symmetric):
    """70 channels, 2 cells, ragged 5x6x4 grid, N = 100 (not a multiple of 64)."""
    _case(f"7 species ragged precision={precision} symmetric={symmetric}")
    f = W.random_f(21, SMALL_7.cells, SMALL_7.nodes)
    r = _run_pair(O, SMALL_7, f, 100, precision, step=3, symmetric=symmetric)
    assert np.allclose(r["m"], r["m_ref"], rtol=1e-13, atol=0)
    _compare(r["A"], r["A_ref"], r["S_ref"], TOL[precision], "A")


@pytest.mark.parametrize("mask", [1 << 6, 0x7F], ids=["gluons", "qg7"])
def test_partial_node_block_fp32(O, mask):
    """105 momenta (3 x 5 x 7): the compacting variant (the gluon channel) and
    the plain ones, where chunks and the last node block end inside a block of
    4 consecutive nodes."""
    _case(f"3x5x7 nodes mask={mask:#x} fp32")
    wl = W.Workload("2cells_3x5x7", (2, 1, 1), (3, 5, 7), (3.0, 3.0, 3.0), (2.0, 2.5, 1.5),
                    mask, 100, "f32", 1, 0.01)
    f = W.random_f(24, wl.cells, wl.nodes, species_mask=mask)
    r = _run_pair(O, wl, f, 100, qgbe.FP32, step=6)
    # odd on every axis: the centre node at p = 0 (E = 0 for a massless lagged mass)
    assert np.allclose(r["m"], r["m_ref"], rtol=1e-13, atol=0)
    _compare(r["A"], r["A_ref"], r["S_ref"], TOL[qgbe.FP32], "A")
    scale_items = np.abs(r["I_ref"]).max()
    assert np.allclose(r["I"], r["I_ref"], rtol=TOL[qgbe.FP32], atol=TOL[qgbe.FP32] * scale_items)
    assert np.all(r["S_ref"][6, :, -1] > 0)   # the bar binds at the last node


@pytest.mark.parametrize("precision", [qgbe.FP64, qgbe.FP32])
def test_conservation(O, precision):
    _case(f"conservation precision={precision}")
    f = W.random_f(22, SMALL_7.cells, SMALL_7.nodes)
    r = _run_pair(O, SMALL_7, f, 64, precision)
    for cell in range(SMALL_7.cells):
        assert abs(r["A"][:, cell].sum()) <= 1e-13 * r["S_ref"][:, cell].sum()


def test_config3_lds_layout_fp32(O):
    """20^3, 7 species (three-slot channels with one f tile outside LDS), N = 8."""
    _case("C3 layout fp32 N=8")
    wl = W.C3
    f = W.initial_f(wl)
    r = _run_pair(O, wl, f, 8, qgbe.FP32)
    _compare(r["A"], r["A_ref"], r["S_ref"], 1e-4, "A")
    assert abs(r["A"].sum()) <= 1e-13 * r["S_ref"].sum()


@pytest.mark.parametrize("n_p,mask,N", [((32, 32, 32), 1 << 6, 4), ((24, 24, 24), 0x7F, 2),
                                         ((28, 28, 28), 0x7F, 1)],
                         ids=["g_32cube", "qg7_24cube", "qg7_28cube"])
def test_large_grid_lds_plans_fp32(O, n_p, mask, N):
    """Grids whose FP64 accumulators do not fit in LDS: 24^3 holds one slot
    per launch; at 32^3 and 28^3 not even one slot fits, and each slot runs
    as two node windows (launches whose accumulators cover half the nodes,
    corners outside left to the other), f from the global node quads."""
    _case(f"large grid {n_p} mask={mask:#x} N={N}")
    wl = W.C3.scaled(n_p=n_p, species_mask=mask)
    f = W.initial_f(wl)
    r = _run_pair(O, wl, f, N, qgbe.FP32)
    _compare(r["A"], r["A_ref"], r["S_ref"], 1e-4, "A")
    assert abs(r["A"].sum()) <= 1e-13 * r["S_ref"].sum()


def test_spatial_small_fp32(O):
    """4x4x1 cells of a Gaussian transverse profile, 8^3 momenta, N = 96."""
    _case("spatial small fp32")
    wl = W.C2.scaled(n_x=(4, 4, 1), n_p=(8, 8, 8), x_half=(6.0, 6.0, 0.375))
    r = _run_pair(O, wl, W.initial_f(wl), 96, qgbe.FP32)
    _compare(r["A"], r["A_ref"], r["S_ref"], 1e-4, "A")


def test_device_pointers_match_host(O):
    """Torch device tensors through the same ABI give the same result."""
    torch = pytest.importorskip("torch")
    _case("device pointers")
    wl = SMALL_7
    f = W.random_f(23, wl.cells, wl.nodes)
    with qgbe.Solver(**_grid_kw(wl), precision=qgbe.FP64, seed=SEED) as s:
        s.set_f(torch.from_numpy(f).cuda())
        A_dev = torch.zeros((7, wl.cells, wl.nodes), dtype=torch.float64, device="cuda")
        qgbe.qgbe_collision_term(s.ctx, 50, qgbe.SAMPLER_UNIFORM, A_dev)
        torch.cuda.synchronize()
        A_host, _, _, _ = s.collision(50)
    assert np.array_equal(A_dev.cpu().numpy(), A_host) or np.allclose(A_dev.cpu().numpy(), A_host, rtol=1e-12)


def test_step_parity_fp64(O):
    """Three upwind steps on a 2x2x1 spatial grid, dynamic masses, 7 species."""
    _case("step parity fp64")
    wl = W.Workload("qg7_2x2x1_6cube", (2, 2, 1), (6, 6, 6), (3.0, 3.0, 3.0), (2.0, 2.0, 2.0),
                    0x7F, 16, "f64", 3, 0.01)
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    f0 = W.smooth_f(wl.cells, wl.n_p, wl.p_half, amp_g=0.5)
    f0[:, 1:] *= 0.7
    st = O.State(f=f0.copy())
    ref = [O.step(g, st, wl.dt_fm, wl.n_samples, SEED) for _ in range(3)]
    with qgbe.Solver(**_grid_kw(wl), precision=qgbe.FP64, seed=SEED) as s:
        s.set_f(f0)
        stats = s.step(wl.dt_fm, wl.n_samples, n_steps=3)
        f_gpu = s.get_f()
    change = np.abs(st.f - f0).max()
    assert np.abs(f_gpu - st.f).max() <= 1e-10 * change
    for a, b in zip(stats, ref):
        assert a["N_total"] == pytest.approx(b["N_total"], rel=1e-13)
        assert a["E_total"] == pytest.approx(b["E_total"], rel=1e-12)
        assert np.allclose(a["mass2_avg"], b["mass2"].mean(axis=1), rtol=1e-12)
        # energy bookkeeping (Eq. current conservation; modified tensor of Sec. IV)
        assert abs(a["E_source"] - b["E_source"]) <= 1e-12 * b["E_total"]
        assert abs(a["E_collide"] - b["E_collide"]) <= 1e-12 * b["E_total"]
        assert a["E_total_mod"] == pytest.approx(b["E_total_mod"], rel=1e-12)
        assert a["entropy"] == pytest.approx(b["entropy"], rel=1e-12)
        assert np.allclose(a["T_ii"], b["T_ii"], rtol=1e-12)
    assert stats[0]["E_source"] == 0.0 and stats[1]["E_source"] != 0.0
    N0 = O.observables(g, f0, O.masses(g, f0))["N_total"]
    assert abs(stats[-1]["N_total"] - N0) <= 1e-13 * N0


def test_energy_source_accounts_for_kinetic_energy_change():
    """The energy test of Sec. IV with dynamic masses: in a homogeneous pure
    gluon system the kinetic energy changes by the mass source term plus the
    collision term's grid residue, step by step (FP32 integrand; the
    bookkeeping itself is FP64)."""
    _case("energy bookkeeping fp32")
    wl = W.Workload("g_1cell_10cube", (1, 1, 1), (10, 10, 10), (3.0, 3.0, 3.0), (2.0, 2.0, 2.0),
                    1 << 6, 128, "f32", 4, 0.01)
    P = W.node_momenta(wl.n_p, wl.p_half)
    f0 = np.zeros((7, 1, wl.nodes))
    f0[6, 0] = 0.5 * (np.linalg.norm(P, axis=1) < 1.5)
    with qgbe.Solver(**_grid_kw(wl), precision=qgbe.FP32, seed=SEED) as s:
        s.set_f(f0)
        stats = s.step(wl.dt_fm, wl.n_samples, n_steps=4)
    for k in range(1, 4):
        change = stats[k]["E_total"] - stats[k - 1]["E_total"]
        parts = stats[k]["E_source"] + stats[k]["E_collide"]
        assert abs(change - parts) <= 1e-12 * stats[k]["E_total"], k
        assert abs(stats[k]["E_collide"]) < 0.05 * abs(stats[k]["E_source"])
    assert all(st["E_total_mod"] < st["E_total"] for st in stats)


def test_step_parity_central_fp32(O):
    _case("step parity central fp32")
    wl = W.Workload("g_3x1x1_8cube", (3, 1, 1), (8, 8, 8), (3.0, 3.0, 3.0), (2.0, 2.0, 2.0),
                    1 << 6, 32, "f32", 2, 0.01, drift="central")
    g = O.Grid(n_x=wl.n_x, n_p=wl.n_p, x_half=wl.x_half, p_half=wl.p_half, species_mask=wl.species_mask)
    f0 = W.smooth_f(wl.cells, wl.n_p, wl.p_half, species_mask=wl.species_mask)
    f0[6, 0] *= 1.3
    st = O.State(f=f0.copy())
    for _ in range(2):
        O.step(g, st, wl.dt_fm, wl.n_samples, SEED, scheme="central")
    with qgbe.Solver(**_grid_kw(wl), precision=qgbe.FP32, drift=qgbe.DRIFT_CENTRAL, seed=SEED) as s:
        s.set_f(f0)
        stats = s.step(wl.dt_fm, wl.n_samples, n_steps=2)
        f_gpu = s.get_f()
    change = np.abs(st.f - f0).max()
    assert np.abs(f_gpu - st.f).max() <= 1e-4 * change
    N0 = O.observables(g, f0, O.masses(g, f0))["N_total"]
    assert abs(stats[-1]["N_total"] - N0) <= 1e-13 * N0


def test_constant_mass_and_flags(O):
    _case("constant mass + flags")
    wl = W.C1
    f = W.initial_f(wl)
    f[6, 0, 0] = -0.1           # a negative occupation must be flagged
    cm = [0.1] * 6 + [0.5]
    with qgbe.Solver(**_grid_kw(wl), precision=qgbe.FP64, mass_mode=qgbe.MASS_CONSTANT,
                     const_mass2=cm, seed=SEED) as s:
        s.set_f(f)
        st = qgbe.Stats()
        qgbe.qgbe_observables(s.ctx, st)
        assert np.allclose(s.masses()[:, 0], cm)
        assert st.flags & qgbe.FLAG_NEGATIVE_F
    g = O.Grid(n_p=wl.n_p, p_half=wl.p_half, species_mask=wl.species_mask)
    ref = O.observables(g, f, O.constant_masses(g, cm))
    assert st.N_total == pytest.approx(ref["N_total"], rel=1e-13)
    assert st.E_total == pytest.approx(ref["E_total"], rel=1e-13)


def test_empty_distribution_gives_zero(O):
    _case("empty f")
    with qgbe.Solver(**_grid_kw(SMALL_7), precision=qgbe.FP32, seed=SEED) as s:
        A, _, _, _ = s.collision(64)
    assert np.all(A == 0.0)


def test_errors_reported():
    _case("error paths")
    with qgbe.Solver(**_grid_kw(SMALL_7), precision=qgbe.FP32, seed=SEED) as s:
        with pytest.raises(qgbe.QgbeError) as e:
            qgbe.qgbe_collision_term(s.ctx, 0, qgbe.SAMPLER_UNIFORM, np.zeros((7, 2, 120)))
        assert e.value.status == qgbe.EINVAL
        with pytest.raises(qgbe.QgbeError):
            qgbe.qgbe_set_distribution(s.ctx, 9, np.zeros((2, 120)))
        with pytest.raises(qgbe.QgbeError):
            qgbe.qgbe_step(s.ctx, -1.0, 8, 0, 1)


@pytest.mark.parametrize("precision", [qgbe.FP64, qgbe.FP32])
def test_mc_error_estimate_matches_replicas(precision):
    """stats.mc_err_est (from each item's own samples) against the spread of
    the item sums over independent replicas (other step indices)."""
    _case(f"mc error estimate precision={precision}")
    wl = W.C3.scaled(n_p=(8, 8, 8))
    R, N = 16, 256
    with qgbe.Solver(**_grid_kw(wl), precision=precision, seed=SEED) as s:
        s.set_f(W.initial_f(wl))
        est, items = [], []
        for r in range(R):
            qgbe.qgbe_set_step_index(s.ctx, 100 + r)
            _, _, I, st = s.collision(N, items=True)
            est.append(st.mc_err_est)
            items.append(I)
    I = np.array(items)
    emp = np.sqrt(I.var(0, ddof=1).sum() / (I.mean(0) ** 2).sum())
    print(f"[mc error] estimate {np.mean(est):.4f} (spread {np.std(est):.4f}), replicas {emp:.4f}", flush=True)
    assert 0.8 < np.mean(est) / emp < 1.25
