"""Pins for the trilinear stencil through which the collision term reads f off
the grid and deposits its symmetric samples (readings R2 and R3).

* Inside the hull of the node centres the stencil interpolates trilinearly on
  the node-centre lattice: scipy's RegularGridInterpolator (method "linear")
  gives the same values for a random f on a ragged grid.
* Trilinear interpolation reproduces every function in
  span{1, x, y, z, xy, yz, zx, xyz} exactly.
* In the band between the outermost node centre and the box face the
  coordinate is clamped (R2): the value is the one at the nearest point of
  the hull.
* The weights are non-negative, sum to 1, and their first moment is the
  clamped momentum: a deposit keeps the sample's number and, inside the hull,
  its momentum (R3: the deposit is the transpose of the interpolation).
* Node indices are in range and follow the layout (ix n_y + iy) n_z + iz.
A transposed axis, a half-cell offset or a wrong clamp fails one of these.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

N_P = (5, 4, 6)
P_HALF = (2.0, 2.5, 1.5)


def _grid(O):
    return O.Grid(n_p=N_P, p_half=P_HALF, species_mask=1 << O.GLUON)


def _axes():
    return [-ph + (np.arange(n) + 0.5) * 2 * ph / n for n, ph in zip(N_P, P_HALF)]


def _inside(rng, n):
    ax = _axes()
    return np.stack([rng.uniform(a[0], a[-1], n) for a in ax], 1)


def test_trilinear_inside_the_hull_matches_scipy(O):
    rng = np.random.Generator(np.random.PCG64(11))
    f = rng.uniform(0.0, 1.0, int(np.prod(N_P)))
    pts = _inside(rng, 2000)
    ref = RegularGridInterpolator(_axes(), f.reshape(N_P), method="linear")(pts)
    got = O.interpolate(_grid(O), f, pts)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_reproduces_multilinear_functions(O):
    rng = np.random.Generator(np.random.PCG64(12))
    c = rng.normal(size=8)

    def h(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * z * x + c[7] * x * y * z

    g = _grid(O)
    pts = _inside(rng, 2000)
    got = O.interpolate(g, h(g.momenta()), pts)
    assert np.allclose(got, h(pts), rtol=1e-12, atol=1e-12)


def test_clamped_in_the_face_band(O):
    rng = np.random.Generator(np.random.PCG64(13))
    f = rng.uniform(0.0, 1.0, int(np.prod(N_P)))
    ph = np.array(P_HALF)
    pts = rng.uniform(-ph, ph, (4000, 3))
    ax = _axes()
    lo = np.array([a[0] for a in ax])
    hi = np.array([a[-1] for a in ax])
    clamped = np.clip(pts, lo, hi)
    band = np.any(pts != clamped, axis=1)
    assert band.sum() > 1000            # a third of the box lies in the face bands here
    g = _grid(O)
    got = O.interpolate(g, f, pts)
    ref = RegularGridInterpolator(ax, f.reshape(N_P), method="linear")(clamped)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-14)
    # the faces themselves
    face = np.array([[ph[0], 0.1, -0.2], [-ph[0], -ph[1], ph[2]]])
    assert np.allclose(O.interpolate(g, f, face), O.interpolate(g, f, np.clip(face, lo, hi)), rtol=1e-13)


def test_weights_partition_unity_and_first_moment(O):
    rng = np.random.Generator(np.random.PCG64(14))
    g = _grid(O)
    ph = np.array(P_HALF)
    pts = rng.uniform(-ph, ph, (3000, 3))
    idx, w = O.stencil(g, pts)
    assert idx.min() >= 0 and idx.max() < g.nodes
    assert np.all(w >= 0.0)
    assert np.allclose(w.sum(1), 1.0, rtol=0, atol=1e-15)
    q = g.momenta()
    ax = _axes()
    clamped = np.clip(pts, [a[0] for a in ax], [a[-1] for a in ax])
    first = np.einsum("nc,nca->na", w, q[idx])
    assert np.allclose(first, clamped, rtol=0, atol=1e-13)
    # the eight corners are the cell's corners, pz fastest in the node layout
    iz = idx % N_P[2]
    iy = (idx // N_P[2]) % N_P[1]
    ix = idx // (N_P[2] * N_P[1])
    for lin in (ix, iy, iz):
        assert np.all(lin.max(1) - lin.min(1) == 1)
