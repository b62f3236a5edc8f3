"""Pins of the bulk and D2d DMI fields of the oracle (CPU only).

Interior cells of spin spirals have closed-form discrete fields: for a spiral
of wave number q on cells of size d, each neighbour pair along the
propagation axis contributes e x (m(+d) - m(-d)) = +-2 sin(qd) m, so the field
is +-(2 D sin(qd) / (mu0 Ms d)) m (the continuum limit is the curl form of the
DMI section, -(2D/(mu0 Ms)) curl m for the bulk class).  Worked by hand:

* bulk, Bloch spirals along x (m in the y-z plane) and along z (m in the x-y
  plane): +(2 D sin(qd) / (mu0 Ms d)) m;
* D2d, the spiral along x with m in the y-z plane and the spiral along y with
  m in the x-z plane: -(2 D sin(qd) / (mu0 Ms d)) m (the opposite handedness
  along x and y that favours antiskyrmions), and no field from z neighbours;

and both fields are gradients of their energies (the discrete operators are
symmetric).
"""
import math

import numpy as np
import pytest

from oracle import fields as F

MU0 = 4e-7 * math.pi
N, D_CELL, Q = 40, 1e-9, 2 * math.pi / 50e-9


def _coef(p):
    return 2 * p.D * math.sin(Q * D_CELL) / (MU0 * p.Ms * D_CELL)


def test_bulk_spirals_along_x_and_z():
    p = F.Params(Ms=5.8e5, D=2e-3, terms=F.DMI_BULK)
    x = np.arange(N) * D_CELL
    m = np.zeros((3, 1, 3, N))
    m[1], m[2] = np.cos(Q * x), np.sin(Q * x)
    H = F.effective_field(m, F.Mesh(N, 3, 1, D_CELL, 3e-9, 1e-9), p)
    sl = (slice(None), 0, 1, slice(1, -1))
    np.testing.assert_allclose(H[sl], _coef(p) * m[sl], rtol=1e-10, atol=1e-6)
    z = np.arange(N) * D_CELL
    m = np.zeros((3, N, 3, 3))
    m[0], m[1] = np.cos(Q * z)[:, None, None], np.sin(Q * z)[:, None, None]
    H = F.effective_field(m, F.Mesh(3, 3, N, 3e-9, 3e-9, D_CELL), p)
    sl = (slice(None), slice(1, -1), 1, 1)
    np.testing.assert_allclose(H[sl], _coef(p) * m[sl], rtol=1e-10, atol=1e-6)


def test_d2d_spirals_along_x_and_y_and_no_z_coupling():
    p = F.Params(Ms=5.8e5, D=2e-3, terms=F.DMI_D2D)
    s = np.arange(N) * D_CELL
    m = np.zeros((3, 1, 3, N))
    m[1], m[2] = np.cos(Q * s), np.sin(Q * s)
    H = F.effective_field(m, F.Mesh(N, 3, 1, D_CELL, 3e-9, 1e-9), p)
    sl = (slice(None), 0, 1, slice(1, -1))
    np.testing.assert_allclose(H[sl], -_coef(p) * m[sl], rtol=1e-10, atol=1e-6)
    m = np.zeros((3, 1, N, 3))
    m[0], m[2] = np.cos(Q * s)[:, None], np.sin(Q * s)[:, None]
    H = F.effective_field(m, F.Mesh(3, N, 1, 3e-9, D_CELL, 1e-9), p)
    sl = (slice(None), 0, slice(1, -1), 1)
    np.testing.assert_allclose(H[sl], -_coef(p) * m[sl], rtol=1e-10, atol=1e-6)
    # a spiral along z has no D2d field (cells with both x and y neighbours)
    m = np.zeros((3, N, 3, 3))
    m[0], m[1] = np.cos(Q * s)[:, None, None], np.sin(Q * s)[:, None, None]
    H = F.effective_field(m, F.Mesh(3, 3, N, 3e-9, 3e-9, D_CELL), p)
    assert np.max(np.abs(H[:, :, 1, 1])) < 1e-6 * _coef(p)


@pytest.mark.parametrize("bit", [F.DMI_BULK, F.DMI_D2D])
def test_fields_are_energy_gradients(bit):
    mesh = F.Mesh(4, 3, 3, 2e-9, 3e-9, 1.5e-9)
    rng = np.random.default_rng(17)
    m = rng.normal(size=(3, 3, 3, 4))
    m /= np.linalg.norm(m, axis=0, keepdims=True)
    p = F.Params(Ms=6e5, D=2.5e-3, terms=bit)
    V = mesh.dx * mesh.dy * mesh.dz
    H = F.effective_field(m, mesh, p)
    g = np.zeros_like(m)
    eps = 1e-6
    for idx in np.ndindex(*m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[idx] += eps
        mm_[idx] -= eps
        g[idx] = (F.energies(mp_, mesh, p)[2] - F.energies(mm_, mesh, p)[2]) / (2 * eps)
    np.testing.assert_allclose(H, -g / (MU0 * p.Ms * V), rtol=1e-6, atol=1e-6 * np.max(np.abs(H)))
