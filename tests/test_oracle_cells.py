"""Pins of the oracle's cell-based material (per-cell Ms, A, D; empty cells), CPU only.

* Constant arrays reproduce the uniform oracle (already pinned) term by term.
* Empty cells are an open boundary: a sample surrounded by Ms = 0 cells has,
  in its cells, exactly the fields and energies of the same sample meshed
  alone (the demag tensor depends only on the displacement), and zero field
  and torque outside.
* A hand-worked two-material chain: the exchange and DMI fields of the
  interface cells with the harmonic means worked out by hand (A_12 = 1.5e-11
  from 1e-11 and 3e-11; D_12 = 3e-3 from 2e-3 and 6e-3), and no DMI coupling
  across opposite chiralities.
* Every term is the gradient of its energy: H_i = -(1/(mu0 Ms_i V)) dE/dm_i
  with random per-cell Ms, A and D (this holds only if the pair couplings are
  symmetric and each field carries its own cell's 1/Ms_i), and the exchange
  energy equals the paper's pair form w_i.
* A uniformly magnetised cube of cubic cells embedded in empty cells has mean
  demag field -Ms/3 exactly.
* An A = 0 layer decouples the exchange of the blocks on either side.
* Interlayer coupling: a hand-worked pair across an empty spacer (fields and
  the energy density -J m_lo.m_hi + D_int.(m_lo x m_hi)), fields as gradients
  of that energy, and the energy recovered from the fields.
* Spin torques folded into the field: the LL result satisfies the paper's
  Gilbert-form equations (Slonczewski/SOT exactly; Zhang-Li on a spiral,
  whose central differences are tangent to the sphere), and with alpha = beta
  the Zhang-Li torque translates a spiral rigidly with velocity u.
"""
import math

import numpy as np
import pytest

from oracle import MU0
from oracle import cells as C
from oracle import fields as F

ALL7 = F.ALL_TERMS | F.DMI_BULK | F.DMI_D2D


def _unit(shape, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3,) + shape)
    return v / np.linalg.norm(v, axis=0)


def _const(shape, Ms, A, D):
    return C.Material(np.full(shape, Ms), np.full(shape, A), np.full(shape, D))


def test_constant_arrays_reduce_to_the_uniform_oracle():
    mesh = F.Mesh(6, 5, 3, 2e-9, 3e-9, 1.5e-9)
    m = _unit((3, 5, 6), 1)
    p = F.Params(Ms=6e5, A=1.2e-11, D=2.5e-3, Ku=4e5, u=(0.3, -0.2, 1.0), H=(1e4, -3e4, 5e4), terms=ALL7)
    mat = _const((3, 5, 6), p.Ms, p.A, p.D)
    ref = F.effective_field_terms(m, mesh, p)
    got = C.effective_field_terms(m, mesh, p, mat)
    assert set(ref) == set(got)
    for k in ref:
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-12, atol=1e-9 * np.max(np.abs(ref[k])))
    np.testing.assert_allclose(C.energies(m, mesh, p, mat), F.energies(m, mesh, p), rtol=1e-12, atol=1e-30)


@pytest.mark.parametrize("box", [((1, 6), (1, 5), (0, 2)), ((0, 5), (2, 6), (1, 3))])
def test_empty_cells_are_an_open_boundary(box):
    (x0, x1), (y0, y1), (z0, z1) = box
    big = F.Mesh(8, 6, 3, 2e-9, 2.5e-9, 3e-9)
    small = F.Mesh(x1 - x0, y1 - y0, z1 - z0, big.dx, big.dy, big.dz)
    p = F.Params(Ms=7e5, A=1.1e-11, D=2e-3, Ku=3e5, u=(0.1, 0.5, 1.0), H=(2e4, 1e4, -4e4), alpha=0.3,
                 terms=ALL7)
    Ms = np.zeros((3, 6, 8))
    Ms[z0:z1, y0:y1, x0:x1] = p.Ms
    mat = C.Material(Ms, np.full(Ms.shape, p.A), np.full(Ms.shape, p.D))  # A, D set everywhere
    m = _unit((3, 6, 8), 2)
    inner = (slice(None), slice(z0, z1), slice(y0, y1), slice(x0, x1))
    ref = F.effective_field_terms(np.ascontiguousarray(m[inner]), small, p)
    got = C.effective_field_terms(m, big, p, mat)
    empty = Ms == 0
    for k in ref:
        np.testing.assert_allclose(got[k][inner], ref[k], rtol=1e-11, atol=1e-10 * np.max(np.abs(ref[k])))
        assert np.all(got[k][:, empty] == 0)
    np.testing.assert_allclose(C.energies(m, big, p, mat), F.energies(np.ascontiguousarray(m[inner]), small, p),
                               rtol=1e-11, atol=1e-30)
    k = C.llg_rhs(m, big, p, mat)
    assert np.all(k[:, empty] == 0)


def test_hand_worked_two_material_chain():
    dx = 2e-9
    mesh = F.Mesh(4, 1, 1, dx, 3e-9, 1e-9)
    Ms1, Ms2 = 8e5, 4e5
    mat = C.Material(np.array([[[Ms1, Ms1, Ms2, Ms2]]]), np.array([[[1e-11, 1e-11, 3e-11, 3e-11]]]),
                     np.array([[[2e-3, 2e-3, 6e-3, 6e-3]]]))
    m = np.zeros((3, 1, 1, 4))
    m[2, 0, 0, :2] = 1.0  # cells 0, 1 along +z
    m[0, 0, 0, 2:] = 1.0  # cells 2, 3 along +x
    ex = C.exchange_field(m, mesh, mat)[:, 0, 0, :]
    A12 = 1.5e-11  # 2 * 1e-11 * 3e-11 / 4e-11, by hand
    np.testing.assert_allclose(ex[:, 0], 0.0, atol=1e-9)
    np.testing.assert_allclose(ex[:, 3], 0.0, atol=1e-9)
    np.testing.assert_allclose(ex[:, 1], 2 * A12 / (MU0 * Ms1 * dx ** 2) * np.array([1.0, 0.0, -1.0]), rtol=1e-12)
    np.testing.assert_allclose(ex[:, 2], 2 * A12 / (MU0 * Ms2 * dx ** 2) * np.array([-1.0, 0.0, 1.0]), rtol=1e-12)
    # interfacial DMI: e_{-x} = -e_y, e_{+x} = +e_y; (-e_y) x e_z = -e_x, e_y x e_x = -e_z; D_12 = 3e-3 by hand
    p = F.Params(Ms=1.0, terms=F.DMI)
    dmi = C.effective_field(m, mesh, p, mat)[:, 0, 0, :]
    np.testing.assert_allclose(dmi[:, 1], np.array([2e-3, 0.0, 3e-3]) / (MU0 * Ms1 * dx), rtol=1e-12)
    np.testing.assert_allclose(dmi[:, 2], np.array([3e-3, 0.0, 6e-3]) / (MU0 * Ms2 * dx), rtol=1e-12)
    # opposite chiralities do not couple
    mat2 = C.Material(mat.Ms, mat.A, np.array([[[2e-3, 2e-3, -6e-3, -6e-3]]]))
    dmi2 = C.effective_field(m, mesh, p, mat2)[:, 0, 0, :]
    np.testing.assert_allclose(dmi2[:, 1], np.array([2e-3, 0.0, 0.0]) / (MU0 * Ms1 * dx), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(dmi2[:, 2], np.array([0.0, 0.0, -6e-3]) / (MU0 * Ms2 * dx), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("bit", [F.EXCHANGE, F.DMI, F.DMI_BULK, F.DMI_D2D, F.ANIS, F.ZEEMAN, F.DEMAG])
def test_cell_fields_are_energy_gradients(bit):
    mesh = F.Mesh(4, 3, 3, 2e-9, 3e-9, 1.5e-9)
    rng = np.random.default_rng(40 + bit)
    Ms = rng.uniform(3e5, 1e6, size=(3, 3, 4))
    Ms[1, 1, 2] = 0.0
    Ms[0, 2, 0] = 0.0
    A = rng.uniform(0.5e-11, 2e-11, size=Ms.shape)
    A[2, 0, 1] = 0.0
    D = rng.uniform(-3e-3, 4e-3, size=Ms.shape)
    mat = C.Material(Ms, A, D)
    m = _unit((3, 3, 4), 9)
    p = F.Params(Ms=1.0, Ku=5e5, u=(0.4, -0.1, 1.0), H=(3e4, 2e4, -1e4), terms=bit)
    V = mesh.dx * mesh.dy * mesh.dz
    kern = F.DemagKernel(mesh)
    H = C.effective_field(m, mesh, p, mat, kern)
    n = F.ENERGY_ORDER.index("dmi" if bit in (F.DMI, F.DMI_BULK, F.DMI_D2D) else
                             {F.EXCHANGE: "exchange", F.ANIS: "anisotropy", F.ZEEMAN: "zeeman",
                              F.DEMAG: "demag"}[bit])
    g = np.zeros_like(m)
    eps = 1e-6
    for idx in np.ndindex(*m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[idx] += eps
        mm_[idx] -= eps
        g[idx] = (C.energies(mp_, mesh, p, mat, kern)[n] - C.energies(mm_, mesh, p, mat, kern)[n]) / (2 * eps)
    mag = Ms > 0
    expect = -g[:, mag] / (MU0 * Ms[mag] * V)
    np.testing.assert_allclose(H[:, mag], expect, rtol=1e-6, atol=1e-6 * np.max(np.abs(H)))
    assert np.all(H[:, ~mag] == 0)
    assert np.all(g[:, ~mag] == 0)  # empty cells carry no energy
    if bit == F.EXCHANGE:
        assert C.exchange_energy_pairs(m, mesh, mat) == pytest.approx(C.energies(m, mesh, p, mat)[0], rel=1e-12)


def test_cube_in_empty_cells_has_mean_field_minus_ms_over_3():
    d = 2e-9
    mesh = F.Mesh(7, 6, 5, d, d, d)
    Ms = np.zeros((5, 6, 7))
    Ms[1:5, 1:5, 2:6] = 8e5
    mat = C.Material(Ms, np.zeros(Ms.shape), np.zeros(Ms.shape))
    m = np.zeros((3, 5, 6, 7))
    m[0] = 1.0
    m[2, Ms == 0] = 1.0  # empty cells point elsewhere: they must not count
    H = C.effective_field(m, mesh, F.Params(Ms=1.0, terms=F.DEMAG), mat)
    mean = H[:, Ms > 0].mean(axis=1)
    np.testing.assert_allclose(mean, [-8e5 / 3, 0.0, 0.0], rtol=1e-12, atol=1e-6)


def test_zero_exchange_layer_decouples():
    mesh = F.Mesh(7, 3, 1, 2e-9, 2e-9, 1e-9)
    A = np.full((1, 3, 7), 1.3e-11)
    A[0, :, 3] = 0.0
    Ms = np.full(A.shape, 8e5)
    mat = C.Material(Ms, A, np.zeros(A.shape))
    m = _unit((1, 3, 7), 5)
    H = C.exchange_field(m, mesh, mat)
    left = F.Mesh(3, 3, 1, 2e-9, 2e-9, 1e-9)
    pl = F.Params(Ms=8e5, A=1.3e-11, terms=F.EXCHANGE)
    np.testing.assert_allclose(H[..., :3], F.exchange_field(np.ascontiguousarray(m[..., :3]), left, pl),
                               rtol=1e-12, atol=1e-6)
    np.testing.assert_allclose(H[..., 4:], F.exchange_field(np.ascontiguousarray(m[..., 4:]), left, pl),
                               rtol=1e-12, atol=1e-6)
    assert np.all(H[..., 3] == 0)


def test_llg_rhs_is_tangent_and_zero_in_empty_cells():
    mesh = F.Mesh(5, 4, 2, 2e-9, 2e-9, 2e-9)
    rng = np.random.default_rng(3)
    Ms = rng.uniform(4e5, 9e5, size=(2, 4, 5))
    Ms[:, 0, 0] = 0.0
    mat = C.Material(Ms, rng.uniform(1e-11, 2e-11, size=Ms.shape), rng.uniform(1e-3, 3e-3, size=Ms.shape))
    m = _unit((2, 4, 5), 4)
    p = F.Params(Ms=1.0, Ku=2e5, H=(0.0, 1e4, 5e4), alpha=0.2, terms=F.ALL_TERMS)
    k = C.llg_rhs(m, mesh, p, mat)
    assert np.max(np.abs(np.sum(m * k, axis=0))) <= 1e-12 * np.max(np.abs(k))
    assert np.all(k[:, Ms == 0] == 0)
    assert math.isfinite(float(np.max(np.abs(k))))


# ----------------------------------------------------------------------------- interlayer, torques

def test_interlayer_hand_worked_pair():
    """Two magnetic layers (z = 0 and z = 2) across an empty spacer: m_lo = e_x,
    m_hi = e_y, J = 1e-3, D_int = 2e-3 e_z.  By hand: w = -J e_x.e_y + D_int.(e_x x e_y)
    = 2e-3 J/m^2 per column; H_lo = (J e_y + D_int x e_y)/(mu0 Ms dz) = (-2e-3, 1e-3, 0)/(mu0 Ms dz),
    H_hi = (J e_x - D_int x e_x)/(mu0 Ms dz) = (1e-3, -2e-3, 0)/(mu0 Ms dz)."""
    mesh = F.Mesh(2, 1, 3, 2e-9, 3e-9, 1e-9)
    Ms = np.array([[[8e5, 8e5]], [[0.0, 0.0]], [[8e5, 8e5]]])
    mat = C.Material(Ms, np.zeros(Ms.shape), np.zeros(Ms.shape))
    m = np.zeros((3, 3, 1, 2))
    m[0, 0] = 1.0
    m[2, 1] = 1.0
    m[1, 2] = 1.0
    ex = C.Extra(k_lo=0, k_hi=2, J=1e-3, D_int=(0.0, 0.0, 2e-3))
    c = 1.0 / (MU0 * 8e5 * 1e-9)
    H = C.interlayer_field(m, mesh, mat, ex)
    np.testing.assert_allclose(H[:, 0, 0, :], c * np.array([[-2e-3] * 2, [1e-3] * 2, [0.0] * 2]), rtol=1e-12)
    np.testing.assert_allclose(H[:, 2, 0, :], c * np.array([[1e-3] * 2, [-2e-3] * 2, [0.0] * 2]), rtol=1e-12)
    assert np.all(H[:, 1] == 0)
    assert C.interlayer_energy(m, mesh, mat, ex) == pytest.approx(2 * 2e-9 * 3e-9 * 2e-3, rel=1e-12)
    p = F.Params(Ms=1.0, terms=C.INTERLAYER)
    E = C.full_energies(m, mesh, p, mat, ex)
    assert E[0] == pytest.approx(0.0, abs=1e-40) and E[2] == pytest.approx(2 * 2e-9 * 3e-9 * 2e-3, rel=1e-12)


def test_interlayer_field_is_energy_gradient():
    mesh = F.Mesh(3, 2, 4, 2e-9, 3e-9, 1.5e-9)
    rng = np.random.default_rng(21)
    Ms = rng.uniform(3e5, 9e5, size=(4, 2, 3))
    Ms[1] = 0.0
    Ms[3, 1, 2] = 0.0
    mat = C.Material(Ms, np.zeros(Ms.shape), np.zeros(Ms.shape))
    m = _unit((4, 2, 3), 22)
    ex = C.Extra(k_lo=0, k_hi=3, J=-1.5e-3, D_int=(0.4e-3, -0.7e-3, 1.1e-3))
    V = mesh.dx * mesh.dy * mesh.dz
    H = C.interlayer_field(m, mesh, mat, ex)
    g = np.zeros_like(m)
    eps = 1e-6
    for idx in np.ndindex(*m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[idx] += eps
        mm_[idx] -= eps
        g[idx] = (C.interlayer_energy(mp_, mesh, mat, ex) - C.interlayer_energy(mm_, mesh, mat, ex)) / (2 * eps)
    mag = Ms > 0
    np.testing.assert_allclose(H[:, mag], -g[:, mag] / (MU0 * Ms[mag] * V), rtol=1e-6,
                               atol=1e-6 * np.max(np.abs(H)))
    assert np.all(H[:, ~mag] == 0)
    # the energies seen through the fields: -(mu0/2) V sum Ms m.H
    assert -0.5 * MU0 * V * np.sum(Ms[None] * m * H) == pytest.approx(C.interlayer_energy(m, mesh, mat, ex),
                                                                       rel=1e-12)


def _cross(a, b):
    return np.cross(a, b, axis=0)


def test_spin_orbit_torque_satisfies_the_printed_equation():
    """dm/dt of the LL form with the torque folded into H satisfies the paper's
    Gilbert form: dm/dt - alpha m x dm/dt = -a_J m x (m x p) - b_J m x p (H = 0 otherwise)."""
    mesh = F.Mesh(4, 3, 2, 2e-9, 2e-9, 2e-9)
    mat = _const((2, 3, 4), 6e5, 0.0, 0.0)
    m = _unit((2, 3, 4), 31)
    ex = C.Extra(a_J=2.3e9, b_J=-0.7e9, p=(0.3, 1.0, -0.2))
    p = F.Params(Ms=1.0, alpha=0.27, terms=C.STT_SOT)
    k = C.full_llg_rhs(m, mesh, p, mat, ex)
    pv = ex.p.reshape(3, 1, 1, 1) * np.ones_like(m)
    lhs = k - p.alpha * _cross(m, k)
    rhs = -ex.a_J * _cross(m, _cross(m, pv)) - ex.b_J * _cross(m, pv)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.max(np.abs(rhs)))


def test_zhang_li_translates_a_spiral_rigidly():
    """With alpha = beta and no other term the Zhang-Li torque moves a texture with
    velocity u: on the interior cells of a spiral m = (sin qx, 0, cos qx) the
    central difference gives (u . grad) m = u sin(q dx)/dx (cos qx, 0, -sin qx) (worked
    by hand), so dm/dt = -that.  For beta != alpha the printed Gilbert form holds:
    dm/dt - alpha m x dm/dt = -(u . grad) m + beta m x (u . grad) m."""
    nx, dx, q, u = 40, 2e-9, 2 * math.pi / 37e-9, 85.0
    mesh = F.Mesh(nx, 3, 1, dx, 2e-9, 1e-9)
    x = np.arange(nx) * dx
    m = np.zeros((3, 1, 3, nx))
    m[0], m[2] = np.sin(q * x), np.cos(q * x)
    mat = _const((1, 3, nx), 7e5, 0.0, 0.0)
    v = np.zeros_like(m)
    v[0], v[2] = np.cos(q * x), -np.sin(q * x)
    v *= u * math.sin(q * dx) / dx
    sl = (slice(None), slice(None), slice(None), slice(1, -1))
    ex = C.Extra(u=(u, 0.0, 0.0), beta=0.3)
    k = C.full_llg_rhs(m, mesh, F.Params(Ms=1.0, alpha=0.3, terms=C.STT_ZL), mat, ex)
    np.testing.assert_allclose(k[sl], -v[sl], rtol=1e-10, atol=1e-10 * np.max(np.abs(v)))
    ex = C.Extra(u=(u, 0.0, 0.0), beta=0.05)
    p = F.Params(Ms=1.0, alpha=0.2, terms=C.STT_ZL)
    k = C.full_llg_rhs(m, mesh, p, mat, ex)
    lhs = k - p.alpha * _cross(m, k)
    rhs = -v + ex.beta * _cross(m, v)
    np.testing.assert_allclose(lhs[sl], rhs[sl], rtol=1e-10, atol=1e-10 * np.max(np.abs(v)))
    # one-sided differences at the ends, none across an empty cell
    d = C.directional_derivative(m, mesh, mat, (u, 0.0, 0.0))
    np.testing.assert_allclose(d[:, :, :, 0], u * (m[:, :, :, 1] - m[:, :, :, 0]) / dx, rtol=1e-12)
    Ms = np.full((1, 3, nx), 7e5)
    Ms[:, :, 10] = 0.0
    d = C.directional_derivative(m, mesh, C.Material(Ms, Ms * 0, Ms * 0), (u, 0.0, 0.0))
    np.testing.assert_allclose(d[:, :, :, 9], u * (m[:, :, :, 9] - m[:, :, :, 8]) / dx, rtol=1e-12)
    assert np.all(d[:, :, :, 10] == 0)
