"""Pins for the oracle's fields, energies and LL right-hand side (CPU only).

What pins what (each derived from the paper's printed formulas or from
textbook facts, not by re-typing the oracle's code):
* exchange: uniform m gives zero field and energy; a spin spiral gives the
  exact discrete field -(4A/(mu0 Ms D^2))(1 - cos qD) m and energy density
  2A(1 - cos qD)/D^2 in interior cells; the energy from the pair form w_i
  equals -(mu0/2) Ms V sum m.H_ex;
* DMI: spirals along x and along y give (2D sin(qD)/(mu0 Ms D)) m in interior
  cells, and the energy per cell tends to the continuum density -Dq of
  w = D(m . grad m_z - m_z div m) (section "Dzyaloshinskii-Moriya Energy");
* every term: H = -(1/(mu0 Ms V)) dE/dm by central differences (ties sign and
  scale of each field to its energy);
* demag: the FFT route equals the O(N^2) direct sum; padding-length
  invariance; a uniformly magnetised cube of n^3 cubic cells has mean field
  -Ms/3 exactly; a wide thin film has N_zz -> 1 at its centre;
* LL: m . dm/dt = 0; dE/dt = -mu0 Ms V alpha gamma/(1+alpha^2) sum |m x H|^2
  (static field) by finite differences.
"""
import math

import numpy as np
import pytest

from oracle import MU0
from oracle import fields as F
from oracle import newell


def _rand_unit(shape, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3,) + shape)
    return v / np.linalg.norm(v, axis=0)


MESH = F.Mesh(6, 5, 3, 2e-9, 3e-9, 1.5e-9)
P_ALL = F.Params(Ms=6e5, A=1.2e-11, D=2.5e-3, Ku=4e5, u=(0.3, -0.2, 1.0),
                 H=(1e4, -3e4, 5e4), alpha=0.2)


def test_uniform_exchange_is_zero():
    m = np.zeros((3, 3, 4, 5))
    m[1] = 1.0
    mesh = F.Mesh(5, 4, 3, 1e-9, 1e-9, 1e-9)
    assert np.all(F.exchange_field(m, mesh, P_ALL) == 0)
    assert F.exchange_energy_pairs(m, mesh, P_ALL) == 0
    assert F.energies(m, mesh, F.Params(Ms=6e5, A=1e-11, terms=F.EXCHANGE))[0] == 0


def _spiral_x(nx, q, dx):
    x = np.arange(nx) * dx
    m = np.zeros((3, 1, 3, nx))
    m[0] = np.sin(q * x)
    m[2] = np.cos(q * x)
    return m


def _spiral_y(ny, q, dy):
    y = np.arange(ny) * dy
    m = np.zeros((3, 1, ny, 3))
    m[1] = np.sin(q * y)[None, :, None]
    m[2] = np.cos(q * y)[None, :, None]
    return m


def test_spiral_exchange_closed_form():
    nx, dx, q = 40, 2e-9, 2 * math.pi / 37e-9
    m = _spiral_x(nx, q, dx)
    mesh = F.Mesh(nx, 3, 1, dx, 5e-9, 1e-9)
    p = F.Params(Ms=8e5, A=1.3e-11, terms=F.EXCHANGE)
    H = F.exchange_field(m, mesh, p)
    exact = -(4 * p.A / (MU0 * p.Ms * dx ** 2)) * (1 - math.cos(q * dx)) * m
    # interior in x; y neighbours are identical so they add nothing
    np.testing.assert_allclose(H[:, :, :, 1:-1], exact[:, :, :, 1:-1], rtol=1e-10, atol=1e-6)
    w = F.exchange_energy_pairs(m, mesh, p)
    V = mesh.dx * mesh.dy * mesh.dz
    # open chain: (nx-1) bonds per row, 3 rows, each bond 2A(1-cos qD)/D^2 * V
    assert w == pytest.approx(3 * (nx - 1) * V * 2 * p.A * (1 - math.cos(q * dx)) / dx ** 2,
                              rel=1e-12)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_spiral_dmi_closed_form_and_continuum_energy(axis):
    n, d, q = 48, 1e-9, 2 * math.pi / 60e-9
    p = F.Params(Ms=5.8e5, D=3e-3, terms=F.DMI)
    if axis == "x":
        m = _spiral_x(n, q, d)
        mesh = F.Mesh(n, 3, 1, d, 4e-9, 1e-9)
        sl = (slice(None), slice(None), slice(1, 2), slice(1, -1))  # interior in x and y
    else:
        m = _spiral_y(n, q, d)
        mesh = F.Mesh(3, n, 1, 4e-9, d, 1e-9)
        sl = (slice(None), slice(None), slice(1, -1), slice(1, 2))
    H = F.dmi_field(m, mesh, p)
    exact = (2 * p.D * math.sin(q * d) / (MU0 * p.Ms * d)) * m
    np.testing.assert_allclose(H[sl], exact[sl], rtol=1e-10, atol=1e-6)
    # energy density of interior cells -> continuum -D q (paper's w_dmi for C_nv)
    dens = -0.5 * MU0 * p.Ms * np.sum(m * H, axis=0)[sl[1:]]   # energy per volume
    np.testing.assert_allclose(dens, -p.D * math.sin(q * d) / d, rtol=1e-10)
    # discretisation error of sin(qD)/D against q is (qD)^2/6 relative
    assert abs(-p.D * math.sin(q * d) / d - (-p.D * q)) < 1.01 * (q * d) ** 2 / 6 * p.D * q
    # chirality: with D > 0 the q > 0 spiral lowers the energy, q < 0 raises it
    E_plus = F.energies(m, mesh, p)[2]
    m_minus = m.copy()
    m_minus[0 if axis == "x" else 1] *= -1
    E_minus = F.energies(m_minus, mesh, p)[2]
    assert E_plus < 0 < E_minus


def _num_grad(Efun, m, eps=1e-6):
    g = np.zeros_like(m)
    it = np.nditer(m[0], flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        for c in range(3):
            mp_, mm_ = m.copy(), m.copy()
            mp_[(c,) + idx] += eps
            mm_[(c,) + idx] -= eps
            g[(c,) + idx] = (Efun(mp_) - Efun(mm_)) / (2 * eps)
    return g


@pytest.mark.parametrize("term,idx", [("exchange", 0), ("demag", 1), ("dmi", 2),
                                      ("anisotropy", 3), ("zeeman", 4)])
def test_field_is_energy_gradient(term, idx):
    mesh = F.Mesh(4, 3, 2, 2e-9, 3e-9, 1.5e-9)
    m = _rand_unit((2, 3, 4), 3)
    bit = {"exchange": F.EXCHANGE, "demag": F.DEMAG, "dmi": F.DMI,
           "anisotropy": F.ANIS, "zeeman": F.ZEEMAN}[term]
    p = F.Params(Ms=P_ALL.Ms, A=P_ALL.A, D=P_ALL.D, Ku=P_ALL.Ku, u=P_ALL.u, H=P_ALL.H,
                 terms=bit)
    kern = F.DemagKernel(mesh)
    V = mesh.dx * mesh.dy * mesh.dz
    H = F.effective_field_terms(m, mesh, p, kern)[term]
    g = _num_grad(lambda mm: F.energies(mm, mesh, p, kern)[idx], m)
    Hnum = -g / (MU0 * p.Ms * V)
    np.testing.assert_allclose(H, Hnum, rtol=1e-6, atol=1e-6 * np.max(np.abs(H)))


def test_exchange_energy_forms_agree():
    m = _rand_unit((3, 5, 6), 4)
    E1 = F.exchange_energy_pairs(m, MESH, P_ALL)
    p = F.Params(Ms=P_ALL.Ms, A=P_ALL.A, terms=F.EXCHANGE)
    E2 = F.energies(m, MESH, p)[0]
    assert E1 == pytest.approx(E2, rel=1e-12)


@pytest.mark.parametrize("mesh", [F.Mesh(5, 4, 3, 2e-9, 3e-9, 1.5e-9),
                                  F.Mesh(16, 16, 1, 4e-9, 4e-9, 3e-9),
                                  F.Mesh(7, 1, 2, 1e-9, 2e-9, 3e-9)])
def test_demag_fft_equals_direct_sum(mesh):
    m = _rand_unit((mesh.nz, mesh.ny, mesh.nx), 5)
    p = F.Params(Ms=8e5, terms=F.DEMAG)
    Hd = F.demag_field_direct(m, mesh, p)
    Hf = F.DemagKernel(mesh).field(m, p.Ms)
    scale = np.max(np.linalg.norm(Hd, axis=0))
    assert np.max(np.linalg.norm(Hf - Hd, axis=0)) <= 1e-12 * scale


def test_demag_padding_invariance():
    mesh = F.Mesh(6, 5, 3, 2e-9, 2e-9, 2e-9)
    m = _rand_unit((3, 5, 6), 6)
    base = F.DemagKernel(mesh).field(m, 1e6)
    for P in [(5, 9, 11), (11, 16, 18), (9, 10, 12)]:
        other = F.DemagKernel(mesh, P=P).field(m, 1e6)
        assert np.max(np.abs(other - base)) <= 1e-12 * np.max(np.abs(base))


@pytest.mark.parametrize("n", [2, 3, 5])
def test_uniform_cube_mean_field_is_minus_third(n):
    mesh = F.Mesh(n, n, n, 3e-9, 3e-9, 3e-9)
    m = np.zeros((3, n, n, n))
    m[0] = 1.0
    Ms = 7e5
    H = F.DemagKernel(mesh).field(m, Ms)
    np.testing.assert_allclose(H.mean(axis=(1, 2, 3)), [-Ms / 3, 0, 0], atol=1e-9 * Ms)


def test_thin_film_perpendicular_demag_tends_to_one():
    n = 64
    mesh = F.Mesh(n, n, 1, 2e-9, 2e-9, 1e-9)
    m = np.zeros((3, 1, n, n))
    m[2] = 1.0
    H = F.DemagKernel(mesh).field(m, 1.0)
    centre = -H[2, 0, n // 2, n // 2]
    assert 0.97 < centre < 1.0
    # in-plane magnetisation: centre field is small
    m2 = np.zeros_like(m)
    m2[0] = 1.0
    H2 = F.DemagKernel(mesh).field(m2, 1.0)
    assert 0 < -H2[0, 0, n // 2, n // 2] < 0.03


def test_llg_rhs_orthogonal_to_m():
    m = _rand_unit((3, 5, 6), 7)
    dm = F.llg_rhs(m, MESH, P_ALL)
    dots = np.sum(m * dm, axis=0)
    assert np.max(np.abs(dots)) <= 1e-12 * np.max(np.abs(dm))


def test_energy_dissipation_rate():
    mesh = F.Mesh(6, 5, 2, 2e-9, 3e-9, 1.5e-9)
    m = _rand_unit((2, 5, 6), 8)
    kern = F.DemagKernel(mesh)
    p = P_ALL
    V = mesh.dx * mesh.dy * mesh.dz
    H = F.effective_field(m, mesh, p, kern)
    dm = F.llg_rhs_from_field(m, H, p)
    Etot = lambda mm: float(np.sum(F.energies(mm, mesh, p, kern)))
    dt = 1e-16
    dEdt = (Etot(m + dt * dm) - Etot(m - dt * dm)) / (2 * dt)
    mxH = np.cross(m, H, axis=0)
    expect = -MU0 * p.Ms * V * p.alpha * p.gamma / (1 + p.alpha ** 2) * np.sum(mxH * mxH)
    assert dEdt == pytest.approx(expect, rel=1e-5)


def test_macrospin_larmor_frequency():
    # one cell, Zeeman only, alpha = 0: |dm/dt| = gamma H sin(theta)
    mesh = F.Mesh(1, 1, 1, 1e-9, 1e-9, 1e-9)
    m = np.zeros((3, 1, 1, 1))
    m[0] = 1.0
    p = F.Params(Ms=8e5, H=(0, 0, 1e5), alpha=0.0, terms=F.ZEEMAN)
    dm = F.llg_rhs(m, mesh, p)
    assert np.linalg.norm(dm[:, 0, 0, 0]) == pytest.approx(p.gamma * 1e5, rel=1e-14)
    # sense of rotation: m x H with H || z and m || x gives -y; -gamma m x H = +y
    assert dm[1, 0, 0, 0] > 0
