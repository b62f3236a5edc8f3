"""Pins of the oracle's scalar-potential demag route (CPU only).

* The face antiderivative integrates 1/r over rectangles as a library
  quadrature does (scipy dblquad), in and out of the rectangle's plane.
* The cuboid potential S matches a library quadrature of its defining volume
  integral near the cell, a 50-digit evaluation of the closed form across
  distances (which also pins the far-field quadrature schedule), the point
  dipole's potential V R / (4 pi |R|^3) far away, and its parities.
* Superposition: the vertex potential of a uniformly magnetised block of
  cells equals that of one big uniformly magnetised cuboid (the closed form
  at the block's size) -- exact, and independent of the convolution.
* The FFT convolution equals the plain sum over cells on tiny meshes, for
  P = 2n and larger P.
* Limits: a uniformly magnetised cube's mean field tends to -Ms/3 and a wide
  film's N_zz to 1; the field tends to the Newell cell-averaged field as the
  mesh is refined (errors that shrink with each halving of the cell).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import fields as F
from oracle import potential as P


@pytest.mark.parametrize("rect", [(-1.0, 2.0, -0.5, 1.5, 0.7), (0.3, 2.0, 0.2, 1.0, 0.0),
                                  (-2.0, -0.4, 0.5, 3.0, -1.3), (-1.0, 1.0, -1.0, 1.0, 0.2)])
def test_face_antiderivative_against_quadrature(rect):
    x1, x2, y1, y2, w = rect
    f = lambda y, x: 1.0 / math.sqrt(x * x + y * y + w * w)
    ref, _ = integrate.dblquad(f, x1, x2, y1, y2, epsabs=1e-13, epsrel=1e-12)
    assert P.face_integral(x1, x2, y1, y2, w) == pytest.approx(ref, rel=1e-9)


def _quad_S(R, d):
    """(1/4pi) int_cell (R - r')/|R - r'|^3 dr' by nested library quadrature."""
    out = []
    for a in range(3):
        def f(z, y, x, a=a):
            v = (R[0] - x, R[1] - y, R[2] - z)
            return v[a] / (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) ** 1.5
        val, _ = integrate.tplquad(f, -d[0] / 2, d[0] / 2, -d[1] / 2, d[1] / 2, -d[2] / 2, d[2] / 2,
                                   epsabs=1e-14, epsrel=1e-11)
        out.append(val / (4 * math.pi))
    return np.array(out)


@pytest.mark.parametrize("R,d", [((1.5, 0.5, 0.5), (1.0, 1.0, 1.0)), ((1.5, -2.5, 0.5), (2.0, 2.0, 1.0)),
                                 ((0.5, 0.5, 1.1), (1.0, 1.0, 0.4))])
def test_kernel_against_library_quadrature(R, d):
    np.testing.assert_allclose(P.kernel(np.array([R]), d)[0], _quad_S(np.array(R), d), rtol=1e-8,
                               atol=1e-10 * max(d) ** 0)


def _mp_S(R, d):
    mp.mp.dps = 50

    def G(x, y, z):
        x, y, z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
        r = mp.sqrt(x * x + y * y + z * z)
        out = mp.mpf(0)
        if x != 0 and x * x + z * z > 0:
            out += x * mp.asinh(y / mp.sqrt(x * x + z * z))
        if y != 0 and y * y + z * z > 0:
            out += y * mp.asinh(x / mp.sqrt(y * y + z * z))
        if z != 0 and r > 0:
            out -= z * mp.atan(x * y / (z * r))
        return out

    res = []
    for a in range(3):
        b, c = [k for k in range(3) if k != a]
        x1, x2 = -mp.mpf(d[b]) / 2 - R[b], mp.mpf(d[b]) / 2 - R[b]
        y1, y2 = -mp.mpf(d[c]) / 2 - R[c], mp.mpf(d[c]) / 2 - R[c]

        def I(w):
            return G(x2, y2, w) - G(x1, y2, w) - G(x2, y1, w) + G(x1, y1, w)
        res.append((I(mp.mpf(R[a]) - mp.mpf(d[a]) / 2) - I(mp.mpf(R[a]) + mp.mpf(d[a]) / 2)) / (4 * mp.pi))
    return np.array([float(v) for v in res])


@pytest.mark.parametrize("d", [(1.0, 1.0, 1.0), (2.0, 2.0, 1.0), (1.0, 1.0, 0.4)])
def test_kernel_against_50_digit_closed_form(d):
    rng = np.random.default_rng(7)
    for rho in (0.8, 2.5, 3.5, 8.0, 20.0, 60.0, 400.0):
        v = rng.normal(size=3)
        R = v / np.linalg.norm(v) * rho * max(d)
        R = (np.round(R / np.array(d) - 0.5) + 0.5) * np.array(d)  # a vertex - cell displacement
        ex = _mp_S(R, d)
        got = P.kernel(R[None], d)[0]
        assert np.max(np.abs(got - ex)) <= 5e-14 * np.max(np.abs(ex)), (rho, got, ex)


def test_kernel_far_field_is_the_dipole_potential():
    d = (2.0, 1.5, 1.0)
    V = d[0] * d[1] * d[2]
    for R in ([1000.5, 0.0, 0.0], [300.5, -400.5, 200.5], [0.5, 0.5, -700.5]):
        R = np.array(R)
        dip = V * R / (4 * math.pi * np.linalg.norm(R) ** 3)
        np.testing.assert_allclose(P.kernel(R[None], d)[0], dip, rtol=1e-5, atol=1e-6 * np.max(np.abs(dip)))


def test_kernel_parities_on_the_lattice():
    g = P.kernel_grid(5, 4, 3, 2.0, 1.5, 1.0)  # [2nz, 2ny, 2nx, 3], index i + n - 1 for i in [-n+1, n]
    flip_x = g[:, :, ::-1]  # i -> 1 - i reverses the lattice (i - 1/2 -> -(i - 1/2))
    np.testing.assert_allclose(flip_x[..., 0], -g[..., 0], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(flip_x[..., 1], g[..., 1], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(flip_x[..., 2], g[..., 2], rtol=1e-14, atol=1e-16)
    flip_z = g[::-1]
    np.testing.assert_allclose(flip_z[..., 2], -g[..., 2], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(flip_z[..., 0], g[..., 0], rtol=1e-14, atol=1e-16)


def test_block_potential_is_one_big_cuboid():
    mesh = F.Mesh(4, 3, 2, 2e-9, 3e-9, 1.5e-9)
    Mv = np.array([3e5, -2e5, 6e5])
    M = np.broadcast_to(Mv.reshape(3, 1, 1, 1), (3, 2, 3, 4)).copy()
    u = P.PotentialKernel(mesh).vertex_potential(M)
    big = (4 * 2e-9, 3 * 3e-9, 2 * 1.5e-9)
    centre = np.array([1.5 * 2e-9, 1.0 * 3e-9, 0.5 * 1.5e-9])
    k, j, i = np.meshgrid(np.arange(3), np.arange(4), np.arange(5), indexing="ij")
    V = np.stack([(i - 0.5) * 2e-9, (j - 0.5) * 3e-9, (k - 0.5) * 1.5e-9], axis=-1) - centre
    ref = P.kernel_closed(V, big) @ Mv
    np.testing.assert_allclose(u, ref, rtol=1e-11, atol=1e-12 * np.max(np.abs(ref)))


@pytest.mark.parametrize("pad", [0, 3])
def test_fft_route_equals_the_plain_sum(pad):
    mesh = F.Mesh(5, 4, 3, 2e-9, 2.5e-9, 1.5e-9)
    rng = np.random.default_rng(11)
    M = 8e5 * rng.normal(size=(3, 3, 4, 5))
    kern = P.PotentialKernel(mesh, P=(6 + pad, 8 + pad, 10 + pad))
    u = kern.vertex_potential(M)
    ref = P.vertex_potential_direct(M, mesh)
    np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_limits_cube_film_and_newell():
    errs = []
    for n in (4, 8, 16):
        mesh = F.Mesh(n, n, n, 1e-9, 1e-9, 1e-9)
        m = np.zeros((3, n, n, n))
        m[0] = 1.0
        H = P.demag_field(m, mesh, 8e5)
        errs.append(abs(H[0].mean() / (-8e5 / 3) - 1))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.01
    nzz = []
    for n in (32, 64):
        mesh = F.Mesh(n, n, 2, 2e-9, 2e-9, 1e-9)
        m = np.zeros((3, 2, n, n))
        m[2] = 1.0
        nzz.append(-P.demag_field(m, mesh, 8e5)[2, 0, n // 2, n // 2] / 8e5)
    assert nzz[0] < nzz[1] < 1.0 and nzz[1] > 0.98
    L, rms = 32e-9, []
    for n in (4, 8, 16):
        d = L / n
        mesh = F.Mesh(n, n, n, d, d, d)
        c = (np.arange(n) + 0.5) * d
        z, y, x = np.meshgrid(c, c, c, indexing="ij")
        m = np.stack([np.sin(np.pi * x / L), np.cos(np.pi * y / L), 0.5 + z / L])
        m /= np.linalg.norm(m, axis=0)
        Hp = P.demag_field(m, mesh, 8e5)
        Hn = F.DemagKernel(mesh).field(m, 8e5)
        rms.append(np.sqrt(np.mean((Hp - Hn) ** 2)) / np.sqrt(np.mean(Hn ** 2)))
    assert rms[0] > 1.8 * rms[1] > 3.2 * rms[2] and rms[2] < 0.02
