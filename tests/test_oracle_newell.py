"""Pins for the oracle's demagnetisation tensor (CPU only).

What pins what:
* cube self term N(0) = I/3 and trace N(0) = 1 for any cell shape (the
  trace of the cell-averaged tensor of a cell with itself is 1);
* trace N(R) = 0 for R != 0 (the dipole kernel is traceless outside its source);
* symmetry / parity of each component under reflections;
* agreement of the two independent evaluations (closed form and quadrature of
  the defining integral) where both are accurate (6 <= rho <= 12);
* far field -> point dipole -V (3 r r^T - r^2 I)/(4 pi r^5) (the paper's
  dipolar-interaction formula, section "Dipolar interaction");
* 60-digit mpmath evaluation of the closed form (FP64 cancellation check) and
  of the quadrature branch against it (1e-10 relative).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import newell

CELLS = [(1.0, 1.0, 1.0), (4.0, 4.0, 3.0), (1.0, 1.0, 0.4), (2.0, 2.0, 1.0), (5.0, 3.0, 2.0)]


def test_cube_self_term_is_one_third():
    t = newell.tensor(0, 0, 0, 1.0, 1.0, 1.0)
    np.testing.assert_allclose(t[:3], [1 / 3, 1 / 3, 1 / 3], rtol=1e-14)
    np.testing.assert_allclose(t[3:], 0.0, atol=1e-15)


@pytest.mark.parametrize("d", CELLS)
def test_self_trace_is_one(d):
    t = newell.tensor(0, 0, 0, *d)
    assert abs(t[0] + t[1] + t[2] - 1.0) < 1e-13
    assert np.all(t[:3] > 0)
    # the flat cell is demagnetised most along its thin axis
    if d[2] < min(d[0], d[1]):
        assert t[2] > t[0] and t[2] > t[1]


@pytest.mark.parametrize("d", CELLS)
def test_trace_vanishes_off_origin(d):
    rng = np.random.default_rng(0)
    I = np.concatenate([rng.integers(-5, 6, 60), rng.integers(-400, 400, 60)])
    J = np.concatenate([rng.integers(-5, 6, 60), rng.integers(-400, 400, 60)])
    K = np.concatenate([rng.integers(-3, 4, 60), rng.integers(-20, 20, 60)])
    keep = (I != 0) | (J != 0) | (K != 0)
    t = newell.tensor(I[keep], J[keep], K[keep], *d)
    scale = np.max(np.abs(t), axis=1)  # (diagonals may all vanish by symmetry)
    assert np.all(np.abs(t[:, 0] + t[:, 1] + t[:, 2]) <= 1e-9 * scale)


@pytest.mark.parametrize("d", CELLS[:3])
def test_parity_of_components(d):
    rng = np.random.default_rng(1)
    I, J, K = rng.integers(1, 30, 40), rng.integers(1, 30, 40), rng.integers(1, 5, 40)
    base = newell.tensor(I, J, K, *d)
    # xx, yy, zz even in each coordinate; xy odd in X,Y; xz odd in X,Z; yz odd in Y,Z
    odd = {"x": (0, 0, 0, 1, 1, 0), "y": (0, 0, 0, 1, 0, 1), "z": (0, 0, 0, 0, 1, 1)}
    for axis, flips in odd.items():
        sI = -I if axis == "x" else I
        sJ = -J if axis == "y" else J
        sK = -K if axis == "z" else K
        t = newell.tensor(sI, sJ, sK, *d)
        sign = np.array([-1.0 if f else 1.0 for f in flips])
        scale = np.max(np.abs(base), axis=1, keepdims=True)
        assert np.all(np.abs(t - base * sign) <= 1e-10 * scale)


def test_exchange_of_axes():
    # N_yy on (dx,dy) equals N_xx with X<->Y, dx<->dy swapped
    a = newell.tensor(3, 1, 2, 2.0, 3.0, 1.0)
    b = newell.tensor(1, 3, 2, 3.0, 2.0, 1.0)
    np.testing.assert_allclose(a[[0, 1, 2, 3, 4, 5]], b[[1, 0, 2, 3, 5, 4]], rtol=1e-12)


@pytest.mark.parametrize("d", CELLS)
def test_closed_form_matches_quadrature_in_overlap(d):
    m = max(d)
    pts = [(6.5, 0.3, 0.2), (7.0, 4.0, 1.0), (0.0, 8.0, 3.0), (5.0, 5.0, 5.0), (9.0, 6.0, 2.0)]
    for p in pts:
        X, Y, Z = (p[0] * m, p[1] * m, p[2] * m)
        # snap to the lattice of cell centres
        I, J, K = round(X / d[0]), round(Y / d[1]), round(Z / d[2])
        X, Y, Z = I * d[0], J * d[1], K * d[2]
        rho = math.sqrt(X * X + Y * Y + Z * Z) / m
        if rho < 6:
            continue
        cf = newell.tensor_closed_form(X, Y, Z, *d)
        q = newell.tensor_quadrature(X, Y, Z, *d, 8)[0]
        scale = np.max(np.abs(q))
        # formula mistakes show up at O(1); FP64 cancellation in the closed form
        # reaches ~1e-8 here for thin and anisotropic cells
        assert np.max(np.abs(cf - q)) < 1e-7 * scale


@pytest.mark.parametrize("d", [(1.0, 1.0, 1.0), (4.0, 4.0, 3.0), (1.0, 1.0, 0.4)])
def test_far_field_is_point_dipole(d):
    V = d[0] * d[1] * d[2]
    for (I, J, K) in [(300, 100, 7), (0, 400, 30), (250, 250, 0)]:
        X, Y, Z = I * d[0], J * d[1], K * d[2]
        r = np.array([X, Y, Z])
        r2 = r @ r
        D = (3 * np.outer(r, r) - r2 * np.eye(3)) / (4 * np.pi * r2 ** 2.5)
        Nd = -V * D
        t = newell.as_matrix(newell.tensor(I, J, K, *d))
        rho = math.sqrt(r2) / max(d)
        assert np.max(np.abs(t - Nd)) <= 3.0 / rho ** 2 * np.max(np.abs(Nd))


# --- 60-digit reference evaluation of the closed form (rounding check) ---
mp.mp.dps = 60


def _f_mp(x, y, z):
    x, y, z = abs(mp.mpf(x)), abs(mp.mpf(y)), abs(mp.mpf(z))
    R = mp.sqrt(x * x + y * y + z * z)
    s = (2 * x * x - y * y - z * z) * R / 6
    if y != 0 and x * x + z * z > 0:
        s += y / 2 * (z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    if z != 0 and x * x + y * y > 0:
        s += z / 2 * (y * y - x * x) * mp.asinh(z / mp.sqrt(x * x + y * y))
    if x != 0 and y != 0 and z != 0:
        s -= x * y * z * mp.atan(y * z / (x * R))
    return s


def _g_mp(x, y, z):
    sg = mp.sign(x) * mp.sign(y)
    if sg == 0:
        return mp.mpf(0)
    x, y, z = abs(mp.mpf(x)), abs(mp.mpf(y)), abs(mp.mpf(z))
    R = mp.sqrt(x * x + y * y + z * z)
    s = -x * y * R / 3
    if z != 0:
        s += x * y * z * mp.asinh(z / mp.sqrt(x * x + y * y))
    if y * y + z * z > 0:
        s += y / 6 * (3 * z * z - y * y) * mp.asinh(x / mp.sqrt(y * y + z * z))
    if x * x + z * z > 0:
        s += x / 6 * (3 * z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    if z != 0:
        s -= z ** 3 / 6 * mp.atan(x * y / (z * R))
        s -= z * y * y / 2 * mp.atan(x * z / (y * R))
        s -= z * x * x / 2 * mp.atan(y * z / (x * R))
    return sg * s


def _stencil_mp(fun, p, q, r, dp, dq, dr):
    w = {-1: -1, 0: 2, 1: -1}
    s = mp.mpf(0)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                s += w[a] * w[b] * w[c] * fun(mp.mpf(p) + a * mp.mpf(dp), mp.mpf(q) + b * mp.mpf(dq),
                                              mp.mpf(r) + c * mp.mpf(dr))
    return s


def tensor_mp(I, J, K, dx, dy, dz):
    X, Y, Z = I * mp.mpf(dx), J * mp.mpf(dy), K * mp.mpf(dz)
    c = 1 / (4 * mp.pi * mp.mpf(dx) * mp.mpf(dy) * mp.mpf(dz))
    return [c * _stencil_mp(_f_mp, X, Y, Z, dx, dy, dz),
            c * _stencil_mp(_f_mp, Y, X, Z, dy, dx, dz),
            c * _stencil_mp(_f_mp, Z, Y, X, dz, dy, dx),
            c * _stencil_mp(_g_mp, X, Y, Z, dx, dy, dz),
            c * _stencil_mp(_g_mp, X, Z, Y, dx, dz, dy),
            c * _stencil_mp(_g_mp, Y, Z, X, dy, dz, dx)]


@pytest.mark.parametrize("d", [(1.0, 1.0, 1.0), (4.0, 4.0, 3.0), (1.0, 1.0, 0.4)])
def test_against_60_digit_reference(d):
    pts = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (2, 1, 1), (3, -2, 1), (5, 2, 0), (4, 4, 2),
           (7, 3, 1), (10, -4, 2), (20, 11, 3), (45, 30, 4), (120, 90, 5), (350, 200, 3)]
    for (I, J, K) in pts:
        ref = np.array([float(v) for v in tensor_mp(I, J, K, *d)])
        got = newell.tensor(I, J, K, *d)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 2e-11 * scale, (I, J, K, got, ref)
