"""Pins of the steepest-descent oracle (CPU only).

* The explicit update solves the implicit midpoint rotation of the paper:
  checked against a 3x3 linear solve of (I - tau/2 [f]x) m' = (I + tau/2 [f]x) m
  per cell, and |m'| = |m|.
* A macrospin with uniaxial anisotropy in a tilted field relaxes to the
  Stoner-Wohlfarth angle, the root of dE/dtheta found by a library root finder.
* On a small film with every term the energy falls and the largest torque
  |m x H| drops by orders of magnitude.
* The step rule: odd iterations take s.s/s.y, even ones s.y/y.y, a negative
  quotient keeps the previous step, and the result is clipped.
"""
import math

import numpy as np
from scipy.optimize import brentq

from oracle import fields as F
from oracle import sd

MU0 = 4e-7 * math.pi


def _cross_matrix(v):
    return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])


def test_update_is_the_implicit_midpoint_rotation():
    rng = np.random.default_rng(5)
    m = rng.normal(size=(3, 2, 3, 4))
    m /= np.linalg.norm(m, axis=0, keepdims=True)
    H = rng.normal(size=(3, 2, 3, 4)) * 1e5
    tau = 3e-6
    got = sd.update(m, H, tau)
    for idx in np.ndindex(2, 3, 4):
        mi, Hi = m[(slice(None),) + idx], H[(slice(None),) + idx]
        Fx = _cross_matrix(np.cross(mi, Hi))
        # m' = m - tau/2 (m + m') x f  <=>  (I - tau/2 [f]x) m' = (I + tau/2 [f]x) m
        want = np.linalg.solve(np.eye(3) - 0.5 * tau * Fx, (np.eye(3) + 0.5 * tau * Fx) @ mi)
        assert np.max(np.abs(got[(slice(None),) + idx] - want)) < 1e-14
    assert np.max(np.abs(np.linalg.norm(got, axis=0) - 1.0)) < 1e-14


def test_macrospin_relaxes_to_stoner_wohlfarth_angle():
    Ms, Ku, Hm, psi = 8e5, 5e4, 4e4, math.radians(30.0)
    mesh = F.Mesh(1, 1, 1, 2e-9, 2e-9, 2e-9)
    p = F.Params(Ms=Ms, Ku=Ku, u=(0, 0, 1), H=(Hm * math.sin(psi), 0.0, Hm * math.cos(psi)),
                 terms=F.ANIS | F.ZEEMAN)
    m = np.zeros((3, 1, 1, 1))
    m[:, 0, 0, 0] = (math.sin(2.0), 0.0, math.cos(2.0))  # 115 degrees from the easy axis
    field = lambda y: F.effective_field(y, mesh, p)
    mm, _ = sd.run(field, m, 200, 1e-6, 1e-9, 1e-3)
    # energy density K sin^2(theta) - mu0 Ms H cos(theta - psi): stationary where
    # K sin(2 theta) + mu0 Ms H sin(theta - psi) = 0, between the field and the axis
    dE = lambda t: Ku * math.sin(2 * t) + MU0 * Ms * Hm * math.sin(t - psi)
    theta = brentq(dE, 0.0, psi)
    got = math.atan2(mm[0, 0, 0, 0], mm[2, 0, 0, 0])
    assert abs(got - theta) < 1e-9
    assert abs(mm[1, 0, 0, 0]) < 1e-12


def test_film_energy_falls_and_torque_vanishes():
    mesh = F.Mesh(12, 10, 1, 2e-9, 2e-9, 2e-9)
    p = F.Params(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=8e5, u=(0, 0, 1), H=(0, 0, 1e5), terms=F.ALL_TERMS)
    kern = F.DemagKernel(mesh)
    rng = np.random.default_rng(2)
    m = np.zeros((3, 1, 10, 12))
    m[2] = 1.0
    m += 0.3 * rng.normal(size=m.shape)
    m /= np.linalg.norm(m, axis=0, keepdims=True)
    field = lambda y: F.effective_field(y, mesh, p, kern)
    t0 = sd.max_torque(m, field(m))
    mm, taus = sd.run(field, m, 300, 1e-7, 1e-10, 1e-3)
    E0, E1 = np.sum(F.energies(m, mesh, p, kern)), np.sum(F.energies(mm, mesh, p, kern))
    assert E1 < E0
    assert sd.max_torque(mm, field(mm)) < 1e-6 * t0
    assert np.max(np.abs(np.linalg.norm(mm, axis=0) - 1)) < 1e-12
    assert len(taus) == 300 and all(1e-10 <= t <= 1e-3 for t in taus)


def test_step_rule():
    s = np.array([1.0, 2.0, 0.0])
    y = np.array([0.5, 0.5, 1.0])
    # s.s = 5, s.y = 1.5, y.y = 1.5
    assert sd.bb_tau(s, y, 1, 7.0, 1e-9, 1e3) == 5.0 / 1.5
    assert sd.bb_tau(s, y, 2, 7.0, 1e-9, 1e3) == 1.0
    assert sd.bb_tau(s, -y, 1, 7.0, 1e-9, 1e3) == 7.0   # s.y < 0: keep the previous step
    assert sd.bb_tau(s, y, 1, 7.0, 1e-9, 2.0) == 2.0    # clipped
    assert sd.bb_tau(s, 0 * y, 2, 7.0, 1e-9, 1e3) == 7.0  # 0 / 0
