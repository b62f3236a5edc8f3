"""Pins of the Heun oracle (CPU only).

* For a macrospin under a static field with no damping the LL right-hand side
  is linear, f(m) = A m with A the cross-product matrix of gamma H, so one
  Heun step is the degree-2 Taylor polynomial of exp(hA) applied to m and
  then normalised: written with matrix powers, independent of the field code.
* The global error against the closed-form damped precession (the paper's
  macrospin, tests/golden/macrospin_paper.json) falls as h^2: halving h
  divides it by about 4 (second order).
* Every step leaves |m| = 1 per cell and a uniform state under a field along
  m does not move.
"""
import json
import math
import os

import numpy as np

from oracle import fields as F
from oracle import heun

PAPER = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "macrospin_paper.json")))
HZ, GAMMA = PAPER["Hz_A_per_m"], PAPER["gamma_m_per_A_s"]


def _macrospin(alpha, H=(0.0, 0.0, HZ)):
    mesh = F.Mesh(1, 1, 1, 1e-9, 1e-9, 1e-9)
    p = F.Params(Ms=8e5, H=H, alpha=alpha, gamma=GAMMA, terms=F.ZEEMAN)
    m0 = np.zeros((3, 1, 1, 1))
    m0[:, 0, 0, 0] = PAPER["m0"]
    return mesh, p, m0


def _analytic(t, alpha):
    g = GAMMA / (1 + alpha ** 2)
    return np.array([math.cos(g * HZ * t) / math.cosh(alpha * g * HZ * t),
                     math.sin(g * HZ * t) / math.cosh(alpha * g * HZ * t),
                     math.tanh(alpha * g * HZ * t)])


def test_undamped_step_is_second_order_taylor_of_rotation():
    H = np.array([2e4, -3e4, 1e5])
    mesh, p, m = _macrospin(0.0, tuple(H))
    m[:, 0, 0, 0] = np.array([0.3, 0.8, -0.2]) / np.linalg.norm([0.3, 0.8, -0.2])
    # dm/dt = -gamma m x H = gamma H x m = A m
    A = GAMMA * np.array([[0, -H[2], H[1]], [H[2], 0, -H[0]], [-H[1], H[0], 0]])
    h = 2e-12
    f = lambda y: F.llg_rhs(y, mesh, p)
    got = heun.step(f, m, h)[:, 0, 0, 0]
    v = (np.eye(3) + h * A + 0.5 * h * h * (A @ A)) @ m[:, 0, 0, 0]
    want = v / np.linalg.norm(v)
    assert np.max(np.abs(got - want)) < 1e-14
    # and not the first-order (Euler) or third-order polynomial
    e1 = (np.eye(3) + h * A) @ m[:, 0, 0, 0]
    assert np.max(np.abs(got - e1 / np.linalg.norm(e1))) > 1e-6


def test_global_error_second_order_against_closed_form():
    a = PAPER["alpha"]
    mesh, p, m = _macrospin(a)
    f = lambda y: F.llg_rhs(y, mesh, p)
    T = 1e-10
    errs = []
    for n in (200, 400, 800):
        mm = heun.run(f, m.copy(), T / n, n)
        errs.append(np.linalg.norm(mm[:, 0, 0, 0] - _analytic(T, a)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (errs, r1, r2)


def test_unit_length_and_fixed_point():
    mesh = F.Mesh(5, 4, 1, 2e-9, 2e-9, 1e-9)
    p = F.Params(Ms=8e5, A=1.3e-11, H=(0, 0, 5e4), alpha=0.1, terms=F.EXCHANGE | F.ZEEMAN)
    rng = np.random.default_rng(3)
    m = rng.normal(size=(3, 1, 4, 5))
    m /= np.linalg.norm(m, axis=0, keepdims=True)
    f = lambda y: F.llg_rhs(y, mesh, p)
    mm = heun.run(f, m, 1e-13, 5)
    assert np.max(np.abs(np.linalg.norm(mm, axis=0) - 1.0)) < 1e-14
    u = np.zeros((3, 1, 4, 5))
    u[2] = 1.0
    assert np.array_equal(heun.run(f, u, 1e-13, 3), u)
