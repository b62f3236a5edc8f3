"""Pins for the oracle's relaxations with the largest-|dm/dt| stopping rule (CPU only).

* the measure is the LL right-hand side's norm: for unit m it equals
  gamma/sqrt(1+alpha^2) |m x H| cell by cell, and one turn per nanosecond
  (2 pi 1e9 rad/s) reads 360 deg/ns;
* on the Stoner-Wohlfarth macrospin of the paper's sim_with example (Ku along
  (1,1,0), field along x; Ms 1e6 A/m, Ku 5e4 J/m^3) both relaxations stop at the
  first check below the threshold, and the state lies within the angle the
  threshold allows of the equilibrium a library root finder gives: at a
  torque |m x H| the deviation is at most |m x H| / kappa, kappa the smaller
  curvature of the energy (in and out of plane) over mu0 Ms; a tenfold smaller
  threshold moves the state closer.
"""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import MU0, dp45, relax
from oracle import fields as F

KU, MS, ALPHA, GAMMA = 5e4, 1e6, 0.5, 2.21e5
HX = 20e-3 / MU0  # 20 mT along x


def _sw():
    mesh = F.Mesh(1, 1, 1, 4e-9, 4e-9, 4e-9)
    p = F.Params(Ms=MS, Ku=KU, u=(1.0, 1.0, 0.0), H=(HX, 0.0, 0.0), alpha=ALPHA, gamma=GAMMA,
                 terms=F.ANIS | F.ZEEMAN)
    return mesh, p


def _equilibrium():
    """In-plane angle phi* of the minimum between 0 and pi/4 and the two curvatures / (mu0 Ms)."""
    de = lambda ph: KU * math.sin(2 * (ph - math.pi / 4)) + MU0 * MS * HX * math.sin(ph)
    ph = scipy.optimize.brentq(de, 0.0, math.pi / 4, xtol=1e-15)
    k_in = (2 * KU * math.cos(2 * (ph - math.pi / 4)) + MU0 * MS * HX * math.cos(ph)) / (MU0 * MS)
    k_out = (2 * KU * math.cos(ph - math.pi / 4) ** 2 + MU0 * MS * HX * math.cos(ph)) / (MU0 * MS)
    return np.array([math.cos(ph), math.sin(ph), 0.0]), min(k_in, k_out)


def _angle(m, ms):
    v = m[:, 0, 0, 0]
    return math.atan2(np.linalg.norm(np.cross(v, ms)), float(np.dot(v, ms)))


def _bound(thr, kappa):
    """Deviation allowed by a stop below thr (deg/ns): |m x H| < thr / DEG_PER_NS * sqrt(1+a^2) / gamma."""
    return thr / relax.DEG_PER_NS * math.sqrt(1 + ALPHA ** 2) / GAMMA / kappa


def _start():
    m = np.zeros((3, 1, 1, 1))
    m[:, 0, 0, 0] = (math.cos(1.2), math.sin(1.2), 0.1)
    return m / np.linalg.norm(m)


def test_measure_is_the_ll_norm_in_degrees_per_ns():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((3, 2, 3, 4))
    m /= np.linalg.norm(m, axis=0)
    H = 1e5 * rng.standard_normal((3, 2, 3, 4))
    p = F.Params(Ms=MS, alpha=ALPHA, gamma=GAMMA)
    k = F.llg_rhs_from_field(m, H, p)
    want = GAMMA / math.sqrt(1 + ALPHA ** 2) * np.linalg.norm(np.cross(m, H, axis=0), axis=0)
    np.testing.assert_allclose(np.linalg.norm(k, axis=0), want, rtol=1e-13)
    assert relax.max_dmdt(k) == pytest.approx(float(np.max(want)), rel=1e-13)
    assert 2 * math.pi * 1e9 * relax.DEG_PER_NS == pytest.approx(360.0, rel=1e-15)


@pytest.mark.parametrize("thr", [0.05, 0.005])
def test_sd_relax_stops_at_the_first_check_below(thr):
    mesh, p = _sw()
    ms, kappa = _equilibrium()
    field = lambda m: F.effective_field(m, mesh, p)
    m, k, meas, taus = relax.sd_relax(field, _start(), p, thr, 5000, 1e-6, 1e-9, 1e-3)
    assert k < 5000 and len(meas) == k + 1 and len(taus) == k
    assert meas[-1] < thr and all(v >= thr for v in meas[:-1])
    assert _angle(m, ms) <= _bound(thr, kappa)


@pytest.mark.parametrize("thr", [0.05, 0.005])
def test_dp45_relax_stops_at_the_first_accepted_step_below(thr):
    mesh, p = _sw()
    ms, kappa = _equilibrium()
    f = lambda y: F.llg_rhs(y, mesh, p)
    st = dp45.State(rtol=1e-6)
    m, stopped, meas = relax.dp45_relax(f, _start(), st, thr, 200000)
    assert stopped and len(meas) == st.n_accept
    assert meas[-1] < thr and all(v >= thr for v in meas[:-1])
    # the stopping slope is the new state's own slope
    assert relax.max_dmdt(f(m)) * relax.DEG_PER_NS == pytest.approx(meas[-1], rel=1e-5)
    assert _angle(m, ms) <= 1.01 * _bound(thr, kappa)


def test_tighter_threshold_lands_closer():
    mesh, p = _sw()
    ms, _ = _equilibrium()
    field = lambda m: F.effective_field(m, mesh, p)
    a = [_angle(relax.sd_relax(field, _start(), p, thr, 5000, 1e-6, 1e-9, 1e-3)[0], ms) for thr in (0.5, 0.005)]
    assert a[1] < 0.1 * a[0]
