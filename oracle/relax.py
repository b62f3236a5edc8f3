"""Relaxation that stops on the largest |dm/dt| (oracle).

TEST INFRASTRUCTURE ONLY.  Section "Design": the relax task of the high-level
interface takes a `stopping_dmdt` value (0.05 in the Stoner-Wohlfarth example
of that section); the paper gives neither the measure nor its unit.  Readings
used on both sides of this project:

* measure: the largest |dm/dt| over the cells, dm/dt being the LL right-hand
  side (eq_llg2) of the state, expressed in degrees per nanosecond (|dm/dt|
  in rad/s times 180/pi * 1e-9, the unit of the stopping rule of that name in
  OOMMF); a relaxation stops once the measure is below the threshold;
* steepest descent: iteration k evaluates H_eff(m_k) anyway, so the measure of
  m_k is taken there; the run stops before the update of the first iteration
  whose measure is below the threshold (m_k is the result, k updates made);
* adaptive Dormand-Prince: after every accepted step the integrator holds the
  slope of the new state (the FSAL slope f(y5), taken before the projection);
  the run stops after the first accepted step whose slope is below the
  threshold (at least one step is taken).
"""
import math

import numpy as np

from . import dp45, sd
from . import fields as F

DEG_PER_NS = 180.0 / math.pi * 1e-9  # (rad/s) -> (deg/ns)


def max_dmdt(k):
    """Largest |dm/dt| over the cells of a slope array k (rad/s)."""
    return float(np.max(np.sqrt(np.sum(k * k, axis=0))))


def sd_relax(field, m, p, stopping_dmdt, max_iter, tau0, tau_min, tau_max):
    """Steepest descent (the rules of oracle.sd) until the state's largest |dm/dt|,
    in deg/ns, is below stopping_dmdt, or max_iter updates.  field(m) -> H_eff.
    Returns (m, iterations, measures in deg/ns, taus)."""
    m_prev = g_prev = None
    tau = tau0
    taus, measures = [], []
    for k in range(max_iter + 1):
        H = field(m)
        measures.append(max_dmdt(F.llg_rhs_from_field(m, H, p)) * DEG_PER_NS)
        if measures[-1] < stopping_dmdt or k == max_iter:
            return m, k, measures, taus
        g = np.cross(m, np.cross(m, H, axis=0), axis=0)
        if k > 0:
            tau = sd.bb_tau(m - m_prev, g - g_prev, k, tau, tau_min, tau_max)
        taus.append(tau)
        m_prev, g_prev = m, g
        m = sd.update(m, H, tau)
    raise AssertionError("unreachable")


def dp45_relax(f, m, st, stopping_dmdt, max_steps):
    """Adaptive Dormand-Prince steps (oracle.dp45) until, after an accepted step, the
    largest |dm/dt| of the FSAL slope, in deg/ns, is below stopping_dmdt, or
    max_steps attempts.  Returns (m, stopped, measures of the accepted steps)."""
    measures = []
    for _ in range(max_steps):
        m, acc = dp45.step(f, m, st)
        if acc:
            measures.append(max_dmdt(st.k1) * DEG_PER_NS)
            if measures[-1] < stopping_dmdt:
                return m, True, measures
    return m, False, measures
