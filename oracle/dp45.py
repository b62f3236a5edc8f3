"""Adaptive Dormand-Prince 5(4) with projection onto the unit sphere (oracle).

TEST INFRASTRUCTURE ONLY.  The paper integrates the LL form of the LLG
equation with "the adaptive Dormand-Prince method" and projects m onto the unit
sphere after each successful step (section "LLG equation"); it prints neither
the tableau nor the step-size controller.  The tableau is Dormand and Prince's
(1980) 5(4) pair.  The controller is the reading used throughout this project:

* error  err = max_i ||e_i||_2 / rtol, e = h sum_j (b_j - bhat_j) k_j
  (absolute tolerance equal to rtol because |m| = 1);
* accept iff err <= 1; after an accepted step m <- y5/|y5| per cell;
* h_new = h * min(5, max(0.2, 0.9 err^(-1/5))), growth capped at 1 on the
  step right after a rejection; h clipped to h_max and to land on t_end;
  a remainder t_end - t not above h_min counts as arrived (no step is taken);
* FSAL: k_7 = f(y5) (before normalisation) is reused as the next k_1;
* a rejected step leaves m and k_1 untouched;
* a non-finite error norm (the stages overflowed, or m holds NaN) counts as a
  rejection with the smallest factor 0.2; ten such attempts in a row stop the
  integration with a non-finite status.
"""
from fractions import Fraction as F

import numpy as np

C = (F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1))
A = (
    (),
    (F(1, 5),),
    (F(3, 40), F(9, 40)),
    (F(44, 45), F(-56, 15), F(32, 9)),
    (F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)),
    (F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)),
    (F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)),
)
B = (F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), F(0))
BHAT = (F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200),
        F(187, 2100), F(1, 40))

SAFETY, FAC_MIN, FAC_MAX = 0.9, 0.2, 5.0


class StepUnderflow(RuntimeError):
    pass


class NonFinite(RuntimeError):
    pass


MAX_NONFINITE = 10


class State:
    """Integrator state: time, next step size, tolerances, counters, FSAL slope."""

    def __init__(self, t=0.0, h=1e-13, rtol=1e-6, h_min=1e-20, h_max=1e-10):
        self.t, self.h, self.rtol = float(t), float(h), float(rtol)
        self.h_min, self.h_max = float(h_min), float(h_max)
        self.n_accept = self.n_reject = self.n_rhs = 0
        self.last_err = 0.0
        self.k1 = None
        self.after_reject = False
        self.accepted_h = []
        self.nonfinite = 0


def _normalize(y):
    return y / np.sqrt(np.sum(y * y, axis=0, keepdims=True))


def attempt(f, m, st, h):
    """One attempted step of size h from (t, m).  Returns (y5, k7, err)."""
    if st.k1 is None:
        st.k1 = f(m)
        st.n_rhs += 1
    k = [st.k1]
    for s in range(1, 7):
        y = m.copy()
        for j, a in enumerate(A[s]):
            if a != 0:
                y = y + (h * float(a)) * k[j]
        k.append(f(y))
        st.n_rhs += 1
    y5 = y  # stage-7 input equals the 5th-order solution (a_7j = b_j)
    e = np.zeros_like(m)
    for j in range(7):
        d = float(B[j] - BHAT[j])
        if d != 0:
            e = e + (h * d) * k[j]
    err = float(np.max(np.sqrt(np.sum(e * e, axis=0)))) / st.rtol
    return y5, k[6], err


def step(f, m, st, t_end=np.inf):
    """One attempted adaptive step; returns (m_new, accepted)."""
    h = min(st.h, st.h_max, t_end - st.t)
    if h < st.h_min:
        raise StepUnderflow("step size %.3e below h_min" % h)
    with np.errstate(over="ignore", invalid="ignore"):
        y5, k7, err = attempt(f, m, st, h)
    st.last_err = err
    if not np.isfinite(err):
        st.nonfinite += 1
        st.n_reject += 1
        st.after_reject = True
        st.h = h * FAC_MIN
        if st.nonfinite >= MAX_NONFINITE:
            raise NonFinite("non-finite error norm in %d attempts in a row" % st.nonfinite)
        return m, False
    st.nonfinite = 0
    if err <= 1.0:
        fac = FAC_MAX if err == 0.0 else min(FAC_MAX, max(FAC_MIN, SAFETY * err ** -0.2))
        if st.after_reject:
            fac = min(fac, 1.0)
        st.t = t_end if h == t_end - st.t else st.t + h
        st.k1 = k7
        st.n_accept += 1
        st.after_reject = False
        st.accepted_h.append(h)
        st.h = min(h * fac, st.h_max)
        return _normalize(y5), True
    fac = max(FAC_MIN, SAFETY * err ** -0.2)
    st.n_reject += 1
    st.after_reject = True
    st.h = h * fac
    return m, False


def run(f, m, st, t_end=np.inf, max_accept=None, max_steps=10 ** 9):
    """Advance until t_end or until max_accept accepted steps."""
    n = 0
    while t_end - st.t > st.h_min and (max_accept is None or st.n_accept < max_accept):
        if n >= max_steps:
            raise RuntimeError("maximum number of attempted steps reached")
        m, _ = step(f, m, st, t_end)
        n += 1
    return m


def replay(f, m, hs, st=None):
    """Take exactly the accepted steps hs (no controller), projecting after each."""
    st = st or State()
    for h in hs:
        y5, k7, err = attempt(f, m, st, h)
        st.k1 = k7
        st.t += h
        st.n_accept += 1
        st.last_err = err
        m = _normalize(y5)
    return m, st
