"""Pins for the oracle's Dormand-Prince 5(4) integrator (CPU only).

* the tableau satisfies the Runge-Kutta order conditions (order 5 for b,
  order 4 for bhat) in exact rational arithmetic, the row-sum condition
  sum_j a_sj = c_s and the FSAL property a_7j = b_j;
* one step on y' = lambda y has local error O(h^6);
* the macrospin under a static field follows the closed form of the paper's
  section "A magnetic moment under an external magnetic field" (eq_llg_m) with
  its printed parameters; the error at t = 1 ns, alpha = 0.05 shrinks with rtol;
* |m| = 1 after each accepted step; energy never increases under damping
  with a static field, and is conserved to tolerance at alpha = 0;
* replaying the accepted step sizes reproduces the adaptive run bit for bit;
* a rejected attempt leaves m untouched;
* the step-size rule: on a problem with a constant error constant the accepted
  error settles at 0.9^5 (fixed by the estimate being O(h^5) and the exponent
  -1/5), a retry after a rejection lands on 0.9^5 too, and an accepted step
  right after a rejection never grows h.
"""
import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import dp45
from oracle import fields as F


def test_tableau_row_sums_and_fsal():
    for s in range(1, 7):
        assert sum(dp45.A[s]) == dp45.C[s]
    assert sum(dp45.B) == 1 and sum(dp45.BHAT) == 1
    assert tuple(dp45.A[6]) + (Fr(0),) == tuple(dp45.B)


def _order_conditions(b, order):
    """Butcher order conditions up to `order` for weights b with the DP45 matrix A."""
    A = [[Fr(0)] * 7 for _ in range(7)]
    for s in range(1, 7):
        for j, a in enumerate(dp45.A[s]):
            A[s][j] = a
    c = list(dp45.C)
    Ac = [sum(A[i][j] * c[j] for j in range(7)) for i in range(7)]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(7)) for i in range(7)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(7)) for i in range(7)]
    conds = [
        (sum(b), Fr(1)),
        (sum(bi * ci for bi, ci in zip(b, c)), Fr(1, 2)),
        (sum(bi * ci ** 2 for bi, ci in zip(b, c)), Fr(1, 3)),
        (sum(bi * x for bi, x in zip(b, Ac)), Fr(1, 6)),
        (sum(bi * ci ** 3 for bi, ci in zip(b, c)), Fr(1, 4)),
        (sum(bi * ci * x for bi, ci, x in zip(b, c, Ac)), Fr(1, 8)),
        (sum(bi * x for bi, x in zip(b, Ac2)), Fr(1, 12)),
        (sum(bi * x for bi, x in zip(b, AAc)), Fr(1, 24)),
    ]
    if order >= 5:
        Ac3 = [sum(A[i][j] * c[j] ** 3 for j in range(7)) for i in range(7)]
        cAc = [c[i] * Ac[i] for i in range(7)]
        AcAc = [sum(A[i][j] * cAc[j] for j in range(7)) for i in range(7)]
        AAc2 = [sum(A[i][j] * Ac2[j] for j in range(7)) for i in range(7)]
        AAAc = [sum(A[i][j] * AAc[j] for j in range(7)) for i in range(7)]
        conds += [
            (sum(bi * ci ** 4 for bi, ci in zip(b, c)), Fr(1, 5)),
            (sum(bi * ci ** 2 * x for bi, ci, x in zip(b, c, Ac)), Fr(1, 10)),
            (sum(bi * x * x for bi, x in zip(b, Ac)), Fr(1, 20)),
            (sum(bi * ci * x for bi, ci, x in zip(b, c, Ac2)), Fr(1, 15)),
            (sum(bi * x for bi, x in zip(b, Ac3)), Fr(1, 20)),
            (sum(bi * ci * x for bi, ci, x in zip(b, c, AAc)), Fr(1, 30)),
            (sum(bi * x for bi, x in zip(b, AcAc)), Fr(1, 40)),
            (sum(bi * x for bi, x in zip(b, AAc2)), Fr(1, 60)),
            (sum(bi * x for bi, x in zip(b, AAAc)), Fr(1, 120)),
        ]
    return conds


def test_order_conditions():
    for got, want in _order_conditions(dp45.B, 5):
        assert got == want
    for got, want in _order_conditions(dp45.BHAT, 4):
        assert got == want
    # bhat is genuinely only 4th order (else there is no error estimate)
    assert any(g != w for g, w in _order_conditions(dp45.BHAT, 5))


def test_local_error_is_sixth_order():
    lam = -1.5
    f = lambda y: lam * y
    errs = []
    for h in (0.2, 0.1, 0.05):
        st = dp45.State(rtol=1.0)
        y5, _, _ = dp45.attempt(f, np.ones((3, 1, 1, 1)), st, h)
        errs.append(abs(y5[0, 0, 0, 0] - np.exp(lam * h)))
    assert 50 < errs[0] / errs[1] < 80 and 50 < errs[1] / errs[2] < 80


PAPER = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "macrospin_paper.json")))
HZ, GAMMA = PAPER["Hz_A_per_m"], PAPER["gamma_m_per_A_s"]


def _macrospin(alpha, Hz=HZ, gamma=GAMMA):
    mesh = F.Mesh(1, 1, 1, 1e-9, 1e-9, 1e-9)
    p = F.Params(Ms=8e5, H=(0, 0, Hz), alpha=alpha, gamma=gamma, terms=F.ZEEMAN)
    m0 = np.zeros((3, 1, 1, 1))
    m0[:, 0, 0, 0] = PAPER["m0"]
    return mesh, p, m0


def _analytic(t, alpha, Hz=HZ, gamma=GAMMA):
    g = gamma / (1 + alpha ** 2)
    return np.array([math.cos(g * Hz * t) / math.cosh(alpha * g * Hz * t),
                     math.sin(g * Hz * t) / math.cosh(alpha * g * Hz * t),
                     math.tanh(alpha * g * Hz * t)])


def test_macrospin_matches_closed_form():
    a = PAPER["alpha"]
    mesh, p, m = _macrospin(a)
    f = lambda y: F.llg_rhs(y, mesh, p)
    for t_end in (5e-11, 2e-10, 5e-10):
        st = dp45.State(rtol=1e-9, h=1e-13)
        mm = dp45.run(f, m.copy(), st, t_end=t_end)
        assert st.t == t_end
        assert np.linalg.norm(mm[:, 0, 0, 0] - _analytic(t_end, a)) < 1e-7


def test_macrospin_error_shrinks_with_rtol():
    a, T = PAPER["error_figure_alpha"], PAPER["error_figure_t_s"]
    mesh, p, m = _macrospin(a)
    f = lambda y: F.llg_rhs(y, mesh, p)
    errs = []
    for rtol in (1e-4, 1e-6, 1e-8):
        st = dp45.State(rtol=rtol)
        mm = dp45.run(f, m.copy(), st, t_end=T)
        errs.append(np.linalg.norm(mm[:, 0, 0, 0] - _analytic(T, a)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-5


def _small_problem(alpha):
    mesh = F.Mesh(6, 5, 1, 3e-9, 3e-9, 2e-9)
    p = F.Params(Ms=8e5, A=1.3e-11, D=1e-3, Ku=2e5, H=(0, 0, 5e4), alpha=alpha)
    rng = np.random.default_rng(11)
    m = rng.standard_normal((3, 1, 5, 6))
    m /= np.linalg.norm(m, axis=0)
    kern = F.DemagKernel(mesh)
    return mesh, p, m, kern


def test_damped_energy_decreases_and_norm_kept():
    mesh, p, m, kern = _small_problem(0.3)
    f = lambda y: F.llg_rhs(y, mesh, p, kern)
    st = dp45.State(rtol=1e-6)
    E_prev = np.sum(F.energies(m, mesh, p, kern))
    for _ in range(40):
        m, acc = dp45.step(f, m, st)
        if acc:
            assert np.max(np.abs(np.linalg.norm(m, axis=0) - 1)) < 1e-14
            E = np.sum(F.energies(m, mesh, p, kern))
            assert E <= E_prev + 1e-12 * abs(E_prev)
            E_prev = E


def test_undamped_energy_conserved():
    mesh, p, m, kern = _small_problem(0.0)
    f = lambda y: F.llg_rhs(y, mesh, p, kern)
    st = dp45.State(rtol=1e-8)
    E0 = np.sum(F.energies(m, mesh, p, kern))
    m = dp45.run(f, m, st, t_end=2e-12)
    E1 = np.sum(F.energies(m, mesh, p, kern))
    assert abs(E1 - E0) < 1e-5 * abs(E0)


def test_replay_reproduces_run_and_reject_keeps_m():
    mesh, p, m0, kern = _small_problem(0.1)
    f = lambda y: F.llg_rhs(y, mesh, p, kern)
    st = dp45.State(rtol=1e-5, h=5e-12)  # too large: the first attempt is rejected
    m = m0.copy()
    m1, acc = dp45.step(f, m, st)
    assert not acc and st.n_reject == 1 and m1 is m
    m = dp45.run(f, m1, st, max_accept=25)
    m_rep, st2 = dp45.replay(f, m0.copy(), st.accepted_h)
    assert np.array_equal(m, m_rep)
    assert st2.n_accept == st.n_accept


def test_underflow_raises():
    mesh, p, m, kern = _small_problem(0.1)
    f = lambda y: F.llg_rhs(y, mesh, p, kern)
    st = dp45.State(rtol=1e-30, h=1e-13, h_min=1e-16)
    with pytest.raises(dp45.StepUnderflow):
        dp45.run(f, m, st, t_end=1e-9, max_steps=200)


def _precession():
    """Undamped macrospin precessing about H = Hz e_z from m = e_x: a uniform rotation,
    so the local error constant of every step is the same."""
    mesh = F.Mesh(1, 1, 1, 1e-9, 1e-9, 1e-9)
    p = F.Params(Ms=8e5, H=(0, 0, 1e5), alpha=0.0, gamma=GAMMA, terms=F.ZEEMAN)
    m0 = np.zeros((3, 1, 1, 1))
    m0[0] = 1.0
    return (lambda y: F.llg_rhs(y, mesh, p)), m0


def test_controller_settles_at_safety_to_the_fifth():
    """The embedded estimate is O(h^5), so with h_new = h * 0.9 err^(-1/5) the error of
    the next step on a problem with a constant error constant is 0.9^5 err / err = 0.9^5
    (an exponent -1/4 would settle at 0.9^4 = 0.656 instead)."""
    f, m = _precession()
    st = dp45.State(rtol=1e-8, h=1e-13)
    errs = []
    for _ in range(60):
        m, acc = dp45.step(f, m, st)
        assert acc  # growing from a small h never overshoots
        errs.append(st.last_err)
    assert st.accepted_h[-1] < 0.05 * st.h_max  # the h_max clip plays no part
    np.testing.assert_allclose(errs[-20:], 0.9 ** 5, rtol=2e-3)


def test_rejection_factor_lands_on_the_target_error():
    """A rejected step retries with h * 0.9 err^(-1/5); in the asymptotic regime the retry
    then has error 0.9^5 whatever the rejected error was (with -1/4: 0.59 err^(-1/4))."""
    f, m = _precession()
    for h0 in (6e-12, 8e-12, 1.1e-11):
        st = dp45.State(rtol=1e-8, h=h0)
        m1, acc = dp45.step(f, m.copy(), st)
        assert not acc and 1.5 < st.last_err < 100.0  # no FAC_MIN clip
        m1, acc = dp45.step(f, m1, st)
        assert acc
        assert abs(st.last_err - 0.9 ** 5) < 0.02


def test_no_growth_right_after_a_rejection():
    """An accepted step right after a rejection never grows h, even where the error
    factor alone would (here by 2-8%): a stiff linear decay towards e_x started from
    steps far outside the stability region."""
    lam = 1e10
    u = np.zeros((3, 1, 1, 1))
    u[0] = 1.0
    f = lambda y: -lam * (y - u)
    m = np.zeros((3, 1, 1, 1))
    m[2] = 1.0
    st = dp45.State(rtol=1e-4, h=1000.0 / lam, h_max=1.0, h_min=1e-30)
    prev_rejected, binding = False, 0
    for _ in range(40):
        m, acc = dp45.step(f, m, st)
        if acc and prev_rejected:
            assert st.h <= st.accepted_h[-1]
            if 0.9 * st.last_err ** -0.2 > 1.02:
                binding += 1
        prev_rejected = not acc
    assert binding >= 2
