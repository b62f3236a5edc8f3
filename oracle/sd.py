"""Steepest-descent energy minimisation with Barzilai-Borwein step sizes (oracle).

TEST INFRASTRUCTURE ONLY.  Section "Steepest descent energy minimization":
per cell, with f = m x H_eff(m) and g = m x (m x H_eff(m)), the update is the
implicit midpoint rotation m' = m - tau (m + m')/2 x f, solved explicitly as

    (1 + tau^2 |f|^2 / 4) m' = (1 - tau^2 |f|^2 / 4) m - tau g,

which keeps |m| (equation eq_update and the one after it).  The step size
follows the two Barzilai-Borwein rules of that section with s = m_k - m_{k-1}
and y = g_k - g_{k-1} summed over all cells.  The paper does not say how the
rules are combined, how the first step is chosen or how a non-positive
quotient is treated; the readings used on both sides of this project:

* iteration 0 uses the caller's tau0;
* iteration k >= 1 uses the first rule (s.s / s.y) for odd k and the second
  (s.y / y.y) for even k;
* a quotient that is not finite or not positive keeps the previous tau;
* tau is clipped to [tau_min, tau_max].
"""
import numpy as np


def update(m, H, tau):
    """One steepest-descent update of every cell for step size tau."""
    f = np.cross(m, H, axis=0)
    g = np.cross(m, f, axis=0)
    a = 0.25 * tau * tau * np.sum(f * f, axis=0, keepdims=True)
    return ((1.0 - a) * m - tau * g) / (1.0 + a)


def bb_tau(s, y, k, tau_prev, tau_min, tau_max):
    """Barzilai-Borwein step size of iteration k >= 1 from s and y (sums over all cells)."""
    ss, sy, yy = float(np.sum(s * s)), float(np.sum(s * y)), float(np.sum(y * y))
    num, den = (ss, sy) if k % 2 == 1 else (sy, yy)
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = num / den if den != 0.0 else np.inf
    if not np.isfinite(tau) or tau <= 0.0:
        tau = tau_prev
    return min(max(tau, tau_min), tau_max)


def run(field, m, n_iter, tau0, tau_min, tau_max):
    """n_iter iterations from m; field(m) returns H_eff.  Returns (m, taus)."""
    m_prev = g_prev = None
    tau = tau0
    taus = []
    for k in range(n_iter):
        H = field(m)
        g = np.cross(m, np.cross(m, H, axis=0), axis=0)
        if k > 0:
            tau = bb_tau(m - m_prev, g - g_prev, k, tau, tau_min, tau_max)
        taus.append(tau)
        m_prev, g_prev = m, g
        m = update(m, H, tau)
    return m, taus


def max_torque(m, H):
    """max over cells of |m x H| (the stopping measure of a relaxation)."""
    f = np.cross(m, H, axis=0)
    return float(np.max(np.sqrt(np.sum(f * f, axis=0))))
