"""Fixed-step Heun integration of the LL equation with projection (oracle).

TEST INFRASTRUCTURE ONLY.  The paper's throughput measurement (section
"Performance", the caption of its throughput figure) integrates N x N x 1
films with demagnetisation, exchange and Zeeman terms using Heun's method; it
prints no formula for it.  The reading used here is the textbook Heun
(explicit trapezoid) step followed by the projection onto the unit sphere that
the paper applies after each step of its Runge-Kutta integrators (section
"LLG equation"):

    k1 = f(m),  m1 = m + h k1,  k2 = f(m1),  m <- (m + h (k1 + k2) / 2) / |...|

per cell, f being the LL right-hand side.  Fixed h, no error control.
"""
import numpy as np


def _normalize(y):
    return y / np.sqrt(np.sum(y * y, axis=0, keepdims=True))


def step(f, m, h):
    """One Heun step of size h from m; returns the projected new state."""
    k1 = f(m)
    m1 = m + h * k1
    k2 = f(m1)
    return _normalize(m + (0.5 * h) * (k1 + k2))


def run(f, m, h, n):
    """n Heun steps of size h."""
    for _ in range(n):
        m = step(f, m, h)
    return m
