"""Nudged-elastic-band force and relaxation iteration (oracle).

TEST INFRASTRUCTURE ONLY.  The paper ("Miscellaneous") describes NEB as a chain
of images with fixed end images, relaxed like LLG with the precession term
switched off, where each image's effective field keeps only the part
perpendicular to the tangent set by its neighbours.  It prints no formulas, so
the following reading is used (parity unpinned physically: the paper prints no
barrier and several minimum-energy paths are valid; the tests pin the
structural invariants listed in tests/test_oracle_neb.py and the update
direction, by the first-order energy decrease of an iteration without
springs):

* distance between images: Euclidean norm over all cells and components;
* tangent: the energy-weighted "improved tangent" of Henkelman and Jonsson
  (2000) built from m^{n+1}-m^n and m^n-m^{n-1}, projected per cell onto the
  tangent plane of m_i^n, then normalised over the image;
* force G = H_eff - (H_eff . t) t + k (d_{n,n+1} - d_{n-1,n}) t, dot products
  over the whole image;
* one iteration: m <- normalize(m + h * (-alpha gamma/(1+alpha^2)) m x (m x G))
  for the inner images; end images never move.
"""
import numpy as np

from . import fields


def image_energy(m, mesh, p, kernel):
    return float(np.sum(fields.energies(m, mesh, p, kernel)))


def tangent(m_prev, m, m_next, E_prev, E, E_next):
    """Energy-weighted tangent, projected per cell and normalised over the image."""
    tp = m_next - m
    tm = m - m_prev
    if E_next > E > E_prev:
        t = tp
    elif E_next < E < E_prev:
        t = tm
    else:
        dmax = max(abs(E_next - E), abs(E_prev - E))
        dmin = min(abs(E_next - E), abs(E_prev - E))
        if E_next > E_prev:
            t = tp * dmax + tm * dmin
        else:
            t = tp * dmin + tm * dmax
    t = t - np.sum(t * m, axis=0, keepdims=True) * m
    return t / np.sqrt(np.sum(t * t))


def neb_force(images, mesh, p, kernel, k_spring):
    """Forces G for the inner images, plus energies of all images.

    Returns (G list aligned with images; None for the end images, energies array).
    """
    n = len(images)
    E = np.array([image_energy(m, mesh, p, kernel) for m in images])
    G = [None] * n
    for i in range(1, n - 1):
        H = fields.effective_field(images[i], mesh, p, kernel)
        t = tangent(images[i - 1], images[i], images[i + 1], E[i - 1], E[i], E[i + 1])
        d_next = np.sqrt(np.sum((images[i + 1] - images[i]) ** 2))
        d_prev = np.sqrt(np.sum((images[i] - images[i - 1]) ** 2))
        G[i] = H - np.sum(H * t) * t + k_spring * (d_next - d_prev) * t
    return G, E


def neb_iteration(images, mesh, p, kernel, k_spring, h):
    """One relaxation iteration of the chain; returns (new images, energies before it)."""
    G, E = neb_force(images, mesh, p, kernel, k_spring)
    g = p.alpha * p.gamma / (1.0 + p.alpha ** 2)
    out = [images[0].copy()]
    for i in range(1, len(images) - 1):
        m = images[i]
        mxG = np.cross(m, G[i], axis=0)
        y = m + h * (-g) * np.cross(m, mxG, axis=0)
        out.append(y / np.sqrt(np.sum(y * y, axis=0, keepdims=True)))
    out.append(images[-1].copy())
    return out, E
