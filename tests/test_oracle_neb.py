"""Structural pins for the oracle's NEB force (CPU only).

The paper prints no NEB formulas, so physical barrier values are "parity
unpinned".  What is pinned: the tangent rule's case analysis on hand-made
energies, |t| = 1 and t_i . m_i = 0, the force identity
G . t = k (d_{n,n+1} - d_{n-1,n}), fixed end images, unit norm after an
iteration, and that the update is perpendicular to m cell by cell before
normalisation.  The update direction is pinned by the first-order energy
change of a k = 0 iteration: dE = -mu0 Ms V h g (|H_perp|^2 - (H_perp . t)^2),
which is never positive.
"""
import numpy as np

from oracle import fields as F
from oracle import neb


def _chain(n_img=5, seed=0):
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((3, 1, 4, 5))
    out = []
    for i in range(n_img):
        v = base + 0.3 * i * rng.standard_normal(base.shape)
        out.append(v / np.linalg.norm(v, axis=0))
    return out


def test_tangent_case_analysis():
    a, b, c = _chain(3)
    tp, tm = c - b, b - a

    def proj_norm(t):
        t = t - np.sum(t * b, axis=0, keepdims=True) * b
        return t / np.linalg.norm(t)

    np.testing.assert_allclose(neb.tangent(a, b, c, 0.0, 1.0, 2.0), proj_norm(tp))
    np.testing.assert_allclose(neb.tangent(a, b, c, 2.0, 1.0, 0.0), proj_norm(tm))
    # maximum at b, E_next > E_prev: dmax = 3 (to prev), dmin = 1 (to next)... weights
    t = neb.tangent(a, b, c, 0.0, 3.0, 2.0)
    np.testing.assert_allclose(t, proj_norm(tp * 3.0 + tm * 1.0))
    t = neb.tangent(a, b, c, 2.0, 3.0, 0.0)
    np.testing.assert_allclose(t, proj_norm(tp * 1.0 + tm * 3.0))


def test_force_identities_and_iteration():
    mesh = F.Mesh(5, 4, 1, 2e-9, 2e-9, 1e-9)
    p = F.Params(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=5e5, H=(0, 0, 1e5), alpha=0.5)
    kern = F.DemagKernel(mesh)
    imgs = _chain(5)
    k = 1e5
    G, E = neb.neb_force(imgs, mesh, p, kern, k)
    assert G[0] is None and G[-1] is None
    for i in range(1, 4):
        t = neb.tangent(imgs[i - 1], imgs[i], imgs[i + 1], E[i - 1], E[i], E[i + 1])
        assert abs(np.linalg.norm(t) - 1) < 1e-14
        assert np.max(np.abs(np.sum(t * imgs[i], axis=0))) < 1e-14
        dn = np.linalg.norm(imgs[i + 1] - imgs[i])
        dp = np.linalg.norm(imgs[i] - imgs[i - 1])
        assert abs(np.sum(G[i] * t) - k * (dn - dp)) <= 1e-9 * np.max(np.abs(G[i]))
    new, E0 = neb.neb_iteration(imgs, mesh, p, kern, k, 1e-14)
    assert np.array_equal(new[0], imgs[0]) and np.array_equal(new[-1], imgs[-1])
    for m in new:
        assert np.max(np.abs(np.linalg.norm(m, axis=0) - 1)) < 1e-14
    np.testing.assert_allclose(E0, E)


def test_relaxation_lowers_the_middle_image_energy():
    """With k = 0 one iteration moves the middle image by h g G_perp (g = alpha gamma /
    (1 + alpha^2)), so to first order dE = -mu0 Ms V h g sum_i H_i . G_perp,i
    = -mu0 Ms V h g (|H_perp|^2 - (H_perp . t)^2) <= 0 (t is a unit vector in the
    cells' tangent planes; Cauchy-Schwarz).  The energy must fall at that rate."""
    mesh = F.Mesh(5, 4, 1, 2e-9, 2e-9, 1e-9)
    p = F.Params(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=5e5, H=(0, 0, 1e5), alpha=0.5)
    kern = F.DemagKernel(mesh)
    imgs = _chain(3, seed=4)
    G, E = neb.neb_force(imgs, mesh, p, kern, 0.0)
    m = imgs[1]
    H = F.effective_field(m, mesh, p, kern)
    t = neb.tangent(imgs[0], m, imgs[2], E[0], E[1], E[2])
    Hp = H - np.sum(H * m, axis=0, keepdims=True) * m
    rate = np.sum(Hp * Hp) - np.sum(Hp * t) ** 2
    assert rate > 0.05 * np.sum(Hp * Hp)  # strictly downhill here
    g = p.alpha * p.gamma / (1 + p.alpha ** 2)
    V = mesh.dx * mesh.dy * mesh.dz
    for h in (1e-16, 1e-17):
        new, _ = neb.neb_iteration(imgs, mesh, p, kern, 0.0, h)
        dE = neb.image_energy(new[1], mesh, p, kern) - E[1]
        want = -F.MU0 * p.Ms * V * h * g * rate
        assert dE < 0
        assert abs(dE - want) <= 1e-3 * abs(want)
