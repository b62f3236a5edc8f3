"""Demagnetising field through the magnetic scalar potential (oracle; test infrastructure only).

The paper (section "Magnetostatic energy") notes that the FFT demag field takes
three forward and three inverse transforms, and that with the magnetic scalar
potential the three inverse transforms become one (citing Abert et al., 2012).
It prints no formulas for this route.  The reading used here:

* H_d = -grad u.  For magnetisation uniform in each cell,
  u(r) = sum_j M_j . S(r - r_j) with S(R) = (1/4 pi) int_cell (R - r') / |R - r'|^3 dr',
  the potential of a uniformly magnetised unit cuboid centred at 0 (M = e_a
  gives S_a).  Integrating along a, S_a is the potential of the cuboid's two
  charged a-faces, (1/4 pi) [I(+a face) - I(-a face)], with I the integral of
  1/|R - r'| over a face, which has a closed form.
* u is evaluated at the cell corners (the (nx+1)(ny+1)(nz+1) vertices).
* The field of a cell: H_a = -(1/(4 d_a)) sum over the cell's four edges along a
  of [u(+ end) - u(- end)].  The exact cell average of -d_a u is the difference
  of u's averages over the two a-faces over d_a (Newell's cell-averaged field);
  here each face average is the trapezoid rule over the face's four corners,
  so the field tends to Newell's as the mesh is refined.
* The sum over j is a convolution over the vertex - cell displacements
  ((i - 1/2) dx, (j - 1/2) dy, (k - 1/2) dz), i in [-nx+1, nx] (2n values per
  axis): a circular convolution on P >= 2n points per axis gives it exactly,
  with three forward transforms of M and one inverse transform of u.

S is evaluated from the closed form for rho = |R| / max(d) < 3 and by
Gauss-Legendre quadrature of its defining volume integral beyond (the closed
form's face differences cancel at large distance).  Pinned in
tests/test_oracle_potential.py.
"""
import numpy as np
import scipy.fft

from . import MU0
from . import fields as F


def face_antiderivative(x, y, z):
    """G with d2G/dxdy = 1/sqrt(x^2 + y^2 + z^2):
    x asinh(y / sqrt(x^2 + z^2)) + y asinh(x / sqrt(y^2 + z^2)) - z atan(x y / (z r));
    terms whose prefactor vanishes are 0 (their limits)."""
    x, y, z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, y, z)))
    r = np.sqrt(x * x + y * y + z * z)
    out = np.zeros(x.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        ax = np.sqrt(x * x + z * z)
        out = out + np.where((x != 0) & (ax > 0), x * np.arcsinh(y / np.where(ax > 0, ax, 1.0)), 0.0)
        ay = np.sqrt(y * y + z * z)
        out = out + np.where((y != 0) & (ay > 0), y * np.arcsinh(x / np.where(ay > 0, ay, 1.0)), 0.0)
        t = (z != 0) & (r > 0)
        out = out - np.where(t, z * np.arctan(x * y / np.where(t, z * r, 1.0)), 0.0)
    return out


def face_integral(x1, x2, y1, y2, w):
    """Integral of 1/sqrt(x^2 + y^2 + w^2) over x in [x1, x2], y in [y1, y2]."""
    G = face_antiderivative
    return G(x2, y2, w) - G(x1, y2, w) - G(x2, y1, w) + G(x1, y1, w)


def kernel_closed(R, d):
    """S(R) for displacements R (array [..., 3]) of a cell of size d = (dx, dy, dz), closed form."""
    R = np.asarray(R, dtype=np.float64)
    out = np.zeros(R.shape)
    for a in range(3):
        b, c = [k for k in range(3) if k != a]
        lo_b, hi_b = -0.5 * d[b] - R[..., b], 0.5 * d[b] - R[..., b]
        lo_c, hi_c = -0.5 * d[c] - R[..., c], 0.5 * d[c] - R[..., c]
        plus = face_integral(lo_b, hi_b, lo_c, hi_c, R[..., a] - 0.5 * d[a])
        minus = face_integral(lo_b, hi_b, lo_c, hi_c, R[..., a] + 0.5 * d[a])
        out[..., a] = (plus - minus) / (4.0 * np.pi)
    return out


def kernel_quadrature(R, d, n):
    """S(R) by n-point Gauss-Legendre quadrature per axis of (1/4pi) int_cell (R - r')/|R - r'|^3 dr'."""
    R = np.asarray(R, dtype=np.float64)
    t, w = np.polynomial.legendre.leggauss(n)
    out = np.zeros(R.shape)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                rp = np.array([0.5 * d[0] * t[i], 0.5 * d[1] * t[j], 0.5 * d[2] * t[k]])
                v = R - rp
                r3 = np.sum(v * v, axis=-1) ** 1.5
                out += (w[i] * w[j] * w[k]) * v / r3[..., None]
    return out * (d[0] * d[1] * d[2] / 8.0) / (4.0 * np.pi)


# nodes per axis of the quadrature by rho = |R| / max(d): [3, 6) -> 14, [6, 16) -> 9,
# [16, 40) -> 6, [40, 300) -> 4, beyond -> 3
_RHO_NODES = ((3.0, 14), (6.0, 9), (16.0, 6), (40.0, 4), (300.0, 3))


def kernel(R, d):
    """S(R): closed form for rho < 3, quadrature beyond."""
    R = np.asarray(R, dtype=np.float64)
    rho = np.sqrt(np.sum(R * R, axis=-1)) / max(d)
    out = np.zeros(R.shape)
    near = rho < _RHO_NODES[0][0]
    if np.any(near):
        out[near] = kernel_closed(R[near], d)
    bounds = [b for b, _ in _RHO_NODES] + [np.inf]
    for (lo, n), hi in zip(_RHO_NODES, bounds[1:]):
        sel = (rho >= lo) & (rho < hi)
        if np.any(sel):
            out[sel] = kernel_quadrature(R[sel], d, n)
    return out


def kernel_grid(nx, ny, nz, dx, dy, dz):
    """S on the vertex - cell displacements ((i - 1/2) dx, (j - 1/2) dy, (k - 1/2) dz),
    i in [-nx+1, nx] (likewise j, k): array [2nz, 2ny, 2nx, 3], index i + nx - 1."""
    i = (np.arange(-nx + 1, nx + 1) - 0.5) * dx
    j = (np.arange(-ny + 1, ny + 1) - 0.5) * dy
    k = (np.arange(-nz + 1, nz + 1) - 0.5) * dz
    R = np.stack(np.meshgrid(i, j, k, indexing="ij"), axis=-1)  # [x, y, z, 3]
    return np.transpose(kernel(R, (dx, dy, dz)), (2, 1, 0, 3))


def padded_shape(mesh):
    """P = 2n per axis (the smallest length that holds the 2n displacements)."""
    return (2 * mesh.nz, 2 * mesh.ny, 2 * mesh.nx)


class PotentialKernel:
    """The displacement lattice wrapped on the padded grid and its spectrum (FP64, complex)."""

    def __init__(self, mesh, P=None):
        self.mesh = mesh
        self.P = tuple(P) if P is not None else padded_shape(mesh)
        for Pd, n in zip(self.P, (mesh.nz, mesh.ny, mesh.nx)):
            if Pd < 2 * n:
                raise ValueError("the potential route needs P >= 2n per axis")
        grid = kernel_grid(mesh.nx, mesh.ny, mesh.nz, mesh.dx, mesh.dy, mesh.dz)
        K = np.zeros(self.P + (3,))
        kk = np.arange(-mesh.nz + 1, mesh.nz + 1) % self.P[0]
        jj = np.arange(-mesh.ny + 1, mesh.ny + 1) % self.P[1]
        ii = np.arange(-mesh.nx + 1, mesh.nx + 1) % self.P[2]
        K[np.ix_(kk, jj, ii)] = grid
        self.spectrum = scipy.fft.fftn(np.moveaxis(K, -1, 0), axes=(1, 2, 3))

    def vertex_potential(self, M):
        """u at the vertices [nz+1, ny+1, nx+1] for M = Ms m (3, nz, ny, nx)."""
        nz, ny, nx = M.shape[1:]
        Mp = np.zeros((3,) + self.P)
        Mp[:, :nz, :ny, :nx] = M
        Mh = scipy.fft.fftn(Mp, axes=(1, 2, 3))
        u = scipy.fft.ifftn(np.sum(self.spectrum * Mh, axis=0)).real
        return u[:nz + 1, :ny + 1, :nx + 1]


def vertex_potential_direct(M, mesh):
    """u at every vertex by the plain sum over cells (O(N^2); small meshes)."""
    nz, ny, nx = M.shape[1:]
    d = (mesh.dx, mesh.dy, mesh.dz)
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([cx.ravel() * mesh.dx, cy.ravel() * mesh.dy, cz.ravel() * mesh.dz], axis=-1)
    Mf = M.reshape(3, -1).T
    u = np.zeros((nz + 1, ny + 1, nx + 1))
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                v = np.array([(i - 0.5) * mesh.dx, (j - 0.5) * mesh.dy, (k - 0.5) * mesh.dz])
                u[k, j, i] = np.sum(kernel(v - cells, d) * Mf)
    return u


def field_from_potential(u, mesh):
    """H of each cell from its eight corner potentials: -(1/(4 d_a)) sum over the
    four a-edges of u(+ end) - u(- end)."""
    Hx = -(u[:-1, :-1, 1:] - u[:-1, :-1, :-1] + u[:-1, 1:, 1:] - u[:-1, 1:, :-1]
           + u[1:, :-1, 1:] - u[1:, :-1, :-1] + u[1:, 1:, 1:] - u[1:, 1:, :-1]) / (4.0 * mesh.dx)
    Hy = -(u[:-1, 1:, :-1] - u[:-1, :-1, :-1] + u[:-1, 1:, 1:] - u[:-1, :-1, 1:]
           + u[1:, 1:, :-1] - u[1:, :-1, :-1] + u[1:, 1:, 1:] - u[1:, :-1, 1:]) / (4.0 * mesh.dy)
    Hz = -(u[1:, :-1, :-1] - u[:-1, :-1, :-1] + u[1:, :-1, 1:] - u[:-1, :-1, 1:]
           + u[1:, 1:, :-1] - u[:-1, 1:, :-1] + u[1:, 1:, 1:] - u[:-1, 1:, 1:]) / (4.0 * mesh.dz)
    return np.stack([Hx, Hy, Hz])


def demag_field(m, mesh, Ms, kern=None):
    """H_d of the scalar-potential route for magnetisation Ms m (uniform Ms)."""
    if kern is None:
        kern = PotentialKernel(mesh)
    return field_from_potential(kern.vertex_potential(Ms * m), mesh)


def effective_field(m, mesh, p, kern=None, newell_kernel=None):
    """H_eff with the demag term (when p.terms has DEMAG) from the potential route;
    every other term as in `fields`."""
    H = np.zeros_like(m, dtype=np.float64)
    q = F.Params(p.Ms, p.A, p.D, p.Ku, p.u, p.H, p.alpha, p.gamma, p.terms & ~F.DEMAG)
    for h in F.effective_field_terms(m, mesh, q).values():
        H += h
    if p.terms & F.DEMAG:
        H += demag_field(m, mesh, p.Ms, kern)
    return H


def energies(m, mesh, p, kern=None):
    """Energies as in `fields.energies`, the demag entry from the potential route's field."""
    q = F.Params(p.Ms, p.A, p.D, p.Ku, p.u, p.H, p.alpha, p.gamma, p.terms & ~F.DEMAG)
    E = F.energies(m, mesh, q)
    if p.terms & F.DEMAG:
        V = mesh.dx * mesh.dy * mesh.dz
        E[1] = -0.5 * MU0 * p.Ms * V * np.sum(m * demag_field(m, mesh, p.Ms, kern))
    return E
