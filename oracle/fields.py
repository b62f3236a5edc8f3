"""Effective field, energies and Landau-Lifshitz right-hand side in FP64 (oracle).

TEST INFRASTRUCTURE ONLY.  Arrays are SoA: m has shape (3, nz, ny, nx), x fastest,
unit vectors per cell.  SI units: fields in A/m, energies in J.

Paper sections followed (MicroMagnetic.jl paper):
* effective field as the functional derivative -1/(mu0 Ms) dE/dm ("Micromagnetics");
* exchange: six-neighbour energy density w_i and field H_ex,i ("Exchange energy");
* demag: E_d = (mu0/2) sum V M_i . N_{i-j} . M_j and H_d,i = -sum_j N_{i-j} M_j
  (eq_demag_energy2, eq_hd1); the FFT route is the convolution theorem applied
  to that sum on a zero-padded grid;
* interfacial DMI: the unified stencil H_dmi,i = -(1/(mu0 Ms)) sum_j D (e_ij x m_j)/Delta_ij
  with e_ij = {-e_y, +e_y, +e_x, -e_x, 0, 0} for the neighbours {-x,+x,-y,+y,-z,+z}
  ("Dzyaloshinskii-Moriya Energy");
* uniaxial anisotropy: the atomistic form H = (2K/mu_s)(m.u)u written for cells,
  mu_s -> mu0 Ms ("Anisotropy");
* Zeeman: the applied field itself ("Zeeman energy");
* LL form of the LLG equation (eq_llg2).

Readings where the paper is silent: open boundaries (missing neighbours drop out
of the exchange and DMI sums), mu0 = 4 pi 1e-7, anisotropy energy -Ku (m.u)^2.
"""
from collections import namedtuple

import numpy as np
import scipy.fft

from . import MU0, GAMMA_DEFAULT
from . import newell

Mesh = namedtuple("Mesh", "nx ny nz dx dy dz")

EXCHANGE, DEMAG, DMI, ANIS, ZEEMAN = 1, 2, 4, 8, 16
ALL_TERMS = EXCHANGE | DEMAG | DMI | ANIS | ZEEMAN
# the other two DMI symmetry classes of the DMI section (same constant D)
DMI_BULK, DMI_D2D = 32, 64


class Params:
    """Uniform material and run parameters (SI)."""

    def __init__(self, Ms, A=0.0, D=0.0, Ku=0.0, u=(0.0, 0.0, 1.0), H=(0.0, 0.0, 0.0),
                 alpha=0.5, gamma=GAMMA_DEFAULT, terms=ALL_TERMS):
        self.Ms, self.A, self.D, self.Ku = float(Ms), float(A), float(D), float(Ku)
        u = np.asarray(u, dtype=np.float64)
        self.u = u / np.linalg.norm(u)
        self.H = np.asarray(H, dtype=np.float64)
        self.alpha, self.gamma = float(alpha), float(gamma)
        self.terms = int(terms)


# neighbour directions: (axis index in the (z, y, x) array, step, cell-size attribute,
# DMI vector e_ij as (ex, ey, ez))
_NEIGHBOURS = (
    (2, -1, "dx", (0.0, -1.0, 0.0)),   # -x : -e_y
    (2, +1, "dx", (0.0, +1.0, 0.0)),   # +x : +e_y
    (1, -1, "dy", (+1.0, 0.0, 0.0)),   # -y : +e_x
    (1, +1, "dy", (-1.0, 0.0, 0.0)),   # +y : -e_x
    (0, -1, "dz", (0.0, 0.0, 0.0)),    # -z : 0
    (0, +1, "dz", (0.0, 0.0, 0.0)),    # +z : 0
)


def _neighbour(m, axis, step):
    """Return (m_j, valid) where m_j[.., i] = m[.., i + step along axis] and valid marks
    cells whose neighbour exists (open boundary)."""
    n = m.shape[1 + axis]
    mj = np.zeros_like(m)
    valid = np.zeros(m.shape[1:], dtype=bool)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if step > 0:
        src[axis], dst[axis] = slice(1, n), slice(0, n - 1)
    else:
        src[axis], dst[axis] = slice(0, n - 1), slice(1, n)
    mj[(slice(None),) + tuple(dst)] = m[(slice(None),) + tuple(src)]
    valid[tuple(dst)] = True
    return mj, valid


def exchange_field(m, mesh, p):
    """H_ex,i = (2A/(mu0 Ms)) sum_{j in N_i} (m_j - m_i)/Delta_ij^2."""
    H = np.zeros_like(m)
    for axis, step, dname, _ in _NEIGHBOURS:
        mj, valid = _neighbour(m, axis, step)
        delta = getattr(mesh, dname)
        H += np.where(valid, (mj - m) / delta ** 2, 0.0)
    return (2.0 * p.A / (MU0 * p.Ms)) * H


def dmi_field(m, mesh, p):
    """H_dmi,i = -(D/(mu0 Ms)) sum_{j in N_i} (e_ij x m_j)/Delta_ij, interfacial e_ij."""
    H = np.zeros_like(m)
    for axis, step, dname, e in _NEIGHBOURS:
        if e == (0.0, 0.0, 0.0):
            continue
        mj, valid = _neighbour(m, axis, step)
        delta = getattr(mesh, dname)
        e = np.asarray(e).reshape(3, 1, 1, 1)
        H += np.where(valid, np.cross(e, mj, axis=0) / delta, 0.0)
    return -(p.D / (MU0 * p.Ms)) * H


# DMI vectors e_ij of the unified DMI form for the neighbours -x, +x, -y, +y, -z, +z
# (same order as _NEIGHBOURS): bulk (classes T, O) e_ij = r_ij; class D2d
# {e_x, -e_x, -e_y, e_y, 0, 0}
_E_BULK = ((-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, -1.0), (0.0, 0.0, 1.0))
_E_D2D = ((1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))


def dmi_field_vectors(m, mesh, p, evecs):
    """H_dmi,i = -(D/(mu0 Ms)) sum_{j in N_i} (e_ij x m_j)/Delta_ij for DMI vectors evecs."""
    H = np.zeros_like(m)
    for (axis, step, dname, _), e in zip(_NEIGHBOURS, evecs):
        if e == (0.0, 0.0, 0.0):
            continue
        mj, valid = _neighbour(m, axis, step)
        delta = getattr(mesh, dname)
        e = np.asarray(e).reshape(3, 1, 1, 1)
        H += np.where(valid, np.cross(e, mj, axis=0) / delta, 0.0)
    return -(p.D / (MU0 * p.Ms)) * H


def anisotropy_field(m, p):
    """H_an,i = (2 Ku/(mu0 Ms)) (m_i . u) u."""
    u = p.u.reshape(3, 1, 1, 1)
    return (2.0 * p.Ku / (MU0 * p.Ms)) * np.sum(m * u, axis=0, keepdims=True) * u


def zeeman_field(m, p):
    """H_Z = H_app (uniform, constant in time)."""
    return np.broadcast_to(p.H.reshape(3, 1, 1, 1), m.shape).copy()


def demag_field_direct(m, mesh, p, tensor_fn=newell.tensor):
    """H_d,i = -Ms sum_j N(r_i - r_j) m_j, the plain O(N^2) sum (self term included)."""
    nz, ny, nx = m.shape[1:]
    cells = np.stack(np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                                 indexing="ij"), axis=-1).reshape(-1, 3)  # (k, j, i)
    mflat = m.reshape(3, -1)
    H = np.zeros((3, cells.shape[0]))
    for t, (k, j, i) in enumerate(cells):
        Nt = newell.as_matrix(tensor_fn(i - cells[:, 2], j - cells[:, 1], k - cells[:, 0],
                                        mesh.dx, mesh.dy, mesh.dz))      # [N, 3, 3]
        H[:, t] = -p.Ms * np.einsum("sab,bs->a", Nt, mflat)
    return H.reshape(m.shape)


def padded_shape(mesh):
    """Zero-padded FFT grid: P = 2n for n > 1, P = 1 for n = 1 (any P >= 2n-1 is exact)."""
    return tuple(1 if n == 1 else 2 * n for n in (mesh.nz, mesh.ny, mesh.nx))


class DemagKernel:
    """Wrapped tensor on the padded grid and its spectrum (FP64, no symmetry folding)."""

    def __init__(self, mesh, P=None, grid=None):
        nz, ny, nx = mesh.nz, mesh.ny, mesh.nx
        self.mesh = mesh
        self.P = tuple(P) if P is not None else padded_shape(mesh)
        for Pd, n in zip(self.P, (nz, ny, nx)):
            if Pd < 2 * n - 1:
                raise ValueError("padded length must be at least 2n-1")
        if grid is None:
            grid = newell.tensor_grid(nx, ny, nz, mesh.dx, mesh.dy, mesh.dz)
        K = np.zeros(self.P + (6,))
        kk = np.arange(-nz + 1, nz) % self.P[0]
        jj = np.arange(-ny + 1, ny) % self.P[1]
        ii = np.arange(-nx + 1, nx) % self.P[2]
        K[np.ix_(kk, jj, ii)] = grid
        self.spectrum = scipy.fft.rfftn(np.moveaxis(K, -1, 0), axes=(1, 2, 3))  # [6, ...]

    def field(self, m, Ms):
        """H_d = -Ms * IFFT( Nhat . FFT(m) ), cropped to the mesh."""
        nz, ny, nx = m.shape[1:]
        mp = np.zeros((3,) + self.P)
        mp[:, :nz, :ny, :nx] = m
        mh = scipy.fft.rfftn(mp, axes=(1, 2, 3))
        S = self.spectrum
        idx = ((0, 3, 4), (3, 1, 5), (4, 5, 2))
        Hh = [sum(S[idx[a][b]] * mh[b] for b in range(3)) for a in range(3)]
        H = np.stack([scipy.fft.irfftn(h, s=self.P, axes=(0, 1, 2)) for h in Hh])
        return -Ms * H[:, :nz, :ny, :nx]


def effective_field_terms(m, mesh, p, kernel=None):
    """Dict term-name -> field for the enabled terms."""
    out = {}
    if p.terms & EXCHANGE:
        out["exchange"] = exchange_field(m, mesh, p)
    if p.terms & DEMAG:
        if kernel is None:
            kernel = DemagKernel(mesh)
        out["demag"] = kernel.field(m, p.Ms)
    if p.terms & DMI:
        out["dmi"] = dmi_field(m, mesh, p)
    if p.terms & DMI_BULK:
        out["dmi_bulk"] = dmi_field_vectors(m, mesh, p, _E_BULK)
    if p.terms & DMI_D2D:
        out["dmi_d2d"] = dmi_field_vectors(m, mesh, p, _E_D2D)
    if p.terms & ANIS:
        out["anisotropy"] = anisotropy_field(m, p)
    if p.terms & ZEEMAN:
        out["zeeman"] = zeeman_field(m, p)
    return out


def effective_field(m, mesh, p, kernel=None):
    """H_eff = sum of the enabled terms."""
    H = np.zeros_like(m, dtype=np.float64)
    for h in effective_field_terms(m, mesh, p, kernel).values():
        H += h
    return H


def llg_rhs_from_field(m, H, p):
    """dm/dt = -gamma/(1+alpha^2) m x H - alpha gamma/(1+alpha^2) m x (m x H)."""
    g = p.gamma / (1.0 + p.alpha ** 2)
    mxH = np.cross(m, H, axis=0)
    return -g * mxH - p.alpha * g * np.cross(m, mxH, axis=0)


def llg_rhs(m, mesh, p, kernel=None):
    return llg_rhs_from_field(m, effective_field(m, mesh, p, kernel), p)


ENERGY_ORDER = ("exchange", "demag", "dmi", "anisotropy", "zeeman")


def energies(m, mesh, p, kernel=None):
    """Energies in J, in the order exchange, demag, dmi, anisotropy, zeeman.

    Quadratic terms: E = -(mu0/2) Ms V sum_i m_i . H_term,i; Zeeman: -mu0 Ms V sum m . H.
    Disabled terms give 0.  Every DMI symmetry class enabled adds to the dmi entry.
    """
    V = mesh.dx * mesh.dy * mesh.dz
    terms = effective_field_terms(m, mesh, p, kernel)
    E = np.zeros(5)
    for name, H in terms.items():
        n = ENERGY_ORDER.index("dmi" if name.startswith("dmi") else name)
        f = 1.0 if name == "zeeman" else 0.5
        E[n] += -f * MU0 * p.Ms * V * np.sum(m * H)
    return E


def exchange_energy_pairs(m, mesh, p):
    """E_ex = V sum_i sum_{j in N_i} A m_i . (m_i - m_j)/Delta_ij^2 written out from w_i."""
    V = mesh.dx * mesh.dy * mesh.dz
    E = 0.0
    for axis, step, dname, _ in _NEIGHBOURS:
        mj, valid = _neighbour(m, axis, step)
        delta = getattr(mesh, dname)
        E += np.sum(np.where(valid, np.sum(m * (m - mj), axis=0) / delta ** 2, 0.0))
    return V * p.A * E
