"""Cell-based material parameters: per-cell Ms, A and D, and empty cells (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).  Arrays as in `fields`:
m has shape (3, nz, ny, nx); Ms, A, D have shape (nz, ny, nx).

Paper sections followed (MicroMagnetic.jl paper):
* "Design": set_Ms accepts a function of position, and a cell whose saturation
  magnetisation is 0 lies outside the sample -- this is how shapes are made;
* "Exchange energy": with a cell-based constant A_i the pair coefficient of
  the six-neighbour form is the harmonic mean A_ij = 2 A_i A_j / (A_i + A_j),
  and H_ex,i = (2/(mu0 Ms_i)) sum_j A_ij (m_j - m_i)/Delta_ij^2;
* "Dzyaloshinskii-Moriya Energy": the unified neighbour form
  H_dmi,i = -(1/(mu0 Ms_i)) sum_j D_ij (e_ij x m_j)/Delta_ij with the harmonic
  mean D_ij = 2 D_i D_j / (D_i + D_j) of cell-based constants;
* "Magnetostatic energy": H_d,i = -sum_j N_{i-j} M_j with M_j = Ms_j m_j, and
  E = -(mu0/2) sum_i V M_i . H_i for every quadratic term.

Readings where the paper is silent:
* an empty cell (Ms_i = 0) has no field, no torque and is nobody's neighbour
  (open boundary towards it); its m is carried along unchanged;
* A_ij = 0 when A_i + A_j = 0; D_ij = 0 unless D_i D_j > 0 (no coupling across
  an interface between opposite chiralities, where the harmonic mean has a pole);
* anisotropy Ku, easy axis u, the applied field, alpha and gamma stay uniform;
  the anisotropy field is 2 Ku / (mu0 Ms_i) (m . u) u;
* energies weight each cell by its own Ms_i (the Zeeman energy -mu0 V sum Ms_i m.H).

Interlayer coupling and spin torques (sections "Interlayer Exchange
Interaction" and "Spin transfer torques"), all as terms of the effective field
(the paper folds the torques into H_eff since each starts with m x):
* interlayer: w = -J m_lo . m_hi + D_int . (m_lo x m_hi) per unit area between
  layers k_lo and k_hi, cell by cell; H = -(1/(mu0 Ms dz)) dw/dm (the paper prints
  the k_lo side; the k_hi side follows from the same w, with -D_int); only pairs
  of magnetic cells couple;
* Slonczewski / spin-orbit torque -a_J m x (m x p) - b_J m x p:
  H = (b_J p + a_J m x p) / gamma;
* Zhang-Li -(u . grad) m + beta m x (u . grad) m, with -(u . grad) m written as
  m x (m x (u . grad) m): H = -(m x v + beta v) / gamma, v = (u . grad) m by central
  differences (one-sided next to a missing or empty neighbour, zero with none);
* torques carry no energy; the interlayer exchange adds to the exchange entry
  and the interlayer DMI to the DMI entry.
"""
import numpy as np

from . import MU0
from . import fields as F


class Material:
    """Per-cell Ms (A/m), A (J/m) and D (J/m^2), arrays of shape (nz, ny, nx)."""

    def __init__(self, Ms, A, D):
        self.Ms = np.asarray(Ms, dtype=np.float64)
        self.A = np.asarray(A, dtype=np.float64)
        self.D = np.asarray(D, dtype=np.float64)
        if not (self.Ms.shape == self.A.shape == self.D.shape) or self.Ms.ndim != 3:
            raise ValueError("Ms, A and D must be (nz, ny, nx) arrays of one shape")
        if np.any(self.Ms < 0) or np.any(self.A < 0):
            raise ValueError("Ms and A must be >= 0")


def _shift(a, axis, step):
    """out[i] = a[i + step] along `axis` of an (nz, ny, nx) array, 0 beyond the mesh."""
    n = a.shape[axis]
    out = np.zeros_like(a)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if step > 0:
        src[axis], dst[axis] = slice(1, n), slice(0, n - 1)
    else:
        src[axis], dst[axis] = slice(0, n - 1), slice(1, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


def harmonic_exchange(Ai, Aj):
    """A_ij = 2 A_i A_j / (A_i + A_j), 0 where A_i + A_j = 0."""
    s = Ai + Aj
    return np.where(s > 0, 2.0 * Ai * Aj / np.where(s > 0, s, 1.0), 0.0)


def harmonic_dmi(Di, Dj):
    """D_ij = 2 D_i D_j / (D_i + D_j) where D_i D_j > 0, else 0."""
    same = Di * Dj > 0
    return np.where(same, 2.0 * Di * Dj / np.where(same, Di + Dj, 1.0), 0.0)


def _pairs(mat, axis, step):
    """Neighbour present (both cells magnetic), A_ij and D_ij towards neighbour i + step."""
    Msj = _shift(mat.Ms, axis, step)
    present = (mat.Ms > 0) & (Msj > 0)
    Aij = np.where(present, harmonic_exchange(mat.A, _shift(mat.A, axis, step)), 0.0)
    Dij = np.where(present, harmonic_dmi(mat.D, _shift(mat.D, axis, step)), 0.0)
    return present, Aij, Dij


def _inv_mu0_ms(mat):
    return np.where(mat.Ms > 0, 1.0 / (MU0 * np.where(mat.Ms > 0, mat.Ms, 1.0)), 0.0)


def exchange_field(m, mesh, mat):
    """H_ex,i = (2/(mu0 Ms_i)) sum_j A_ij (m_j - m_i)/Delta_ij^2."""
    H = np.zeros_like(m)
    for axis, step, dname, _ in F._NEIGHBOURS:
        mj = np.stack([_shift(m[c], axis, step) for c in range(3)])
        _, Aij, _ = _pairs(mat, axis, step)
        H += Aij * (mj - m) / getattr(mesh, dname) ** 2
    return 2.0 * _inv_mu0_ms(mat) * H


def dmi_field(m, mesh, mat, evecs):
    """H_dmi,i = -(1/(mu0 Ms_i)) sum_j D_ij (e_ij x m_j)/Delta_ij for the DMI vectors evecs."""
    H = np.zeros_like(m)
    for (axis, step, dname, _), e in zip(F._NEIGHBOURS, evecs):
        if tuple(e) == (0.0, 0.0, 0.0):
            continue
        mj = np.stack([_shift(m[c], axis, step) for c in range(3)])
        _, _, Dij = _pairs(mat, axis, step)
        ev = np.asarray(e, dtype=np.float64).reshape(3, 1, 1, 1)
        H += Dij * np.cross(ev, mj, axis=0) / getattr(mesh, dname)
    return -_inv_mu0_ms(mat) * H


_E_INTERFACIAL = tuple(nb[3] for nb in F._NEIGHBOURS)


def effective_field_terms(m, mesh, p, mat, kernel=None):
    """Dict term-name -> field for the terms enabled in p.terms (p.Ms, p.A, p.D unused)."""
    out = {}
    magnetic = (mat.Ms > 0)[None]
    if p.terms & F.EXCHANGE:
        out["exchange"] = exchange_field(m, mesh, mat)
    if p.terms & F.DEMAG:
        if kernel is None:
            kernel = F.DemagKernel(mesh)
        out["demag"] = np.where(magnetic, kernel.field(mat.Ms[None] * m, 1.0), 0.0)
    if p.terms & F.DMI:
        out["dmi"] = dmi_field(m, mesh, mat, _E_INTERFACIAL)
    if p.terms & F.DMI_BULK:
        out["dmi_bulk"] = dmi_field(m, mesh, mat, F._E_BULK)
    if p.terms & F.DMI_D2D:
        out["dmi_d2d"] = dmi_field(m, mesh, mat, F._E_D2D)
    if p.terms & F.ANIS:
        u = p.u.reshape(3, 1, 1, 1)
        out["anisotropy"] = 2.0 * p.Ku * _inv_mu0_ms(mat)[None] * np.sum(m * u, axis=0, keepdims=True) * u
    if p.terms & F.ZEEMAN:
        out["zeeman"] = np.where(magnetic, p.H.reshape(3, 1, 1, 1), 0.0)
    return out


def effective_field(m, mesh, p, mat, kernel=None):
    H = np.zeros_like(m, dtype=np.float64)
    for h in effective_field_terms(m, mesh, p, mat, kernel).values():
        H += h
    return H


def llg_rhs(m, mesh, p, mat, kernel=None):
    """The LL right-hand side of the cell-based field (zero in empty cells, where H = 0)."""
    return F.llg_rhs_from_field(m, effective_field(m, mesh, p, mat, kernel), p)


def energies(m, mesh, p, mat, kernel=None):
    """Energies in J ordered exchange, demag, dmi, anisotropy, zeeman:
    -(mu0/2) V sum_i Ms_i m_i . H_term,i (Zeeman -mu0 V sum Ms_i m_i . H)."""
    V = mesh.dx * mesh.dy * mesh.dz
    E = np.zeros(5)
    for name, H in effective_field_terms(m, mesh, p, mat, kernel).items():
        n = F.ENERGY_ORDER.index("dmi" if name.startswith("dmi") else name)
        f = 1.0 if name == "zeeman" else 0.5
        E[n] += -f * MU0 * V * np.sum(mat.Ms[None] * m * H)
    return E


def exchange_energy_pairs(m, mesh, mat):
    """E_ex = V sum_i sum_{j in N_i} A_ij m_i . (m_i - m_j)/Delta_ij^2 (the paper's w_i)."""
    V = mesh.dx * mesh.dy * mesh.dz
    E = 0.0
    for axis, step, dname, _ in F._NEIGHBOURS:
        mj = np.stack([_shift(m[c], axis, step) for c in range(3)])
        _, Aij, _ = _pairs(mat, axis, step)
        E += np.sum(Aij * np.sum(m * (m - mj), axis=0)) / getattr(mesh, dname) ** 2
    return V * E


# ---------------------------------------------------------------------------
# Interlayer coupling and spin torques written as effective fields
# ---------------------------------------------------------------------------
class Extra:
    """Per-instance parameters of the interlayer and spin-torque terms.

    Interlayer (section "Interlayer Exchange Interaction"): layers z = k_lo and
    z = k_hi couple cell by cell with w = -J m_lo . m_hi + D_int . (m_lo x m_hi)
    per unit area (J, D_int in J/m^2).  Slonczewski / spin-orbit torque (section
    "Spin transfer torques", eq_llg_stt2): -a_J m x (m x p) - b_J m x p (a_J, b_J
    in 1/s, p normalised).  Zhang-Li (eq_llg_stt): -(u . grad) m + beta m x (u . grad) m
    (u in m/s)."""

    def __init__(self, k_lo=0, k_hi=0, J=0.0, D_int=(0.0, 0.0, 0.0), a_J=0.0, b_J=0.0, p=(0.0, 0.0, 1.0),
                 u=(0.0, 0.0, 0.0), beta=0.0):
        self.k_lo, self.k_hi = int(k_lo), int(k_hi)
        self.J = float(J)
        self.D_int = np.asarray(D_int, dtype=np.float64)
        self.a_J, self.b_J = float(a_J), float(b_J)
        p = np.asarray(p, dtype=np.float64)
        self.p = p / np.linalg.norm(p)
        self.u = np.asarray(u, dtype=np.float64)
        self.beta = float(beta)


INTERLAYER, STT_SOT, STT_ZL = 256, 512, 1024


def interlayer_field(m, mesh, mat, ex):
    """H at layer k_lo: (J m_hi + D_int x m_hi) / (mu0 Ms dz); at layer k_hi:
    (J m_lo - D_int x m_lo) / (mu0 Ms dz) (the derivative of w with respect to each
    layer's m), where both cells of a pair are magnetic; zero elsewhere."""
    H = np.zeros_like(m)
    lo, hi = ex.k_lo, ex.k_hi
    both = (mat.Ms[lo] > 0) & (mat.Ms[hi] > 0)
    inv = _inv_mu0_ms(mat) / mesh.dz
    D = ex.D_int.reshape(3, 1, 1)
    H[:, lo] = np.where(both, inv[lo] * (ex.J * m[:, hi] + np.cross(D, m[:, hi], axis=0)), 0.0)
    H[:, hi] = np.where(both, inv[hi] * (ex.J * m[:, lo] - np.cross(D, m[:, lo], axis=0)), 0.0)
    return H


def interlayer_energy(m, mesh, mat, ex):
    """E = dx dy sum over the pairs of [-J m_lo . m_hi + D_int . (m_lo x m_hi)], magnetic pairs only."""
    lo, hi = ex.k_lo, ex.k_hi
    both = (mat.Ms[lo] > 0) & (mat.Ms[hi] > 0)
    w = -ex.J * np.sum(m[:, lo] * m[:, hi], axis=0) + np.einsum("a,a...->...", ex.D_int,
                                                                 np.cross(m[:, lo], m[:, hi], axis=0))
    return mesh.dx * mesh.dy * float(np.sum(np.where(both, w, 0.0)))


def sot_field(m, mat, ex, gamma):
    """Slonczewski / spin-orbit torque as a field: (b_J p + a_J m x p) / gamma (magnetic cells)."""
    p = ex.p.reshape(3, 1, 1, 1)
    H = (ex.b_J * np.broadcast_to(p, m.shape) + ex.a_J * np.cross(m, p, axis=0)) / gamma
    return np.where((mat.Ms > 0)[None], H, 0.0)


def directional_derivative(m, mesh, mat, u):
    """(u . grad) m by differences: central where both neighbours along an axis are
    present (inside the mesh and magnetic), one-sided where one is, zero where none is."""
    v = np.zeros_like(m)
    mag = mat.Ms > 0
    for axis, ua, dname in ((2, u[0], "dx"), (1, u[1], "dy"), (0, u[2], "dz")):
        if ua == 0.0:
            continue
        d = getattr(mesh, dname)
        mp = np.stack([_shift(m[c], axis, +1) for c in range(3)])
        mm_ = np.stack([_shift(m[c], axis, -1) for c in range(3)])
        hp = mag & (_shift(mat.Ms, axis, +1) > 0)
        hm = mag & (_shift(mat.Ms, axis, -1) > 0)
        g = np.where((hp & hm)[None], (mp - mm_) / (2 * d),
                     np.where(hp[None], (mp - m) / d, np.where(hm[None], (m - mm_) / d, 0.0)))
        v += ua * g
    return v


def zhang_li_field(m, mesh, mat, ex, gamma):
    """Zhang-Li torque as a field: -(m x v + beta v) / gamma with v = (u . grad) m."""
    v = directional_derivative(m, mesh, mat, ex.u)
    H = -(np.cross(m, v, axis=0) + ex.beta * v) / gamma
    return np.where((mat.Ms > 0)[None], H, 0.0)


def full_field(m, mesh, p, mat, ex, kernel=None):
    """The cell-based effective field plus the terms of p.terms among INTERLAYER,
    STT_SOT and STT_ZL."""
    H = effective_field(m, mesh, p, mat, kernel)
    if p.terms & INTERLAYER:
        H = H + interlayer_field(m, mesh, mat, ex)
    if p.terms & STT_SOT:
        H = H + sot_field(m, mat, ex, p.gamma)
    if p.terms & STT_ZL:
        H = H + zhang_li_field(m, mesh, mat, ex, p.gamma)
    return H


def full_llg_rhs(m, mesh, p, mat, ex, kernel=None):
    return F.llg_rhs_from_field(m, full_field(m, mesh, p, mat, ex, kernel), p)


def full_energies(m, mesh, p, mat, ex, kernel=None):
    """Energies of the conservative terms; the interlayer exchange adds to the
    exchange entry and the interlayer DMI to the DMI entry (torques carry none)."""
    E = energies(m, mesh, p, mat, kernel)
    if p.terms & INTERLAYER:
        Jonly = Extra(ex.k_lo, ex.k_hi, J=ex.J)
        Donly = Extra(ex.k_lo, ex.k_hi, D_int=ex.D_int)
        E[0] += interlayer_energy(m, mesh, mat, Jonly)
        E[2] += interlayer_energy(m, mesh, mat, Donly)
    return E
