"""Cell-averaged demagnetisation tensor in FP64 (oracle; test infrastructure only).

The paper writes the demag field as a discrete convolution H_d,i = -sum_j N_{i-j} M_j
with a 3x3 symmetric tensor that depends only on the displacement between cells
(section "Magnetostatic energy", equations eq_demag_energy2 and eq_hd1), and cites
Newell, Williams and Dunlop (1993) for it without printing the formulas.

The tensor is defined as the average over target cell i of the field produced
by a uniformly magnetised source cell j:

    N(R) = -(1/V) int_{cell i} int_{cell j} D(r - r') dr dr',
    D(r) = (3 r r^T - |r|^2 I) / (4 pi |r|^5),

and, with u the difference of the two in-cell offsets (whose density is the
product of tent functions), equivalently

    N(R) = - int_{[-d,d]^3} D(R + u) prod_a (1 - |u_a|/d_a) du.

Two evaluations of this one definition are used (a reading of a point on which
the paper is silent; plain FP64 closed forms cancel catastrophically at large
distance):

* rho = |R| / max(d) < 3: Newell's closed forms f and g, differenced with the
  27-point (2,-1,-1)^3 stencil;
* rho >= 3: Gauss-Legendre quadrature of the integral above, each interval
  [-d_a, 0] and [0, d_a] taking n nodes (n = 10, 6, 4, 3, 2 for rho in [3,6),
  [6,16), [16,40), [40,300), [300, inf)).  For rho >= 3 the integrand is
  smooth on each sub-box, and this schedule is within ~1e-14 of a 60-digit
  evaluation of the closed form, while the FP64 closed form itself loses up to
  ~1e-10 relative by rho ~ 5 on flat cells.

Both are pinned in tests/test_oracle_newell.py against 60-digit mpmath
evaluations of the closed form, the trace identities, the cube value 1/3, the
parity of each component and the point-dipole far field.
"""
import numpy as np

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


def newell_f(x, y, z):
    """Newell's f(x,y,z) (even in each argument); zero-prefactor terms are 0."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    y = np.abs(np.asarray(y, dtype=np.float64))
    z = np.abs(np.asarray(z, dtype=np.float64))
    x, y, z = np.broadcast_arrays(x, y, z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    with np.errstate(divide="ignore", invalid="ignore"):
        m = (y > 0) & (x2 + z2 > 0)
        out = out + np.where(m, 0.5 * y * (z2 - x2) * np.arcsinh(y / np.sqrt(x2 + z2)), 0.0)
        m = (z > 0) & (x2 + y2 > 0)
        out = out + np.where(m, 0.5 * z * (y2 - x2) * np.arcsinh(z / np.sqrt(x2 + y2)), 0.0)
        m = (x > 0) & (y > 0) & (z > 0)
        out = out - np.where(m, x * y * z * np.arctan(y * z / (x * R)), 0.0)
    return out


def newell_g(x, y, z):
    """Newell's g(x,y,z): odd in x and in y, even in z; zero-prefactor terms are 0."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    x, y, z = np.broadcast_arrays(x, y, z)
    sgn = np.sign(x) * np.sign(y)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3.0
    with np.errstate(divide="ignore", invalid="ignore"):
        m = (z > 0) & (x2 + y2 > 0)
        out = out + np.where(m, x * y * z * np.arcsinh(z / np.sqrt(x2 + y2)), 0.0)
        m = (y2 + z2 > 0)
        out = out + np.where(m, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(x / np.sqrt(y2 + z2)), 0.0)
        m = (x2 + z2 > 0)
        out = out + np.where(m, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(y / np.sqrt(x2 + z2)), 0.0)
        m = (z > 0) & (R > 0)
        out = out - np.where(m, z2 * z / 6.0 * np.arctan(x * y / (z * R)), 0.0)
        m = (y > 0) & (z > 0)
        out = out - np.where(m, 0.5 * z * y2 * np.arctan(x * z / (y * R)), 0.0)
        m = (x > 0) & (z > 0)
        out = out - np.where(m, 0.5 * z * x2 * np.arctan(y * z / (x * R)), 0.0)
    return sgn * out


_W = {-1: -1.0, 0: 2.0, 1: -1.0}


def _stencil(fun, p, q, r, dp, dq, dr):
    """sum over a,b,c in {-1,0,1} of w_a w_b w_c fun(p + a dp, q + b dq, r + c dr)."""
    s = 0.0
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                s = s + _W[a] * _W[b] * _W[c] * fun(p + a * dp, q + b * dq, r + c * dr)
    return s


def tensor_closed_form(X, Y, Z, dx, dy, dz):
    """Newell tensor at physical displacements (X,Y,Z) from the closed forms.

    Returns an array [..., 6] ordered xx, yy, zz, xy, xz, yz.
    """
    X, Y, Z = np.broadcast_arrays(np.asarray(X, float), np.asarray(Y, float), np.asarray(Z, float))
    c = 1.0 / (4.0 * np.pi * dx * dy * dz)
    out = np.empty(X.shape + (6,))
    out[..., 0] = c * _stencil(newell_f, X, Y, Z, dx, dy, dz)
    out[..., 1] = c * _stencil(newell_f, Y, X, Z, dy, dx, dz)
    out[..., 2] = c * _stencil(newell_f, Z, Y, X, dz, dy, dx)
    out[..., 3] = c * _stencil(newell_g, X, Y, Z, dx, dy, dz)
    out[..., 4] = c * _stencil(newell_g, X, Z, Y, dx, dz, dy)
    out[..., 5] = c * _stencil(newell_g, Y, Z, X, dy, dz, dx)
    return out


def _tent_gauss(n):
    """Nodes s in [-1,1] and weights for int_{-1}^{1} phi(s) (1 - |s|) ds, n nodes per half."""
    t, w = np.polynomial.legendre.leggauss(n)
    s_half = 0.5 * (1.0 + t)            # nodes on [0, 1]
    w_half = 0.5 * w * (1.0 - s_half)   # Gauss weight * tent factor
    return np.concatenate([-s_half, s_half]), np.concatenate([w_half, w_half])


def tensor_quadrature(X, Y, Z, dx, dy, dz, n):
    """Newell tensor from Gauss-Legendre quadrature of its defining integral.

    Valid when the integrand is smooth on [-d,d]^3 around R (far field).
    Returns [..., 6] in the order xx, yy, zz, xy, xz, yz.
    """
    X = np.asarray(X, float).ravel()
    Y = np.asarray(Y, float).ravel()
    Z = np.asarray(Z, float).ravel()
    s, w = _tent_gauss(n)
    ux, uy, uz = np.meshgrid(s * dx, s * dy, s * dz, indexing="ij")
    wx, wy, wz = np.meshgrid(w * dx, w * dy, w * dz, indexing="ij")
    ux, uy, uz = ux.ravel(), uy.ravel(), uz.ravel()
    ww = (wx * wy * wz).ravel()
    out = np.empty((X.size, 6))
    chunk = max(1, 4_000_000 // ww.size)
    for lo in range(0, X.size, chunk):
        hi = min(X.size, lo + chunk)
        rx = X[lo:hi, None] + ux[None, :]
        ry = Y[lo:hi, None] + uy[None, :]
        rz = Z[lo:hi, None] + uz[None, :]
        r2 = rx * rx + ry * ry + rz * rz
        k = ww[None, :] / (4.0 * np.pi * r2 * r2 * np.sqrt(r2))
        out[lo:hi, 0] = -np.sum(k * (3.0 * rx * rx - r2), axis=1)
        out[lo:hi, 1] = -np.sum(k * (3.0 * ry * ry - r2), axis=1)
        out[lo:hi, 2] = -np.sum(k * (3.0 * rz * rz - r2), axis=1)
        out[lo:hi, 3] = -np.sum(k * (3.0 * rx * ry), axis=1)
        out[lo:hi, 4] = -np.sum(k * (3.0 * rx * rz), axis=1)
        out[lo:hi, 5] = -np.sum(k * (3.0 * ry * rz), axis=1)
    return out


# (rho lower bound, Gauss nodes per half interval)
QUAD_SCHEDULE = ((300.0, 2), (40.0, 3), (16.0, 4), (6.0, 6), (3.0, 10))
NEAR_RHO = 3.0


def tensor(I, J, K, dx, dy, dz):
    """Newell tensor at integer cell displacements (I, J, K): [..., 6].

    Closed form for rho < 3, quadrature beyond (schedule in QUAD_SCHEDULE).
    """
    I, J, K = np.broadcast_arrays(np.asarray(I), np.asarray(J), np.asarray(K))
    shape = I.shape
    X = (I * dx).astype(float).ravel()
    Y = (J * dy).astype(float).ravel()
    Z = (K * dz).astype(float).ravel()
    rho = np.sqrt(X * X + Y * Y + Z * Z) / max(dx, dy, dz)
    out = np.empty((X.size, 6))
    near = rho < NEAR_RHO
    if near.any():
        out[near] = tensor_closed_form(X[near], Y[near], Z[near], dx, dy, dz)
    upper = np.inf
    for lower, n in QUAD_SCHEDULE:
        sel = (rho >= lower) & (rho < upper)
        if sel.any():
            out[sel] = tensor_quadrature(X[sel], Y[sel], Z[sel], dx, dy, dz, n)
        upper = lower
    return out.reshape(shape + (6,))


def _grid_rows(nx, nz, j0, j1, dx, dy, dz):
    """Rows J in [j0, j1) of the displacement grid, every I and K: [2nz-1, j1-j0, 2nx-1, 6]."""
    K, J, I = np.meshgrid(np.arange(-nz + 1, nz), np.arange(j0, j1),
                          np.arange(-nx + 1, nx), indexing="ij")
    return tensor(I, J, K, dx, dy, dz)


def _grid_rows_star(a):
    return _grid_rows(*a)


def tensor_grid(nx, ny, nz, dx, dy, dz, workers=1):
    """Tensor for every displacement (I,J,K), |I|<nx, |J|<ny, |K|<nz.

    Returns an array [2nz-1, 2ny-1, 2nx-1, 6]; index [K+nz-1, J+ny-1, I+nx-1].
    workers > 1 evaluates bands of J rows in that many processes (every entry is
    computed on its own, so the result is the same bit for bit).
    """
    if workers <= 1 or ny < 2:
        return _grid_rows(nx, nz, -ny + 1, ny, dx, dy, dz)
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    edges = np.linspace(-ny + 1, ny, min(2 * ny - 1, 4 * workers) + 1).round().astype(int)
    parts = [(nx, nz, int(a), int(b), dx, dy, dz) for a, b in zip(edges[:-1], edges[1:]) if b > a]
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        return np.concatenate(list(ex.map(_grid_rows_star, parts)), axis=1)


def as_matrix(t6):
    """[..., 6] -> symmetric [..., 3, 3]."""
    t6 = np.asarray(t6)
    M = np.empty(t6.shape[:-1] + (3, 3))
    M[..., 0, 0], M[..., 1, 1], M[..., 2, 2] = t6[..., 0], t6[..., 1], t6[..., 2]
    M[..., 0, 1] = M[..., 1, 0] = t6[..., 3]
    M[..., 0, 2] = M[..., 2, 0] = t6[..., 4]
    M[..., 1, 2] = M[..., 2, 1] = t6[..., 5]
    return M
