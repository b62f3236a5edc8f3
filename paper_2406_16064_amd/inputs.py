"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds only input recipes (random unit vectors, skyrmion and
S-state textures, geodesic NEB chains, parameter-sweep draws).  It contains
none of the method's arithmetic and imports neither the HIP binding nor the
oracle.  All arrays are FP64 NumPy, SoA (3, nz, ny, nx), x fastest.

Seeds: base seed 2406 + workload index; instance or image i of a workload uses
base * 1000 + i.  Generator: NumPy PCG64.
"""
import math

import numpy as np

MU0 = 4e-7 * math.pi
BASE_SEED = 2406

# term bits (same values as the C interface)
EXCHANGE, DEMAG, DMI, ANIS, ZEEMAN = 1, 2, 4, 8, 16
ALL_TERMS = 31


def rng_for(workload, instance=None):
    seed = BASE_SEED + workload
    if instance is not None:
        seed = seed * 1000 + instance
    return np.random.Generator(np.random.PCG64(seed))


def _unit(v):
    return v / np.sqrt(np.sum(v * v, axis=0, keepdims=True))


def random_unit(nx, ny, nz, rng):
    """Per-cell unit vectors from normalised N(0,1)^3 draws."""
    return _unit(rng.standard_normal((3, nz, ny, nx)))


def add_noise(m, sigma, rng):
    return _unit(m + sigma * rng.standard_normal(m.shape))


def skyrmion_profile(px, py, cx, cy, R, w, c):
    """Neel skyrmion: theta(r) = 2 atan(exp((R-r)/w)); m = (c sin cos phi, c sin sin phi, cos)."""
    dx, dy = px - cx, py - cy
    r = np.hypot(dx, dy)
    th = 2.0 * np.arctan(np.exp((R - r) / w))
    ph = np.arctan2(dy, dx)
    return np.stack([c * np.sin(th) * np.cos(ph), c * np.sin(th) * np.sin(ph), np.cos(th)])


def skyrmion_film(nx, ny, nz, dx, dy, centres, R=10e-9, w=2e-9, c=-1.0):
    """+z film with skyrmions at the given centres (metres); each cell takes its nearest centre."""
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    px, py = np.meshgrid(x, y, indexing="xy")  # (ny, nx)
    best = np.full(px.shape, np.inf)
    m2 = np.zeros((3, ny, nx))
    m2[2] = 1.0
    for (cx, cy) in centres:
        d = np.hypot(px - cx, py - cy)
        sel = d < best
        prof = skyrmion_profile(px, py, cx, cy, R, w, c)
        m2[:, sel] = prof[:, sel]
        best = np.minimum(best, d)
    return np.repeat(m2[:, None], nz, axis=1)


def place_skyrmions(n, Lx, Ly, R, rng, max_tries=100000):
    """n centres, pairwise >= 4R apart and >= 2R from the edges (rejection sampling)."""
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("cannot place skyrmions")
        c = (rng.uniform(2 * R, Lx - 2 * R), rng.uniform(2 * R, Ly - 2 * R))
        if all(math.hypot(c[0] - o[0], c[1] - o[1]) >= 4 * R for o in out):
            out.append(c)
    return out


def s_state(nx, ny, nz, dx):
    """In-plane S-state m = (cos phi(x), sin phi(x), 0), phi(x) = -(pi/4) cos(pi x / L)."""
    L = nx * dx
    x = (np.arange(nx) + 0.5) * dx
    ph = -(math.pi / 4.0) * np.cos(math.pi * x / L)
    m = np.zeros((3, nz, ny, nx))
    m[0] = np.cos(ph)[None, None, :]
    m[1] = np.sin(ph)[None, None, :]
    return m


def slerp_chain(mA, mB, n_images):
    """Per-cell geodesic interpolation; antiparallel cells rotate about the part of e_x
    perpendicular to m_A (e_y if m_A is along x)."""
    out = []
    dot = np.clip(np.sum(mA * mB, axis=0), -1.0, 1.0)
    cross = np.cross(mA, mB, axis=0)
    cn = np.sqrt(np.sum(cross * cross, axis=0))
    om = np.arctan2(cn, dot)
    degenerate = cn < 1e-12
    ex = np.zeros_like(mA)
    ex[0] = 1.0
    ax = ex - np.sum(ex * mA, axis=0, keepdims=True) * mA
    axn = np.sqrt(np.sum(ax * ax, axis=0, keepdims=True))
    ey = np.zeros_like(mA)
    ey[1] = 1.0
    ax = np.where(axn < 1e-6, ey - np.sum(ey * mA, axis=0, keepdims=True) * mA, ax)
    ax = _unit(ax)
    for i in range(n_images):
        s = i / (n_images - 1)
        with np.errstate(divide="ignore", invalid="ignore"):
            a = np.sin((1 - s) * om) / np.sin(om)
            b = np.sin(s * om) / np.sin(om)
        m = a * mA + b * mB
        # degenerate cells: parallel -> stay; antiparallel -> rotate by s*pi about ax
        th = s * math.pi
        rot = mA * math.cos(th) + np.cross(ax, mA, axis=0) * math.sin(th)
        par = np.where(dot > 0, mA, rot)
        m = np.where(degenerate, par, m)
        out.append(_unit(m))
    return out


# ---------------------------------------------------------------------------
# Workloads (the five configurations of the benchmark description)
# ---------------------------------------------------------------------------

def workload(idx):
    """Dict describing workload idx (0..4): mesh, parameters, terms, run length, precision."""
    if idx == 0:
        return dict(name="plain-fp64-16x16x1", mesh=(16, 16, 1, 4e-9, 4e-9, 3e-9),
                    params=dict(Ms=8e5, A=1.3e-11, D=0.0, Ku=0.0, u=(0, 0, 1),
                                H=(0.0, 0.0, 1e5), alpha=0.5),
                    terms=EXCHANGE | DEMAG | ZEEMAN, rtol=1e-6, accepted_steps=200,
                    precision="f64")
    if idx == 1:
        return dict(name="thinfilm-256x256x1", mesh=(256, 256, 1, 2e-9, 2e-9, 1e-9),
                    params=dict(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=8e5, u=(0, 0, 1),
                                H=(0.0, 0.0, 2e5), alpha=0.3),
                    terms=ALL_TERMS, rtol=1e-6, t_end=5e-9, precision="f32")
    if idx == 2:
        Hmag = 25e-3 / MU0
        th = math.radians(170.0)
        return dict(name="3d-512x512x16", mesh=(512, 512, 16, 5e-9, 5e-9, 5e-9),
                    params=dict(Ms=8e5, A=1.3e-11, D=0.0, Ku=0.0, u=(0, 0, 1),
                                H=(Hmag * math.cos(th), Hmag * math.sin(th), 0.0), alpha=0.02),
                    terms=EXCHANGE | DEMAG | ZEEMAN, rtol=1e-6, t_end=1e-9, precision="f32")
    if idx == 3:
        return dict(name="neb-32x128x128x1", mesh=(128, 128, 1, 1e-9, 1e-9, 0.4e-9),
                    params=dict(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=5e5, u=(0, 0, 1),
                                H=(0.0, 0.0, 1e5), alpha=0.5),
                    terms=ALL_TERMS, n_images=32, n_iter=2000, k_spring=1e5, h=2e-14,
                    precision="f32")
    if idx == 4:
        return dict(name="sweep-256", n_instances=256, t_end=1e-9, rtol=1e-6,
                    terms=ALL_TERMS, precision="f32")
    raise ValueError(idx)


def initial_state(idx, mesh=None):
    """Seeded initial magnetisation of workload idx (0..3) on its mesh (or a given one)."""
    w = workload(idx)
    nx, ny, nz, dx, dy, dz = mesh if mesh is not None else w["mesh"]
    rng = rng_for(idx)
    if idx == 0:
        return random_unit(nx, ny, nz, rng)
    if idx == 1:
        R = 10e-9
        if nx * dx >= 256e-9 and ny * dy >= 256e-9:
            cs = place_skyrmions(8, nx * dx, ny * dy, R, rng)
        else:  # reduced test meshes: one skyrmion at the centre
            cs = [(nx * dx / 2, ny * dy / 2)]
        return add_noise(skyrmion_film(nx, ny, nz, dx, dy, cs, R=R), 1e-3, rng)
    if idx == 2:
        return add_noise(s_state(nx, ny, nz, dx), 1e-2, rng)
    if idx == 3:
        return neb_chain(mesh)
    raise ValueError(idx)


def neb_chain(mesh=None):
    w = workload(3)
    nx, ny, nz, dx, dy, dz = mesh if mesh is not None else w["mesh"]
    mA = skyrmion_film(nx, ny, nz, dx, dy, [(nx * dx / 2, ny * dy / 2)], R=10e-9)
    mB = np.zeros_like(mA)
    mB[2] = 1.0
    return slerp_chain(mA, mB, w["n_images"])


# ---------------------------------------------------------------------------
# The paper's throughput setting: N x N x 1 films with demagnetisation,
# exchange and Zeeman terms, integrated with Heun (fixed step).  The paper
# gives neither material nor cell size; permalloy-like values on 2 nm cubic
# cells (below the exchange length) and a seeded random start stand in.
# ---------------------------------------------------------------------------

HEUN_SIZES = (256, 512, 1024)


def heun_film(n):
    """Workload of the throughput setting for an n x n x 1 film."""
    return dict(name="heun-%dx%dx1" % (n, n), mesh=(n, n, 1, 2e-9, 2e-9, 2e-9),
                params=dict(Ms=8e5, A=1.3e-11, D=0.0, Ku=0.0, u=(0, 0, 1),
                            H=(0.0, 0.0, 1e5), alpha=0.5),
                terms=EXCHANGE | DEMAG | ZEEMAN, h=5e-14, precision="f32")


def heun_initial(n, mesh=None):
    """Seeded random unit start of the n x n x 1 throughput film (or of a given mesh)."""
    nx, ny, nz = (mesh or heun_film(n)["mesh"])[:3]
    return random_unit(nx, ny, nz, rng_for(5, n))


def sp4():
    """Standard Problem 4 as the paper states it (section "Standard Problem 4"): a
    500 x 125 x 3 nm Permalloy film relaxed from the uniform m0 = (1, 0.25, 0.1),
    then driven by mu0 H = (-24.6, 4.3, 0) mT.  Cells 2.5 x 2.5 x 3 nm (200 x 50 x 1);
    Ms, A and the damping of the dynamics (0.02) are the problem's usual Permalloy
    values, which the paper does not print; exchange + demag (+ Zeeman in the
    dynamics)."""
    mesh = (200, 50, 1, 2.5e-9, 2.5e-9, 3e-9)
    H = (-24.6e-3 / MU0, 4.3e-3 / MU0, 0.0)
    return dict(name="sp4-200x50x1", mesh=mesh,
                relax=dict(Ms=8e5, A=1.3e-11, D=0.0, Ku=0.0, u=(0, 0, 1), H=(0.0, 0.0, 0.0), alpha=0.5),
                dynamics=dict(Ms=8e5, A=1.3e-11, D=0.0, Ku=0.0, u=(0, 0, 1), H=H, alpha=0.02),
                relax_terms=EXCHANGE | DEMAG, terms=EXCHANGE | DEMAG | ZEEMAN, t_end=1e-9, rtol=1e-6)


def sp4_initial():
    """The uniform start m0 = (1, 0.25, 0.1) / |.| of every cell."""
    nx, ny, nz = sp4()["mesh"][:3]
    m = np.zeros((3, nz, ny, nx))
    m[0], m[1], m[2] = 1.0, 0.25, 0.1
    return _unit(m)


SWEEP_SIZES = (32, 64, 96, 128, 192, 256)


def sweep_instance(i):
    """Instance i of the parameter sweep: mesh, parameters and seeded random m."""
    rng = rng_for(4, i)
    n = int(rng.choice(SWEEP_SIZES))
    nz = int(rng.integers(1, 3))
    Ms = rng.uniform(4e5, 1.2e6)
    A = rng.uniform(5e-12, 2e-11)
    D = rng.uniform(0.0, 4e-3)
    Ku = rng.uniform(0.0, 1e6)
    Hm = rng.uniform(0.0, 3e5)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    alpha = rng.uniform(0.01, 0.5)
    mesh = (n, n, nz, 2e-9, 2e-9, 2e-9)
    m = random_unit(n, n, nz, rng)
    return dict(mesh=mesh, params=dict(Ms=Ms, A=A, D=D, Ku=Ku, u=(0, 0, 1), H=tuple(Hm * d),
                                       alpha=alpha), m=m)


def disk_material(nx, ny, nz, dx, dy, rng, Ms=(8e5, 5.8e5), A=(1.3e-11, 1.5e-11), D=(0.0, 3e-3),
                  spread=0.05, radius_frac=0.45):
    """Cell-based material of a two-grain disk: cells farther than radius_frac * min(Lx, Ly)
    from the film's centre are empty (Ms = 0, a shape made by the magnetisation as with a
    function-valued set_Ms); inside, the left half is grain 0 and the right half grain 1,
    each value scaled per cell by 1 + spread * U(-1, 1).  Returns (Ms, A, D), each
    (nz, ny, nx) FP64."""
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    px, py = np.meshgrid(x, y, indexing="xy")
    cx, cy = 0.5 * nx * dx, 0.5 * ny * dy
    inside = np.hypot(px - cx, py - cy) <= radius_frac * min(nx * dx, ny * dy)
    right = px >= cx
    out = []
    for pair in (Ms, A, D):
        v = np.where(right, pair[1], pair[0])[None].repeat(nz, axis=0)
        v = v * (1.0 + spread * rng.uniform(-1.0, 1.0, size=v.shape))
        out.append(v)
    out[0] = np.where(inside[None], out[0], 0.0)
    return tuple(out)
