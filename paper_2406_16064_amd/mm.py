"""Thin ctypes binding of the C interface in include/mm.h (argument marshalling only).

Every computation runs in the HIP library libmmx.so; this module only converts
Python values and torch tensors to the C structures and device pointers.
Importing it raises if the library has not been built: there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmx.so")

MM_OK, MM_E_ARG, MM_E_NOMEM, MM_E_HIP = 0, -1, -2, -3
MM_E_NONFINITE, MM_E_STEP_UNDERFLOW, MM_E_MAXSTEPS, MM_E_STATE = -4, -5, -6, -7
MM_F32, MM_F64 = 0, 1
# launch shapes: x-forward rows and threads, y columns, threads per column and threads, x-inverse rows and threads
SHAPE_KEYS = ("ty_f", "nt_f", "cb_y", "tpc_y", "nt_y", "ty_x", "nt_i")
EXCHANGE, DEMAG, DMI, ANIS, ZEEMAN = 1, 2, 4, 8, 16
ALL_TERMS = 31
DMI_BULK, DMI_D2D = 32, 64  # the other DMI symmetry classes (same D)
CELLS = 128  # cell-based Ms, A, D of the instance (Plan.set_cells)
INTERLAYER, STT_SOT, STT_ZL = 256, 512, 1024  # interlayer coupling, spin-orbit / Slonczewski and Zhang-Li torques
DEMAG_POTENTIAL = 2048  # demag through the magnetic scalar potential (in place of DEMAG)

if not os.path.exists(LIB_PATH):
    raise ImportError("libmmx.so is not built; run `python -m paper_2406_16064_amd.build` "
                      "(the HIP library is required, there is no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)


class Mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("Ms", ctypes.c_double), ("A", ctypes.c_double), ("D", ctypes.c_double),
                ("Ku", ctypes.c_double), ("u", ctypes.c_double * 3), ("H", ctypes.c_double * 3),
                ("alpha", ctypes.c_double), ("gamma", ctypes.c_double), ("terms", ctypes.c_uint32),
                ("k_lo", ctypes.c_int32), ("k_hi", ctypes.c_int32), ("J_rkky", ctypes.c_double),
                ("D_int", ctypes.c_double * 3), ("a_J", ctypes.c_double), ("b_J", ctypes.c_double),
                ("p", ctypes.c_double * 3), ("u_zl", ctypes.c_double * 3), ("beta", ctypes.c_double)]


class RK45State(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h", ctypes.c_double), ("rtol", ctypes.c_double),
                ("h_min", ctypes.c_double), ("h_max", ctypes.c_double),
                ("n_accept", ctypes.c_int64), ("n_reject", ctypes.c_int64), ("n_rhs", ctypes.c_int64),
                ("last_err", ctypes.c_double), ("last_accepted", ctypes.c_int32),
                ("fsal_valid", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("mesh_id", ctypes.c_int32), ("p", Params), ("m", ctypes.c_void_p), ("st", RK45State),
                ("t_end", ctypes.c_double), ("status", ctypes.c_int32)]


_vp, _i32, _i64, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_P = ctypes.POINTER
_sigs = {
    "mm_plan_create": [_P(_vp), _P(Mesh), ctypes.c_int, ctypes.c_uint32, _i32, _vp],
    "mm_plan_destroy": [_vp],
    "mm_plan_padded": [_vp, _P(_i32), _P(_i32), _P(_i32)],
    "mm_plan_set_cells": [_vp, _i32, _P(_dbl), _P(_dbl), _P(_dbl), _vp],
    "mm_demag_tensor": [_P(Mesh), _vp, _i64, _vp, _vp],
    "mm_scalar_potential_kernel": [_P(Mesh), _vp, _i64, _vp, _vp],
    "mm_effective_field": [_vp, _P(Params), _i32, _vp, _vp, _vp],
    "mm_llg_rhs": [_vp, _P(Params), _i32, _vp, _vp, _vp],
    "mm_energy": [_vp, _P(Params), _i32, _vp, _P(_dbl), _vp],
    "mm_rk45_step": [_vp, _P(Params), _i32, _vp, _P(RK45State), _vp],
    "mm_rk45_run": [_vp, _P(Params), _i32, _vp, _P(RK45State), _dbl, _i64, _P(_dbl), _i64, _vp],
    "mm_neb_run": [_vp, _P(Params), _vp, _i32, _dbl, _dbl, _i64, _P(_dbl), _vp],
    "mm_heun_run": [_vp, _P(Params), _i32, _vp, _dbl, _i64, _vp],
    "mm_sd_run": [_vp, _P(Params), _i32, _vp, _i64, _dbl, _dbl, _dbl, _P(_dbl), _vp],
    "mm_sd_run_noalloc": [_vp, _P(Params), _i32, _vp, _i64, _dbl, _dbl, _dbl, _P(_dbl), _vp],
    "mm_sd_relax": [_vp, _P(Params), _i32, _vp, _dbl, _i64, _dbl, _dbl, _dbl, _P(_i64), _P(_dbl), _P(_dbl), _vp],
    "mm_rk45_relax": [_vp, _P(Params), _i32, _vp, _P(RK45State), _dbl, _i64, _P(_dbl), _vp],
    "mm_profile_passes": [_vp, _P(Params), _i32, _vp, _vp, _i32, _P(_dbl), _P(_i32), _P(_dbl), _vp],
    "mm_profile_step": [_vp, _P(Params), _i32, _vp, _P(RK45State), _i32, _P(_dbl), _P(_i32), _P(_i32), _P(_dbl),
                        _vp],
    "mm_plan_autotune": [_vp, _P(Params), _i32, _vp, _vp, _i32, _P(_i32), _vp],
    "mm_plan_tune_padding": [_vp, _P(Params), _i32, _vp, _vp, _i32, _P(_i32), _vp],
    "mm_plan_shapes": [_vp, _P(_i32)],
    "mm_plan_set_shapes": [_vp, _P(_i32)],
    "mm_batch_create": [_P(_vp), _P(Mesh), _i32, ctypes.c_int, ctypes.c_uint32, _vp],
    "mm_batch_run": [_vp, _P(Instance), _i32, _i64, _vp],
    "mm_batch_destroy": [_vp],
}
for _n, _a in _sigs.items():
    _f = getattr(_lib, _n)
    _f.argtypes = _a
    _f.restype = ctypes.c_int
_lib.mm_status_string.argtypes = [ctypes.c_int]
_lib.mm_status_string.restype = ctypes.c_char_p
_lib.mm_last_error.argtypes = []
_lib.mm_last_error.restype = ctypes.c_char_p

EXPORTED = tuple(_sigs) + ("mm_status_string", "mm_last_error")


class MMError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.mm_last_error().decode()
        super().__init__("%s: %s (%d): %s" % (where, _lib.mm_status_string(status).decode(), status, msg))


def _check(st, where):
    if st != MM_OK:
        raise MMError(st, where)


def status_string(st):
    return _lib.mm_status_string(st).decode()


def make_params(Ms, A=0.0, D=0.0, Ku=0.0, u=(0.0, 0.0, 1.0), H=(0.0, 0.0, 0.0), alpha=0.5,
                gamma=2.21e5, terms=ALL_TERMS, k_lo=0, k_hi=0, J_rkky=0.0, D_int=(0.0, 0.0, 0.0), a_J=0.0,
                b_J=0.0, p=(0.0, 0.0, 1.0), u_zl=(0.0, 0.0, 0.0), beta=0.0):
    """mm_params of one instance (SI units; see include/mm.h for every field)."""
    q = Params()
    q.Ms, q.A, q.D, q.Ku = Ms, A, D, Ku
    for k in range(3):
        q.u[k] = u[k]
        q.H[k] = H[k]
        q.D_int[k] = D_int[k]
        q.p[k] = p[k]
        q.u_zl[k] = u_zl[k]
    q.alpha, q.gamma, q.terms = alpha, gamma, terms
    q.k_lo, q.k_hi, q.J_rkky = k_lo, k_hi, J_rkky
    q.a_J, q.b_J, q.beta = a_J, b_J, beta
    return q


def _params_array(params):
    if isinstance(params, Params):
        params = [params]
    arr = (Params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p if isinstance(p, Params) else make_params(**p)
    return arr


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def new_states(n, t=0.0, h=1e-13, rtol=1e-6, h_min=1e-20, h_max=1e-10):
    arr = (RK45State * n)()
    for s in arr:
        s.t, s.h, s.rtol, s.h_min, s.h_max = t, h, rtol, h_min, h_max
    return arr


class Plan:
    """A plan for up to max_batch instances sharing one mesh (mm_plan_create)."""

    def __init__(self, mesh, precision="f32", terms=ALL_TERMS, max_batch=1, stream=None):
        self.mesh = Mesh(*mesh)
        self.prec = MM_F32 if precision in ("f32", MM_F32) else MM_F64
        self.terms = terms
        self.max_batch = max_batch
        self._h = ctypes.c_void_p()
        _check(_lib.mm_plan_create(ctypes.byref(self._h), ctypes.byref(self.mesh), self.prec,
                                   terms, max_batch, _stream(stream)), "mm_plan_create")

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.prec == MM_F32 else torch.float64

    def padded(self):
        a, b, c = _i32(), _i32(), _i32()
        _check(_lib.mm_plan_padded(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "mm_plan_padded")
        return a.value, b.value, c.value

    def _batch(self, m):
        return 1 if m.dim() == 4 else m.shape[0]

    def set_cells(self, instance, Ms, A, D, stream=None):
        """Cell-based Ms, A, D (arrays of nz x ny x nx, FP64 on the host) of instance slot `instance`."""
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (Ms, A, D)]
        n = self.mesh.nx * self.mesh.ny * self.mesh.nz
        for a in arrs:
            if a.size != n:
                raise ValueError("cell arrays must hold nx * ny * nz values")
        ptrs = [a.ctypes.data_as(_P(_dbl)) for a in arrs]
        _check(_lib.mm_plan_set_cells(self._h, instance, ptrs[0], ptrs[1], ptrs[2], _stream(stream)),
               "mm_plan_set_cells")

    def effective_field(self, params, m, out=None, stream=None):
        import torch
        out = torch.empty_like(m) if out is None else out
        pa = _params_array(params)
        _check(_lib.mm_effective_field(self._h, pa, self._batch(m), _ptr(m), _ptr(out), _stream(stream)),
               "mm_effective_field")
        return out

    def llg_rhs(self, params, m, out=None, stream=None):
        import torch
        out = torch.empty_like(m) if out is None else out
        pa = _params_array(params)
        _check(_lib.mm_llg_rhs(self._h, pa, self._batch(m), _ptr(m), _ptr(out), _stream(stream)),
               "mm_llg_rhs")
        return out

    def energy(self, params, m, stream=None):
        b = self._batch(m)
        E = (ctypes.c_double * (5 * b))()
        pa = _params_array(params)
        _check(_lib.mm_energy(self._h, pa, b, _ptr(m), E, _stream(stream)), "mm_energy")
        return np.array(E[:]).reshape(b, 5)

    def rk45_step(self, params, m, states, stream=None):
        pa = _params_array(params)
        st = _lib.mm_rk45_step(self._h, pa, self._batch(m), _ptr(m), states, _stream(stream))
        _check(st, "mm_rk45_step")
        return states

    def rk45_run(self, params, m, states, t_end=math.inf, max_steps=10 ** 9, replay_h=None,
                 stream=None, check=True):
        pa = _params_array(params)
        if replay_h is not None:
            rh = (ctypes.c_double * len(replay_h))(*replay_h)
            n = len(replay_h)
        else:
            rh, n = None, 0
        st = _lib.mm_rk45_run(self._h, pa, self._batch(m), _ptr(m), states, t_end, max_steps, rh, n,
                              _stream(stream))
        if check:
            _check(st, "mm_rk45_run")
        return st

    def heun_run(self, params, m, h, n_steps, stream=None):
        """n_steps fixed Heun steps of size h with projection, m advanced in place."""
        _check(_lib.mm_heun_run(self._h, _params_array(params), self._batch(m), _ptr(m), h, n_steps,
                                _stream(stream)), "mm_heun_run")

    def sd_run(self, params, m, n_iter, tau0, tau_min, tau_max, stream=None):
        """n_iter steepest-descent (Barzilai-Borwein) iterations, m in place; returns the last tau per instance."""
        nb = self._batch(m)
        tau = (ctypes.c_double * nb)()
        _check(_lib.mm_sd_run(self._h, _params_array(params), nb, _ptr(m), n_iter, tau0, tau_min, tau_max, tau,
                              _stream(stream)), "mm_sd_run")
        return np.array(tau[:])

    def sd_run_noalloc(self, params, m, n_iter, tau0, tau_min, tau_max, stream=None, check=True):
        """sd_run without device allocation (mm_sd_run_noalloc: the library's fixed scratch).
        Returns (status, last tau per instance)."""
        nb = self._batch(m)
        tau = (ctypes.c_double * nb)()
        st = _lib.mm_sd_run_noalloc(self._h, _params_array(params), nb, _ptr(m), n_iter, tau0, tau_min, tau_max,
                                    tau, _stream(stream))
        if check:
            _check(st, "mm_sd_run_noalloc")
        return st, np.array(tau[:])

    def sd_relax(self, params, m, stopping_dmdt, max_iter, tau0, tau_min, tau_max, stream=None, check=True):
        """Steepest descent until the largest |dm/dt| (deg/ns) is below stopping_dmdt (mm_sd_relax).
        Returns (status, iterations, last measures in deg/ns, last taus) per instance arrays."""
        nb = self._batch(m)
        it = (ctypes.c_int64 * nb)()
        dm = (ctypes.c_double * nb)()
        tau = (ctypes.c_double * nb)()
        st = _lib.mm_sd_relax(self._h, _params_array(params), nb, _ptr(m), stopping_dmdt, max_iter, tau0, tau_min,
                              tau_max, it, dm, tau, _stream(stream))
        if check:
            _check(st, "mm_sd_relax")
        return st, np.array(it[:]), np.array(dm[:]), np.array(tau[:])

    def rk45_relax(self, params, m, states, stopping_dmdt, max_steps=10 ** 9, stream=None, check=True):
        """Adaptive Dormand-Prince until the largest |dm/dt| (deg/ns) after an accepted step is below
        stopping_dmdt (mm_rk45_relax).  Returns (status, last measures in deg/ns)."""
        nb = self._batch(m)
        dm = (ctypes.c_double * nb)()
        st = _lib.mm_rk45_relax(self._h, _params_array(params), nb, _ptr(m), states, stopping_dmdt, max_steps, dm,
                                _stream(stream))
        if check:
            _check(st, "mm_rk45_relax")
        return st, np.array(dm[:])

    def neb_run(self, params, images, k_spring, h, n_iter, stream=None):
        n_img = images.shape[0]
        E = (ctypes.c_double * n_img)()
        _check(_lib.mm_neb_run(self._h, _params_array(params), _ptr(images), n_img, k_spring, h, n_iter,
                               E, _stream(stream)), "mm_neb_run")
        return np.array(E[:])

    def autotune(self, params, m, reps=10, stream=None):
        """Pick the fastest launch shape of every pass on the device; returns the shapes."""
        import torch
        work = torch.empty_like(m)
        shape = (ctypes.c_int32 * 8)()
        _check(_lib.mm_plan_autotune(self._h, _params_array(params), self._batch(m), _ptr(m), _ptr(work), reps,
                                     shape, _stream(stream)), "mm_plan_autotune")
        return dict(zip(SHAPE_KEYS, shape[:7]))

    def tune_padding(self, params, m, reps=5, stream=None):
        """Pick the padded FFT grid by timing dm/dt on the candidates (mm_plan_tune_padding);
        returns (Px, Py, Pz).  Launch shapes go back to their defaults."""
        import torch
        work = torch.empty_like(m)
        out = (ctypes.c_int32 * 3)()
        _check(_lib.mm_plan_tune_padding(self._h, _params_array(params), self._batch(m), _ptr(m), _ptr(work), reps,
                                         out, _stream(stream)), "mm_plan_tune_padding")
        return tuple(out[:])

    def shapes(self):
        """The plan's current launch shapes (as autotune reports them)."""
        shape = (ctypes.c_int32 * 8)()
        _check(_lib.mm_plan_shapes(self._h, shape), "mm_plan_shapes")
        return dict(zip(SHAPE_KEYS, shape[:7]))

    def set_shapes(self, shapes):
        """Set the launch shapes (a dict as shapes() returns; unnamed keys keep their value)."""
        cur = self.shapes()
        cur.update(shapes)
        shape = (ctypes.c_int32 * 8)(*[int(cur[k]) for k in SHAPE_KEYS], 0)
        _check(_lib.mm_plan_set_shapes(self._h, shape), "mm_plan_set_shapes")

    def profile_passes(self, params, m, reps=20, stream=None, in_order=False):
        """Mean duration (us) of each kernel pass of one dm/dt evaluation, each pass launched
        back to back; with in_order also the passes of whole evaluations timed in their own
        order (returns (back_to_back, in_order))."""
        import torch
        work = torch.empty_like(m)
        us = (ctypes.c_double * 8)()
        seq = (ctypes.c_double * 8)()
        n = _i32()
        _check(_lib.mm_profile_passes(self._h, _params_array(params), self._batch(m), _ptr(m), _ptr(work),
                                      reps, us, ctypes.byref(n), seq, _stream(stream)), "mm_profile_passes")
        if in_order:
            return list(us[:n.value]), list(seq[:n.value])
        return list(us[:n.value])

    def profile_step(self, params, m, states, reps=20, stream=None, in_order=False):
        """Mean duration (us) of each kernel of one adaptive attempt, launched back to back:
        returns (begin_us, [stage pass us...], error_x_inverse_us, fused); with in_order also
        the same figures from whole attempts timed in their own order (a fifth item, a tuple
        of the first three)."""
        us = (ctypes.c_double * 8)()
        seq = (ctypes.c_double * 8)()
        n = _i32()
        fused = _i32()
        _check(_lib.mm_profile_step(self._h, _params_array(params), self._batch(m), _ptr(m), states, reps, us,
                                    ctypes.byref(n), ctypes.byref(fused), seq, _stream(stream)), "mm_profile_step")
        v = list(us[:n.value])
        out = (v[0], v[1:-1], v[-1], bool(fused.value))
        if in_order:
            w = list(seq[:n.value])
            out = out + ((w[0], w[1:-1], w[-1]),)
        return out

    def close(self):
        if self._h:
            _lib.mm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Instances of up to 16 different meshes advanced together (mm_batch_*)."""

    def __init__(self, meshes, precision="f32", terms=ALL_TERMS, stream=None):
        self.meshes = [tuple(msh) for msh in meshes]
        arr = (Mesh * len(meshes))(*[Mesh(*msh) for msh in meshes])
        self.prec = MM_F32 if precision in ("f32", MM_F32) else MM_F64
        self._h = ctypes.c_void_p()
        _check(_lib.mm_batch_create(ctypes.byref(self._h), arr, len(meshes), self.prec, terms, _stream(stream)),
               "mm_batch_create")

    def run(self, instances, max_steps=10 ** 9, stream=None, check=True):
        """instances: list of dicts with mesh_id, params (Params), m (device tensor), t_end
        and optional state (RK45State).  Returns (status, list of (state, status))."""
        arr = (Instance * len(instances))()
        for i, d in enumerate(instances):
            arr[i].mesh_id = d["mesh_id"]
            arr[i].p = d["params"]
            arr[i].m = _ptr(d["m"])
            arr[i].st = d.get("state") or new_states(1, rtol=d.get("rtol", 1e-6))[0]
            arr[i].t_end = d["t_end"]
        st = _lib.mm_batch_run(self._h, arr, len(instances), max_steps, _stream(stream))
        if check:
            _check(st, "mm_batch_run")
        return st, [(arr[i].st, arr[i].status) for i in range(len(instances))]

    def close(self):
        if self._h:
            _lib.mm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def demag_tensor(mesh, disp, stream=None):
    """Newell tensor at integer displacements disp (array [n,3]) -> numpy [n,6] (FP64, device-computed)."""
    import torch
    d = torch.as_tensor(np.ascontiguousarray(disp, dtype=np.int32)).cuda()
    out = torch.empty((d.shape[0], 6), dtype=torch.float64, device="cuda")
    _check(_lib.mm_demag_tensor(ctypes.byref(Mesh(*mesh)), _ptr(d), d.shape[0], _ptr(out), _stream(stream)),
           "mm_demag_tensor")
    return out.cpu().numpy()


def scalar_potential_kernel(mesh, disp, stream=None):
    """Cuboid potential S at the vertex - cell displacements ((I - 1/2) dx, (J - 1/2) dy, (K - 1/2) dz)
    for disp (array [n,3] of I, J, K) -> numpy [n,3] (FP64, device-computed)."""
    import torch
    d = torch.as_tensor(np.ascontiguousarray(disp, dtype=np.int32)).cuda()
    out = torch.empty((d.shape[0], 3), dtype=torch.float64, device="cuda")
    _check(_lib.mm_scalar_potential_kernel(ctypes.byref(Mesh(*mesh)), _ptr(d), d.shape[0], _ptr(out),
                                           _stream(stream)), "mm_scalar_potential_kernel")
    return out.cpu().numpy()
