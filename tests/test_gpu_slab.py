"""GPU parity of the demag-dominated 512x512x16 slab (5 nm cells, Ms 8e5 A/m,
A 1.3e-11 J/m, alpha 0.02, 25 mT at 170 degrees in plane; S-state + 1e-2 noise).

* Full size, in the launch shapes bench.py times: the dense effective field and
  dm/dt of the S-state against the oracle's FFT convolution (FP32 <= 1e-5,
  FP64 <= 1e-10 in the max-norm form).  The oracle's tensor grid (32.4M
  displacements) is built in worker processes; every entry is computed on its
  own, so the grid is the same as a single-process build.
* Reduced meshes that reach the slab's kernel instantiations and that the oracle
  integrates in seconds: 512x4x16 (512-point x transforms: the fixed-length
  forward and inverse x kernels; Pz = 32: the register z pass of half-zero
  columns) and 8x512x16 (Py = 1024: the fixed-length y kernels; Pz = 32):
  dense fields in FP32 and FP64, an FP32 trajectory of 20 accepted oracle
  steps replayed on the device (m within 1e-4), and an FP32 batched run of
  both meshes against the free-running oracle.
"""
import os

import numpy as np
import pytest

from oracle import dp45, newell
from oracle import fields as F
from paper_2406_16064_amd import inputs

from _util import field_err, gpu_params, oracle_params, representable, to_dev

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f32": 1e-5, "f64": 1e-10}
W = inputs.workload(2)
REDUCED = [(512, 4, 16) + tuple(W["mesh"][3:]), (8, 512, 16) + tuple(W["mesh"][3:])]


@pytest.fixture(scope="module")
def mm():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2406_16064_amd import mm as m
    return m


_kern = {}


def _kernel(mesh, workers=1):
    if mesh not in _kern:
        msh = F.Mesh(*mesh)
        grid = newell.tensor_grid(msh.nx, msh.ny, msh.nz, msh.dx, msh.dy, msh.dz, workers=workers)
        _kern[mesh] = F.DemagKernel(msh, grid=grid)
    return _kern[mesh]


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def _bench_shapes(mm, plan, mesh, prec, gp, md):
    """The launch shapes bench.py times: the committed tuned table, else the autotuner."""
    from paper_2406_16064_amd import tuned
    sh = tuned.lookup(mesh, prec)
    if sh is not None:
        plan.set_shapes(sh)
    else:
        plan.autotune(gp, md, reps=2)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_slab_full_size_dense(mm, prec):
    mesh = tuple(W["mesh"])
    print("slab dense %s: oracle tensor grid" % prec, flush=True)
    kern = _kernel(mesh, _workers())
    m = representable(inputs.initial_state(2), DT[prec])
    op = oracle_params(W["params"], W["terms"])
    print("slab dense %s: oracle field" % prec, flush=True)
    Href = F.effective_field(m, F.Mesh(*mesh), op, kern)
    kref = F.llg_rhs_from_field(m, Href, op)
    plan = mm.Plan(mesh, prec, terms=W["terms"])
    gp = gpu_params(mm, W["params"], W["terms"])
    md = to_dev(m, DT[prec])
    _bench_shapes(mm, plan, mesh, prec, gp, md)
    print("slab dense %s: device field" % prec, flush=True)
    assert field_err(plan.effective_field(gp, md).cpu().numpy(), Href) <= TOL[prec]
    assert field_err(plan.llg_rhs(gp, md).cpu().numpy(), kref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mesh", REDUCED, ids=["512x4x16", "8x512x16"])
def test_slab_instantiations_dense(mm, prec, mesh):
    m = representable(inputs.initial_state(2, mesh), DT[prec])
    op = oracle_params(W["params"], W["terms"])
    Href = F.effective_field(m, F.Mesh(*mesh), op, _kernel(mesh))
    plan = mm.Plan(mesh, prec, terms=W["terms"])
    gp = gpu_params(mm, W["params"], W["terms"])
    md = to_dev(m, DT[prec])
    plan.autotune(gp, md, reps=2)
    assert plan.padded()[2] == 32
    assert field_err(plan.effective_field(gp, md).cpu().numpy(), Href) <= TOL[prec]
    kref = F.llg_rhs_from_field(m, Href, op)
    assert field_err(plan.llg_rhs(gp, md).cpu().numpy(), kref) <= TOL[prec]


@pytest.mark.parametrize("mesh", REDUCED, ids=["512x4x16", "8x512x16"])
def test_slab_instantiations_replay_fp32(mm, mesh):
    """20 accepted oracle steps (rtol 1e-6, from h = 1e-13 s) replayed by the FP32 graph."""
    m0 = representable(inputs.initial_state(2, mesh), torch.float32)
    op = oracle_params(W["params"], W["terms"])
    f = lambda y: F.llg_rhs(y, F.Mesh(*mesh), op, _kernel(mesh))
    ost = dp45.State(rtol=W["rtol"])
    mo = dp45.run(f, m0.copy(), ost, max_accept=20)
    assert ost.n_accept == 20
    plan = mm.Plan(mesh, "f32", terms=W["terms"])
    gp = gpu_params(mm, W["params"], W["terms"])
    md = to_dev(m0, torch.float32)
    plan.autotune(gp, md, reps=2)
    st = mm.new_states(1, rtol=W["rtol"])
    plan.rk45_run(gp, md, st, replay_h=ost.accepted_h)
    assert st[0].n_accept == 20
    assert np.max(np.linalg.norm(md.cpu().numpy() - mo, axis=0)) <= 1e-4


def test_slab_instantiations_batched_fp32(mm):
    """Both reduced meshes in one FP32 batch, free running to 3 ps, against the oracle
    integrator (FP32 error norms move the step sizes by ~1e-5 relative only)."""
    t_end = 3e-12
    m0 = [representable(inputs.initial_state(2, msh), torch.float32) for msh in REDUCED]
    batch = mm.Batch(REDUCED, "f32", terms=W["terms"])
    devs = [to_dev(m, torch.float32) for m in m0]
    gp = gpu_params(mm, W["params"], W["terms"])
    _, res = batch.run([dict(mesh_id=k, params=gp, m=devs[k], t_end=t_end) for k in range(2)])
    op = oracle_params(W["params"], W["terms"])
    for k, msh in enumerate(REDUCED):
        f = lambda y: F.llg_rhs(y, F.Mesh(*msh), op, _kernel(msh))
        ost = dp45.State(rtol=W["rtol"])
        mo = dp45.run(f, m0[k].copy(), ost, t_end=t_end)
        st, status = res[k]
        assert status == mm.MM_OK and st.t == t_end
        assert st.n_accept == ost.n_accept and st.n_reject == ost.n_reject, k
        assert np.max(np.linalg.norm(devs[k].cpu().numpy() - mo, axis=0)) <= 1e-4, k


@pytest.mark.parametrize("shape", [dict(ty_x=4, nt_i=512), dict(ty_x=2, nt_i=512), dict(ty_x=2, nt_i=256)],
                         ids=["4rows512", "2rows512", "2rows256"])
def test_slab_stage_epilogue_shapes_replay_fp32(mm, shape):
    """The FP32 stage and error kernels in three inverse-x launch shapes (4 or 2
    rows of 512 cells a workgroup, one cell or several a thread) on 512 x 6 x 16,
    whose y tiles end in a partial one: 10 accepted oracle steps replayed, m
    within 1e-4."""
    mesh = (512, 6, 16) + tuple(W["mesh"][3:])
    m0 = representable(inputs.initial_state(2, mesh), torch.float32)
    op = oracle_params(W["params"], W["terms"])
    f = lambda y: F.llg_rhs(y, F.Mesh(*mesh), op, _kernel(mesh))
    ost = dp45.State(rtol=W["rtol"])
    mo = dp45.run(f, m0.copy(), ost, max_accept=10)
    plan = mm.Plan(mesh, "f32", terms=W["terms"])
    gp = gpu_params(mm, W["params"], W["terms"])
    md = to_dev(m0, torch.float32)
    base = plan.shapes()
    plan.set_shapes(dict(base, **shape))
    assert plan.shapes()["ty_x"] == shape["ty_x"] and plan.shapes()["nt_i"] == shape["nt_i"]
    st = mm.new_states(1, rtol=W["rtol"])
    plan.rk45_run(gp, md, st, replay_h=ost.accepted_h)
    assert st[0].n_accept == 10
    assert np.max(np.linalg.norm(md.cpu().numpy() - mo, axis=0)) <= 1e-4
