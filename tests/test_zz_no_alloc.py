"""mm_sd_run_noalloc (steepest descent without device allocation) against
mm_sd_run through the C interface: two calls in a row, the second on a smaller
mesh and batch, each compared with mm_sd_run from the same start.  Both run the
same kernels with fixed-order reductions, so the results must agree bit for bit
(well inside the FP32 1e-4 bar of the trajectories).  Also the host-side
refusals: a batch beyond the fixed scratch, and a plan whose stage buffers do
not hold the batch yet."""
import numpy as np
import pytest

from _util import gpu_params, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAR = dict(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=8e5, u=(0, 0, 1), H=(1e4, 0.0, 1e5), alpha=0.5)
ALL = 31
SD = (1e-7, 1e-10, 1e-3)


@pytest.fixture(scope="module")
def mm():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2406_16064_amd import mm as m
    return m


def _start(mesh, batch, seed):
    rng = np.random.default_rng(seed)
    m = np.zeros((batch, 3, mesh[2], mesh[1], mesh[0]))
    m[:, 2] = 1.0
    m += 0.3 * rng.normal(size=m.shape)
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def test_noalloc_matches_sd_run_twice(mm):
    big = (40, 24, 3, 3e-9, 3e-9, 3e-9)
    small = (16, 12, 1, 2e-9, 2e-9, 2e-9)
    cases = []
    for mesh, batch, seed in ((big, 2, 11), (small, 1, 12)):
        plan = mm.Plan(mesh, "f32", terms=ALL, max_batch=batch)
        ps = [gpu_params(mm, dict(PAR, Ms=PAR["Ms"] * (1 + 0.2 * b)), ALL) for b in range(batch)]
        m0 = _start(mesh, batch, seed)
        ref = to_dev(m0, torch.float32)
        tau_ref = plan.sd_run(ps, ref, 25, *SD)  # also allocates the plan's stage buffers
        torch.cuda.synchronize()
        cases.append((plan, ps, m0, ref, tau_ref))
    outs = []
    for plan, ps, m0, _, _ in cases:  # the two allocation-free calls, back to back
        md = to_dev(m0, torch.float32)
        st, tau = plan.sd_run_noalloc(ps, md, 25, *SD)
        assert st == mm.MM_OK
        outs.append((md, tau))
    torch.cuda.synchronize()
    for (plan, ps, m0, ref, tau_ref), (md, tau) in zip(cases, outs):
        assert torch.equal(md, ref)
        assert np.array_equal(tau, tau_ref)
        assert float((md - torch.tensor(m0, dtype=torch.float32, device="cuda")).abs().max()) > 1e-3  # it moved


def test_noalloc_refusals(mm):
    mesh = (16, 12, 1, 2e-9, 2e-9, 2e-9)
    plan = mm.Plan(mesh, "f32", terms=ALL, max_batch=2)
    gp = gpu_params(mm, PAR, ALL)
    md = to_dev(_start(mesh, 2, 3), torch.float32)
    before = md.clone()
    st, _ = plan.sd_run_noalloc([gp, gp], md, 5, *SD, check=False)
    assert st == mm.MM_E_STATE  # no stage buffers yet: nothing launched
    assert torch.equal(md, before)
    # 1024 x 1024 x 4 cells: 512 KiB of partial sums per instance, 40 instances > 16 MiB
    bigmesh = (1024, 1024, 4, 2e-9, 2e-9, 2e-9)
    bp = mm.Plan(bigmesh, "f32", terms=1, max_batch=40)
    ex = gpu_params(mm, PAR, 1)
    mb = torch.zeros((40, 3, 4, 1024, 1024), dtype=torch.float32, device="cuda")
    st, _ = bp.sd_run_noalloc([ex] * 40, mb, 1, *SD, check=False)
    assert st == mm.MM_E_ARG
    assert "scratch" in mm._lib.mm_last_error().decode()
