"""Seeded input recipes: determinism, unit norms, layout (CPU only)."""
import numpy as np

from paper_2406_16064_amd import inputs


def test_seeded_and_unit():
    for idx in (0, 1):
        a = inputs.initial_state(idx)
        b = inputs.initial_state(idx)
        assert np.array_equal(a, b)
        nx, ny, nz = inputs.workload(idx)["mesh"][:3]
        assert a.shape == (3, nz, ny, nx)
        assert np.max(np.abs(np.linalg.norm(a, axis=0) - 1)) < 1e-14


def test_skyrmion_cores_point_down():
    m = inputs.initial_state(1)
    assert m[2].min() < -0.99 and np.mean(m[2]) > 0.9


def test_neb_chain_ends_and_monotone_distance():
    mesh = (32, 32, 1, 1e-9, 1e-9, 0.4e-9)
    ch = inputs.neb_chain(mesh)
    assert len(ch) == 32
    assert np.all(ch[-1][2] == 1.0)
    d = [np.linalg.norm(ch[i + 1] - ch[i]) for i in range(31)]
    assert max(d) < 3 * min(d)
    for m in ch:
        assert np.max(np.abs(np.linalg.norm(m, axis=0) - 1)) < 1e-12


def test_sweep_instances_in_range():
    sizes = set()
    for i in range(40):
        w = inputs.sweep_instance(i)
        n, _, nz = w["mesh"][:3]
        sizes.add(n)
        assert n in inputs.SWEEP_SIZES and nz in (1, 2)
        assert 4e5 <= w["params"]["Ms"] <= 1.2e6
    assert len(sizes) >= 4
