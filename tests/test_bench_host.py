"""Host logic of bench.py: algorithmic byte counts, the roofline's choice of
kernel, the counter lookup and the one-GPU guard (no GPU, no library calls)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_pass_bytes_thin_film_by_hand():
    # 256 x 256 x 1 padded to 512 x 512 x 1, FP32: X' = 257 kept x columns,
    # spectrum of 3 components x 257 x 256 rows, 4 folded tensor components of
    # 257 x 257 reals
    mesh, P, w = (256, 256, 1), (512, 512, 1), 4
    m = 3 * 256 * 256 * 4
    sx = 3 * 257 * 256 * 8
    K = 4 * 1 * 257 * 257 * 4
    assert bench.pass_bytes(mesh, P, w) == [m + sx, 2 * sx + K, sx + 2 * m]


def test_pass_bytes_slab_by_hand():
    mesh, P, w = (512, 512, 16), (1024, 1024, 32), 8
    m = 3 * 512 * 512 * 16 * 8
    sx = 3 * 16 * 513 * 512 * 16
    sy = 3 * 16 * 513 * 1024 * 16
    K = 6 * 17 * 513 * 513 * 8
    assert bench.pass_bytes(mesh, P, w) == [m + sx, sx + sy, 2 * sy + K, sy + sx, sx + 2 * m]


def _res(mesh, shapes, kernel="x_inv_stage_fused_fwd"):
    att = [{"kernel": "y_fwd", "per_attempt": 6, "us": 1.0, "alg_bytes": 10, "gbs": 10.0, "us_per_attempt": 6.0},
           {"kernel": kernel, "per_attempt": 5, "us": 2.0, "alg_bytes": 4000, "gbs": 2000.0,
            "us_per_attempt": 10.0}]
    return {"attempt_kernels": att, "attempt_kernel_us": 16.0, "mesh": list(mesh), "launch_shapes": shapes}


@pytest.fixture
def counters(tmp_path, monkeypatch):
    """A counter summary for the current sources in a scratch copy of the root."""
    os.makedirs(tmp_path / "profiles")
    rec = {"source_hash": bench.source_hash(), "workloads": {"thin": {
        "x_inv_stage_fused_fwd": {"kernel": "k", "launch": "grid 32768, workgroup 512, LDS 0",
                                  "bytes_per_launch": 123.0, "by_launch": {
                                      "grid 32768, workgroup 512, LDS 0": {"bytes_per_launch": 123.0},
                                      "grid 65536, workgroup 256, LDS 0": {"bytes_per_launch": 150.0}}},
        "x_inv_error": {"kernel": "k", "launch": "grid 32768, workgroup 512, LDS 512", "bytes_per_launch": 9.0},
        "y_fwd": {"kernel": "k", "bytes_per_launch": 7.0}}}}
    with open(tmp_path / "profiles" / "traffic_counters.json", "w") as f:
        json.dump(rec, f)
    h = bench.source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    return rec


def test_roofline_takes_largest_time_per_attempt(counters):
    r = bench.roofline(_res((256, 256, 1), {"ty_x": 4, "nt_i": 512}), "thin")
    assert r["kernel"] == "x_inv_stage_fused_fwd"
    assert r["frac"] == round(2000.0 / 8000.0, 4)
    assert r["share_of_attempt"] == round(10.0 / 16.0, 3)


def test_traffic_needs_the_launch_shape_it_was_counted_at(counters):
    # 64 workgroups of 512 threads: the shape the timed counter run used
    assert bench.roofline(_res((256, 256, 1), {"ty_x": 4, "nt_i": 512}), "thin")["traffic"] == 123.0
    # one row per workgroup, 256 threads: an autotuner candidate the counters also read
    assert bench.roofline(_res((256, 256, 1), {"ty_x": 1, "nt_i": 256}), "thin")["traffic"] == 150.0
    # one row per workgroup, 512 threads: no counters for it
    assert bench.roofline(_res((256, 256, 1), {"ty_x": 1, "nt_i": 512}), "thin")["traffic"] is None
    # a record without per-shape entries matches its own launch only
    res = _res((256, 256, 1), {"ty_x": 4, "nt_i": 512}, "x_inv_error")
    assert bench.roofline(res, "thin")["traffic"] == 9.0
    res = _res((256, 256, 1), {"ty_x": 2, "nt_i": 512}, "x_inv_error")
    assert bench.roofline(res, "thin")["traffic"] is None
    # pass kernels carry no launch shape
    assert bench.load_traffic("thin", "y_fwd") == 7.0


def test_traffic_null_when_sources_changed(counters, tmp_path):
    counters["source_hash"] = "0" * 16
    with open(tmp_path / "profiles" / "traffic_counters.json", "w") as f:
        json.dump(counters, f)
    assert bench.load_traffic("thin", "y_fwd") is None


def test_more_than_one_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr or "1 GPU" in p.stderr or "single" in p.stderr


def _csv(path, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Counter_Value,Grid_Size,Workgroup_Size,LDS_Block_Size\n")
        for k, v, g, w in rows:
            f.write('"%s",%s,%d,%d,0\n' % (k, v, g, w))


def test_ingest_scales_by_copy_and_keeps_shapes_read_in_both_runs(tmp_path, monkeypatch):
    h = bench.source_hash()
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    copy = "__amd_rocclr_copyBuffer"
    kib = bench.COPY_BYTES / 1024.0
    # the copy's fetch counter reads half its bytes, its write counter all of them
    _csv(tmp_path / "cf.csv", [(copy, kib / 2, 1, 1)])
    _csv(tmp_path / "cw.csv", [(copy, kib, 1, 1)])
    st4 = "void mmx::k_inv_x<float, true, 2, 4, true, false>(mmx::Launch<float>)"
    st1 = "void mmx::k_inv_x<float, true, 2, 1, true, false>(mmx::Launch<float>)"
    yk = "void mmx::k_ypass_s<float, 512, 8>(mmx::Launch<float>)"
    yk16 = "void mmx::k_ypass_s<float, 512, 16>(mmx::Launch<float>)"
    fetch = [(st4, 10, 100, 50)] * 3 + [(st1, 20, 400, 100)] * 2 + [(yk, 3, 1, 1)] * 4 + [(yk16, 5, 1, 1)]
    write = [(st4, 7, 100, 50)] * 3 + [(yk, 1, 1, 1)] * 4
    _csv(tmp_path / "f.csv", fetch)
    _csv(tmp_path / "w.csv", write)
    d = bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                              str(tmp_path / "cw.csv"), "thin", 2, 1)
    rec = d["workloads"]["thin"]
    # y: the instantiation launched most and read in both runs; fetch x 2, write x 1
    assert rec["y_fused_product"]["kernel"] == yk
    assert rec["y_fused_product"]["bytes_per_launch"] == 3 * 1024 * 2 + 1 * 1024
    st = rec["x_inv_stage_fused_fwd"]
    assert st["launch"] == "grid 100, workgroup 50, LDS 0" and st["dispatches"] == 3
    assert st["bytes_per_launch"] == 10 * 1024 * 2 + 7 * 1024
    # the shape only the fetch run saw has no record (its write bytes are unknown)
    assert list(st["by_launch"]) == ["grid 100, workgroup 50, LDS 0"]


def test_demag_pipeline_counts_every_pass_of_an_evaluation():
    """The pipeline figure covers the inverse-x complex-to-real pass too (with its
    fused epilogue), not only the forward transforms, the product and inverse y."""
    names = bench.pass_names(16)
    res = {"passes": [{"kernel": n, "us": 1.0 + i, "alg_bytes": 1000 * (i + 1)} for i, n in enumerate(names)]}
    dp = bench.demag_pipeline(res)
    assert list(dp["passes"]) == names and "x_inv_fused_llg" in dp["passes"]
    assert dp["alg_bytes"] == 15000 and dp["us"] == 15.0
    assert dp["frac"] == round(15000 / 15e-6 / 1e9 / 8000.0, 4)


def test_tuned_table_round_trip(tmp_path):
    from paper_2406_16064_amd import tuned
    path = str(tmp_path / "t.json")
    assert tuned.lookup((512, 512, 16), "f32", path) is None
    sh = {"ty_f": 4, "nt_f": 256, "cb_y": 4, "tpc_y": 64, "nt_y": 256, "ty_x": 4, "nt_i": 512}
    tuned.store((512, 512, 16, 5e-9, 5e-9, 5e-9), "f32", sh, path)
    assert tuned.lookup((512, 512, 16), "f32", path) == sh
    assert tuned.lookup((512, 512, 16), "f64", path) is None
