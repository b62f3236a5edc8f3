"""Benchmark of the micromagnetic hot path on one MI355X.

Headline workload: the demag-dominated 512x512x16 slab (5x5x5 nm cells, Ms
8e5 A/m, A 1.3e-11 J/m, alpha 0.02, 25 mT at 170 degrees in plane; S-state plus
1e-2 noise; padded FFT grid 1024x1024x32) integrated with adaptive
Dormand-Prince in FP32.  One step = one attempted adaptive step of the whole
path (six effective-field + LL evaluations with the fused stage combinations,
the FP64 error norm, the device controller and the projection), run under the
library's captured HIP graph.  value = cells x RHS evaluations / second over
the timed steps, with m resident in HBM.  Launch shapes come from the tuned
table (paper_2406_16064_amd/tuned_shapes.json), so the profiled and the timed
kernels are the same instantiations.

Also reported: FP64 on the same workload, the 256x256x1 thin film (FP32 and
FP64), per-kernel roofline figures measured with HIP events, the uneven
parameter sweep batched vs one by one, the 32-image NEB chain, the Heun and
steepest-descent records, and the FP64 CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LLG RHS cell-evals/s, FP32 vs FP64 (field rel err ≤1e-5); batched vs 1-by-1"
HBM_PEAK_GBS = 8000.0


def pass_names(nz):
    if nz == 1:
        return ["x_fwd", "y_fused_product", "x_inv_fused_llg"]
    return ["x_fwd", "y_fwd", "z_product", "y_inv", "x_inv_fused_llg"]


def pass_bytes(mesh, P, w):
    """Algorithmic HBM bytes of each pass of one dm/dt evaluation (read + write).

    w: bytes per real.  Complex = 2w.  Xp = Px/2+1 spectral columns kept in x;
    tensor spectrum K = ncomp * (Pz/2+1) * Xp * (Py/2+1) reals.  The fused last
    pass reads the x spectrum and m (with its halo from cache) and writes dm/dt.
    """
    nx, ny, nz = mesh[:3]
    Px, Py, Pz = P
    N = nx * ny * nz
    Xp = Px // 2 + 1
    sx = 3 * nz * Xp * ny * 2 * w
    sy = 3 * nz * Xp * Py * 2 * w
    ncomp = 4 if nz == 1 else 6
    K = ncomp * (Pz // 2 + 1) * Xp * (Py // 2 + 1) * w
    m = 3 * N * w
    if nz == 1:
        return [m + sx, sx + K + sx, sx + m + m]
    return [m + sx, sx + sy, sy + K + sy, sy + sx, sx + m + m]


POT_PASSES = ["x_fwd", "y_fwd", "z_potential", "y_inv_potential", "x_inv_potential_llg"]


def pot_pass_bytes(mesh, P, w):
    """Algorithmic HBM bytes of each pass of one dm/dt evaluation through the
    scalar potential: the forward x and y passes as for the Newell route; z reads
    the 3 spectra and the folded kernel spectrum (3 (Pz/2+1) Xp (Py/2+1) reals)
    and writes the potential's nz + 1 vertex planes; the inverse y pass reads those
    and writes ny + 1 vertex rows per plane; the last pass reads each vertex row
    once and m, and writes dm/dt."""
    nx, ny, nz = mesh[:3]
    Px, Py, Pz = P
    N = nx * ny * nz
    Xp = Px // 2 + 1
    sx = 3 * nz * Xp * ny * 2 * w
    sy = 3 * nz * Xp * Py * 2 * w
    K = 3 * (Pz // 2 + 1) * Xp * (Py // 2 + 1) * w
    u_z = (nz + 1) * Xp * Py * 2 * w
    u_y = (nz + 1) * (ny + 1) * Xp * 2 * w
    m = 3 * N * w
    return [m + sx, sx + sy, sy + K + u_z, u_z + u_y, u_y + m + m]


# Dormand-Prince slopes read by the stage combinations of stages 2..6 (entries
# of a_{s+1,j}, j < s, that are non-zero) and by the error combination
STAGE_KPREV = (1, 2, 3, 4, 4)
ERROR_KPREV = 5


def step_kernel_bytes(mesh, P, w, fused):
    """Algorithmic HBM bytes per launch of the attempt-only kernels: the step
    begin after an accepted attempt (read y5 and k7; write the projected m, k1 = k7
    and the stage-2 input; after a rejection it reads m and k1 and writes the input
    only), the inverse-x pass with the
    stage epilogue (read Sx, stage input, m, the slopes of its combination;
    write k_s and the next stage input, and the next x spectrum when fused;
    mean over stages 2..6) and with the error epilogue (read Sx, stage input,
    five slopes; write k7)."""
    nx, ny, nz = mesh[:3]
    Xp = P[0] // 2 + 1
    sx = 3 * nz * Xp * ny * 2 * w
    f = 3 * nx * ny * nz * w  # one m-like array
    kp = sum(STAGE_KPREV) / len(STAGE_KPREV)
    return {"step_begin": 5 * f,
            "x_inv_stage": sx + (2 + kp) * f + 2 * f + (sx if fused else 0),
            "x_inv_error": sx + (1 + ERROR_KPREV) * f + f}


def attempt_breakdown(mesh, P, w, passes_us, step):
    """Time of each kernel kind per adaptive attempt from the back-to-back
    launch timings: (name, launches per attempt, us per launch, alg bytes)."""
    b_us, stage_us, err_us, fused = step
    names = pass_names(mesh[2])
    kb = step_kernel_bytes(mesh, P, w, fused)
    pb = dict(zip(names, pass_bytes(mesh, P, w)))
    rows = [("step_begin", 1, b_us, kb["step_begin"])]
    for name, us in zip(names[:-1], stage_us[:-1]):
        n = (1 if fused else 6) if name == "x_fwd" else 6
        rows.append((name, n, us, pb[name]))
    rows.append(("x_inv_stage" + ("_fused_fwd" if fused else ""), 5, stage_us[-1], kb["x_inv_stage"]))
    rows.append(("x_inv_error", 1, err_us, kb["x_inv_error"]))
    return rows


def source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2406_16064_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2406_16064_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def set_shapes(plan, params, m, mesh, prec, retune=None):
    """Launch shapes of the tuned table (the same instantiations every run), else the
    autotuner's pick on this device (not timed).  retune: autotune and store the pick
    in the table file `retune`.  Returns (shapes, source)."""
    from paper_2406_16064_amd import tuned
    sh = None if retune else tuned.lookup(mesh, prec)
    if sh is not None:
        plan.set_shapes(sh)
        return plan.shapes(), "tuned table"
    sh = plan.autotune(params, m, reps=20)
    if retune:
        tuned.store(mesh, prec, sh, retune)
    return sh, "autotuned in this run"


def run_workload(mm, inputs, torch, idx, prec, steps, warmup, mesh=None, retune=None):
    w = inputs.workload(idx)
    mesh = tuple(mesh or w["mesh"])
    dt = torch.float32 if prec == "f32" else torch.float64
    plan = mm.Plan(mesh, prec, terms=w["terms"])
    params = mm.make_params(terms=w["terms"], **w["params"])
    m = torch.tensor(inputs.initial_state(idx, mesh), dtype=dt, device="cuda")
    shapes, shapes_src = set_shapes(plan, params, m, mesh, prec, retune)
    st = mm.new_states(1, rtol=w["rtol"])
    t_end = w["t_end"]
    s = plan.rk45_run(params, m, st, t_end=t_end, max_steps=warmup, check=False)
    if s not in (mm.MM_OK, mm.MM_E_MAXSTEPS):
        raise RuntimeError("warmup failed: %s" % mm.status_string(s))
    torch.cuda.synchronize()
    n0, a0 = st[0].n_rhs, st[0].n_accept + st[0].n_reject
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    s = plan.rk45_run(params, m, st, t_end=t_end, max_steps=steps, check=False)
    e1.record()
    torch.cuda.synchronize()
    if s not in (mm.MM_OK, mm.MM_E_MAXSTEPS):
        raise RuntimeError("timed run failed: %s" % mm.status_string(s))
    ms = e0.elapsed_time(e1)
    evals = st[0].n_rhs - n0
    attempts = st[0].n_accept + st[0].n_reject - a0
    N = mesh[0] * mesh[1] * mesh[2]
    P = plan.padded()
    # kernel durations from whole evaluations and attempts timed in their own order
    # (each kernel after the one whose output it reads, as in the timed run); the
    # back-to-back repeats of one kernel, whose inputs stay in the 256 MB cache,
    # are kept beside them
    us_b2b, us = plan.profile_passes(params, m, reps=30, in_order=True)
    b0, st_b2b, e0_, fused, (b1, st_seq, e1_) = plan.profile_step(params, m, st, reps=20, in_order=True)
    step, step_b2b = (b1, st_seq, e1_, fused), (b0, st_b2b, e0_, fused)
    w_bytes = 4 if prec == "f32" else 8
    pb = pass_bytes(mesh, P, w_bytes)
    passes = []
    for name, t, t2, b in zip(pass_names(mesh[2]), us, us_b2b, pb):
        passes.append({"kernel": name, "us": round(t, 3), "alg_bytes": b,
                       "gbs": round(b / (t * 1e-6) / 1e9, 1), "us_back_to_back": round(t2, 3)})
    attempt = []
    for (name, n, t, b), (_, _, t2, _) in zip(attempt_breakdown(mesh, P, w_bytes, us, step),
                                              attempt_breakdown(mesh, P, w_bytes, us_b2b, step_b2b)):
        attempt.append({"kernel": name, "per_attempt": n, "us": round(t, 3), "alg_bytes": int(b),
                        "gbs": round(b / (t * 1e-6) / 1e9, 1), "us_per_attempt": round(n * t, 2),
                        "us_back_to_back": round(t2, 3)})
    out = {
        "workload": w["name"], "mesh": list(mesh), "padded": list(P), "dtype": prec,
        "cell_evals_per_s": N * evals / (ms * 1e-3), "ms_per_step": ms / max(attempts, 1),
        "steps": attempts, "rhs_evals": evals, "t_sim": st[0].t, "h": st[0].h,
        "passes": passes,
        "attempt_kernels": attempt,
        "attempt_kernel_us": round(sum(a["us_per_attempt"] for a in attempt), 2),
        "launch_shapes": shapes,
        "launch_shapes_source": shapes_src,
        "eval_us": round(sum(us), 3),
        "demag_pipeline_gbs": round(sum(pb) / (sum(us) * 1e-6) / 1e9, 1),
    }
    return out, plan, params, m, mesh


def sweep_bench(mm, inputs, torch, n_inst=256, steps=16, warmup=8):
    """Parameter sweep of n_inst instances of uneven meshes: one batched run (one
    launch per pass across all meshes) against the same instances run one by one
    through one plan per mesh.  Both time `steps` adaptive attempts per instance."""
    w = inputs.workload(4)
    insts = [inputs.sweep_instance(i) for i in range(n_inst)]
    meshes = sorted({tuple(x["mesh"]) for x in insts})
    mid = {msh: i for i, msh in enumerate(meshes)}
    params = [mm.make_params(terms=w["terms"], **x["params"]) for x in insts]
    cells = [x["mesh"][0] * x["mesh"][1] * x["mesh"][2] for x in insts]
    batch = mm.Batch(meshes, "f32", terms=w["terms"])
    devs = [torch.tensor(x["m"], dtype=torch.float32, device="cuda") for x in insts]
    states = [mm.new_states(1, rtol=w["rtol"])[0] for _ in insts]

    def one_batched(k):
        desc = [dict(mesh_id=mid[tuple(x["mesh"])], params=params[i], m=devs[i], t_end=w["t_end"],
                     state=states[i]) for i, x in enumerate(insts)]
        _, res = batch.run(desc, max_steps=k, check=False)
        for i, (st, status) in enumerate(res):
            states[i] = st
            if status not in (mm.MM_OK, mm.MM_E_MAXSTEPS):
                raise RuntimeError("sweep instance %d failed: %s" % (i, mm.status_string(status)))

    one_batched(warmup)
    n0 = [s.n_rhs for s in states]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    one_batched(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    evals_b = sum(c * (s.n_rhs - n) for c, s, n in zip(cells, states, n0))
    # one by one, same instances, one plan and one state buffer per mesh (set-up
    # not timed): each instance is copied into its mesh's buffer, run, and copied
    # back, and only the runs are timed.  The plan's captured graph is keyed by the
    # state buffer, so it is captured once per mesh (in the warm-up), not per instance.
    plans = {msh: mm.Plan(msh, "f32", terms=w["terms"]) for msh in meshes}
    bufs = {msh: torch.empty((3, msh[2], msh[1], msh[0]), dtype=torch.float32, device="cuda") for msh in meshes}
    devs1 = [torch.tensor(x["m"], dtype=torch.float32, device="cuda") for x in insts]
    st1 = [mm.new_states(1, rtol=w["rtol"]) for _ in insts]

    def one_by_one(k):
        spent = 0.0
        for i, x in enumerate(insts):
            msh = tuple(x["mesh"])
            bufs[msh].copy_(devs1[i])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plans[msh].rk45_run(params[i], bufs[msh], st1[i], t_end=w["t_end"], max_steps=k, check=False)
            spent += time.perf_counter() - t0  # rk45_run synchronises
            devs1[i].copy_(bufs[msh])
        return spent

    one_by_one(warmup)
    n1 = [s[0].n_rhs for s in st1]
    ms_1 = 1e3 * one_by_one(steps)
    evals_1 = sum(c * (s[0].n_rhs - n) for c, s, n in zip(cells, st1, n1))
    rb = evals_b / (ms_b * 1e-3)
    r1 = evals_1 / (ms_1 * 1e-3)
    return {"workload": w["name"], "instances": n_inst, "meshes": [list(m) for m in meshes],
            "cells_total": sum(cells), "attempts_per_instance": steps,
            "batched_cell_evals_per_s": rb, "batched_ms": ms_b,
            "one_by_one_cell_evals_per_s": r1, "one_by_one_ms": ms_1,
            "batched_over_one_by_one": rb / r1}


def neb_bench(mm, inputs, torch, relax_dmdt=1.0):
    """32-image NEB chain on 128x128x1, the configured 2000 iterations (one launch
    per pass for all images).  The seeded skyrmion and the uniform +z end images
    are first relaxed by steepest descent until the largest |dm/dt| is below
    relax_dmdt (deg/ns; not timed), and the chain is the geodesic interpolation
    between the relaxed ends, so that the image energies after the run give the
    skyrmion's collapse barrier: the highest image above the skyrmion end."""
    import numpy as np
    w = inputs.workload(3)
    params = mm.make_params(terms=w["terms"], **w["params"])
    ends = np.stack(inputs.neb_chain())[[0, -1]]
    one = mm.Plan(w["mesh"], "f32", terms=w["terms"], max_batch=2)
    dend = torch.tensor(ends, dtype=torch.float32, device="cuda")
    st, it, _, _ = one.sd_relax([params, params], dend, relax_dmdt, 20000, 1e-7, 1e-10, 1e-3, check=False)
    relaxed = dend.cpu().numpy().astype(np.float64)
    del one
    chain = np.stack(inputs.slerp_chain(relaxed[0], relaxed[1], w["n_images"]))
    plan = mm.Plan(w["mesh"], "f32", terms=w["terms"], max_batch=w["n_images"])
    warm = torch.tensor(chain, dtype=torch.float32, device="cuda")
    plan.neb_run(params, warm, w["k_spring"], w["h"], 4)  # graph capture and first launches, not timed
    dev = torch.tensor(chain, dtype=torch.float32, device="cuda")
    iters = w["n_iter"]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    E = plan.neb_run(params, dev, w["k_spring"], w["h"], iters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = w["n_images"] * w["mesh"][0] * w["mesh"][1]
    imax = int(np.argmax(E))
    return {"workload": w["name"], "iterations": iters, "ms_per_iteration": ms / iters,
            "cell_evals_per_s": cells * iters / (ms * 1e-3),
            "end_relaxation": {"status": int(st), "iterations": [int(v) for v in it],
                               "stopping_dmdt_deg_ns": relax_dmdt},
            "image_energies_J": [float(e) for e in E],
            "highest_image": imax, "barrier_J": float(E[imax] - E[0]),
            "barrier_kT_300K": float(E[imax] - E[0]) / (1.380649e-23 * 300.0)}


def sp4_bench(mm, inputs, torch, stop=0.01, samples=100):
    """Standard Problem 4 as the paper describes it, in FP32: steepest-descent
    relaxation from the uniform start until the largest |dm/dt| is below `stop`
    (deg/ns), then 1 ns of adaptive Dormand-Prince dynamics in the applied field,
    <m> sampled every 10 ps.  Reports the wall times, the relaxed S-state's <m>,
    <m>(t) and the first time <m_x> changes sign (the OOMMF curves the paper
    compares with are not available here: no reference values)."""
    import numpy as np
    w = inputs.sp4()
    mesh = w["mesh"]
    plan = mm.Plan(mesh, "f32", terms=w["terms"])
    pr = mm.make_params(terms=w["relax_terms"], **w["relax"])
    pd = mm.make_params(terms=w["terms"], **w["dynamics"])
    m = torch.tensor(inputs.sp4_initial(), dtype=torch.float32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    st, it, dm, _ = plan.sd_relax(pr, m, stop, 200000, 1e-7, 1e-10, 1e-3, check=False)
    e1.record()
    torch.cuda.synchronize()
    relax_ms = e0.elapsed_time(e1)
    m_relaxed = [float(v) for v in m.mean(dim=(1, 2, 3)).cpu()]
    states = mm.new_states(1, rtol=w["rtol"])
    ts, mt = [0.0], [m_relaxed]
    torch.cuda.synchronize()
    e0.record()
    for k in range(1, samples + 1):
        plan.rk45_run(pd, m, states, t_end=w["t_end"] * k / samples)
        mt.append([float(v) for v in m.mean(dim=(1, 2, 3)).cpu()])
        ts.append(states[0].t)
    e1.record()
    torch.cuda.synchronize()
    dyn_ms = e0.elapsed_time(e1)
    mx = np.array([v[0] for v in mt])
    cross = next((i for i in range(1, len(mx)) if mx[i] < 0 <= mx[i - 1]), None)
    t0 = None
    if cross is not None:  # linear interpolation between the samples
        t0 = ts[cross - 1] + (ts[cross] - ts[cross - 1]) * mx[cross - 1] / (mx[cross - 1] - mx[cross])
    return {"workload": w["name"], "relax_status": int(st), "relax_iterations": int(it[0]),
            "relax_final_dmdt_deg_ns": float(dm[0]), "relax_ms": relax_ms, "s_state_mean_m": m_relaxed,
            "dynamics_ms_per_ns": dyn_ms / (w["t_end"] * 1e9), "accepted_steps": int(states[0].n_accept),
            "rejected_steps": int(states[0].n_reject), "rhs_evals": int(states[0].n_rhs),
            "first_mx_zero_crossing_ns": None if t0 is None else t0 * 1e9,
            "mean_m_every_100ps": [[round(x, 5) for x in mt[i]] for i in range(0, len(mt), 10)]}


def heun_bench(mm, inputs, torch, steps=100):
    """The paper's throughput setting: N x N x 1 films, demag + exchange + Zeeman,
    fixed-step Heun with projection in FP32, m resident in HBM.  cells_per_s =
    cells x Heun steps / s (two dm/dt evaluations per step)."""
    out = {"paper_context": "up to ~1e9 cells/s on an NVIDIA A800 (MicroMagnetic.jl and MuMax3, "
                            "Heun; whether steps or evaluations are counted is not stated)"}
    for n in inputs.HEUN_SIZES:
        w = inputs.heun_film(n)
        plan = mm.Plan(w["mesh"], "f32", terms=w["terms"])
        params = mm.make_params(terms=w["terms"], **w["params"])
        m = torch.tensor(inputs.heun_initial(n), dtype=torch.float32, device="cuda")
        plan.autotune(params, m)
        plan.heun_run(params, m, w["h"], 4)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        plan.heun_run(params, m, w["h"], steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        cells = n * n
        # algorithmic bytes of one step on an N x N x 1 film (FP32): two fused y
        # passes (spectrum in and out, tensor in), two inverse-x stage kernels
        # that read the spectrum and write the next input's spectrum, the
        # stage-1 epilogue (read m, write k1 and m1) and the stage-2 epilogue
        # (read m1, m, k1; write m): 8 sx + 2 K + 7 x 3wN
        Px, Py = plan.padded()[:2]
        Xp = Px // 2 + 1
        sx = 3 * Xp * n * 8
        K = 4 * Xp * (Py // 2 + 1) * 4
        b = 8 * sx + 2 * K + 7 * 3 * 4 * cells
        gbs = b / (ms / steps * 1e-3) / 1e9
        out[w["name"]] = {"steps": steps, "ms_per_step": ms / steps,
                          "cells_per_s": cells * steps / (ms * 1e-3),
                          "cell_evals_per_s": 2 * cells * steps / (ms * 1e-3),
                          "alg_bytes_per_step": b, "achieved_gbs": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "launch_shapes": plan.shapes()}
        del plan
    return out


def padding_bench(mm, inputs, torch, sizes=(96, 192), reps=20):
    """Padded-grid choice by measurement (mm_plan_tune_padding) on sweep meshes
    n x n x 2 (2 nm cells, the sweep's terms) whose default 3-smooth grid has a
    power-of-two alternative (n = 96: 192 or 256 along x and y): dm/dt evaluation
    time (sum of the passes in evaluation order) at the default grid and at the
    grid kept."""
    import numpy as np
    w = inputs.workload(4)
    terms = w["terms"]
    p = mm.make_params(terms=terms, Ms=8e5, A=1.3e-11, D=1e-3, Ku=2e5, u=(0, 0, 1), H=(1e4, 0, 5e4), alpha=0.1)
    out = []
    for n in sizes:
        mesh = (n, n, 2, 2e-9, 2e-9, 2e-9)
        plan = mm.Plan(mesh, "f32", terms=terms)
        m = torch.tensor(inputs.random_unit(n, n, 2, np.random.default_rng(n)), dtype=torch.float32, device="cuda")
        P0 = plan.padded()
        t0 = sum(plan.profile_passes(p, m, reps=reps, in_order=True)[1])
        P1 = plan.tune_padding(p, m, reps=reps)
        t1 = sum(plan.profile_passes(p, m, reps=reps, in_order=True)[1])
        out.append({"mesh": [n, n, 2], "default_padded": list(P0), "eval_us_default": round(t0, 2),
                    "kept_padded": list(P1), "eval_us_kept": round(t1, 2)})
        del plan
    return out


def sd_bench(mm, inputs, torch, iters=200):
    """Steepest-descent (Barzilai-Borwein) relaxation of the 256x256x1 thin film
    (all five terms, FP32): iterations per second and cells x iterations / s
    (one field evaluation per iteration), m resident in HBM."""
    w = inputs.workload(1)
    plan = mm.Plan(w["mesh"], "f32", terms=w["terms"])
    params = mm.make_params(terms=w["terms"], **w["params"])
    m = torch.tensor(inputs.initial_state(1), dtype=torch.float32, device="cuda")
    plan.autotune(params, m)
    plan.sd_run(params, m.clone(), 4, 1e-7, 1e-10, 1e-3)
    t0 = time.perf_counter()
    tau = plan.sd_run(params, m, iters, 1e-7, 1e-10, 1e-3)  # synchronises
    s = time.perf_counter() - t0
    cells = w["mesh"][0] * w["mesh"][1]
    return {"workload": "sd-" + w["name"], "iterations": iters, "ms_per_iteration": 1e3 * s / iters,
            "cell_iterations_per_s": cells * iters / s, "last_tau": float(tau[0])}


def potential_bench(mm, inputs, torch, newell=None, reps=30):
    """The 512 x 512 x 16 slab's dm/dt through the scalar potential (three
    forward transforms and one inverse, FP32) next to the Newell route's
    evaluation: back-to-back pass times, algorithmic bytes and the fraction of
    8 TB/s, and the relative RMS difference of the two demag fields (a
    discretisation difference that shrinks with the cell size, not an error)."""
    w = inputs.workload(2)
    mesh = tuple(w["mesh"])
    terms = (w["terms"] & ~mm.DEMAG) | mm.DEMAG_POTENTIAL
    plan = mm.Plan(mesh, "f32", terms=terms)
    params = mm.make_params(terms=terms, **w["params"])
    m = torch.tensor(inputs.initial_state(2, mesh), dtype=torch.float32, device="cuda")
    from paper_2406_16064_amd import tuned
    sh = tuned.lookup(mesh, "f32")  # the slab's shapes of the forward passes and tiles
    if sh is not None:
        plan.set_shapes(sh)
    us_b2b, us = plan.profile_passes(params, m, reps=reps, in_order=True)
    pb = pot_pass_bytes(mesh, plan.padded(), 4)
    passes = [{"kernel": n, "us": round(t, 3), "alg_bytes": b, "gbs": round(b / (t * 1e-6) / 1e9, 1),
               "us_back_to_back": round(t2, 3)} for n, t, t2, b in zip(POT_PASSES, us, us_b2b, pb)]
    b, t = sum(pb), sum(us)
    out = {"workload": "potential-" + w["name"], "padded": list(plan.padded()), "passes": passes,
           "launch_shapes": plan.shapes(),
           "eval_us": round(t, 3), "alg_bytes": b, "achieved_gbs": round(b / (t * 1e-6) / 1e9, 1),
           "frac": round(b / (t * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
           "cell_evals_per_s": mesh[0] * mesh[1] * mesh[2] / (t * 1e-6)}
    # adaptive Dormand-Prince attempts on the route (the headline's step, with
    # the potential passes in every stage), timed as the headline is
    st = mm.new_states(1, rtol=w["rtol"])
    mr = m.clone()  # the field comparison below uses the initial state
    s = plan.rk45_run(params, mr, st, t_end=w["t_end"], max_steps=8, check=False)
    if s not in (mm.MM_OK, mm.MM_E_MAXSTEPS):
        raise RuntimeError("potential-route warmup failed: %s" % mm.status_string(s))
    n0, a0 = st[0].n_rhs, st[0].n_accept + st[0].n_reject
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    s = plan.rk45_run(params, mr, st, t_end=w["t_end"], max_steps=16, check=False)
    e1.record()
    torch.cuda.synchronize()
    if s not in (mm.MM_OK, mm.MM_E_MAXSTEPS):
        raise RuntimeError("potential-route run failed: %s" % mm.status_string(s))
    ms = e0.elapsed_time(e1)
    att = st[0].n_accept + st[0].n_reject - a0
    out["rk45"] = {"attempts": att, "ms_per_step": ms / max(att, 1),
                   "cell_evals_per_s": mesh[0] * mesh[1] * mesh[2] * (st[0].n_rhs - n0) / (ms * 1e-3)}
    if newell is not None:
        out["rk45"]["speedup_over_newell"] = round(newell["ms_per_step"] / out["rk45"]["ms_per_step"], 3)
    # the demag fields of the two routes on this state
    pd = mm.Plan(mesh, "f32", terms=mm.DEMAG_POTENTIAL)
    Hp = pd.effective_field(mm.make_params(terms=mm.DEMAG_POTENTIAL, **w["params"]), m)
    del pd
    pn = mm.Plan(mesh, "f32", terms=mm.DEMAG)
    Hn = pn.effective_field(mm.make_params(terms=mm.DEMAG, **w["params"]), m)
    del pn
    out["demag_rms_difference_vs_newell"] = float(torch.sqrt(torch.mean((Hp - Hn) ** 2) / torch.mean(Hn ** 2)))
    if newell is not None:
        out["newell_eval_us"] = newell["eval_us"]
        out["newell_alg_bytes"] = newell["demag_pipeline"]["alg_bytes"]
        out["speedup_over_newell"] = round(newell["eval_us"] / t, 3)
        out["byte_ratio_to_newell"] = round(b / newell["demag_pipeline"]["alg_bytes"], 3)
    return out


def roofline(res, workload):
    """Roofline of the kernel that takes the most time per adaptive attempt
    (launches per attempt x launch duration, from whole attempts timed in their
    own order with HIP events on the launch stream)."""
    dom = max(res["attempt_kernels"], key=lambda p: p["us_per_attempt"])
    ach = dom["gbs"]
    launch = None
    sh = res.get("launch_shapes")
    if dom["kernel"].startswith("x_inv") and sh:  # the inverse x kernels' grid follows ty_x / nt_i
        mesh = res["mesh"]
        launch = "grid %d, workgroup %d," % (mesh[2] * -(-mesh[1] // sh["ty_x"]) * sh["nt_i"], sh["nt_i"])
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic(workload, dom["kernel"], launch),
            "kernel": dom["kernel"], "alg_bytes_per_launch": dom["alg_bytes"], "us_per_launch": dom["us"],
            "launches_per_attempt": dom["per_attempt"], "share_of_attempt": round(
                dom["us_per_attempt"] / res["attempt_kernel_us"], 3),
            "us_per_launch_back_to_back": dom.get("us_back_to_back")}


def demag_pipeline(res):
    """Every pass of one dm/dt evaluation: the demag FFT passes (forward x, y, z
    with the tensor product, inverse y) and the inverse-x complex-to-real pass,
    which also holds the local terms and the LL epilogue (its bytes: read the x
    spectrum and m, write dm/dt).  Algorithmic bytes over the summed pass
    times of whole evaluations timed in their own order."""
    names = tuple(p["kernel"] for p in res["passes"])
    ps = res["passes"]
    b = sum(p["alg_bytes"] for p in ps)
    us = sum(p["us"] for p in ps)
    gbs = b / (us * 1e-6) / 1e9
    return {"passes": list(names), "alg_bytes": b, "us": round(us, 3), "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def load_traffic(workload, kernel, launch=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the summary is missing, the kernels changed since it was taken,
    or the counters were read at another launch shape than `launch`
    ("grid G, workgroup W," of this run, when given)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    rec = d.get("workloads", {}).get(workload, {}).get(kernel)
    if rec is None:
        return None
    if launch and "launch" in rec:
        for sig, r in rec.get("by_launch", {rec["launch"]: rec}).items():
            if sig.startswith(launch):
                return r.get("bytes_per_launch")
        return None
    return rec.get("bytes_per_launch")


# kernel-name fragments of each pass in rocprofv3 output
# (the y passes: kernels compiled for one length, k_*_s, or the general ones)
PASS_KERNELS = {"x_fwd": ("k_fwd_x<",), "y_fused_product": ("k_ypass_s<", "k_ypass<"),
                "y_fwd": ("k_ypass_s<", "k_ypass<"),
                "z_product": ("k_z3d_reg_half<", "k_z3d_reg<", "k_z3d_s<", "k_z3d_pair<", "k_z3d<"),
                "y_inv": ("k_yinv_s<", "k_yinv<"), "x_inv_fused_llg": ("k_inv_x<",)}
COPY_BYTES = 1 << 30


def copy_reference(torch):
    """Plain device-to-device copies of COPY_BYTES: the reference the HBM
    counters are scaled by (bytes read = bytes written = COPY_BYTES each)."""
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes": COPY_BYTES, "copies": 5}


def copy_bandwidth(torch, reps=10):
    """Attainable HBM bandwidth: a plain 1 GiB device-to-device copy (torch's copy
    kernel), bytes read + written per second, best of `reps` timed with events."""
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * COPY_BYTES / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return round(best, 1)


def _counter_rows(path, full=False):
    """Kernel name -> counter values in dispatch order (full: also the launch
    signature (grid, workgroup, LDS) of each dispatch)."""
    import csv
    rows = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            v = float(r["Counter_Value"])
            if full:
                v = (v, (r["Grid_Size"], r["Workgroup_Size"], r["LDS_Block_Size"]))
            rows.setdefault(r["Kernel_Name"], []).append(v)
    return rows


def ingest_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, workload, reps, mesh_nz):
    """Per-launch HBM bytes of each pass from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    (KiB per dispatch; the last `reps` dispatches of each kernel are the timed
    dm/dt evaluations), scaled by what the same counters read for a copy of
    COPY_BYTES.  Writes profiles/traffic_counters.json for this source hash."""
    cf = _counter_rows(copy_fetch_csv)
    cw = _counter_rows(copy_write_csv)
    big_f = max(v for k, vs in cf.items() if "copyBuffer" in k for v in vs)
    big_w = max(v for k, vs in cw.items() if "copyBuffer" in k for v in vs)
    kf = COPY_BYTES / (big_f * 1024.0)
    kw = COPY_BYTES / (big_w * 1024.0)
    fr = _counter_rows(fetch_csv)
    wr = _counter_rows(write_csv)
    out = {}

    def per_launch(f, w):
        fb = sum(f) / len(f) * 1024.0 * kf
        wb = sum(w) / len(w) * 1024.0 * kw
        return {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb}

    for name in pass_names(mesh_nz):
        frags = PASS_KERNELS[name]
        if name == "x_inv_fused_llg":  # the dm/dt (MODE_RHS = 1) instance with the demag transform
            keys = [k for k in fr if frags[0] in k and ", true, 1," in k and k.split("(")[0].endswith("false>")]
        else:
            keys = [k for f in frags for k in fr if f in k]
        # read in both runs; the instantiation the timed run used is the one
        # launched most (graph replays and the pass timings)
        keys = [k for k in keys if k in wr]
        if not keys:
            continue
        k = max(keys, key=lambda kk: len(fr[kk]))
        out[name] = dict(kernel=k, **per_launch(fr[k][-reps:], wr[k][-reps:]))
    # the attempt-only kernels, per instantiation and launch shape read in both
    # runs (the autotuner's candidates included); the headline record is the
    # shape launched most (the autotuner's pick: the stage kernel runs stages
    # 2..6 in equal numbers in the graph replays and in the step timing)
    frf = _counter_rows(fetch_csv, True)
    wrf = _counter_rows(write_csv, True)
    def inv_x_args(k):  # k_inv_x<T, demag, mode, cells per thread, fused, cell material>
        if "k_inv_x<" not in k:
            return [None] * 6
        a = [x.strip() for x in k.split("k_inv_x<", 1)[1].split(">", 1)[0].split(",")]
        return a + ["false"] * (6 - len(a))  # builds without the cell-material argument

    def is_stage(k, fused):
        a = inv_x_args(k)
        return a[1:3] == ["true", "2"] and a[4] == ("true" if fused else "false") and a[5] == "false"

    step_kinds = {"step_begin": lambda k: "k_begin<" in k,
                  "x_inv_stage": lambda k: is_stage(k, False),
                  "x_inv_stage_fused_fwd": lambda k: is_stage(k, True),
                  "x_inv_error": lambda k: inv_x_args(k)[1:3] == ["true", "3"] and inv_x_args(k)[5] == "false"}
    for name, sel in step_kinds.items():
        combos = {}
        for src, col in ((frf, 0), (wrf, 1)):
            for k, vs in src.items():
                if sel(k):
                    for v, g in vs:
                        combos.setdefault((k, g), ([], []))[col].append(v)
        both = {kg: fw for kg, fw in combos.items() if fw[0] and fw[1]}
        if not both:
            continue
        sig = lambda g: "grid %s, workgroup %s, LDS %s" % g
        by = {sig(g): dict(kernel=k, dispatches=len(f), **per_launch(f, w)) for (k, g), (f, w) in both.items()}
        k, g = max(both, key=lambda kg: len(both[kg][0]))
        out[name] = dict(by[sig(g)], launch=sig(g), by_launch=by)
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    d = {}
    if os.path.exists(path):
        try:
            d = json.load(open(path))
        except ValueError:
            d = {}
    if d.get("source_hash") != source_hash():
        d = {"source_hash": source_hash(), "workloads": {}}
    d["calibration"] = {"copy_bytes": COPY_BYTES, "fetch_kib": big_f, "write_kib": big_w,
                        "fetch_scale": kf, "write_scale": kw}
    d["workloads"][workload] = out
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    return d


def oracle_workers():
    """Host threads / processes the oracle may use: the machine's CPU share for one GPU
    (16) at most, whatever os.cpu_count() reports."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(inputs, idx=2, budget_s=12.0, budget1_s=8.0):
    """The FP64 oracle's dm/dt evaluation of workload idx timed on this host, as it
    stands: NumPy elementwise work (single-threaded) and scipy.fft with
    `workers` threads (also a one-worker figure).  The tensor setup (the Newell
    grid in worker processes, its spectrum) is not timed.  Median evaluation
    time over at least 5 (one worker: 2) evaluations after one warm-up."""
    import numpy as np
    import scipy.fft
    from oracle import fields as F
    from oracle import newell
    w = inputs.workload(idx)
    mesh = tuple(w["mesh"])
    p = F.Params(terms=w["terms"], **w["params"])
    msh = F.Mesh(*mesh)
    nw = oracle_workers()
    t0 = time.perf_counter()
    grid = newell.tensor_grid(msh.nx, msh.ny, msh.nz, msh.dx, msh.dy, msh.dz, workers=nw)
    with scipy.fft.set_workers(nw):
        kern = F.DemagKernel(msh, grid=grid)
    del grid
    setup = time.perf_counter() - t0
    m = inputs.initial_state(idx)

    def timed(workers, budget, n_min):
        ts = []
        with scipy.fft.set_workers(workers):
            F.llg_rhs(m, msh, p, kern)
            t_all = time.perf_counter()
            while len(ts) < n_min or time.perf_counter() - t_all < budget:
                t = time.perf_counter()
                F.llg_rhs(m, msh, p, kern)
                ts.append(time.perf_counter() - t)
        return float(np.median(ts)), len(ts)

    tm, n = timed(nw, budget_s, 5)
    t1, n1 = timed(1, budget1_s, 2)
    N = mesh[0] * mesh[1] * mesh[2]
    one = {"value": N / t1, "unit": "cell-evals/s", "cores": 1, "evaluations": n1, "median_s": t1}
    return {"value": N / tm, "unit": "cell-evals/s", "cores": nw, "kind": "oracle",
            "sample": "median of %d dm/dt evaluations of the %s mesh (%dx%dx%d) after one warm-up, %.2f s each; "
                      "scipy.fft with %d workers, NumPy elementwise work single-threaded (os.cpu_count() = %s); "
                      "one worker: %.2f s per evaluation; tensor setup %.1f s in %d processes, not timed"
                      % (n, w["name"], mesh[0], mesh[1], mesh[2], tm, nw, os.cpu_count(), t1, setup, nw),
            "one_worker": one}, kern


def field_error(mm, torch, plan, params, inputs, idx, kern):
    """max-norm relative error of the FP32 effective field of workload idx's initial
    state (rounded to FP32, the oracle's input) against the oracle."""
    import numpy as np
    from oracle import fields as F
    w = inputs.workload(idx)
    m = torch.tensor(inputs.initial_state(idx), dtype=torch.float32)
    H = plan.effective_field(params, m.cuda()).cpu().double().numpy()
    ref = F.effective_field(m.double().numpy(), F.Mesh(*w["mesh"]), F.Params(terms=w["terms"], **w["params"]),
                            kern)
    d = np.sqrt(np.sum((H - ref) ** 2, axis=0))
    return float(np.max(d) / np.max(np.sqrt(np.sum(ref ** 2, axis=0))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--only", choices=["slab3d", "slab3d_f64", "thinfilm", "copy", "heun", "sd", "sweep", "neb",
                                       "potential", "padding", "sp4"],
                    default=None,
                    help="profiling aids: slab3d (slab3d_f64) runs only the 512x512x16 slab in FP32 (FP64), "
                         "thinfilm only the 256x256x1 film in FP32, and prints its record; copy runs only the "
                         "plain 1 GiB copies the HBM counters are scaled by; heun, sd, sweep, neb, potential, "
                         "padding, sp4 run "
                         "only that record")
    ap.add_argument("--retune", default=None, metavar="TABLE",
                    help="autotune the launch shapes of the workloads run and store them in the table file TABLE")
    ap.add_argument("--ingest-counters", nargs=5, default=None,
                    metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="turn rocprofv3 FETCH_SIZE/WRITE_SIZE counter files into per-launch HBM bytes "
                         "(profiles/traffic_counters.json); WORKLOAD is thinfilm_f32 or slab3d_f32")
    args = ap.parse_args()
    if args.ingest_counters:
        wl, fcsv, wcsv, cfcsv, cwcsv = args.ingest_counters
        d = ingest_counters(fcsv, wcsv, cfcsv, cwcsv, wl, 30, 16 if wl.startswith("slab") else 1)
        print(json.dumps(d, indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2406_16064_amd import inputs
    from paper_2406_16064_amd import mm

    torch.cuda.set_device(0)
    rt = args.retune
    if args.only == "copy":
        print(json.dumps(copy_reference(torch)))
        return
    if args.only == "heun":
        print(json.dumps(heun_bench(mm, inputs, torch, args.steps)))
        return
    if args.only == "sd":
        print(json.dumps(sd_bench(mm, inputs, torch)))
        return
    if args.only == "sweep":
        print(json.dumps(sweep_bench(mm, inputs, torch)))
        return
    if args.only == "neb":
        print(json.dumps(neb_bench(mm, inputs, torch)))
        return
    if args.only == "potential":
        print(json.dumps(potential_bench(mm, inputs, torch)))
        return
    if args.only == "sp4":
        print(json.dumps(sp4_bench(mm, inputs, torch)))
        return
    if args.only == "padding":
        print(json.dumps(padding_bench(mm, inputs, torch)))
        return
    if args.only in ("slab3d", "slab3d_f64", "thinfilm"):
        idx = 1 if args.only == "thinfilm" else 2
        r, *_ = run_workload(mm, inputs, torch, idx, "f64" if args.only == "slab3d_f64" else "f32", args.steps,
                             args.warmup, retune=rt)
        r["demag_pipeline"] = demag_pipeline(r)
        print(json.dumps(r))
        return
    print("bench: 3d slab fp32", file=sys.stderr, flush=True)
    res, plan, params, m, mesh = run_workload(mm, inputs, torch, 2, "f32", args.steps, args.warmup, retune=rt)
    res["demag_pipeline"] = demag_pipeline(res)
    extra = {}
    if not args.no_extra:
        print("bench: 3d slab fp64", file=sys.stderr, flush=True)
        r64, *_ = run_workload(mm, inputs, torch, 2, "f64", max(8, args.steps // 2), 8, retune=rt)
        r64["demag_pipeline"] = demag_pipeline(r64)
        extra["slab3d_f64"] = r64
        extra["fp32_over_fp64"] = res["cell_evals_per_s"] / r64["cell_evals_per_s"]
        for prec in ("f32", "f64"):
            print("bench: thin film %s" % prec, file=sys.stderr, flush=True)
            rt_, *_ = run_workload(mm, inputs, torch, 1, prec, 48 if prec == "f32" else 24, 16, retune=rt)
            rt_["demag_pipeline"] = demag_pipeline(rt_)
            extra["thinfilm_" + prec] = rt_
        extra["thinfilm_fp32_over_fp64"] = (extra["thinfilm_f32"]["cell_evals_per_s"] /
                                            extra["thinfilm_f64"]["cell_evals_per_s"])
        extra["thinfilm_f32"]["roofline"] = roofline(extra["thinfilm_f32"], "thinfilm_f32")
        print("bench: sweep batched vs one by one", file=sys.stderr, flush=True)
        extra["sweep"] = sweep_bench(mm, inputs, torch)
        print("bench: neb", file=sys.stderr, flush=True)
        extra["neb"] = neb_bench(mm, inputs, torch)
        print("bench: heun", file=sys.stderr, flush=True)
        extra["heun"] = heun_bench(mm, inputs, torch)
        print("bench: steepest descent", file=sys.stderr, flush=True)
        extra["sd"] = sd_bench(mm, inputs, torch)
        print("bench: standard problem 4", file=sys.stderr, flush=True)
        extra["sp4"] = sp4_bench(mm, inputs, torch)
        print("bench: padded-grid choice", file=sys.stderr, flush=True)
        extra["padding"] = padding_bench(mm, inputs, torch)
        print("bench: scalar-potential demag", file=sys.stderr, flush=True)
        extra["potential_f32"] = potential_bench(mm, inputs, torch, newell=res)
    cpu = None
    if not args.no_cpu:
        print("bench: cpu oracle", file=sys.stderr, flush=True)
        cpu, kern = cpu_baseline(inputs, 2)
        print("bench: fp32 field error", file=sys.stderr, flush=True)
        extra["field_rel_err_f32"] = field_error(mm, torch, plan, params, inputs, 2, kern)
        del kern
    rl = roofline(res, "slab3d_f32")
    # fractions of the attainable bandwidth (a plain copy) next to those of the spec peak
    cbw = copy_bandwidth(torch)
    extra["copy_gbs"] = cbw
    rl["frac_of_copy"] = round(rl["achieved"] / cbw, 4)
    dps = [res["demag_pipeline"]] + [extra[k]["demag_pipeline"] for k in ("slab3d_f64", "thinfilm_f32",
                                                                          "thinfilm_f64") if k in extra]
    for dp in dps:
        dp["copy_gbs"] = cbw
        dp["frac_of_copy"] = round(dp["achieved"] / cbw, 4)
    if "thinfilm_f32" in extra:
        extra["thinfilm_f32"]["roofline"]["frac_of_copy"] = round(
            extra["thinfilm_f32"]["roofline"]["achieved"] / cbw, 4)
    line = {
        "metric": METRIC,
        "value": res["cell_evals_per_s"],
        "unit": "cell-evals/s",
        "n_gpus": 1,
        "steps": res["steps"],
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3d-512x512x16 fp32, adaptive Dormand-Prince (rtol 1e-6), exchange+demag+Zeeman "
                               "(25 mT at 170 deg in plane), S-state + 1e-2 noise",
                   "mesh": list(mesh), "padded": res["padded"], "cells": mesh[0] * mesh[1] * mesh[2],
                   "rhs_evals_timed": res["rhs_evals"]},
        "roofline": rl,
        "cpu_baseline": cpu,
        "demag_pipeline": res["demag_pipeline"],
        "passes": res["passes"],
        "attempt_kernels": res["attempt_kernels"],
        "launch_shapes": res["launch_shapes"],
        "launch_shapes_source": res["launch_shapes_source"],
        "extra": extra,
        "source_hash": source_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
