"""Benchmark of the WENO-ZN hot path on one MI355X.

Default workload: 1D Euler, component-wise global Lax-Friedrichs WENO-ZN, N = 2^20 cells on
[-5, 5] (Shu-Osher-like data), transmissive boundaries, fp64, TVD-RK3 at CFL 0.5.  One
"step" is one TVD-RK3 step (three fused stage kernels: BC map, flux, LF split, WENO-ZN
reconstruction of every interface, flux difference, stage combination, and the max wave
speed for the next stage's alpha / next step's dt).  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--graph] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# launch-shape layouts of the 1D stage kernel (wzn_set_row_tuning)
LAYOUT_NAMES = {0: "tile", 1: "split"}
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X fp64 vector (FMA = 2 flop)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Sources each profiled kernel is built from: a committed counter profile is used only while
# the hash of these files is the one it was taken on.
ROW_KERNEL_SOURCES = ("wzn_rows.hip", "wzn_rows.hpp", "wzn_tile.hpp", "wzn_device.hpp",
                      "wzn_1d.hip", "wzn_host.hpp")
CHAR_KERNEL_SOURCES = ("wzn_char.hip", "wzn_rows.hpp", "wzn_tile.hpp", "wzn_device.hpp",
                       "wzn_host.hpp")
EULER2D_KERNEL_SOURCES = ("wzn_2d.hip", "wzn_rows.hip", "wzn_rows.hpp", "wzn_tile.hpp",
                          "wzn_device.hpp", "wzn_host.hpp")
CHAR2D_KERNEL_SOURCES = ("wzn_char2d.hip", "wzn_rows.hpp", "wzn_tile.hpp", "wzn_device.hpp",
                         "wzn_host.hpp")
VJP_KERNEL_SOURCES = ("wzn_vjp.hip", "wzn_rows.hpp", "wzn_tile.hpp", "wzn_device.hpp",
                      "wzn_host.hpp")


def kernel_source_hash(files):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2004_07954_amd", "csrc")
    for f in sorted(files):
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def committed_profile(kind, kernel, workload, key, sources):
    """A figure from a committed rocprofv3 --pmc summary (profiles/<kind>_<kernel>_<workload>.md,
    line '<KIND>_JSON {...}'), if it was taken on the kernel's current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s.md" % (kind, kernel, workload))
    if not os.path.exists(path):
        return None
    rec = None
    tag = kind.upper() + "_JSON "
    for line in open(path):
        if line.startswith(tag):
            rec = json.loads(line[len(tag):])
    if rec is None or rec.get("source_hash") != kernel_source_hash(sources):
        return None
    return rec.get(key)


# Algorithmic fp64 flops of one 1D Euler cell-stage, counted on the scheme's literal formulas
# (+, -, *, / and a square root one flop each): 6 reconstructions of 86 (indicators 33, tau5 1,
# tau8 8, C 7, alpha 12, normalisation 5, candidate polynomials 15, combination 5), flux 10,
# Lax-Friedrichs split 15, flux difference 9, stage combination 12 (mean of 6, 15, 15) and
# the wave speed for the next alpha and dt 11.
FLOPS_PER_CELL_STAGE = 6 * 86 + 10 + 15 + 9 + 12 + 11
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9  # fp64 VALU lane-instructions/s (FMA = 1 instruction)


def cpu_baseline(n, budget_s=12.0, serial_budget_s=10.0):
    """The oracle as it stands, on the host cores, over a bounded sample of the same
    workload (whole RK3 steps at the full N): on every host core (the reported value), and
    serially on one core beside it."""
    import numpy as np  # noqa: F401
    from oracle import binding as orc
    from paper_2004_07954_amd import inputs as I
    u, dx = I.shu_osher_like(n)
    orc.lib()
    cores = orc.num_threads()

    def sample(budget):
        t0 = time.perf_counter()
        u1, _, _ = orc.rk3_run_1d(u, dx, 1, cfl=0.5)
        t1 = time.perf_counter() - t0
        steps = max(1, min(400, int(budget / max(t1, 1e-3))))
        t0 = time.perf_counter()
        orc.rk3_run_1d(u1, dx, steps, cfl=0.5)
        return steps, time.perf_counter() - t0

    steps, el = sample(budget_s)
    orc.set_num_threads(1)
    try:
        steps1, el1 = sample(serial_budget_s)
    finally:
        orc.set_num_threads(cores)
    return {"value": n * 3 * steps / el, "unit": "cell-RHS/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d TVD-RK3 steps (%d RHS evaluations) of the N=%d 1D Euler workload, "
                      "%.1f s" % (steps, 3 * steps, n, el),
            "serial": {"value": n * 3 * steps1 / el1, "unit": "cell-RHS/s", "cores": 1,
                       "sample": "%d TVD-RK3 steps at N=%d on one thread, %.1f s"
                                 % (steps1, n, el1)}}


def bench_2d(steps, dtype_name, warmup=3, split="lf"):
    """Secondary figure: 2D Euler dimension-by-dimension WENO-ZN, transmissive, CFL 0.5 (one
    step = row kernel + column kernel per stage): the global Lax-Friedrichs split on 4096^2
    four-quadrant data, or the paper's own setup, the Steger-Warming split on its second
    Riemann case at its finest grid, 2400^2 (Sec. 4.4)."""
    import torch
    from paper_2004_07954_amd import api, inputs as I
    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    if split == "sw":
        nx = ny = 2400
        u0, dx, dy = I.riemann_2d(2, nx)
        wl = "euler2d_riemann_case2_steger_warming_%dx%d" % (nx, ny)
    else:
        nx = ny = 4096
        u0, dx, dy = I.four_quadrant_random(nx, ny, seed=3)
        wl = "euler2d_four_quadrant_%dx%d" % (nx, ny)
    u0t = torch.tensor(u0, dtype=tdt, device="cuda")
    u = u0t.clone()
    stage = torch.empty((2, 4, ny, nx), dtype=tdt, device="cuda")
    prm = api.params("euler", dtype="fp64" if dtype_name == "f64" else "fp32",
                     eps=1e-40 if dtype_name == "f64" else 1e-30, split=split)
    api.rk3_run_2d(u, dx, dy, warmup, prm=prm, stage=stage)
    u.copy_(u0t)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    api.rk3_run_2d(u, dx, dy, steps, prm=prm, stage=stage)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    assert torch.isfinite(u).all().item()
    esz = 8 if dtype_name == "f64" else 4
    # algorithmic bytes per cell and stage of a fused stage: read U^(s) (+ U^n), write
    bytes_stage = nx * ny * 4 * esz * (2 + 3 + 3) / 3.0
    stage_ms = ms / (3 * steps)
    gbs = bytes_stage / (stage_ms * 1e-3) / 1e9
    rec = {"workload": wl, "dtype": dtype_name,
           "steps": steps, "ms_per_step": ms / steps,
           "value": nx * ny * 3 * steps / (ms * 1e-3), "unit": "cell-RHS/s",
           "stage_ms": stage_ms, "hbm_gbs_algorithmic": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    # VALU and measured-traffic side: the x sweep plus the column kernel per stage, from the
    # committed counter profile of the 2D kernels (Steger-Warming steps run the column kernel
    # with the wave-speed epilogue in their last stage only)
    sfx = "_" + dtype_name
    per_cell = meas = None
    v = committed_profile("counters", "euler2d", "kernels", "valu_per_cell",
                          EULER2D_KERNEL_SOURCES)
    hb = committed_profile("counters", "euler2d", "kernels", "hbm_bytes_per_cell",
                           EULER2D_KERNEL_SOURCES)

    def stage_mean(d):
        if split == "lf":
            return d["x_lf" + sfx] + d["col_lf" + sfx + "_speed"]
        return d["x_sw" + sfx] + (2 * d["col_sw" + sfx] + d["col_sw" + sfx + "_speed"]) / 3.0
    if v:
        per_cell = stage_mean(v)
    if hb:
        meas = stage_mean(hb)
    ach = per_cell * nx * ny / (stage_ms * 1e-3) if per_cell else None
    # fp32 VALU instructions issue at twice the fp64 rate (the vector peaks are 157.3 and
    # 78.6 TFLOP/s; the fp32 lines measure above the fp64 lane rate, so it is not the same)
    peak = VALU_LANE_PEAK * (2 if dtype_name == "f32" else 1)
    rec["roofline_alu"] = {"bound": "alu", "unit": "VALU lane-instr/s",
                           "valu_instr_per_cell_stage": per_cell, "achieved": ach,
                           "peak": peak, "frac": ach / peak if ach else None}
    rec["hbm_bytes_per_cell_stage_measured"] = meas
    return rec


def bench_batched(steps, baseline_sample=48, use_graph=True):
    """Secondary figure: 4096 independent 1D Euler shock tubes (N_i ~ U{256..16384}, seed 4)
    advanced by `steps` TVD-RK3 steps in one persistent launch (autotuned, longest first,
    captured in a HIP graph), against one launch per instance and stage (wzn_rk3_run_1d per
    instance, timed on a random sample of instances and scaled to the whole batch)."""
    import numpy as np
    import torch
    from paper_2004_07954_amd import api, autotune, inputs as I
    U, offs, dx = I.shock_tube_batch(4096, seed=4)
    lens = np.diff(offs)
    dev = "cuda"
    U0 = torch.tensor(U, dtype=torch.float64, device=dev)
    Ug = U0.clone()
    offg = torch.tensor(offs, dtype=torch.int64, device=dev)
    dxg = torch.tensor(dx, dtype=torch.float64, device=dev)
    order = api.lpt_order(lens)
    stage = torch.empty((2, 3, U.shape[1]), dtype=torch.float64, device=dev)
    tn, timings = autotune.tune_batched(Ug, offg, dxg, order=order, use_cache=False, log=log)
    log("batched tuning: nt=%d k=%d blocks/cu=%d" % (tn.nt, tn.k, tn.blocks_per_cu))
    graph = None
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            api.batched_rk3_run_1d(Ug, offg, dxg, steps, order=order, tuning=tn, stage=stage)
    Ug.copy_(U0)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    if graph is not None:
        graph.replay()
    else:
        api.batched_rk3_run_1d(Ug, offg, dxg, steps, order=order, tuning=tn, stage=stage)
    e.record()
    torch.cuda.synchronize()
    ms_batched = s.elapsed_time(e)
    # instances that lost positivity (a property of the scheme on this random batch: the CPU
    # oracle run of instance 1767 alone reaches rho < 0 too); counted, not hidden
    fin = torch.isfinite(Ug).all(dim=0).cpu().numpy()
    bad_inst = sorted(set((np.searchsorted(offs, np.nonzero(~fin)[0], side="right") - 1).tolist()))
    # baseline: one launch per instance and stage, on a random sample of instances
    pick = np.random.default_rng(11).choice(len(lens), baseline_sample, replace=False)
    singles = [torch.tensor(np.ascontiguousarray(U[:, offs[b]:offs[b + 1]]),
                            dtype=torch.float64, device=dev) for b in pick]
    st1 = [torch.empty((2,) + tuple(t.shape), dtype=torch.float64, device=dev) for t in singles]
    torch.cuda.synchronize()
    s.record()
    for t, stg, b in zip(singles, st1, pick):
        api.rk3_run_1d(t, float(dx[b]), steps, cfl=0.5, stage=stg)
    e.record()
    torch.cuda.synchronize()
    ms_sample = s.elapsed_time(e)
    ms_baseline = ms_sample * len(lens) / baseline_sample
    # the same per-instance launches captured in one HIP graph and replayed: the GPU time of
    # one launch per instance and stage without the host's launch cost
    pg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(pg):
        for t, stg, b in zip(singles, st1, pick):
            api.rk3_run_1d(t, float(dx[b]), steps, cfl=0.5, stage=stg)
    for t, b in zip(singles, pick):
        t.copy_(torch.tensor(np.ascontiguousarray(U[:, offs[b]:offs[b + 1]]),
                             dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    s.record()
    pg.replay()
    e.record()
    torch.cuda.synchronize()
    ms_sample_graph = s.elapsed_time(e)
    ms_baseline_graph = ms_sample_graph * len(lens) / baseline_sample
    cells = float(lens.sum())
    return {"workload": "batched_shock_tubes_B4096_seed4", "instances": int(len(lens)),
            "total_cells": int(cells), "steps": steps, "ms_batched": ms_batched,
            "value": cells * 3 * steps / (ms_batched * 1e-3), "unit": "cell-RHS/s",
            "tuning": {"nt": tn.nt, "k": tn.k, "blocks_per_cu": tn.blocks_per_cu,
                       "layout": "split" if tn.layout == 1 else "tile"},
            "launch": "hip_graph" if graph is not None else "stream",
            "baseline_ms_estimate": ms_baseline, "baseline_sample": baseline_sample,
            "baseline_sample_ms": ms_sample,
            "speedup_vs_one_launch_per_instance": ms_baseline / ms_batched,
            "baseline_graph_ms_estimate": ms_baseline_graph,
            "baseline_graph_sample_ms": ms_sample_graph,
            "speedup_vs_graph_launch_per_instance": ms_baseline_graph / ms_batched,
            "nonfinite_instances": bad_inst}


def bench_char(n, steps, warmup=3, cpu_steps=3):
    """Secondary figure: the paper's own 1D Euler setup (Sec. 4.3), WENO-ZN in local
    characteristic fields with per-field Lax-Friedrichs alphas, same data, grid and CFL as the
    headline workload.  The stage kernel is fp64-VALU bound: the roofline reports its
    measured VALU instructions per interface (committed counter profile) against the issue
    peak.  The oracle's characteristic run on the same grid is timed beside it."""
    import torch
    from paper_2004_07954_amd import api, inputs as I
    u0, dx = I.shu_osher_like(n)
    base = torch.tensor(u0, dtype=torch.float64, device="cuda")
    u = base.clone()
    stage = torch.empty((2, 3, n), dtype=torch.float64, device="cuda")
    api.rk3_run_1d_char(u, dx, warmup, cfl=0.5, stage=stage)
    u.copy_(base)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    api.rk3_run_1d_char(u, dx, steps, cfl=0.5, stage=stage)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    assert torch.isfinite(u).all().item() and u[0].min().item() > 0
    kernel_ms = ms / (3 * steps)
    workload = "euler1d_n%d" % n
    valu = committed_profile("valu", "char_kernel_256", workload, "valu_instr_per_cell",
                             CHAR_KERNEL_SOURCES)
    traffic = committed_profile("traffic", "char_kernel_256", workload, "hbm_bytes_per_launch",
                                CHAR_KERNEL_SOURCES)
    rec = {"workload": "euler1d_shu_osher_like_characteristic", "n_cells": n, "steps": steps,
           "ms_per_step": ms / steps, "value": n * 3 * steps / (ms * 1e-3),
           "unit": "cell-RHS/s", "kernel": "char_kernel<256, field-outer>",
           "kernel_ms": kernel_ms,
           "hbm_gbs_algorithmic": n * (48 + 72 + 72) / 3.0 / (kernel_ms * 1e-3) / 1e9,
           "hbm_bytes_per_launch_measured": traffic,
           "roofline": {"bound": "alu", "unit": "VALU lane-instr/s",
                        "valu_instr_per_cell_stage": valu,
                        "achieved": valu * n / (kernel_ms * 1e-3) if valu else None,
                        "peak": VALU_LANE_PEAK,
                        "frac": valu * n / (kernel_ms * 1e-3) / VALU_LANE_PEAK if valu else None}}
    if cpu_steps:
        from oracle import binding as orc
        t0 = time.perf_counter()
        orc.rk3_run_1d_char(u0, dx, cpu_steps, cfl=0.5)
        el = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": n * 3 * cpu_steps / el, "unit": "cell-RHS/s",
                               "cores": orc.num_threads(), "kind": "oracle",
                               "sample": "%d characteristic TVD-RK3 steps at N=%d, %.1f s"
                                         % (cpu_steps, n, el)}
    return rec


def bench_char2d(steps, warmup=3):
    """Secondary figure: 2D Euler with each sweep's reconstruction in local characteristic
    fields (the 1D procedure of Sec. 4.3 along x and y), on the paper's second Riemann case at
    2400^2, transmissive, CFL 0.5, fp64.  One stage = the column kernel (the y sweep) and the
    x sweep with the stage epilogue."""
    import torch
    from paper_2004_07954_amd import api, inputs as I
    nx = ny = 2400
    u0, dx, dy = I.riemann_2d(2, nx)
    u0t = torch.tensor(u0, dtype=torch.float64, device="cuda")
    u = u0t.clone()
    stage = torch.empty((2, 4, ny, nx), dtype=torch.float64, device="cuda")
    work = torch.empty(4 * nx * ny, dtype=torch.float64, device="cuda")
    api.rk3_run_2d_char(u, dx, dy, warmup, stage=stage, work=work)
    u.copy_(u0t)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    api.rk3_run_2d_char(u, dx, dy, steps, stage=stage, work=work)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    assert torch.isfinite(u).all().item()
    stage_ms = ms / (3 * steps)
    # algorithmic bytes per cell and stage: the y sweep (read U, write its part of L), the
    # fused x sweep (read U and the y part, U^n in stages 2 and 3, write the stage output)
    alg = 4 * 8 * (2 + (2 + 3 + 3) / 3.0 + 1)
    rec = {"workload": "euler2d_riemann_case2_characteristic_%dx%d" % (nx, ny), "dtype": "f64",
           "steps": steps, "ms_per_step": ms / steps,
           "value": nx * ny * 3 * steps / (ms * 1e-3), "unit": "cell-RHS/s",
           "stage_ms": stage_ms,
           "hbm_gbs_algorithmic": alg * nx * ny / (stage_ms * 1e-3) / 1e9,
           "hbm_bytes_per_cell_stage_algorithmic": alg}
    rec["hbm_frac"] = rec["hbm_gbs_algorithmic"] / HBM_PEAK_GBS
    c = committed_profile("counters", "char2d", "kernels_riemann2_2400", "stage_valu_per_cell",
                          CHAR2D_KERNEL_SOURCES)
    b = committed_profile("counters", "char2d", "kernels_riemann2_2400",
                          "stage_hbm_bytes_per_cell", CHAR2D_KERNEL_SOURCES)
    ach = c * nx * ny / (stage_ms * 1e-3) if c else None
    rec["roofline_alu"] = {"bound": "alu", "unit": "VALU lane-instr/s",
                           "valu_instr_per_cell_stage": c, "achieved": ach,
                           "peak": VALU_LANE_PEAK, "frac": ach / VALU_LANE_PEAK if ach else None}
    rec["hbm_bytes_per_cell_stage_measured"] = b
    return rec


def bench_strip(evals=100):
    """Secondary figure: one GPU's share of a row decomposition of the 4096^2 grid over eight
    GPUs, a 4096 x 512 strip (fp64, Lax-Friedrichs), its right-hand side with ghost rows and
    the global alphas supplied (wzn_rhs_2d_strip), against the whole-grid right-hand side on
    this GPU.  The halo a neighbour would send per stage is 3 rows x 4096 x 4 x 8 B each way."""
    import torch
    from paper_2004_07954_amd import api, inputs as I
    U, dx, dy = I.four_quadrant_random(4096, 4096, seed=3)
    full = torch.tensor(U, dtype=torch.float64, device="cuda")
    r0, r1 = 1536, 2048
    strip = full[:, r0:r1].contiguous()
    lo, hi = full[:, r0 - 3:r0].contiguous(), full[:, r1:r1 + 3].contiguous()
    alpha2 = api.speed_max_2d(full)
    out = torch.empty_like(strip)
    outf = torch.empty_like(full)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(n):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / n

    ms_strip = timed(lambda: api.rhs_2d_strip(strip, lo, hi, dx, dy, alpha2=alpha2, out=out),
                     evals)
    ms_full = timed(lambda: api.rhs_2d(full, dx, dy, out=outf), max(1, evals // 8))
    cells = 4096 * (r1 - r0)
    return {"workload": "euler2d_strip_4096x512_of_4096x4096", "dtype": "f64",
            "rhs_evals": evals, "ms_per_rhs": ms_strip,
            "value": cells / (ms_strip * 1e-3), "unit": "cell-RHS/s",
            "whole_grid_ms_per_rhs": ms_full,
            "whole_grid_value": 4096 * 4096 / (ms_full * 1e-3),
            "halo_bytes_per_neighbour_per_stage": 3 * 4096 * 4 * 8}


def bench_large_1d(n=1 << 25, steps=20):
    """Secondary figure: the 1D stage at N = 2^25 (805 MB per state, 2.4 GB in flight), where
    the working set cannot stay in the 256 MB Infinity Cache, against the headline's 2^20."""
    import torch
    from paper_2004_07954_amd import api, inputs as I
    u0, dx = I.shu_osher_like(n)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    del u0
    stage = torch.empty((2, 3, n), dtype=torch.float64, device="cuda")
    api.rk3_run_1d(u, dx, 2, cfl=0.5, stage=stage)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    api.rk3_run_1d(u, dx, steps, cfl=0.5, stage=stage)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    assert torch.isfinite(u).all().item()
    stage_ms = ms / (3 * steps)
    gbs = n * 64.0 / (stage_ms * 1e-3) / 1e9
    return {"workload": "euler1d_shu_osher_like_n%d" % n, "steps": steps,
            "value": n * 3 * steps / (ms * 1e-3), "unit": "cell-RHS/s",
            "stage_ms": stage_ms, "hbm_gbs_algorithmic": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "launch_shape": list(__import__("paper_2004_07954_amd.autotune",
                                            fromlist=["x"]).get_row_tuning(3, n))}


def bench_adjoint(n=65536, nsteps=400, ckpt=20, reps=3):
    """Secondary figure: the discrete adjoint of a periodic 1D Euler run (N = 65536, 400 steps,
    checkpoints every 20; loss 1/2 ||rho_T - rho_target||^2).  Reports the forward time (run
    with checkpoints and the recorded schedule) and the backward time (segment recomputation
    plus the adjoint kernels), medians of `reps` repetitions."""
    import numpy as np
    import torch
    from paper_2004_07954_amd import adjoint, api, inputs as I
    u0, ut, dx = I.adjoint_case(n=n, seed=5)
    U0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    rho_t = torch.tensor(ut[0], dtype=torch.float64, device="cuda")
    prm = api.params("euler", bc="periodic")
    fw, bw = [], []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        UT, dts, als, ckpts = adjoint.forward_checkpointed(U0, dx, nsteps, 0.5, prm, ckpt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lamT = torch.zeros_like(UT)
        lamT[0] = UT[0] - rho_t
        lam0 = adjoint.backward_checkpointed(lamT, dx, dts, als, ckpts, ckpt, prm)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fw.append(t1 - t0)
        bw.append(t2 - t1)
    fw, bw = float(np.median(fw[1:])), float(np.median(bw[1:]))
    assert torch.isfinite(lam0).all().item()
    # the same passes captured once in HIP graphs and replayed: GPU time without the host's
    # per-kernel launch cost (a stage kernel at this N runs about as long as its launch takes)
    cap = adjoint.CapturedAdjoint(U0, dx, nsteps, 0.5, prm, ckpt)
    fg, bg = [], []
    for _ in range(reps + 1):
        s0, s1, s2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        s0.record()
        UTg = cap.forward(U0)
        s1.record()
        lamTg = torch.zeros_like(UTg)
        lamTg[0] = UTg[0] - rho_t
        torch.cuda.synchronize()
        s1b = torch.cuda.Event(enable_timing=True)
        s1b.record()
        lamg = cap.backward(lamTg)
        s2.record()
        torch.cuda.synchronize()
        fg.append(s0.elapsed_time(s1))
        bg.append(s1b.elapsed_time(s2))
    fg, bg = float(np.median(fg[1:])), float(np.median(bg[1:]))
    return {"workload": "adjoint_euler1d_periodic_n%d_%dsteps_ckpt%d" % (n, nsteps, ckpt),
            "forward_ms": fw * 1e3, "backward_ms": bw * 1e3, "adjoint_fwd_ratio": bw / fw,
            "timing": "host wall clock around synchronised GPU work, median of %d" % reps,
            "forward_ms_graph": fg, "backward_ms_graph": bg, "adjoint_fwd_ratio_graph": bg / fg,
            "graph_equals_eager": bool(torch.equal(lamg, lam0)),
            "timing_graph": "HIP events around replays of the captured passes, median of %d"
                            % reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=7,
                    help="timed repeats of the K steps (median reported; at least 5)")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--graph", action="store_true", help="replay the steps as a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the secondary 2D figures")
    ap.add_argument("--steps-2d", type=int, default=100)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--steps-batched", type=int, default=500)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-char", action="store_true",
                    help="skip the characteristic-field secondary figure")
    ap.add_argument("--steps-char", type=int, default=300)
    ap.add_argument("--no-strip", action="store_true",
                    help="skip the one-share-of-eight 2D strip figure")
    ap.add_argument("--no-large", action="store_true", help="skip the 1D N = 2^25 figure")
    ap.add_argument("--no-char2d", action="store_true",
                    help="skip the 2D characteristic-field figure")
    ap.add_argument("--steps-char2d", type=int, default=100)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, fill and copy 256 MiB (reference kernels "
                         "for rocprof FETCH_SIZE / WRITE_SIZE scaling)")
    ap.add_argument("--traffic-calibration", action="store_true",
                    help="after the timed region, three times each: fill 256 MiB, sum it, "
                         "copy it (reference kernels of known traffic for the byte counters)")
    args = ap.parse_args()
    args.repeats = max(5, args.repeats)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2004_07954_amd import api, inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, K, W = args.n, args.steps, args.warmup
    u0, dx = I.shu_osher_like(n)
    u = torch.tensor(u0, dtype=torch.float64, device=dev)
    stage = torch.empty((2, 3, n), dtype=torch.float64, device=dev)
    prm = api.params("euler", bc="transmissive")
    stream = torch.cuda.current_stream()

    # launch shape of the stage kernel, chosen by timing the candidates before the timed run
    from paper_2004_07954_amd import autotune
    tune_best, tune_ms = autotune.tune_rows(n, steps=100, shapes=[(256, 4, 1), (128, 4, 1),
                                                                  (256, 2, 1), (256, 2, 0)],
                                            log=log, apply=True, rounds=3)
    log("warmup", W, "steps, N =", n)
    if W:
        api.rk3_run_1d(u, dx, W, cfl=0.5, prm=prm, stage=stage)
    torch.cuda.synchronize()
    u.copy_(torch.tensor(u0, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()

    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            api.rk3_run_1d(u, dx, K, cfl=0.5, prm=prm, stage=stage)
        u.copy_(torch.tensor(u0, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()

    # the K timed steps are repeated (each repeat from the initial state, restored outside the
    # timed region); the median repeat is the reported figure
    u_init = torch.tensor(u0, dtype=torch.float64, device=dev)
    reps_ms = []
    log("timed", K, "steps x", args.repeats, "repeats", "(graph)" if graph else "(eager)")
    for _ in range(args.repeats):
        u.copy_(u_init)
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        if graph is not None:
            graph.replay()
        else:
            api.rk3_run_1d(u, dx, K, cfl=0.5, prm=prm, stage=stage)
        end.record(stream)
        torch.cuda.synchronize()
        reps_ms.append(start.elapsed_time(end))
    ms = float(np.median(reps_ms))
    uf = u.cpu().numpy()
    assert np.isfinite(uf).all() and uf[0].min() > 0, "non-physical state after the run"

    launches = 3 * K
    kernel_ms = ms / launches  # upper bound of the stage kernel's mean duration
    # algorithmic HBM bytes per cell: stage 1 reads U, writes U1 (48 B); stages 2 and 3 read
    # U^(s) and U^n and write (72 B): mean 64 B per cell per stage launch
    bytes_per_launch = n * (48 + 72 + 72) / 3.0
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    value = n * 3 * K / (ms * 1e-3)
    nt, kk, lay = autotune.get_row_tuning(3, n)
    autotune.set_row_tuning(0, 0)  # the other workloads use the size-based shapes
    lname = LAYOUT_NAMES[lay]
    kname = "row_kernel<%d, %d, EULER1, double, %s>" % (nt, kk, lname)
    workload = "euler1d_n%d" % n
    ktag = "row_kernel_%dx%d_%s" % (nt, kk, lname)
    traffic = committed_profile("traffic", ktag, workload, "hbm_bytes_per_launch",
                                ROW_KERNEL_SOURCES)
    valu = committed_profile("valu", ktag, workload, "valu_instr_per_cell", ROW_KERNEL_SOURCES)
    flops = FLOPS_PER_CELL_STAGE * n / (kernel_ms * 1e-3) / 1e12
    rec = {
        "metric": "WENO-ZN RHS cell-updates/s (1D Euler, fused TVD-RK3 stages)",
        "value": value,
        "unit": "cell-RHS/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "euler1d_shu_osher_like", "n_cells": n, "nvar": 3,
                   "launch_shape": {"nt": tune_best[0], "k": tune_best[1],
                                    "layout": LAYOUT_NAMES[tune_best[2]],
                                    "autotune_ms_per_step": tune_ms},
                   "bc": "transmissive", "cfl": 0.5, "eps": 1e-40, "A": 10.0,
                   "launch": "hip_graph" if graph else "stream", "kernels_per_step": 3},
        "timing": {"repeats": len(reps_ms), "statistic": "median",
                   "ms_per_step_repeats": [r / K for r in reps_ms],
                   "ms_per_step_min": min(reps_ms) / K, "ms_per_step_max": max(reps_ms) / K},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": kname, "kernel_ms": kernel_ms},
        # the stage kernel's fp64 VALU side (algorithmic flops of the literal formulas, and the
        # measured VALU instructions per cell from the committed counter profile)
        "roofline_alu": {"bound": "alu", "achieved": flops, "peak": FP64_VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": flops / FP64_VALU_PEAK_TFLOPS,
                         "flops_per_cell_stage": FLOPS_PER_CELL_STAGE,
                         "valu_instr_per_cell_stage": valu,
                         "valu_issue_frac": (valu * n / (kernel_ms * 1e-3) / VALU_LANE_PEAK
                                             if valu else None)},
        "cpu_baseline": None,
    }
    if args.copy_calibration or args.traffic_calibration:
        # reference kernels of known traffic for the rocprof byte counters, after the timed
        # region: a fill (writes 256 MiB), a sum (reads 256 MiB) and a copy (reads and writes
        # 256 MiB), each kernel run three times
        a = torch.empty(32 << 20, dtype=torch.float64, device=dev)  # 256 MiB
        b = torch.empty_like(a)
        reps = 3 if args.traffic_calibration else 1
        for _ in range(reps):
            a.fill_(1.0)
            if args.traffic_calibration:
                a.sum()
            b.copy_(a)
        torch.cuda.synchronize()
        rec["calibration_bytes"] = a.numel() * 8
    if not args.no_2d:
        log("2D fp64 and fp32, 4096^2")
        rec["secondary"] = {"euler2d_f64": bench_2d(args.steps_2d, "f64"),
                            "euler2d_f32": bench_2d(args.steps_2d, "f32"),
                            "euler2d_sw_f64": bench_2d(args.steps_2d, "f64", split="sw"),
                            "euler2d_sw_f32": bench_2d(args.steps_2d, "f32", split="sw")}
    if not args.no_batched:
        log("batched: 4096 shock tubes")
        rec.setdefault("secondary", {})["batched"] = bench_batched(args.steps_batched)
        rec["batched_speedup"] = rec["secondary"]["batched"]["speedup_vs_one_launch_per_instance"]
    if not args.no_adjoint:
        log("adjoint: N=65536, 400 steps")
        rec.setdefault("secondary", {})["adjoint"] = bench_adjoint()
        rec["adjoint_fwd_ratio"] = rec["secondary"]["adjoint"]["adjoint_fwd_ratio"]
    if not args.no_strip:
        log("2D strip 4096 x 512 (one share of eight)")
        rec.setdefault("secondary", {})["strip"] = bench_strip()
    if not args.no_large:
        log("1D at N = 2^25")
        rec.setdefault("secondary", {})["euler1d_large"] = bench_large_1d()
    if not args.no_char:
        log("characteristic fields, N =", n)
        rec.setdefault("secondary", {})["characteristic"] = bench_char(
            n, args.steps_char, cpu_steps=0 if args.no_cpu_baseline else 3)
    if not args.no_char2d:
        log("2D characteristic fields, 2400^2")
        rec.setdefault("secondary", {})["characteristic_2d"] = bench_char2d(args.steps_char2d)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
