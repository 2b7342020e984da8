#!/usr/bin/env python3
"""Benchmark of the acoustic_iso_cd forward propagator on one MI355X.

One bench step = one full forward modelling run of the workload: reset the
state, then T leapfrog steps with CPML, source injection and recording of
the receiver plane (all in the HIP library).  Inputs (model, wavelet, trace
buffer) are resident in HBM before timing starts.  The default workload is
the 1024 x 1024 x 512 layered model with a 32-cell CPML and 500 steps, whose
working set (about 7.5 GB) is far beyond the 256 MiB Infinity Cache.

Prints ONE JSON line:
  value     = grid points x T / wall time of one run (Gpoint-updates/s)
  roofline  = algorithmic bytes of one time step (16 B per point plus 16 B
              per point and damped CPML axis) / the average duration of a
              step (start of its first kernel to end of its last, stamped by
              the launches into HIP events on the library's stream), vs
              8 TB/s; traffic = the bytes the step's kernels actually move
              (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by calibration
              kernels), from the committed counter summary of the same
              kernel source
  cpu_baseline = the FP64 oracle timed on the host cores on a bounded sample
                 of the same workload (cpu_baseline_1thread: one thread, on
                 a sample of the 240^3 workload)
  paper_context = the paper's own serial CPU rate for a 240^3 run (context only)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# names of the forward CPML strategies (mm_get_cpml_kernel)
CPML_NAMES = {0: None, 1: "layer pass + stencil", 2: "fused"}
ALG_BYTES_STENCIL = 16  # read p^n, p^{n-1}, (dt v)^2; write p^{n+1}  (bytes per grid point)
ALG_BYTES_ISO = 40      # acoustic_iso: read and write p and the three face velocities, read rho v^2 and buoyancy


def kernel_hash():
    """Hash of the kernel source and of the host runtime that plans their launches (tile tables,
    z-chunking, strategy choice), which the counter and duration summaries depend on."""
    h = hashlib.sha256()
    for f in ("mm_kernels.hip", "mm_internal.h", "mm_api.cpp"):
        with open(os.path.join(ROOT, "paper_2007_06048_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_workload(name):
    from paper_2007_06048_amd import workloads as W
    if name == "smooth240":
        return W.smooth_240()
    if name == "layered1024":
        return W.layered_1024()
    if name == "twolayer64":
        return W.two_layer_64()
    if name == "smoothiso":
        return W.smooth_iso()
    raise SystemExit(f"unknown workload {name}")


def traffic_entry(workload_name):
    """The committed rocprofv3 summary of a workload's time step (counters and
    per-kernel durations), if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "step_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(workload_name)
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e


def traffic_for(workload_name):
    """HBM bytes per time step (all kernels of the step) from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    e = traffic_entry(workload_name)
    return e.get("bytes_per_step") if e else None


def launch_kind(name):
    """Which part of a forward CPML step (fused strategy) a kernel
    instantiation runs: the plain stencil over the interior box, or the fused
    kernel over the frame (template XY, not LZ), the z-layer chunks away from
    the x / y faces (LZ, not XY) or the z-layer corners (both)."""
    if name.startswith("void mm::k_step<") or name.startswith("mm::k_step<"):
        return "interior"
    if "k_cstep<" in name:
        args = [a.strip() for a in name.split("<", 1)[1].split(">", 1)[0].split(",")]
        xy, lz = args[4] == "true", args[5] == "true"
        return {(True, False): "frame", (False, True): "z_layer", (True, True): "z_corners"}.get((xy, lz))
    return None


def region_alg_bytes(wl):
    """Algorithmic bytes of each part of a forward CPML step (fused strategy):
    16 B per point (p^n, p^{n-1}, (dt v)^2 read, p^{n+1} written) plus 16 B
    per point and damped axis (psi and zeta, read and written).  The parts
    are the interior box (no layer), the frame of the x / y layers in the
    middle z range, the z-layer chunks away from the x / y layers, and the
    z-layer corners; they sum to step_alg_bytes."""
    nx, ny, nz, nb = wl.nx, wl.ny, wl.nz, wl.nb
    fs = getattr(wl, "free_surface", 0)
    zlo, zhi = (0 if fs else nb), nz - nb
    mid = zhi - zlo
    zl = nz - mid  # planes of the z layers
    ix, iy = nx - 2 * nb, ny - 2 * nb
    xy_all, xy_in = nx * ny, ix * iy
    xl_cells = 2 * nb * ny     # xy cells in an x layer
    yl_cells = 2 * nb * nx     # in a y layer
    ring = xy_all - xy_in
    return {"interior": 16 * xy_in * mid,
            "frame": 16 * ring * mid + 16 * (xl_cells + yl_cells) * mid,
            "z_layer": 32 * xy_in * zl,
            "z_corners": 32 * ring * zl + 16 * (xl_cells + yl_cells) * zl}


def step_alg_bytes(wl, alg_pt):
    """Algorithmic bytes of one time step: alg_pt per grid point plus, for
    CPML, 16 B (psi and zeta, read and write) per point and damped axis."""
    damped_axis_pts = 0
    if wl.bc == 2:
        for m in (wl.ny * wl.nz, wl.nx * wl.nz, wl.nx * wl.ny):
            damped_axis_pts += 2 * wl.nb * m
    return alg_pt * wl.nx * wl.ny * wl.nz + 16 * damped_axis_pts


def cpu_baseline(wl, budget_s, threads=0):
    """Time the FP64 oracle on a bounded sample: the same grid, model,
    boundary and source, for as many steps as fit in about budget_s, on
    `threads` OpenMP threads (0: the runtime's default, all host cores)."""
    import numpy as np
    from oracle import c_oracle as C
    from paper_2007_06048_amd import minimod as mm
    default_threads = C.num_threads()
    if threads > 0:
        C.set_num_threads(threads)
    try:
        return _cpu_baseline(wl, budget_s, C, mm, np)
    finally:
        C.set_num_threads(default_threads)


def _cpu_baseline(wl, budget_s, C, mm, np):
    s = wl.shots[0]
    p = mm.default_params(nx=wl.nx, ny=wl.ny, nz=wl.nz, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=wl.bc, nb=wl.nb)
    vmax = float(s.vel.max())
    dt = mm.dt_for(p, vmax)
    g = C.Grid(wl.nx, wl.ny, wl.nz, wl.h, wl.h, wl.h, dt, bc=wl.bc, nb=wl.nb, sigma=wl.sigma, R=wl.cpml_R,
               f0=wl.f0, vmax=vmax)
    vel = s.vel.astype(np.float64)
    w = C.ricker(wl.f0, wl.t0, dt, wl.nsteps)[:, None]
    t0 = time.perf_counter()
    _, pm, pc, mem = C.forward(g, vel, s.src, w[:1], s.rec, 1)
    t1 = time.perf_counter()
    per = max(t1 - t0, 1e-3)
    n = int(max(1, min(wl.nsteps - 1, budget_s / per)))
    t0 = time.perf_counter()
    C.forward(g, vel, s.src, w[1:1 + n], s.rec, n, p_prev=pm, p_cur=pc, cpml_mem=mem)
    t1 = time.perf_counter()
    pts = wl.nx * wl.ny * wl.nz
    return {"value": pts * n / (t1 - t0) / 1e9, "unit": "Gpt/s", "cores": C.num_threads(), "kind": "oracle",
            "sample": f"{n} steps (of {wl.nsteps}) of the same {wl.nx}x{wl.ny}x{wl.nz} run, FP64, "
                      f"after 1 warm-up step"}


# kernels that advance the forward wavefields by one time level (one launch each per step; with CPML
# either the fused kernel over the frame of the faces and the z-layer chunks beside the interior
# stencil, or the layer pass before the stencil over the whole grid)
STEP_KERNELS = ("k_step<", "k_cstep<", "k_cpml_fwd<", "k_iso_u<", "k_iso_p<")


def pmc_summary(fetch_dir, write_dir, workload, out_path, stats_dir=None):
    """HBM traffic of one time step from two rocprofv3 --pmc passes
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch): the mean per dispatch of
    every kernel of the step, summed, each counter scaled by what it reads
    for kernels of known size in the same program: k_vcheck reads exactly
    4 N bytes (the velocity model), k_vdt2 writes exactly 4 N bytes.  With
    stats_dir (a rocprofv3 --kernel-trace --stats run of the same command)
    each kernel's average duration is kept beside its bytes."""
    import csv
    import numpy as np
    from paper_2007_06048_amd import workloads as W
    # a workload name, or an object with its name and geometry
    wl = workload if hasattr(workload, "nx") else {"smooth240": W.smooth_240, "layered1024": W.layered_1024}[workload]()
    n = wl.nx * wl.ny * wl.nz

    def per_kernel(d, counter):
        vals = {}
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return vals

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")

    def one(vals, key):
        ks = [k for k in vals if key in k]
        assert len(ks) == 1, (key, ks)
        return float(np.mean(vals[ks[0]]))

    f_fac = 4.0 * n / one(fetch, "k_vcheck")
    w_fac = 4.0 * n / one(write, "k_vdt2")
    kernels = {}
    for fam in STEP_KERNELS:
        # the instantiation the timed steps ran: the one with the most dispatches (the autotuner's
        # trials of the other tile variants come first and are fewer)
        names = [k for k in set(fetch) | set(write) if fam in k]
        if not names:
            continue
        top = max(len(fetch.get(k, [])) for k in names)
        for name in names:
            if len(fetch.get(name, [])) != top:
                continue
            kernels[name] = {"dispatches": len(fetch.get(name, [])),
                             "fetch_bytes": round(float(np.mean(fetch.get(name, [0.0]))) * f_fac),
                             "write_bytes": round(float(np.mean(write.get(name, [0.0]))) * w_fac)}
    if stats_dir:
        with open(os.path.join(stats_dir, "run_kernel_stats.csv")) as f:
            for r in csv.DictReader(f):
                if r["Name"] in kernels:
                    kernels[r["Name"]]["avg_ns"] = round(float(r["AverageNs"]), 1)
                    kernels[r["Name"]]["calls"] = int(r["Calls"])
    fb = sum(k["fetch_bytes"] for k in kernels.values())
    wb = sum(k["write_bytes"] for k in kernels.values())
    entry = {"kernels": kernels, "kernel_hash": kernel_hash(), "points": n,
             "fetch_scale": round(f_fac, 4), "write_scale": round(w_fac, 4),
             "fetch_bytes_per_step": fb, "write_bytes_per_step": wb, "bytes_per_step": fb + wb,
             "alg_bytes_per_step": step_alg_bytes(wl, ALG_BYTES_STENCIL),
             "note": "bytes below L2 (FETCH_SIZE/WRITE_SIZE; Infinity Cache hits are included), per time step "
                     "(every kernel of the step once); calibration kernels k_vcheck (read 4N B) and k_vdt2 "
                     "(write 4N B)"}
    try:
        with open(out_path) as f:
            allv = json.load(f)
    except (OSError, ValueError):
        allv = {}
    allv[wl.name] = entry
    with open(out_path, "w") as f:
        json.dump(allv, f, indent=1)
    print(json.dumps(entry, indent=1))


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def gradient_leg(dev, reps=2):
    """FWI gradient on the 200^3 workload (sponge-20, 1000 steps, checkpoints
    every 32): seconds per shot for the plain forward run and for the
    gradient (forward with checkpoints + residual + adjoint with segment
    replay and imaging) with FP32 and BF16 snapshots.  d_obs is the library's
    own forward run on the true model (input data for timing only)."""
    import torch
    from paper_2007_06048_amd import minimod as mm
    from paper_2007_06048_amd import workloads as W
    wl = W.fwi_200()
    s = wl.shots[0]
    T = wl.nsteps
    res = {"workload": wl.name, "shots_timed": 1}
    base = dict(nx=wl.nx, ny=wl.ny, nz=wl.nz, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=wl.bc, nb=wl.nb,
                sponge_sigma=wl.sigma, vmax=wl.vmax, tile=-1)
    p0 = mm.default_params(**base)
    vt = torch.from_numpy(wl.vel_true).to(dev)
    v0 = torch.from_numpy(s.vel).to(dev)
    ct = mm.Context.single(p0, vt, s.src, s.rec)
    w = torch.from_numpy(mm.ricker(wl.f0, wl.t0, ct.dt, T)).to(dev).reshape(T, 1)
    d_obs = torch.empty((T, len(s.rec)), dtype=torch.float32, device=dev)
    ct.forward(T, w, d_obs)
    del ct
    cf = mm.Context.single(p0, v0, s.src, s.rec)
    tr = torch.empty_like(d_obs)

    def fwd():
        cf.reset()
        cf.forward(T, w, tr)

    res["forward_s"] = round(_timed(fwd, reps), 4)
    del cf
    for name, snap in (("fp32", mm.SNAP_FP32), ("bf16", mm.SNAP_BF16)):
        pg = mm.default_params(**base, ckpt_every=wl.ckpt_every, snap=snap, nsteps_max=T)
        cg = mm.Context.single(pg, v0, s.src, s.rec)
        g = torch.empty(s.vel.shape, dtype=torch.float32, device=dev)
        res[f"gradient_{name}_s"] = round(_timed(lambda: cg.gradient(T, w, d_obs, g, tr), reps), 4)
        res[f"workspace_{name}_GB"] = round(cg.ws_bytes / 1e9, 2)
        del cg, g
        torch.cuda.empty_cache()
    res["gradient_fp32_vs_forward"] = round(res["gradient_fp32_s"] / res["forward_s"], 2)
    res["gradient_bf16_vs_forward"] = round(res["gradient_bf16_s"] / res["forward_s"], 2)
    # the same shot with a 20-cell CPML (adjoint through the transposed memory recursions)
    cbase = dict(base, bc=2, cpml_f0=wl.f0)
    cc = mm.Context.single(mm.default_params(**cbase), v0, s.src, s.rec)

    def fwd_cpml():
        cc.reset()
        cc.forward(T, w, tr)

    res["forward_cpml_s"] = round(_timed(fwd_cpml, reps), 4)
    del cc
    cg = mm.Context.single(mm.default_params(**cbase, ckpt_every=wl.ckpt_every, nsteps_max=T), v0, s.src, s.rec)
    g = torch.empty(s.vel.shape, dtype=torch.float32, device=dev)
    res["gradient_cpml_fp32_s"] = round(_timed(lambda: cg.gradient(T, w, d_obs, g, tr), reps), 4)
    res["workspace_cpml_fp32_GB"] = round(cg.ws_bytes / 1e9, 2)
    res["gradient_cpml_vs_forward"] = round(res["gradient_cpml_fp32_s"] / res["forward_cpml_s"], 2)
    del cg, g
    torch.cuda.empty_cache()
    return res


def iso_leg(dev, reps=2, bc=1):
    """acoustic_iso (first-order variable-density system, staggered grid) on
    the 240^3 smooth model with Gardner density, 20-cell sponge (bc 1) or
    CPML (bc 2), 1000 steps.  Algorithmic bytes per point and step: 40 (read
    and write p and the three face velocities, read rho v^2 and the
    buoyancy), with CPML 16 more per damped cell and axis (the memory of the
    face and of the cell derivative, each read and written); the two kernels
    move 56 + the memory (p and u are each read by both kernels)."""
    import torch
    from paper_2007_06048_amd import minimod as mm
    from paper_2007_06048_amd import workloads as W
    wl = W.smooth_iso(240, 1000)
    s = wl.shots[0]
    T = wl.nsteps
    p = mm.default_params(nx=wl.nx, ny=wl.ny, nz=wl.nz, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=bc, nb=wl.nb,
                          sponge_sigma=wl.sigma, cpml_R=wl.cpml_R, cpml_f0=wl.f0, model=mm.MODEL_ISO, tile=-1)
    ctx = mm.Context.single(p, torch.from_numpy(s.vel).to(dev), s.src, s.rec, rho=torch.from_numpy(s.rho).to(dev))
    w = torch.from_numpy(mm.ricker(wl.f0, wl.t0, ctx.dt, T)).to(dev).reshape(T, 1)
    tr = torch.empty((T, len(s.rec)), dtype=torch.float32, device=dev)

    def run():
        ctx.reset()
        ctx.forward(T, w, tr)

    t = _timed(run, reps)
    ctx.profile(10)
    ctx.profile_read()
    run()
    k_ms, k_n = ctx.profile_read()
    ctx.profile(0)
    pts = wl.nx * wl.ny * wl.nz
    step_s = t / T
    from types import SimpleNamespace as NS
    bytes_step = step_alg_bytes(NS(nx=wl.nx, ny=wl.ny, nz=wl.nz, bc=bc, nb=wl.nb), ALG_BYTES_ISO)
    ach = bytes_step / step_s / 1e9
    return {"workload": wl.name.replace("sponge", "cpml") if bc == 2 else wl.name, "run_s": round(t, 4),
            "gpts": round(pts * T / t / 1e9, 2), "us_per_step": round(step_s * 1e6, 2),
            "tile": mm.tile_name(ctx.info()["tile"]), "kernels_us_per_step": round(k_ms / max(k_n, 1) * 1e3, 2),
            "roofline": {"bound": "hbm", "alg_bytes_per_point": round(bytes_step / pts, 3), "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}}


def iso_cpml_leg(dev, reps=2):
    return iso_leg(dev, reps, bc=2)


def free_surface_leg(dev, reps=2):
    """The bench workload (240^3, CPML-20, 1000 steps) with a free surface on
    the top face instead of the top CPML layer."""
    import torch
    from paper_2007_06048_amd import minimod as mm
    from paper_2007_06048_amd import workloads as W
    wl = W.smooth_240()
    s = wl.shots[0]
    T = wl.nsteps
    p = mm.default_params(nx=wl.nx, ny=wl.ny, nz=wl.nz, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=wl.bc, nb=wl.nb,
                          cpml_R=wl.cpml_R, cpml_f0=wl.f0, tile=-1, free_surface=1)
    ctx = mm.Context.single(p, torch.from_numpy(s.vel).to(dev), s.src, s.rec)
    w = torch.from_numpy(mm.ricker(wl.f0, wl.t0, ctx.dt, T)).to(dev).reshape(T, 1)
    tr = torch.empty((T, len(s.rec)), dtype=torch.float32, device=dev)

    def run():
        ctx.reset()
        ctx.forward(T, w, tr)

    t = _timed(run, reps)
    return {"workload": wl.name + "_free_surface", "run_s": round(t, 4),
            "gpts": round(wl.nx * wl.ny * wl.nz * T / t / 1e9, 2), "tile": mm.tile_name(ctx.info()["tile"]),
            "cpml_kernel": CPML_NAMES[ctx.cpml_kernel()]}


def batched_leg(dev, reps=2):
    """32 shots on uneven sub-volumes (CPML-16, 800 steps): one context over
    all shots launched as one HIP graph, against the plain single-shot path
    run 32 times in sequence (same kernels, bitwise-identical traces)."""
    import torch
    from paper_2007_06048_amd import minimod as mm
    from paper_2007_06048_amd import workloads as W
    wl = W.batched_shots()
    T = wl.nsteps
    pts = wl.points
    base = dict(dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=wl.bc, nb=wl.nb, cpml_R=wl.cpml_R, cpml_f0=wl.f0,
                vmax=wl.vmax)
    p = mm.default_params(**base, tile=-1)
    vels = [torch.from_numpy(sh.vel).to(dev) for sh in wl.shots]
    ctx = mm.Context(p, [(v, sh.src, sh.rec) for v, sh in zip(vels, wl.shots)])
    dt = ctx.dt
    w1 = mm.ricker(wl.f0, wl.t0, dt, T)
    w = torch.from_numpy(w1).to(dev).reshape(T, 1).repeat(1, len(wl.shots)).contiguous()
    tr = torch.empty((T, ctx.nrec), dtype=torch.float32, device=dev)

    def batch():
        ctx.reset()
        ctx.forward(T, w, tr, graph=True)

    t_batch = _timed(batch, reps)
    tile = mm.tile_name(ctx.info()["tile"])
    cpml = CPML_NAMES[ctx.cpml_kernel()]
    del ctx, tr
    torch.cuda.empty_cache()
    singles = []
    for v, sh in zip(vels, wl.shots):
        q = mm.default_params(**base, tile=-1)
        c = mm.Context.single(q, v, sh.src, sh.rec)
        singles.append((c, torch.empty((T, len(sh.rec)), dtype=torch.float32, device=dev)))
    ws = torch.from_numpy(w1).to(dev).reshape(T, 1)

    def seq():
        for c, t in singles:
            c.reset()
            c.forward(T, ws, t)

    t_seq = _timed(seq, reps)
    return {"workload": wl.name, "shots": len(wl.shots), "points": pts, "time_steps": T, "tile": tile,
            "cpml_kernel": cpml,
            "batched_graph_s": round(t_batch, 4), "batched_gpts": round(pts * T / t_batch / 1e9, 2),
            "sequential_single_s": round(t_seq, 4), "sequential_gpts": round(pts * T / t_seq / 1e9, 2),
            "speedup": round(t_seq / t_batch, 3)}


def run_forward_workload(dev, wl, tile=-1, graph=False, steps=1, warmup=1, prof_stride=10):
    """Times full modelling runs of a single-shot workload: returns the
    context's description, the seconds per run and the step timing."""
    import torch
    from paper_2007_06048_amd import minimod as mm
    s = wl.shots[0]
    T = wl.nsteps
    iso = s.rho is not None  # the acoustic_iso workload carries a density model
    p = mm.default_params(nx=wl.nx, ny=wl.ny, nz=wl.nz, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=wl.bc, nb=wl.nb,
                          sponge_sigma=wl.sigma, cpml_R=wl.cpml_R, cpml_f0=wl.f0, tile=tile,
                          model=mm.MODEL_ISO if iso else mm.MODEL_ISO_CD)
    vel = torch.from_numpy(s.vel).to(dev)
    t_init0 = time.perf_counter()
    ctx = mm.Context.single(p, vel, s.src, s.rec, rho=torch.from_numpy(s.rho).to(dev) if iso else None)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init0
    dt = ctx.dt
    w = torch.from_numpy(mm.ricker(wl.f0, wl.t0, dt, T)).to(dev).reshape(T, 1)
    traces = torch.empty((T, len(s.rec)), dtype=torch.float32, device=dev)

    def run():
        ctx.reset()
        ctx.forward(T, w, traces, graph=graph)

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    if prof_stride > 0 and not graph:
        ctx.profile(prof_stride)
        ctx.profile_read()  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n = (ctx.profile_read() if prof_stride > 0 and not graph else (0.0, 0))
    ctx.profile(0)
    info = {"tile": mm.tile_name(ctx.info()["tile"]), "cpml_kernel": CPML_NAMES[ctx.cpml_kernel()],
            "init_s": round(t_init, 3), "dt_s": dt}
    del ctx, traces, vel
    torch.cuda.empty_cache()
    return info, (t1 - t0) / steps, k_ms, k_n


def kernel_breakdown(wl):
    """Per-launch fractions of a forward CPML step (fused strategy) from the
    committed profile of the current kernels: each part's algorithmic bytes
    over its average rocprofv3 duration, and its counter-measured bytes."""
    e = traffic_entry(wl.name)
    if not e or wl.bc != 2:
        return None
    alg = region_alg_bytes(wl)
    out = {}
    for name, k in e["kernels"].items():
        kind = launch_kind(name)
        if kind is None or "avg_ns" not in k:
            continue
        ach = alg[kind] / (k["avg_ns"] * 1e-9) / 1e9
        out[kind] = {"kernel": name.split("(")[0].replace("void ", ""), "avg_launch_us": round(k["avg_ns"] / 1e3, 1),
                     "alg_bytes": alg[kind], "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": k["fetch_bytes"] + k["write_bytes"],
                     "traffic_per_alg": round((k["fetch_bytes"] + k["write_bytes"]) / alg[kind], 3)}
    return out or None


def step_roofline(wl, alg_pt, step_ms, n_timed, stride, kernels):
    """Roofline of one time step: its algorithmic bytes over the average
    duration of the timed steps."""
    bytes_step = step_alg_bytes(wl, alg_pt)
    ach = bytes_step / (step_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_for(wl.name),
            "kernel": kernels, "avg_launch_us": round(step_ms * 1e3, 2),
            "alg_bytes_per_launch": bytes_step,
            "alg_bytes_per_point": round(bytes_step / (wl.nx * wl.ny * wl.nz), 3),
            "timed_launches": n_timed, "timed_every": stride}
    if roof["traffic"]:
        # the bytes the step's kernels actually move below L2, at the measured step time
        roof["traffic_GBs"] = round(roof["traffic"] / (step_ms / 1e3) / 1e9, 1)
        roof["traffic_per_alg"] = round(roof["traffic"] / bytes_step, 3)
        parts = kernel_breakdown(wl)
        if parts:
            # per launch, from the profile summary committed with the counters (same kernel source)
            roof["kernels"] = parts
    return roof


def step_kernels_name(wl, iso, cpml=None):
    if iso:
        return "time step: k_iso_u + k_iso_p (face velocities, then pressure)"
    if wl.bc == 2 and cpml == CPML_NAMES[1]:
        return ("time step: k_cpml_fwd over the damping layers (CPML memory update and correction) + k_step over "
                "the whole grid (stencil adding the correction, leapfrog, record)")
    if wl.bc == 2:
        return ("time step: k_step over the interior box (stencil, leapfrog, record) + k_cstep over the frame of "
                "the x / y faces and k_cstep over the z-layer chunks (stencil with the CPML memory update fused)")
    return "time step: k_step (stencil, damping, leapfrog, source, record)"


def cache_resident_leg(dev, reps=2):
    """The 240^3 CPML-20 workload (1000 steps): a working set of about
    250 MB, which the 256 MiB Infinity Cache can hold, so its rate is not an
    HBM figure; reported beside the headline for comparison with the paper's
    240^3 example."""
    from paper_2007_06048_amd import workloads as W
    wl = W.smooth_240()
    info, t, k_ms, k_n = run_forward_workload(dev, wl, steps=reps, warmup=1)
    out = {"workload": wl.name, "run_s": round(t, 4),
           "gpts": round(wl.nx * wl.ny * wl.nz * wl.nsteps / t / 1e9, 2), "tile": info["tile"],
           "cpml_kernel": info["cpml_kernel"],
           "note": "working set about 250 MB: Infinity-Cache resident, not an HBM figure"}
    if k_n > 0:
        out["roofline"] = step_roofline(wl, ALG_BYTES_STENCIL, k_ms / k_n, k_n, 10,
                                        step_kernels_name(wl, False, info["cpml_kernel"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered1024")
    ap.add_argument("--tile", type=int, default=-1, help="tile variant, -1 = autotune")
    ap.add_argument("--prof-stride", type=int, default=10,
                    help="time every k-th time step with HIP events stamped by its first and last launch (0: "
                         "none); sampling keeps the whole-run figure unperturbed")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graph", action="store_true", help="launch the step loop as one HIP graph")
    ap.add_argument("--calib", action="store_true", help="also run a 1 GiB copy (counter calibration)")
    ap.add_argument("--time-steps", type=int, default=0, help="override the workload's step count (profiling)")
    ap.add_argument("--legs", default="",
                    help="comma-separated subset of the extra legs to run (cache_resident_240, gradient, batched, "
                         "free_surface, acoustic_iso, acoustic_iso_cpml); default all")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 240^3, gradient, batched, free-surface and acoustic_iso legs")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                    help="FETCH_DIR WRITE_DIR [STATS_DIR]: summarise two rocprofv3 --pmc runs (and a "
                         "--kernel-trace --stats run of the same command) into profiles/step_traffic.json "
                         "and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        if len(args.pmc_summary) not in (2, 3):
            raise SystemExit("--pmc-summary takes FETCH_DIR WRITE_DIR [STATS_DIR]")
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.workload,
                    os.path.join(ROOT, "profiles", "step_traffic.json"),
                    args.pmc_summary[2] if len(args.pmc_summary) == 3 else None)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (shots and z-slabs would shard "
              "across GPUs; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    wl = load_workload(args.workload)
    s = wl.shots[0]
    if args.time_steps > 0:
        wl.nsteps = args.time_steps
    T = wl.nsteps
    iso = s.rho is not None
    info, t_run, k_ms, k_n = run_forward_workload(dev, wl, tile=args.tile, graph=args.graph, steps=args.steps,
                                                  warmup=args.warmup, prof_stride=args.prof_stride)
    ms_step = t_run * 1e3
    pts = wl.nx * wl.ny * wl.nz
    value = pts * T / t_run / 1e9

    if args.calib:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    alg_pt = ALG_BYTES_ISO if iso else ALG_BYTES_STENCIL
    roof = None
    if k_n > 0:
        roof = step_roofline(wl, alg_pt, k_ms / k_n, k_n, args.prof_stride,
                             step_kernels_name(wl, iso, info["cpml_kernel"]))
    # the same over the whole run (wall clock of a run / T): launch gaps, the trace record and reset included
    bytes_step = step_alg_bytes(wl, alg_pt)
    run_ach = bytes_step / (t_run / T) / 1e9
    run_roof = {"achieved": round(run_ach, 1), "frac": round(run_ach / HBM_PEAK_GBS, 4),
                "us_per_step": round(t_run / T * 1e6, 2)}

    out = {
        "metric": "Gpoint-updates/s and % HBM roofline (fwd); FWI gradient s/shot vs plain",
        "value": round(value, 3),
        "unit": "Gpt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "time_steps_per_run": T, "h_m": wl.h,
                   "bc": {0: "none", 1: "sponge", 2: "cpml"}[wl.bc], "nb": wl.nb, "receivers": len(s.rec),
                   "tile": info["tile"], "cpml_kernel": info["cpml_kernel"], "graph": bool(args.graph), "init_s": info["init_s"], "dt_s": info["dt_s"]},
        "roofline": roof,
        "run_roofline": run_roof,
    }
    legs = {"cache_resident_240": cache_resident_leg, "gradient": gradient_leg, "batched": batched_leg,
            "free_surface": free_surface_leg, "acoustic_iso": iso_leg, "acoustic_iso_cpml": iso_cpml_leg}
    if args.legs:
        unknown = set(args.legs.split(",")) - set(legs)
        if unknown:
            raise SystemExit(f"unknown legs {sorted(unknown)}; known: {sorted(legs)}")
    for name, leg in legs.items():
        if args.no_extras or (args.legs and name not in args.legs.split(",")):
            continue
        out[name] = leg(dev)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
        from paper_2007_06048_amd import workloads as W
        out["cpu_baseline_1thread"] = cpu_baseline(W.smooth_240(), args.cpu_budget * 2.0 / 3.0, threads=1)
    # the paper's only timing of this propagator, as context (a different grid, spacing, step count
    # and boundary width, one CPU thread on unstated hardware): section "Compilation and usage"
    # reports 30.47 s of kernel time for 240^3 points x 300 steps
    out["paper_context"] = {"value": round(240 ** 3 * 300 / 30.47 / 1e9, 3), "unit": "Gpt/s",
                            "what": "paper's serial CPU run: 240^3, h 20 m, 300 steps, ndamping 27, "
                                    "1 thread, hardware unstated; kernel time 30.47 s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
