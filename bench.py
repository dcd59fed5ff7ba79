#!/usr/bin/env python3
"""Benchmark of the implicit ray-by-ray MGFLD transport step on one MI355X.

Workload: 16384 rays x 540 zones x 20 groups x 4 species (707,788,800 cells), the
synthetic stellar-profile recipe of `synth`, generated directly in HBM.  One bench
step = one implicit time step: the mixed-precision Newton iteration (FP32 block
factorisation, FP64 residual/update/sums) refined to a 1e-12 relative residual.
Alongside, the FP64 path is timed to the same tolerance (time-to-tolerance and the
mixed-vs-FP64 error are reported), the FP64 adjoint of the outer luminosity, and the
configuration's multi-step job (10 drifting steps, then the adjoint over all of them with
one checkpoint per step), the FP64 Y_e-coupled step of species 0 and 1 (blocks of 2N+1
rows coupling the electron neutrinos, antineutrinos and the electron fraction of each zone), and
the energy-advection update of every zone (Lagrangian energy shift, PPM remap, over-fill limiter).

Metric: Newton updates/s = sum over systems of (Newton updates applied) x I x N / time.
Output: one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray·zone·group Newton updates/s, mixed vs FP64 at ≤1e-8 rel err; % roofline"
TAU = 1e-30
# MI355X published peaks: FP64 vector/matrix 78.6 TFLOP/s; FP32 157.3 TFLOP/s (matrix cores, or packed
# FP32 on the vector units); HBM3E 8 TB/s
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
KERNEL_F32 = "k_factor_q<20, false, true, 0>"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def iteration_flops_per_cell(N: int) -> float:
    """Algorithmic flops per cell per Newton iteration: 2N^2 + 20N (1200 at N = 20; the block inverse is
    2N^2 of it)."""
    return 2.0 * N * N + 20.0 * N


def iteration_bytes_per_cell() -> float:
    """Compulsory FP64 HBM bytes per cell per Newton iteration: read psi^n, psi, kappa_a, eta, kappa_s and
    write the new psi (6 x 8 B).  Stored block factors are not algorithmic traffic: they are what a design
    pays on top."""
    return 48.0


def stored_factor_bytes_per_cell(N: int, factor_bytes: int) -> float:
    """HBM bytes per cell of the stored block-Thomas factors: C_i (N values per cell) and y_i (one), written
    by the forward sweep and read back by the backward sweep."""
    return 2.0 * (N + 1) * factor_bytes


def roofline_time(cells: int, N: int, mixed: bool) -> dict:
    """T_roof = max(bytes / HBM, sum_p flops_p / peak_p) of one Newton iteration over `cells` cells.

    FP64 path: all 2N^2 + 20N flops at the FP64 peak.  Mixed path: the block elimination (2N^2 + 10N,
    1000 at N = 20) at the FP32 peak and the rest (10N, 200) at the FP64 peak."""
    tot = iteration_flops_per_cell(N)
    f32 = (2.0 * N * N + 10.0 * N) if mixed else 0.0
    f64 = tot - f32
    t_hbm = iteration_bytes_per_cell() * cells / (PEAK_HBM_GBS * 1e9)
    t_alu = cells * (f32 / (PEAK_FP32_TFLOPS * 1e12) + f64 / (PEAK_FP64_TFLOPS * 1e12))
    return dict(t_roof=max(t_hbm, t_alu), t_hbm=t_hbm, t_alu=t_alu, flops=tot * cells, flops_fp32=f32 * cells,
                flops_fp64=f64 * cells, bytes=iteration_bytes_per_cell() * cells)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Cores this process may run on, at most 16 (the host share of one GPU on the benchmark machine)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def source_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_record(kernel_src, record="k_factor_traffic.json"):
    """HBM traffic per launch measured with rocprofv3 --pmc, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_16") != source_hash(kernel_src):
        return None
    return rec


def rel_err_gpu(a, ref):
    import torch
    return float(torch.max((a - ref).abs() / ref.abs().clamp_min(TAU)).item())


def run_newton_leg(tm, torch, w, f, precision, steps, warmup, rtol, max_iter):
    ctx = tm.Context(tm.problem_of(w, precision))
    psi = torch.empty_like(w.psi_n)
    cells_per_sys = w.I * w.N
    times, updates = [], []
    stats = None
    for s in range(warmup + steps):
        psi.copy_(w.psi_n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, stats = ctx.newton_step(f, w.psi_n, psi, max_iter, rtol, with_stats=True, raise_on_status=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if st != 0:
            log("newton status", tm.STATUS_NAMES.get(st, st))
        it = stats["iters"].to(torch.int64)
        if s >= warmup:
            times.append(t1 - t0)
            updates.append(int(it.sum().item()) * cells_per_sys)
        log(f"  {'warm' if s < warmup else 'step'} {s}: {1e3 * (t1 - t0):.1f} ms, iters "
            f"min {int(it.min())} max {int(it.max())}, status {tm.STATUS_NAMES.get(st, st)}")
    return ctx, psi, stats, times, updates


def time_kernel(torch, fn, reps):
    """Average duration of `fn` (one kernel launch plus trivial setup) with HIP events on the current stream."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps / 1e3


def time_factor_kernel(ctx, fn, reps):
    """Average duration of the diagonal-pivot factor launch inside `fn` (one factor solve): HIP events that
    the library records on its own stream right before and after that launch (kernel timing)."""
    ctx.set_kernel_timing(True)
    fn()
    ms = []
    for _ in range(reps):
        fn()
        ms.append(ctx.kernel_time_ms())
    ctx.set_kernel_timing(False)
    return sum(ms) / len(ms) / 1e3


def prealloc_workspace(torch, ctx):
    """Hand the context its factor workspace before timing: all systems if they fit in 70% of the
    free device memory, else the largest halving that does (the library then batches)."""
    free = torch.cuda.mem_get_info()[0]
    b = ctx.problem.n_species * ctx.problem.n_rays
    while b > 1 and ctx.workspace_bytes(b) > 0.7 * free:
        b = (b + 1) // 2
    ctx.set_workspace(ctx.workspace_bytes(b))
    return b


def multistep_leg(tm, torch, synth, dev, rays, steps, rtol, max_iter):
    """The configuration's multi-step job: `steps` consecutive implicit steps with drifting inputs
    (mixed-precision Newton, one checkpoint per step), then the checkpointed FP64 adjoint of
    J = sum_s L_N(psi^s) over all steps.  A step's drifted inputs are regenerated on the GPU when
    needed (held one step at a time); that generation is excluded from the reported times."""
    from paper_1809_05608_amd import multistep
    gen = [0.0]
    held = {}
    marks = []                                   # (call start, call end) of each input generation

    def fields_at(s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        marks.append([t0, t0])
        held.clear()
        ws = synth.make(4, rays=rays, step=s, device=dev)
        held["w"] = ws
        f = tm.DeviceFields.of(ws)
        torch.cuda.synchronize()
        marks[-1][1] = time.perf_counter()
        gen[0] += marks[-1][1] - t0
        return f

    w0 = synth.make(4, rays=rays, step=0, device=dev)
    psi0 = w0.psi_n.clone()
    prob_m, prob_d = tm.problem_of(w0, tm.PREC_MIXED), tm.problem_of(w0, tm.PREC_FP64)
    cells_per_sys = w0.I * w0.N
    del w0
    torch.cuda.empty_cache()
    ctx = tm.Context(prob_m)
    cps = [torch.empty_like(psi0) for _ in range(steps)]   # one checkpoint per step, allocated up front
    prealloc_workspace(torch, ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats = multistep.forward(ctx, fields_at, psi0, steps, max_iter=max_iter, rtol=rtol, checkpoints=cps)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    t_fwd = t_end - t0 - gen[0]
    per = [b[0] - a[1] for a, b in zip(marks, marks[1:] + [[t_end, t_end]])]
    log("  forward steps (ms): " + " ".join(f"{1e3 * x:.0f}" for x in per))
    marks.clear()
    updates = sum(int(st["iters"].to(torch.int64).sum().item()) for st in stats) * cells_per_sys
    iters = [float(st["iters"].double().mean()) for st in stats]
    ctx.close()
    torch.cuda.empty_cache()
    log(f"  forward: {steps} steps in {1e3 * t_fwd:.0f} ms (generation {1e3 * gen[0]:.0f} ms excluded)")
    ctx = tm.Context(prob_d)
    batch = prealloc_workspace(torch, ctx)
    # The FP64 plain path over the same steps (psi carried over on its own), each step's state compared
    # with the mixed checkpoint on every cell (tau metric); untimed.
    prev, cur, vs64 = psi0.clone(), torch.empty_like(psi0), []
    for s in range(steps):
        f = fields_at(s)
        cur.copy_(prev)
        ctx.newton_step(f, prev, cur, max_iter, rtol)
        vs64.append(rel_err_gpu(cps[s], cur))
        prev, cur = cur, prev
    del prev, cur
    log("  mixed vs FP64 per step: " + " ".join(f"{e:.1e}" for e in vs64))
    gen[0] = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d0 = multistep.adjoint(ctx, fields_at, psi0, cps)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0 - gen[0]
    finite = bool(torch.isfinite(d0).all().item())
    log(f"  adjoint: {steps} steps in {1e3 * t_adj:.0f} ms (generation {1e3 * gen[0]:.0f} ms excluded, "
        f"factor batches of {batch} systems)")
    ctx.close()
    held.clear()
    del cps, d0
    torch.cuda.empty_cache()
    return dict(steps=steps, forward_ms=1e3 * t_fwd, adjoint_ms=1e3 * t_adj,
                forward_updates_per_s=updates / t_fwd, mean_iters_per_step=iters,
                mixed_vs_fp64_per_step=vs64, adjoint_precision="fp64", adjoint_factor_batch=batch,
                checkpoints=steps, gradient_finite=finite)


def ye_factor_flops_per_zone(N: int) -> float:
    """Algorithmic flops of one coupled block of M = 2N+1 rows (nu_e, anti-nu_e, Y_e) per zone and
    Newton update: in-place Gauss-Jordan on [A | diag(b) | g], M steps of (M-1) row updates of M+1
    entries (2M(M^2-1)), plus the Schur update diag(bm) C and the back substitution (4M^2)."""
    M = 2 * N + 1
    return 2.0 * M * (M * M - 1) + 4.0 * M * M


def ye_factor_bytes_per_zone(N: int) -> float:
    """Algorithmic HBM bytes of one coupled block per zone and launch: 2N cells reading psi, kappa_a,
    eta, kappa_s, the residual and the two Y_e derivatives and writing the update (8 x 8 B), plus the
    stored factors C_i and y_i ((2N+1) x (2N+1) doubles) written forward and read back."""
    M = 2 * N + 1
    return 2 * N * 64.0 + 2.0 * M * M * 8


def ye_leg(tm, torch, synth, w, f, rays, steps, warmup, rtol, max_iter):
    """FP64 Y_e-coupled Newton step of species 0 and 1 of every ray (block 2N+1) to the same rule."""
    y = synth.ye_inputs(w, 4, rays=rays)
    ctx = tm.Context(tm.problem_of(w, tm.PREC_FP64))
    ctx.set_workspace(ctx.ye_workspace_bytes(0))
    psi = torch.empty_like(w.psi_n)
    ye = torch.empty_like(y.ye_n)
    times, iters, st, stats = [], None, None, None
    for s in range(warmup + steps):
        psi.copy_(w.psi_n)
        ye.copy_(y.ye_n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, stats = ctx.ye_newton_step(f, y, w.psi_n, psi, ye, max_iter, rtol, raise_on_status=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        iters = stats["iters"].to(torch.int64)
        log(f"  {'warm' if s < warmup else 'step'} {s}: {1e3 * (t1 - t0):.1f} ms, iters min {int(iters.min())} "
            f"max {int(iters.max())}, status {tm.STATUS_NAMES.get(st, st)}")
        if s >= warmup:
            times.append(t1 - t0)
    upd = int(iters.sum().item())                      # coupled block updates (ray x update)
    t = sum(times) / len(times)
    zones_upd = upd * w.I
    res = dict(status=tm.STATUS_NAMES.get(st, st), flags_max=int(stats["flags"].max().item()))
    ctx.close()
    del psi, ye, y
    torch.cuda.empty_cache()
    return dict(ms_per_step=1e3 * t, value=zones_upd * 2 * w.N / t, unit="updates/s (nu_e and anti-nu_e cells)",
                mean_iters=float(iters.double().mean()), precision="fp64", block=2 * w.N + 1,
                factor_flops_per_update=ye_factor_flops_per_zone(w.N) * w.R * w.I,
                factor_bytes_per_update=ye_factor_bytes_per_zone(w.N) * w.R * w.I,
                **res)


def energy_bytes(cells: int, zones: int) -> float:
    """Algorithmic HBM bytes of one energy-advection launch: read psi and the Eddington factor and write
    psi (3 x 8 B per cell), and six zone arrays (rho, lapse before and after, dR/R, db/b) once per zone."""
    return 24.0 * cells + 48.0 * zones


def energy_leg(tm, torch, synth, w, rays, reps):
    """Energy-advection update (Lagrangian energy shift, PPM remap, over-fill limiter) of every zone of
    the workload: one launch timed with HIP events on the library's stream, `reps` times."""
    e = synth.eadv_inputs(w, 4, rays=rays)
    ctx = tm.Context(tm.problem_of(w, tm.PREC_FP64))
    psi = w.psi_n.clone()
    kw = dict(rho_old=e.rho_old, rho_new=e.rho_new, lapse_old=e.lapse_old, lapse_new=e.lapse_new, dlnR=e.dlnR,
              dlnb=e.dlnb, eddington=e.eddington)
    t = time_kernel(torch, lambda: ctx.energy_advect(w.e_edge, psi, **kw), reps)
    ctx.close()
    del psi, e
    torch.cuda.empty_cache()
    cells, zones = w.n_cells, w.R * w.I
    b = energy_bytes(cells, zones)
    # counters taken on the full 16384-ray launch; a reduced run reports none
    tr = traffic_record(os.path.join(ROOT, "paper_1809_05608_amd", "csrc", "tm_energy.hip"),
                        "k_energy_advect_traffic.json") if rays is None else None
    return dict(kernel="k_energy_advect<20>", kernel_ms=1e3 * t, cells_per_s=cells / t,
                zone_updates_per_s=w.S * zones / t, algorithmic_bytes_per_launch=b, achieved_gbs=b / t / 1e9,
                hbm_frac=b / t / 1e9 / PEAK_HBM_GBS, traffic=(tr or {}).get("bytes_per_launch"))


def cpu_baseline(sample_systems: int, workers: int):
    """The FP64 oracle (as written, untuned) on a bounded sample of systems of the same workload."""
    import multiprocessing as mp
    import numpy as np
    import synth
    rays = list(range(0, 16384, 16384 // max(1, sample_systems // 4)))[: max(1, sample_systems // 4)]
    w = synth.make(4, rays=rays, device="cpu").numpy()
    jobs = [(s, r) for r in range(len(rays)) for s in range(4)][:sample_systems]
    args = []
    for s, r in jobs:
        one = {k: (v[s:s + 1, r:r + 1] if k in ("kappa_a", "eta", "kappa_s", "psi_n") else
                   v[s:s + 1, r:r + 1] if k == "nes_amp" else v[r:r + 1] if k in ("r_edge", "temp") else v)
               for k, v in w.items()}
        one.update(S=1, R=1)
        args.append(one)
    # one single-threaded worker process per core (fresh interpreters: no inherited thread pools)
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            pool.map(_noop, range(workers))            # interpreter start-up outside the timed region
            t0 = time.perf_counter()
            res = pool.map(_oracle_one, args, chunksize=1)
            dt = time.perf_counter() - t0
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    upd = sum(it for it in res) * w["I"] * w["N"]
    return upd / dt, dt, len(jobs), upd


def _pool_map(fn, args, workers):
    """Map `fn` over `args` on `workers` single-threaded spawned processes; returns (results, wall s)."""
    import multiprocessing as mp
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            pool.map(_noop, range(workers))            # interpreter start-up outside the timed region
            t0 = time.perf_counter()
            res = pool.map(fn, args, chunksize=1)
            dt = time.perf_counter() - t0
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return res, dt


def cpu_baseline_ye(sample_rays: int, workers: int):
    """The Y_e-coupled oracle (FP64 Newton to the same rule) on `sample_rays` rays of the workload."""
    import synth
    rays = list(range(0, 16384, 16384 // sample_rays))[:sample_rays]
    w = synth.make(4, rays=rays, device="cpu")
    y = synth.ye_inputs(w, 4, rays=rays)
    wn, yn = w.numpy(), y.numpy()
    args = [({k: (v[:, r:r + 1] if k in ("kappa_a", "eta", "kappa_s", "psi_n", "nes_amp") else
                  v[r:r + 1] if k in ("r_edge", "temp") else v) for k, v in wn.items()},
             {k: (v[:, r:r + 1] if k in ("dka_dye", "deta_dye") else v[r:r + 1]) for k, v in yn.items()})
            for r in range(len(rays))]
    for a in args:
        a[0].update(R=1)
    res, dt = _pool_map(_ye_oracle_one, args, workers)
    upd = sum(res) * 2 * w.I * w.N
    return dict(value=upd / dt, unit="updates/s (nu_e and anti-nu_e cells)", cores=workers, kind="oracle",
                sample=f"{len(rays)} rays of the workload, coupled FP64 Newton to 1e-12, {sum(res)} block "
                       f"updates in {dt:.1f} s wall")


def _ye_oracle_one(a):
    from oracle import ye_coupled as yc
    wn, yn = a
    cs = yc.coupled_systems(wn, yn)[0]
    u_n = yc.pack(wn["psi_n"][0, 0], wn["psi_n"][1, 0], cs.ye_n)
    return yc.newton(cs, u_n, max_iter=30, rtol=1e-12).iters


def cpu_baseline_energy(sample_rays: int):
    """The energy-advection oracle (vectorised NumPy, one process) on `sample_rays` rays of the workload."""
    import synth
    from oracle import energy_advection as ea
    rays = list(range(0, 16384, 16384 // sample_rays))[:sample_rays]
    w = synth.make(4, rays=rays, device="cpu")
    e = synth.eadv_inputs(w, 4, rays=rays)
    wn, en = w.numpy(), e.numpy()
    t0 = time.perf_counter()
    ea.energy_advect(wn["psi_n"], wn["e_edge"], rho_old=en["rho_old"], rho_new=en["rho_new"], a_old=en["lapse_old"],
                     a_new=en["lapse_new"], dlnR=en["dlnR"], dlnb=en["dlnb"], eddington=en["eddington"])
    dt = time.perf_counter() - t0
    cells = wn["psi_n"].size
    return dict(value=cells / dt, unit="cells/s", cores=1, kind="oracle",
                sample=f"{len(rays)} rays x 540 zones x 4 species ({cells // w.N} zones) of the workload in "
                       f"{dt:.1f} s")


def _noop(_):
    import oracle  # noqa: F401
    return 0


def _oracle_one(w):
    import oracle
    sysm = oracle.systems_from_workload(w)[0][0]
    return oracle.newton(sysm, w["psi_n"][0, 0], max_iter=30, rtol=1e-12).iters


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--max-iter", type=int, default=30)
    ap.add_argument("--rays", type=int, default=16384, help="rays of the 16384-ray workload to use")
    ap.add_argument("--kernel-reps", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--multistep", type=int, default=10,
                    help="steps of the multi-step leg (drifting inputs, checkpointed adjoint); 0 skips it")
    ap.add_argument("--ye-steps", type=int, default=1,
                    help="timed steps of the FP64 Y_e-coupled leg (species 0 and 1 with Y_e); 0 skips it")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--profile-pass", action="store_true",
                    help="short pass for rocprofv3: one mixed step, one launch of each timed kernel, "
                         "and a plain 1 GiB device copy that calibrates the HBM byte counters")
    a = ap.parse_args(argv)
    if a.profile_pass:
        a.steps, a.warmup, a.kernel_reps, a.no_fp64, a.no_cpu, a.multistep = 1, 0, 1, True, True, 0
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {a.gpus} requested); the transport systems of a "
              "multi-GPU run would be sharded by ray with no exchange inside a step", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_1809_05608_amd import tm

    torch.cuda.init()
    dev = torch.device("cuda", 0)
    log("generating inputs in HBM")
    rays = None if a.rays >= 16384 else range(a.rays)
    w = synth.make(4, rays=rays, device=dev)
    f = tm.DeviceFields.of(w)
    torch.cuda.synchronize()
    cells = w.n_cells
    log(f"workload {w.name}: {w.S}x{w.R}x{w.I}x{w.N} = {cells} cells")

    if a.profile_pass:
        # calibration: a plain copy of exactly 1 GiB (reads 1 GiB, writes 1 GiB)
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 1 GiB device-to-device copy done")

    # ---------------- mixed-precision leg (headline)
    log("mixed-precision Newton")
    ctx_m, psi_m, st_m, t_m, u_m = run_newton_leg(tm, torch, w, f, tm.PREC_MIXED, a.steps, a.warmup, a.rtol,
                                                  a.max_iter)
    mixed_iters = st_m["iters"].to(torch.float64)
    # dominant kernel: the FP32 fused assembly + block-Thomas factor/solve, one launch per call
    G = torch.empty_like(psi_m)
    ctx_m.assemble(f, w.psi_n, w.psi_n, G)
    x = torch.empty_like(psi_m)
    t_fac = time_factor_kernel(ctx_m, lambda: ctx_m.factor_solve(f, w.psi_n, G, x), a.kernel_reps)
    t_res = time_kernel(torch, lambda: ctx_m.assemble(f, w.psi_n, w.psi_n, G), a.kernel_reps)
    del G, x
    ctx_m.close()
    torch.cuda.empty_cache()

    out_fp64 = None
    out_adj = None
    err_mixed = None
    if not a.no_fp64:
        log("FP64 Newton")
        ctx_d, psi_d, st_d, t_d, u_d = run_newton_leg(tm, torch, w, f, tm.PREC_FP64, a.steps, a.warmup, a.rtol,
                                                      a.max_iter)
        err_mixed = rel_err_gpu(psi_m, psi_d)
        xs = torch.empty_like(psi_d)
        t_fac64 = time_factor_kernel(ctx_d, lambda: ctx_d.factor_solve(f, w.psi_n, psi_m, xs), 1)
        del xs
        out_fp64 = dict(value=sum(u_d) / sum(t_d), ms_per_step=1e3 * sum(t_d) / len(t_d),
                        mean_iters=float(st_d["iters"].double().mean()), factor_kernel_ms=1e3 * t_fac64)
        if not a.no_adjoint:
            log("FP64 adjoint")
            seed = torch.empty_like(psi_d)
            ctx_d.luminosity_seed(f, seed)
            mu = torch.empty_like(psi_d)
            g = [torch.empty_like(psi_d) for _ in range(3)]
            gamp = torch.empty_like(w.nes_amp)
            tadj = time_kernel(torch, lambda: ctx_d.adjoint_step(f, w.psi_n, psi_d, seed, mu, *g, gamp),
                               max(1, a.steps))
            out_adj = dict(ms_per_step=1e3 * tadj, finite=bool(torch.isfinite(g[0]).all().item()))
            del seed, mu, g, gamp
        ctx_d.close()
        del psi_d
        torch.cuda.empty_cache()

    log("energy advection (Lagrangian shift, PPM remap, over-fill limiter)")
    out_energy = energy_leg(tm, torch, synth, w, rays, a.kernel_reps)

    out_ye = None
    if a.ye_steps > 0:
        log("FP64 Y_e-coupled Newton (species 0 and 1 with Y_e)")
        out_ye = ye_leg(tm, torch, synth, w, f, rays, a.ye_steps, 0 if a.profile_pass else 1, a.rtol, a.max_iter)

    value = sum(u_m) / sum(t_m)
    ms = 1e3 * sum(t_m) / len(t_m)
    # roofline of one Newton iteration at the algorithmic count (48 B and 2N^2 + 20N flops per cell),
    # charged to the dominant kernel (the float32 factor/solve launch) and to the whole step
    rm = roofline_time(cells, w.N, mixed=True)
    kernel_src = os.path.join(ROOT, "paper_1809_05608_amd", "csrc", "tm_factor_q.hip")
    # the counters were taken on the full 16384-ray launch; a reduced run reports none
    tr = traffic_record(kernel_src) if rays is None else None
    traffic = (tr or {}).get("bytes_per_launch")
    iters_mean = float(mixed_iters.mean())
    if rm["t_alu"] >= rm["t_hbm"]:
        # compute-bound: achieved flop rate against the blended peak of the FP32 and FP64 parts
        peak = rm["flops"] / rm["t_alu"] / 1e12
        roof = dict(bound="alu", achieved=rm["flops"] / t_fac / 1e12, peak=peak, unit="TFLOP/s")
    else:
        roof = dict(bound="hbm", achieved=rm["bytes"] / t_fac / 1e9, peak=PEAK_HBM_GBS, unit="GB/s")
    roof.update(frac=rm["t_roof"] / t_fac, traffic=traffic,
                traffic_over_algorithmic=(traffic / rm["bytes"]) if traffic else None,
                kernel=KERNEL_F32, kernel_ms=1e3 * t_fac, roofline_ms=1e3 * rm["t_roof"],
                roofline_hbm_ms=1e3 * rm["t_hbm"], roofline_alu_ms=1e3 * rm["t_alu"],
                algorithmic_bytes_per_launch=rm["bytes"], flops_per_launch=rm["flops"],
                flops_fp32_per_launch=rm["flops_fp32"], flops_fp64_per_launch=rm["flops_fp64"],
                peaks=dict(fp32_tflops=PEAK_FP32_TFLOPS, fp64_tflops=PEAK_FP64_TFLOPS, hbm_gbs=PEAK_HBM_GBS),
                stored_factor_bytes_per_launch=stored_factor_bytes_per_cell(w.N, 4) * cells,
                step_roofline_ms=1e3 * rm["t_roof"] * iters_mean, step_frac=(rm["t_roof"] * iters_mean) / (ms / 1e3),
                residual_kernel_ms=1e3 * t_res)
    if out_fp64 is not None:
        rd = roofline_time(cells, w.N, mixed=False)
        out_fp64["roofline"] = dict(kernel_frac=rd["t_roof"] / (out_fp64["factor_kernel_ms"] / 1e3),
                                    roofline_ms=1e3 * rd["t_roof"],
                                    step_frac=rd["t_roof"] * out_fp64["mean_iters"] / (out_fp64["ms_per_step"] / 1e3))

    wmeta = dict(name=w.name, R=w.R, I=w.I, N=w.N, S=w.S)
    multi = None
    if a.multistep > 0:
        log(f"multi-step leg: {a.multistep} drifting steps, then the checkpointed adjoint")
        del psi_m, f, w
        torch.cuda.empty_cache()
        multi = multistep_leg(tm, torch, synth, dev, rays, a.multistep, a.rtol, a.max_iter)

    cpu = None
    if not a.no_cpu:
        log("CPU oracle baseline")
        workers = host_cores()
        v, dt, nsys, upd = cpu_baseline(a.cpu_sample, workers)
        cpu = dict(value=v, unit="updates/s", cores=workers, kind="oracle", cpu_model=cpu_model(),
                   sample=f"{nsys} systems (species x rays spread over the 16384 rays) of the same workload, "
                          f"FP64 Newton to 1e-12, {upd} updates in {dt:.1f} s wall")
        if out_ye is not None:
            log("CPU oracle baseline of the Y_e-coupled step")
            out_ye["cpu_oracle"] = cpu_baseline_ye(16, workers)
        log("CPU oracle baseline of the energy advection")
        out_energy["cpu_oracle"] = cpu_baseline_energy(16)

    res = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 factor + f64 residual", "data": "synthetic",
        "config": {"workload": f"{wmeta['name']}: one implicit step, mixed precision Newton to rtol {a.rtol:g}",
                   "rays": wmeta["R"], "zones": wmeta["I"], "groups": wmeta["N"], "species": wmeta["S"],
                   "cells": cells,
                   "mean_newton_iters": float(mixed_iters.mean())},
        "mixed_err_vs_fp64": err_mixed,
        "fp64": out_fp64,
        "mixed_vs_fp64_speedup": (out_fp64["ms_per_step"] / ms) if out_fp64 else None,
        "adjoint_fp64": out_adj,
        "ye_coupled_fp64": out_ye,
        "energy_advection": out_energy,
        "multistep": multi,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
