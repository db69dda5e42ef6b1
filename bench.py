"""Benchmark: site*ray*wavelength updates per second of the formal solution on a
262,144-site Voronoi grid (64 wavelengths 400-900 nm, 24 rays), one GPU.

One step = grey LTE source assembly (chi = kappa0 rho^2 T^9, S = B_lambda(T),
a site's two rows side by side in one [n][2][64] array unless --rows separate)
+ the FP32 formal solution of all 24 rays in the launch mode and layout the
library's autotuner picks (the persistent sweep or graph-captured level steps)
+ the angle quadrature of J (double accumulation) + the emergent-intensity
gather. Inputs (T, rho) are resident on the GPU before the
timed region. The grid, its quadrature and the per-ray schedules are built
once, outside the timed region.

Printed as one JSON line with, besides the headline value:
  roofline     the sweep kernel's algorithmic bytes per launch over its mean
               launch time (HIP events on the library's stream), vs 8 TB/s;
  fp64_plain   the plain FP64 GPU path (one launch per ray and level) and the
               FP32-batched speed-up over it;
  bezier_segment  the formal solution with the quadratic Bezier segment and
               its time relative to the linear one;
  adjoint      forward and reverse-sweep times of the differentiable emergent
               intensity (32 wavelengths 500-700 nm on the same grid) and
               their ratio;
  regular_grid the same formal solution on the regular 128 x 128 x 256 grid
               (short characteristics), FP32 graph-launched and plain FP64;
  synthesis    the final synthesis from the Voronoi grid to that regular grid
               with the 101-point line: the nearest-site map (once per grid
               pair) and the mu = 1 long-characteristics line synthesis in FP32
               and FP64, with its algorithmic HBM rate;
  cpu_baseline the FP64 CPU oracle timed on this host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sites N] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (first processor entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def sweep_bytes_per_update(nl: int, fp: int) -> float:
    """Algorithmic HBM bytes of the sweep kernel per site*ray*wavelength update:
    read S_i and chi_i, write I_i (3 * fp bytes), plus the per-(ray, site) sweep
    record (16 B of indices + 4 * fp bytes of weights and lengths) shared by
    the nl wavelengths. Upwind gathers are not counted (served on chip in the
    ideal streaming model)."""
    return 3.0 * fp + (16.0 + 4.0 * fp) / nl


LAYOUT_KEYS = ("record_order", "shared_levels", "xcd_chunks", "ray_affinity", "chains", "lane_bytes", "interleave",
               "pipeline", "rows")
# layout values of summaries that predate a key
LAYOUT_DEFAULTS = {"rows": "separate"}


def counter_traffic(nl, n, mode, layout):
    """HBM bytes per sweep launch measured by rocprofv3 counters (FETCH_SIZE x
    its copy-kernel calibration + WRITE_SIZE), read from the committed profile
    summary, or None when that summary was taken on another workload, another
    launch layout or kernel sources that have changed since."""
    import hashlib

    persistent = mode == "persistent"
    name = "persistent_sweep_c1_counters.json" if persistent else "sweep_kernel_c1_counters.json"
    path = os.path.join(ROOT, "profiles", name)
    if nl != 64 or n != 262144 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    srcs = ("k_persist.hip", "persist.h", "segment.h") if persistent else ("k_sweep.hip", "segment.h")
    for f in srcs:
        h.update(open(os.path.join(ROOT, "paper_2306_01041_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    # one entry per measured layout: the persistent sweep reads the per-ray
    # record order or, with an interleaved copy built, that copy (wave items
    # then mix rays), and its work items follow the level steps
    keys = ("shared_levels", "interleave", "rows") if persistent else LAYOUT_KEYS
    for e in rec.get("entries", [rec]):
        if all(e.get("layout", {}).get(k, LAYOUT_DEFAULTS.get(k, 0)) == layout.get(k, LAYOUT_DEFAULTS.get(k, 0))
               for k in keys):
            return e["sweep_bytes_per_launch"]["total"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sites", type=int, default=262144)
    ap.add_argument("--nl", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward timing")
    ap.add_argument("--no-regular", action="store_true", help="skip the regular-grid and synthesis timings")
    ap.add_argument("--no-synthesis", action="store_true", help="skip the final-synthesis timing")
    ap.add_argument("--no-bezier", action="store_true", help="skip the quadratic-segment timing")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the grid's default launch layout (for profiler runs that average over dispatches)")
    ap.add_argument("--interleave", type=int, choices=[0, 1, 2], default=0,
                    help="with a fixed layout (c1: --no-autotune; c2/c3: --mode other than auto): sweep the "
                         "interleaved record copy, in Morton order (1) or in site-index order (2)")
    ap.add_argument("--shared-levels", type=int, choices=[0, 1], default=0,
                    help="with a fixed layout: one level schedule for the rays of one azimuth and hemisphere")
    ap.add_argument("--pipeline", type=int, choices=[0, 2, 4, 8], default=0,
                    help="with a fixed layout: interior level steps launch the pipelined sweep kernel with this "
                         "many groups of records in flight per wavefront (0: the plain level-step kernel)")
    ap.add_argument("--rows", choices=["paired", "separate"], default="paired",
                    help="timed formal solutions: chi and S of a site in one [2][n_lambda] row pair "
                         "(vrt_formal_solution_ld, the layout of the two-level iteration) or in separate arrays")
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "synth", "design"], default="c1",
                    help="c1: the formal solution (default line); c2: the two-level Lambda iteration on 1,048,576 "
                         "sites; c3: 48 atmospheres of 32,768-524,288 sites solved as one batch; synth: only the "
                         "final synthesis from the 262,144-site grid to the regular 128 x 128 x 256 grid; "
                         "design: the grid-design accuracy workload (searchlight beams, LTE continuum "
                         "intensities against site count and sampling density)")
    ap.add_argument("--accel", action="store_true",
                    help="c2/c3: the Jacobi-accelerated iteration (local operator) instead of the plain one")
    ap.add_argument("--max-iter", type=int, default=None,
                    help="iteration cap of the timed plain c2/c3 Lambda iterations (default 20 for c2, 10 for c3; "
                         "the accelerated iteration runs to convergence)")
    ap.add_argument("--mode", choices=["auto", "graph", "batched", "persistent"], default="auto",
                    help="launch mode of the timed steps (auto: the faster of graph and persistent)")
    ap.add_argument("--workers", type=int, default=16,
                    help="processes that build the c3 batch's atmospheres (1: in this process, e.g. under a profiler)")
    ap.add_argument("--no-accel", action="store_true",
                    help="c2/c3 alone: skip the accelerated iteration to convergence (short profiler runs)")
    ap.add_argument("--inputs-cache", default=None, metavar="DIR",
                    help="c2/c3: read the atmospheres from DIR/<workload>.npz, or build and write them there (a "
                         "run that reads the cache starts no worker processes)")
    ap.add_argument("--no-lambda", action="store_true",
                    help="default run: skip the c2 and c3 two-level iteration blocks")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (to scale HBM counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        a = torch.ones(args.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "synth":
        run_synthesis_only(args)
        return
    if args.workload == "design":
        run_design(args)
        return
    if args.workload != "c1":
        run_lambda(args)
        return

    import torch

    import paper_2306_01041_amd
    import synth

    v = paper_2306_01041_amd.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    seed = 1041
    nl = args.nl
    lam = np.linspace(400e-9, 900e-9, nl)

    t0 = time.time()
    atm = synth.make_atmosphere(args.sites, seed=seed)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature()
    R = len(dirs)
    log(f"grid {g.n} sites, {g.m / g.n:.2f} neighbours/site, built in {time.time() - t0:.1f} s")

    ctx = v.Context(0)
    stream = torch.cuda.current_stream()
    G = v.Grid.from_synth(ctx, g)
    t0 = time.time()
    G.set_rays(dirs, w, 7.0)
    info = G.info()
    setup_s = time.time() - t0
    log(f"rays set in {setup_s:.2f} s: {info}")

    T = torch.as_tensor(atm.T, device=dev)
    rho = torch.as_tensor(atm.rho, device=dev)
    f32 = torch.float32
    chi = torch.empty((g.n, nl), dtype=f32, device=dev)
    S = torch.empty_like(chi)
    J = torch.empty_like(chi)
    # the timed steps' opacity and source: a site's two rows side by side
    # (views of one [n][2][nl] array) or the separate arrays above
    if args.rows == "paired":
        cs = torch.empty((g.n, 2, nl), dtype=f32, device=dev)
        chi_t, S_t = cs[:, 0], cs[:, 1]
    else:
        chi_t, S_t = chi, S
    off, _ = G.emergent_index()
    em = torch.empty((int(off[-1]), nl), dtype=f32, device=dev)

    modes = {"graph": v.VRT_EXEC_GRAPH, "batched": v.VRT_EXEC_BATCHED, "persistent": v.VRT_EXEC_PERSISTENT}
    # the library's autotuner times the launch layouts and the persistent sweep
    # on this workload and keeps the fastest on the grid (its launch mode too)
    v.lte_continuum(G, lam, atm.kappa0, T, rho, chi, S)
    if chi_t is not chi:
        v.lte_continuum(G, lam, atm.kappa0, T, rho, chi_t, S_t)
    # (the autotuner takes arrays of n x n_lambda)
    tuning = None if args.no_autotune else v.autotune(G, chi, S, J, reps=5)
    log(f"autotune: {tuning}")
    if tuning is None:
        G.tune(v.VRT_TUNE_SHARED_LEVELS, args.shared_levels)
        G.tune(v.VRT_TUNE_INTERLEAVE, args.interleave)
        G.tune(v.VRT_TUNE_PIPELINE, args.pipeline)
    layout = dict(tuning["chosen"]) if tuning else {"record_order": 1, "shared_levels": args.shared_levels,
                                                    "xcd_chunks": 8, "ray_affinity": 0, "chains": 1,
                                                    "lane_bytes": 16, "interleave": args.interleave,
                                                    "pipeline": args.pipeline}
    layout.setdefault("chains", 1)  # the autotuner times one launch chain
    layout["rows"] = args.rows
    mode_times = {}
    if args.mode == "auto" and tuning:
        args.mode = tuning["chosen"]["exec"]
        for c in tuning["candidates"]:
            if c["ms"] is not None and c["ms"] < mode_times.get(c["exec"], float("inf")):
                mode_times[c["exec"]] = c["ms"]
        log(f"launch modes (best ms per formal solution in the autotuner): {mode_times} -> {args.mode}")
    elif args.mode == "auto":
        for name in ("graph", "persistent"):
            try:
                for _ in range(2):
                    v.formal_solution(G, chi_t, S_t, J, exec_mode=modes[name])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    v.formal_solution(G, chi_t, S_t, J, exec_mode=modes[name])
                G.device_status()
                mode_times[name] = (time.perf_counter() - t0) * 1e3 / 5
            except v.VrtError as e:  # a mode that reports an error is not a candidate
                log(f"launch mode {name} failed: {e}")
        args.mode = min(mode_times, key=mode_times.get)
        log(f"launch modes (ms per formal solution): {mode_times} -> {args.mode}")
    mode = modes[args.mode]

    def step():
        v.lte_continuum(G, lam, atm.kappa0, T, rho, chi_t, S_t)
        v.formal_solution(G, chi_t, S_t, J, exec_mode=mode)
        v.emergent_gather(G, em)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warm-up done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    G.device_status()
    ms_step = (t1 - t0) * 1e3 / args.steps
    updates = g.n * R * nl
    value = updates / (ms_step * 1e-3)
    log(f"FP32 {args.mode} step {ms_step:.3f} ms -> {value:.3e} updates/s")

    # roofline of the dominant kernel (the sweep): HIP events on the library's
    # stream around the formal solution as launched in the timed steps, minus the
    # angle-quadrature kernel timed on its own (one launch), over the sweep launches
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nprof = 10
    ev0.record(stream)
    for _ in range(nprof):
        v.formal_solution(G, chi_t, S_t, J, exec_mode=mode)
    ev1.record(stream)
    ev1.synchronize()
    fs_ms = ev0.elapsed_time(ev1) / nprof
    ctx.profile_reset()
    ctx.set_profiling(True)
    for _ in range(3):
        v.formal_solution(G, chi_t, S_t, J, exec_mode=v.VRT_EXEC_BATCHED)
    sw_ms_ev, sw_launches, sw_units = ctx.profile(0)
    jr_ms, jr_launches, jr_units = ctx.profile(1)
    ctx.set_profiling(False)
    torch.cuda.synchronize()
    jr_one = jr_ms / jr_launches
    launches = sw_launches // 3 if args.mode != "persistent" else 1
    sweep_ms = fs_ms - jr_one
    bpu = sweep_bytes_per_update(nl, 4)
    avg_launch_ms = sweep_ms / launches
    bytes_per_launch = bpu * updates / launches
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    jr_bytes = (4.0 + 4.0 / R) * jr_units / jr_launches  # read every ray's I once, write J once
    traffic = counter_traffic(nl, g.n, args.mode, layout)
    log(f"sweep: {launches} launches/step, {sweep_ms:.3f} ms, mean {avg_launch_ms * 1e3:.2f} us/launch, "
        f"{achieved:.0f} GB/s algorithmic (counters: {traffic}); J quadrature {jr_one:.3f} ms "
        f"({jr_bytes / (jr_one * 1e-3) / 1e9:.0f} GB/s)")

    # plain FP64 GPU path: one launch per (ray, level), on each ray's own level
    # schedule (levels shared by a group of rays would add launches here)
    fp64 = None
    if not args.no_fp64:
        if layout.get("shared_levels"):
            G.tune(v.VRT_TUNE_SHARED_LEVELS, 0)
        f64 = torch.float64
        chi64 = torch.empty((g.n, nl), dtype=f64, device=dev)
        S64 = torch.empty_like(chi64)
        J64 = torch.empty_like(chi64)
        v.lte_continuum(G, lam, atm.kappa0, T, rho, chi64, S64)
        v.formal_solution(G, chi64, S64, J64, exec_mode=v.VRT_EXEC_PLAIN)
        torch.cuda.synchronize()
        k64 = 3
        t0 = time.perf_counter()
        for _ in range(k64):
            v.lte_continuum(G, lam, atm.kappa0, T, rho, chi64, S64)
            v.formal_solution(G, chi64, S64, J64, exec_mode=v.VRT_EXEC_PLAIN)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / k64
        # error of the FP32 path against the FP64 GPU path on this workload
        jerr = float(((J.double() - J64).abs() / J64.abs()).max().item())
        fp64 = {"ms_per_step": round(ms64, 3), "value": updates / (ms64 * 1e-3),
                "speedup_fp32_batched": round(ms64 / ms_step, 2), "fp32_vs_fp64_max_rel_err_J": jerr}
        log(f"FP64 plain step {ms64:.2f} ms; FP32 {args.mode} speed-up {ms64 / ms_step:.1f}x; FP32 J err {jerr:.2e}")
        del chi64, S64, J64
        if layout.get("shared_levels"):
            G.tune(v.VRT_TUNE_SHARED_LEVELS, 1)

    # the quadratic Bezier segment on the same grid and fields (FP32, graph-launched)
    bezier = None
    if not args.no_bezier:
        G.tune(v.VRT_TUNE_SEGMENT, 1)
        ms_by_mode = {}
        for name, m in (("graph", v.VRT_EXEC_GRAPH), ("persistent", v.VRT_EXEC_PERSISTENT)):
            try:
                v.formal_solution(G, chi_t, S_t, J, exec_mode=m)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(5):
                    v.formal_solution(G, chi_t, S_t, J, exec_mode=m)
                e1.record(stream)
                e1.synchronize()
                G.device_status()
                ms_by_mode[name] = e0.elapsed_time(e1) / 5
            except v.VrtError as e:
                log(f"Bezier launch mode {name} not used: {e}")
        G.tune(v.VRT_TUNE_SEGMENT, 0)
        mode_b = min(ms_by_mode, key=ms_by_mode.get)
        ms_b = ms_by_mode[mode_b]
        bezier = {"workload": "the same formal solution with the quadratic Bezier segment (FP32)",
                  "launch_mode": mode_b, "ms": round(ms_b, 3), "updates_per_s": updates / (ms_b * 1e-3),
                  "ms_by_mode": {k: round(t, 3) for k, t in ms_by_mode.items()},
                  "over_linear": round(ms_b / fs_ms, 2)}
        log(f"Bezier segment: {ms_b:.3f} ms per formal solution ({mode_b}; {ms_by_mode}; "
            f"{ms_b / fs_ms:.2f}x the linear one)")

    # adjoint of the LTE formal solution (same grid, 32 wavelengths 500-700 nm):
    # forward = continuum + formal solution keeping per-ray intensities + emergent
    # gather; backward = emergent scatter + reverse sweep + LTE chain rule
    adjoint = None
    if not args.no_adjoint:
        nl4 = 32
        lam4 = np.linspace(500e-9, 700e-9, nl4)
        rng = np.random.Generator(np.random.PCG64(seed + 1))
        T_tgt = torch.as_tensor(atm.T * (1.0 + 0.02 * rng.standard_normal(g.n)), device=dev)
        with torch.no_grad():
            target = v.lte_emergent(T_tgt, rho, G, lam4, atm.kappa0)
        Tq = T.clone().requires_grad_(True)
        rq = rho.clone().requires_grad_(True)

        def timed(emergent_dtype, **kw):
            def fwd():
                em4 = v.lte_emergent(Tq, rq, G, lam4, atm.kappa0, emergent_dtype=emergent_dtype, **kw)
                return ((em4.double() - target.double()) ** 2).sum()

            for _ in range(2):
                fwd().backward()
            torch.cuda.synchronize()
            fw_ms = bw_ms = 0.0
            k4 = 5
            for _ in range(k4):
                Tq.grad = rq.grad = None
                t0 = time.perf_counter()
                L = fwd()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                L.backward()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                fw_ms += (t1 - t0) * 1e3 / k4
                bw_ms += (t2 - t1) * 1e3 / k4
            return fw_ms, bw_ms

        u4 = g.n * R * nl4
        # the default pipeline (FP32 sweeps, the misfit's emergent intensities
        # from an FP64 forward sweep: gradients within 1e-4 of central
        # differences); the reverse sweep as level-step launches and as one
        # persistent launch, the faster reported as the adjoint time
        fw_l, bw_l = timed(None)
        G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 1)
        try:
            fw_p, bw_p = timed(None)
            G.device_status()
        except v.VrtError as e:
            log(f"persistent reverse sweep not used: {e}")
            fw_p = bw_p = float("inf")
        reverse_mode = "persistent" if bw_p < bw_l else "level steps"
        G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 1 if bw_p < bw_l else 0)
        fw_ms, bw_ms = (fw_p, bw_p) if bw_p < bw_l else (fw_l, bw_l)
        fw2, bw2 = timed(torch.float32)  # all-FP32
        G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 0)
        # memory-bounded backward: forward intensities dropped after the forward
        # pass and recomputed from per-level-chunk checkpoints (16 steps)
        ck = 16
        fw3, bw3 = timed(None, keep_intensities=False, checkpoint_levels=ck)
        mem = {key: v.formal_solution_vjp_scratch(G, torch.float32, nl4, keep_intensities=keep,
                                                  checkpoint_levels=kk)
               for key, keep, kk in (("kept", True, 0), ("recomputed", False, 0), ("checkpointed", False, ck))}
        adjoint = {"workload": f"adjoint of the LTE formal solution, {g.n} sites, {nl4} wavelengths 500-700 nm, "
                               f"{R} rays, FP32 sweeps, FP64 ray accumulation, loss sum (I_em - I_target)^2 with "
                               f"I_em from an FP64 forward sweep (gradient within 1e-4 of central differences)",
                   "forward_ms": round(fw_ms, 3), "adjoint_ms": round(bw_ms, 3),
                   "adjoint_over_forward": round(bw_ms / fw_ms, 3), "reverse_sweep": reverse_mode,
                   "adjoint_ms_by_reverse_sweep": {"level steps": round(bw_l, 3),
                                                   "persistent": None if bw_p == float("inf") else round(bw_p, 3)},
                   "forward_updates_per_s": u4 / (fw_ms * 1e-3), "adjoint_updates_per_s": u4 / (bw_ms * 1e-3),
                   "all_fp32": {"note": "misfit from the FP32 forward sweep (faster forward; gradient within "
                                        "2e-3 of central differences when the residuals are small)",
                                "forward_ms": round(fw2, 3), "adjoint_ms": round(bw2, 3),
                                "adjoint_over_forward": round(bw2 / fw2, 3)},
                   "checkpointed": {"note": f"forward intensities not kept; the reverse sweep recomputes them from "
                                            f"per-level-chunk checkpoints every {ck} level steps",
                                    "checkpoint_levels": ck, "forward_ms": round(fw3, 3),
                                    "adjoint_ms": round(bw3, 3), "adjoint_over_forward": round(bw3 / fw3, 3),
                                    "scratch_bytes": mem},
                   "grad_finite": bool(torch.isfinite(Tq.grad).all() and torch.isfinite(rq.grad).all())}
        log(f"adjoint: forward {fw_ms:.3f} ms, backward {bw_ms:.3f} ms ({reverse_mode}; level steps {bw_l:.3f}, "
            f"persistent {bw_p:.3f}), ratio {bw_ms / fw_ms:.2f}; all-FP32: {fw2:.3f} / {bw2:.3f} ms; "
            f"checkpointed every {ck} steps: {fw3:.3f} / {bw3:.3f} ms, scratch {mem}")
        del Tq, rq, target, T_tgt

    # the regular 128 x 128 x 256 grid of the same recipe (short characteristics):
    # FP32 graph-launched and plain FP64, 64 wavelengths, 24 rays
    regular = None
    synthesis = None
    if not args.no_regular:
        del chi, S, J, chi_t, S_t
        nx = ny = 128
        nz = 256
        dxr, dyr, zr, xyz = regular_recipe(atm.box, nx, ny, nz)
        atr = synth.make_atmosphere(len(xyz), seed=seed, xyz=xyz)
        Gr = v.Grid.regular(ctx, nx, ny, zr, dxr, dyr)
        Gr.set_rays(dirs, w)
        Tr, rr = torch.as_tensor(atr.T, device=dev), torch.as_tensor(atr.rho, device=dev)
        ur = len(xyz) * R * nl
        regular = {"workload": f"regular grid {nx}x{ny}x{nz}, {nl} wavelengths 400-900 nm, {R} rays, short "
                               f"characteristics with bilinear upwind interpolation"}
        for name, dt, mode, reps in (("fp32_graph", torch.float32, v.VRT_EXEC_GRAPH, 5),
                                     ("fp64_plain", torch.float64, v.VRT_EXEC_PLAIN, 2)):
            chr_ = torch.empty((len(xyz), nl), dtype=dt, device=dev)
            Sr = torch.empty_like(chr_)
            Jr = torch.empty_like(chr_)
            v.lte_continuum(Gr, lam, atr.kappa0, Tr, rr, chr_, Sr)
            if mode == v.VRT_EXEC_GRAPH:
                # the autotuner picks the plane kernel (rows or LDS tiles) for this workload
                regular["tuning"] = v.autotune(Gr, chr_, Sr, Jr, reps=2)["chosen"]
            v.formal_solution(Gr, chr_, Sr, Jr, exec_mode=mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                v.formal_solution(Gr, chr_, Sr, Jr, exec_mode=mode)
            torch.cuda.synchronize()
            ms_r = (time.perf_counter() - t0) * 1e3 / reps
            regular[name] = {"ms": round(ms_r, 3), "updates_per_s": ur / (ms_r * 1e-3)}
            Gr.tune(v.VRT_TUNE_REGULAR_TILE, 2)  # the FP64 plain path keeps the library default
            log(f"regular grid {name}: {ms_r:.2f} ms -> {ur / (ms_r * 1e-3):.3e} updates/s")
            del chr_, Sr, Jr
        regular["speedup_fp32_graph"] = round(regular["fp64_plain"]["ms"] / regular["fp32_graph"]["ms"], 2)
        # the two plane kernels (LDS-tiled upwind blocks, per-point rows) in both
        # precisions; the default takes the tiles in FP64 and the rows in FP32
        kernels = {}
        for name, dt, mode in (("fp32_graph", torch.float32, v.VRT_EXEC_GRAPH),
                               ("fp64_plain", torch.float64, v.VRT_EXEC_PLAIN)):
            chr_ = torch.empty((len(xyz), nl), dtype=dt, device=dev)
            Sr = torch.empty_like(chr_)
            Jr = torch.empty_like(chr_)
            v.lte_continuum(Gr, lam, atr.kappa0, Tr, rr, chr_, Sr)
            for tiled, key in ((1, "lds_tiles"), (0, "rows")):
                Gr.tune(v.VRT_TUNE_REGULAR_TILE, tiled)
                v.formal_solution(Gr, chr_, Sr, Jr, exec_mode=mode)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(2):
                    v.formal_solution(Gr, chr_, Sr, Jr, exec_mode=mode)
                torch.cuda.synchronize()
                kernels.setdefault(name, {})[key] = round((time.perf_counter() - t0) * 1e3 / 2, 3)
            del chr_, Sr, Jr
        Gr.tune(v.VRT_TUNE_REGULAR_TILE, 2)
        regular["plane_kernels_ms"] = kernels
        log(f"regular grid plane kernels (ms): {kernels}")
        if not args.no_synthesis:
            synthesis = run_synthesis(v, G, Gr, g, atm, atr, nx, ny, zr, stream)
        Gr.close()

    # CPU oracle on a bounded sample: the same formal solution (all sites, rays and
    # wavelengths), repeated until about 10 s of host time have been spent
    cpu = None
    if not args.no_cpu:
        import oracle

        chi_o, S_o = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
        sel = oracle.select(g, dirs)
        reps, dt = 0, 0.0
        while reps < 4 and dt < 10.0:
            t0 = time.perf_counter()
            oracle.fs_voronoi(g, dirs, w, sel, chi_o, S_o, S_o)
            dt += time.perf_counter() - t0
            reps += 1
        cpu = {"value": reps * updates / dt, "unit": "site*ray*lambda updates/s",
               "cores": oracle.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
               "sample": f"{reps} FP64 formal solution(s) of the full workload ({g.n} sites x {R} rays x {nl} "
                         f"wavelengths), {dt:.1f} s"}
        log(f"CPU oracle {cpu['value']:.3e} updates/s on {cpu['cores']} threads ({dt:.1f} s)")

    out = {
        "metric": "site*ray*lambda updates/s, FP32 batched formal solution (vs FP64 plain) + %HBM roofline; "
                  "adjoint/fwd",
        "value": value,
        "unit": "site*ray*lambda updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "launch_mode": args.mode,
        "mode_ms": mode_times,
        "data": "synthetic (seeded Bifrost-like stratified atmosphere, rejection-sampled Voronoi sites)",
        "config": {"workload": f"LTE continuum formal solution, Voronoi grid {g.n} sites, {nl} wavelengths "
                               f"400-900 nm, {R} rays, FP32 sweeps with FP64 J accumulation",
                   "sites": g.n, "rays": R, "wavelengths": nl, "levels_max": info["max_levels"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "algorithmic_bytes_per_launch": round(bytes_per_launch),
                     "kernel": sweep_kernel_names(args.mode, layout, 16), "bytes_per_update": round(bpu, 4),
                     "mean_launch_us": round(avg_launch_ms * 1e3, 2), "launches_per_step": launches,
                     "sweep_ms_per_step": round(sweep_ms, 4), "j_quadrature_ms": round(jr_one, 4)},
        "whole_step_effective_GBs": round(updates * (20.0 + 20.0 / nl) / (ms_step * 1e-3) / 1e9, 1),
        "fp64_plain": fp64,
        "bezier_segment": bezier,
        "adjoint": adjoint,
        "regular_grid": regular,
        "synthesis": synthesis,
        "cpu_baseline": cpu,
        "setup_s": round(setup_s, 3),
        "tuning": tuning,
        "layout": {k: layout.get(k) for k in LAYOUT_KEYS},
    }
    G.close()
    ctx.close()
    del stream, T, rho, em
    torch.cuda.empty_cache()
    # the two-level iteration workloads, whose sweeps read more than the 256 MB
    # of the last-level cache holds: 1,048,576 sites, and 48 atmospheres in one batch
    if not args.no_lambda:
        out["c2"] = lambda_block("c2", max_iter=20, accel_iter=1000, workers=args.workers, rows=args.rows)
        out["c3"] = lambda_block("c3", max_iter=5, accel_iter=200, workers=args.workers, rows=args.rows)
    print(json.dumps(out))


def synthesis_bytes(m, ncol, nl, fp):
    """Algorithmic HBM bytes of one line synthesis on m regular points: the
    packing pass reads the two site indices and the weight (16 B), chi_line,
    chi_cont and B (24 B) and two S_line values (16 B) and writes 4 values per
    point; the column pass reads the profile (m nl values) and the packed
    point data once and writes the top-plane intensities."""
    pack = m * (16 + 24 + 16 + 4 * fp)
    columns = m * nl * fp + m * 4 * fp + ncol * nl * fp
    return pack + columns


def run_synthesis(v, G, Gr, g, atm, atr, nx, ny, zr, stream):
    """Final synthesis (the paper's last step): S_line on the Voronoi sites is
    carried to the regular points by two-nearest-site inverse-distance weights
    and the emergent line intensity at mu = 1 follows from long characteristics
    up every column. S_line is B times a seeded factor (the timing does not
    depend on the values)."""
    import torch

    from synth.nlte import LAMBDA0_NM, line_setup

    dev = "cuda:0"
    nl = 101
    m = len(atr.T)
    ncol = nx * ny
    t0 = time.time()
    line = line_setup(atr.T, atr.rho, n_lambda=nl, workers=16)
    lam0 = np.array([LAMBDA0_NM * 1e-9])
    f64 = torch.float64

    def continuum(grid, a):
        """grey continuum opacity and B at line centre, assembled by the library on the device"""
        n = len(a.T)
        chi = torch.empty((n, 1), dtype=f64, device=dev)
        B = torch.empty_like(chi)
        v.lte_continuum(grid, lam0, a.kappa0, torch.as_tensor(a.T, device=dev), torch.as_tensor(a.rho, device=dev),
                        chi, B)
        return chi[:, 0].contiguous(), B[:, 0].contiguous()

    chi_c, B = continuum(Gr, atr)
    _, Bs = continuum(G, atm)
    S_line = Bs * torch.as_tensor(0.5 + np.random.default_rng(1048).random(g.n), device=dev)
    log(f"synthesis inputs built in {time.time() - t0:.1f} s")
    d = {"S": S_line, "chiL": torch.as_tensor(np.ascontiguousarray(line.chi_line), dtype=f64, device=dev),
         "chic": chi_c, "B": B}
    v.idw_map(G, Gr)  # first call pays one-time costs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, w1 = v.idw_map(G, Gr)
    map_ms = (time.perf_counter() - t0) * 1e3
    res = {"workload": f"final synthesis: S_line on {g.n} Voronoi sites -> regular {nx}x{ny}x{len(zr)} points "
                       f"(two nearest sites, inverse distance), {nl}-point line, mu = 1 long characteristics",
           "points": m, "columns": ncol, "wavelengths": nl, "idw_map_ms": round(map_ms, 3)}
    for name, dt in (("fp32", torch.float32), ("fp64", f64)):
        phi = torch.as_tensor(line.phi, dtype=dt, device=dev)
        out = torch.empty((ncol, nl), dtype=dt, device=dev)
        for _ in range(2):
            v.synthesis_vertical(G, Gr, idx, w1, d["S"], phi, d["chiL"], d["chic"], d["B"], out=out)
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            v.synthesis_vertical(G, Gr, idx, w1, d["S"], phi, d["chiL"], d["chic"], d["B"], out=out)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = synthesis_bytes(m, ncol, nl, 4 if dt == torch.float32 else 8)
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "point_lambda_per_s": m * nl / (ms * 1e-3),
                     "algorithmic_bytes": nbytes, "achieved_GBs": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"synthesis {name}: {ms:.3f} ms -> {gbs:.0f} GB/s algorithmic ({gbs / HBM_PEAK_GBS:.2f} of HBM)")
        del phi, out
    log(f"nearest-site map of {m} points: {map_ms:.2f} ms")
    return res


def regular_recipe(box, nx=128, ny=128, nz=256):
    """Spacings, planes and points of the regular grid over the recipe's box
    (point (k ny + j) nx + i at (lo_x + i dx, lo_y + j dy, z_k))."""
    dxr = (box.hi[0] - box.lo[0]) / nx
    dyr = (box.hi[1] - box.lo[1]) / ny
    zr = box.lo[2] + (box.hi[2] - box.lo[2]) * np.arange(nz) / (nz - 1)
    X, Y, Z = np.meshgrid(box.lo[0] + dxr * np.arange(nx), box.lo[1] + dyr * np.arange(ny), zr, indexing="xy")
    xyz = np.stack([a.transpose(2, 0, 1).ravel() for a in (X, Y, Z)], 1)
    return dxr, dyr, zr, xyz


def run_synthesis_only(args):
    import torch

    import paper_2306_01041_amd
    import synth

    v = paper_2306_01041_amd.load()
    seed = 1041
    t0 = time.time()
    atm = synth.make_atmosphere(args.sites, seed=seed)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    nx = ny = 128
    dxr, dyr, zr, xyz = regular_recipe(atm.box, nx, ny, 256)
    atr = synth.make_atmosphere(len(xyz), seed=seed, xyz=xyz)
    log(f"grids built in {time.time() - t0:.1f} s")
    ctx = v.Context(0)
    G = v.Grid.from_synth(ctx, g)
    Gr = v.Grid.regular(ctx, nx, ny, zr, dxr, dyr)
    res = run_synthesis(v, G, Gr, g, atm, atr, nx, ny, zr, torch.cuda.current_stream())
    print(json.dumps({"workload": "synth", "synthesis": res}))
    Gr.close()
    G.close()
    ctx.close()


def _design_grid(args):
    """Sites of one sampling density, their Voronoi grid and state (process pool)."""
    import synth
    from synth import design

    name, n, seed = args
    xyz = synth.sample_sites(n, seed) if name == "dlntau" else design.sample_sites_density(n, seed, name)
    atm = synth.make_atmosphere(n, seed=1041, xyz=xyz)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    return name, n, atm, g


def run_design(args):
    """Grid-design workload (accuracy, not throughput):
    * searchlight beams (Sect. 3.1): 51^3 uniformly random sites and the 51^3
      lattice in a periodic 1 m box, chi = S = 0, a beam of radius 0.2 m on the
      bottom face, one ray at 20, 45 and 60 degrees from the vertical: peak and
      edge width of the beam at the top, and the shift of its centre against
      tan(theta);
    * LTE continuum at 500 nm and mu = 1 (Sect. 3.2): the opacity at the sites of
      grids sampled from several densities and site counts is carried to the
      regular 128 x 128 x 256 grid by two-nearest-site inverse distances and the
      columns are integrated; the result is compared with the same columns on
      the exact regular-grid opacity."""
    from multiprocessing import get_context

    import torch

    import paper_2306_01041_amd
    import synth
    from synth import design

    v = paper_2306_01041_amd.load()
    dev = "cuda:0"
    f64 = torch.float64
    ctx = v.Context(0)
    out = {"workload": "design", "searchlight": [], "lte_sweep": []}

    # searchlight
    xyz, lo, hi, _, _, beam = design.searchlight()
    t0 = time.time()
    g = synth.voronoi_neighbours(xyz, lo, hi, periodic_xy=True)
    log(f"searchlight grid {g.n} sites in {time.time() - t0:.1f} s")
    n_side = 51
    zr = np.linspace(0.0, 1.0, n_side)
    dxr = 1.0 / n_side
    Xr, Yr = np.meshgrid(np.arange(n_side) * dxr, np.arange(n_side) * dxr, indexing="xy")
    for theta in (20.0, 45.0, 60.0):
        th = np.deg2rad(theta)
        d = np.array([[np.sin(th), 0.0, np.cos(th)]])
        row = {"theta_deg": theta}
        for kind in ("voronoi", "regular"):
            if kind == "voronoi":
                G = v.Grid.from_synth(ctx, g)
                m = g.n
                Ib = beam(g.xyz[:, 0], g.xyz[:, 1])
            else:
                G = v.Grid.regular(ctx, n_side, n_side, zr, dxr, dxr)
                m = n_side ** 3
                Ib = np.zeros(m)
                Ib[: n_side * n_side] = beam(Xr.ravel(), Yr.ravel())
            G.set_rays(d, np.array([1.0]))
            zero = torch.zeros((m, 1), dtype=f64, device=dev)
            J = torch.empty_like(zero)
            I = torch.empty((1, m, 1), dtype=f64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v.formal_solution(G, zero, zero, J, I_bottom=torch.as_tensor(Ib[:, None], device=dev), I_rays=I)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            _, sites = G.emergent_index()
            It = I[0, :, 0].cpu().numpy()[sites]
            if kind == "voronoi":
                xt = g.xyz[sites, 0]
            else:
                xt = (sites % n_side) * dxr
            cx = (np.angle(np.sum(It * np.exp(2j * np.pi * xt))) / (2 * np.pi)) % 1.0
            want = (0.5 + np.tan(th)) % 1.0
            shift_err = (cx - want + 0.5) % 1.0 - 0.5
            # edge width: the area where 0.1 < I < 0.9, over the beam circumference
            frac_edge = float(np.mean((It > 0.1) & (It < 0.9)))
            row[kind] = {"peak": float(It.max()), "edge_width_m": frac_edge / (2 * np.pi * 0.2),
                         "centre_error_m": float(shift_err), "ms": round(ms, 3)}
            G.close()
        out["searchlight"].append(row)
        log(f"searchlight {theta:.0f} deg: {row}")

    # LTE continuum against site count and sampling density
    box = synth.BoxSpec()
    nx = ny = 128
    dxr, dyr, zr, xyz_r = regular_recipe(box, nx, ny, 256)
    atr = synth.make_atmosphere(len(xyz_r), seed=1041, xyz=xyz_r)
    R = v.Grid.regular(ctx, nx, ny, zr, dxr, dyr)
    lam = np.array([500e-9])
    Tr, rr = torch.as_tensor(atr.T, device=dev), torch.as_tensor(atr.rho, device=dev)
    chi_r = torch.empty((len(xyz_r), 1), dtype=f64, device=dev)
    S_r = torch.empty_like(chi_r)
    v.lte_continuum(R, lam, atr.kappa0, Tr, rr, chi_r, S_r)
    I_ref = v.lc_vertical(R, chi_r, S_r).cpu().numpy()[:, 0]
    jobs = [(name, n, 1041) for n in (65536, 262144) for name in ("dlntau", "log_nh_t", "log_nhii", "alpha_c")]
    with get_context("spawn").Pool(min(8, len(jobs))) as pool:
        for name, n, atm, gd in pool.imap(_design_grid, jobs):
            G = v.Grid.from_synth(ctx, gd)
            chi_s = torch.empty((n, 1), dtype=f64, device=dev)
            S_s = torch.empty_like(chi_s)
            v.lte_continuum(G, lam, atm.kappa0, torch.as_tensor(atm.T, device=dev),
                            torch.as_tensor(atm.rho, device=dev), chi_s, S_s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            idx, w1 = v.idw_map(G, R)
            chi_i = v.idw_apply(G, R, idx, w1, chi_s[:, 0].contiguous())
            I_int = v.lc_vertical(R, chi_i[:, None].contiguous(), S_r)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            I_int = I_int.cpu().numpy()[:, 0]
            rel = np.abs(I_int - I_ref) / I_ref
            row = {"density": name, "sites": n, "mean_rel_err": float(rel.mean()),
                   "p99_rel_err": float(np.quantile(rel, 0.99)), "max_rel_err": float(rel.max()),
                   "contrast_ref": float(I_ref.std() / I_ref.mean()), "contrast": float(I_int.std() / I_int.mean()),
                   "correlation": float(np.corrcoef(I_ref, I_int)[0, 1]), "map_and_solve_ms": round(ms, 3)}
            out["lte_sweep"].append(row)
            log(f"LTE sweep {name} {n}: mean err {row['mean_rel_err']:.3e}, p99 {row['p99_rel_err']:.3e}, "
                f"corr {row['correlation']:.4f}")
            G.close()
    R.close()
    ctx.close()
    print(json.dumps(out))


LAMBDA_LAYOUT_KEYS = ("record_order", "shared_levels", "xcd_chunks", "ray_affinity", "lane_bytes", "interleave",
                      "pipeline", "rows")


def sweep_kernel_names(mode, layout, c):
    """The sweep kernels one formal solution launches in this launch mode and layout."""
    if mode == "persistent":
        return f"persistent_sweep_kernel<float,{c},4,true>"
    pp = layout.get("pipeline", 0)
    if pp:
        return f"sweep_pipe_kernel<float,{c},4,{pp}> (interior level steps) + sweep_kernel<float,{c},4>"
    return f"sweep_kernel<float,{c},4>"


def lambda_counter_traffic(workload, mode, layout):
    """HBM bytes per formal solution's sweep launches (rocprofv3 FETCH_SIZE x
    its copy-kernel calibration + WRITE_SIZE, summed over the launches of one
    formal solution) from the committed summary of this workload, or None when
    it was taken on another launch mode, another launch layout or on kernel
    sources that have changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"sweep_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("launch_mode") != mode:
        return None
    if mode != "persistent" and ({k: rec.get("layout", {}).get(k, LAYOUT_DEFAULTS.get(k)) for k in LAMBDA_LAYOUT_KEYS}
                                 != {k: layout.get(k, LAYOUT_DEFAULTS.get(k)) for k in LAMBDA_LAYOUT_KEYS}):
        return None
    if mode == "persistent" and rec.get("layout", {}).get("rows", "separate") != layout.get("rows", "separate"):
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    return rec["sweep_bytes_per_formal_solution"]["total"]


def lambda_inputs(workload, workers, cache_dir=None):
    """The seeded atmospheres of a two-level workload as one union grid:
    (grid, site offsets, T, rho, kappa0, LineSetup). With cache_dir, the grid,
    T and rho are read from (or written to) <cache_dir>/<workload>.npz and the
    line data are recomputed from T and rho with threads, so a run that reads
    the cache starts no worker processes (e.g. under a profiler)."""
    import synth
    from synth.nlte import line_case, line_setup

    path = os.path.join(cache_dir, f"{workload}.npz") if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        U = synth.VoronoiGrid(xyz=z["xyz"], nbr_ptr=z["ptr"], nbr_idx=z["idx"], nbr_shift=z["shift"], wall=z["wall"],
                              lo=z["lo"], hi=z["hi"], periodic_xy=True)
        off, T, rho, kappa0 = z["off"], z["T"], z["rho"], float(z["kappa0"])
        log(f"{workload}: inputs read from {path}")
        return U, off, T, rho, kappa0, line_setup(T, rho, n_lambda=101, workers=16)
    seed = 1041
    if workload == "c2":
        jobs = [(1048576, seed)]
    else:
        # atmosphere j of the batch uses seed + 1 + j
        jobs = [(n, seed + 1 + j) for j, n in enumerate(synth.batch_sizes(48, 32768, 524288, seed))]
    made = []
    if len(jobs) == 1 or workers <= 1:
        for k, job in enumerate(jobs):
            made.append(line_case(job))
            log(f"atmosphere {k + 1}/{len(jobs)}: {made[-1][1].n} sites")
    else:
        import multiprocessing as mp

        with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
            for k, r in enumerate(pool.imap(line_case, jobs)):
                made.append(r)
                log(f"atmosphere {k + 1}/{len(jobs)}: {r[1].n} sites")
    grids = [m[1] for m in made]
    U, off = synth.concat_grids(grids) if len(grids) > 1 else (grids[0], np.array([0, grids[0].n], np.int64))
    T = np.concatenate([m[0].T for m in made])
    rho = np.concatenate([m[0].rho for m in made])
    kappa0 = float(made[0][0].kappa0)
    if len(made) == 1:
        line = made[0][2]
    else:
        line = made[0][2]
        line.phi = np.concatenate([m[2].phi for m in made])
        line.chi_line = np.concatenate([m[2].chi_line for m in made])
    del made
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(path, xyz=U.xyz, ptr=U.nbr_ptr, idx=U.nbr_idx, shift=U.nbr_shift, wall=U.wall, lo=U.lo, hi=U.hi,
                 off=off, T=T, rho=rho, kappa0=kappa0)
        log(f"{workload}: inputs written to {path}")
    return U, off, T, rho, kappa0, line


def lambda_block(workload, max_iter=None, accel_iter=None, mode_pref="auto", interleave=0, pipeline=0, workers=16,
                 cache_dir=None, shared_levels=0, rows="paired"):
    """Two-level Lambda iteration on 1,048,576 sites (c2) or on a batch of 48
    atmospheres of 32,768-524,288 sites (c3): 101 line wavelengths (rows padded
    to 104), 24 rays, eps = 1e-4, FP32 sweeps, FP64 line update, graph-captured
    iterations. Times the formal solution alone in the iteration's layout (the
    launch mode that is faster of graph and persistent), a bounded number of
    plain iterations, and the accelerated (Jacobi) iteration to convergence;
    returns the block's dictionary, with the roofline of the formal solution on
    two byte bases: the whole-solution model (20 B + 20 B / Nlambda per update:
    read S and chi, write I, read-modify-write J) over the whole formal
    solution, and the sweep kernel's own bytes (read S_i and chi_i, write I_i,
    the record shared by the wavelengths) over the sweep launches alone."""
    import torch

    import paper_2306_01041_amd
    import synth
    from synth.nlte import LAMBDA0_NM

    v = paper_2306_01041_amd.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    t0 = time.time()
    U, off, T, rho, kappa0, line = lambda_inputs(workload, workers, cache_dir)
    n_atm = len(off) - 1
    nl = 101
    wlam = line.wlam
    phi = torch.as_tensor(line.phi, device=dev)
    chi_L = torch.as_tensor(line.chi_line, device=dev)
    del line
    dirs, w = synth.gauss_legendre_quadrature()
    R = len(dirs)
    build_s = time.time() - t0
    log(f"{workload}: {n_atm} atmosphere(s), {U.n} sites, inputs built in {build_s:.1f} s")

    ctx = v.Context(0)
    stream = torch.cuda.current_stream()
    G = v.Grid.from_synth(ctx, U)
    t0 = time.time()
    G.set_rays(dirs, w)
    setup_s = time.time() - t0
    info = G.info()
    log(f"rays set in {setup_s:.2f} s: {info}")
    d = torch.float64
    lam0 = np.array([LAMBDA0_NM * 1e-9])
    # one continuum constant for the batch (a recipe constant)
    chi_c = torch.empty((U.n, 1), dtype=d, device=dev)
    B = torch.empty_like(chi_c)
    v.lte_continuum(G, lam0, kappa0, torch.as_tensor(T, device=dev), torch.as_tensor(rho, device=dev), chi_c, B)
    chi_c, B = chi_c[:, 0].contiguous(), B[:, 0].contiguous()
    eps = 1e-4

    # the formal solution alone, on the fields of the first iteration, in the
    # library's own layout inside the iteration: rows padded to 104 entries
    # (16-byte multiples) with the continuum in the padding, a site's chi and S
    # rows side by side (rows="paired"; "separate": two arrays); only the 101
    # line wavelengths count as updates
    f32 = torch.float32
    ld = (nl + 3) // 4 * 4
    chi = torch.empty((U.n, ld), dtype=f32, device=dev)
    S = torch.empty_like(chi)
    chi[:, :nl] = chi_c[:, None] + chi_L[:, None] * phi
    S[:, :nl] = (chi_L[:, None] * phi * B[:, None] + chi_c[:, None] * B[:, None]) / (chi_c[:, None] +
                                                                                 chi_L[:, None] * phi)
    chi[:, nl:] = chi_c[:, None]
    S[:, nl:] = B[:, None]
    J = torch.empty_like(chi)
    if rows == "paired":
        cs = torch.empty((U.n, 2, ld), dtype=f32, device=dev)
        cs[:, 0] = chi
        cs[:, 1] = S
        chi_t, S_t = cs[:, 0], cs[:, 1]
    else:
        chi_t, S_t = chi, S
    # launch modes: the autotuner (auto) times the graph of level steps under
    # its layouts and the persistent sweep, and keeps the fastest on the grid
    modes = {"graph": v.VRT_EXEC_GRAPH, "batched": v.VRT_EXEC_BATCHED, "persistent": v.VRT_EXEC_PERSISTENT}
    tuning = None
    if mode_pref == "auto":
        t1 = time.time()
        tuning = v.autotune(G, chi, S, J, reps=3)  # (on arrays of n x ld)
        log(f"{workload}: autotune in {time.time() - t1:.1f} s, chosen {tuning['chosen']}")
        mode_pref = tuning["chosen"]["exec"]
        layout = dict(tuning["chosen"])
    else:
        G.tune(v.VRT_TUNE_SHARED_LEVELS, shared_levels)
        G.tune(v.VRT_TUNE_INTERLEAVE, interleave)
        G.tune(v.VRT_TUNE_PIPELINE, pipeline)
        layout = {"record_order": 1, "shared_levels": shared_levels, "xcd_chunks": 8, "ray_affinity": 0,
                  "lane_bytes": 16, "interleave": interleave, "pipeline": pipeline}
    layout["rows"] = rows
    fs_by_mode = {}
    if tuning:
        for c in tuning["candidates"]:
            if c["ms"] is not None and c["ms"] < fs_by_mode.get(c["exec"], float("inf")):
                fs_by_mode[c["exec"]] = c["ms"]
    for name in (mode_pref,):
        try:
            for _ in range(2):
                v.formal_solution(G, chi_t, S_t, J, exec_mode=modes[name])
            torch.cuda.synchronize()
            k = 5
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(k):
                v.formal_solution(G, chi_t, S_t, J, exec_mode=modes[name])
            e1.record(stream)
            e1.synchronize()
            G.device_status()
            fs_ms = e0.elapsed_time(e1) / k
        except v.VrtError as e:
            log(f"launch mode {name} not used: {e}")
            raise
    mode_name = mode_pref
    # the angle quadrature of J on its own (one eager launch, HIP events on the library stream)
    ctx.profile_reset()
    ctx.set_profiling(True)
    v.formal_solution(G, chi_t, S_t, J, exec_mode=v.VRT_EXEC_BATCHED)
    jr_ms, jr_launches, _ = ctx.profile(1)
    sw_ms_b, sw_launches, _ = ctx.profile(0)
    ctx.set_profiling(False)
    torch.cuda.synchronize()
    jr_one = jr_ms / max(jr_launches, 1)
    sweep_ms = fs_ms - jr_one
    launches = 1 if mode_name == "persistent" else sw_launches
    updates = U.n * R * nl
    upd_s = updates / (fs_ms * 1e-3)
    whole_bpu = 20.0 + 20.0 / nl
    sweep_bpu = sweep_bytes_per_update(nl, 4) * ld / nl  # the sweep moves ld-entry rows
    sweep_gbs = sweep_bpu * updates / (sweep_ms * 1e-3) / 1e9
    traffic = lambda_counter_traffic(workload, mode_name, layout)
    del chi, S, J, chi_t, S_t
    if rows == "paired":
        del cs
    torch.cuda.empty_cache()  # the library allocates the iteration's scratch itself
    log(f"{workload}: formal solution (ms by launch mode): {fs_by_mode} -> {mode_name}: {fs_ms:.3f} ms, "
        f"{upd_s:.3e} updates/s; sweep {sweep_ms:.3f} ms ({sweep_gbs:.0f} GB/s own bytes), J {jr_one:.3f} ms")

    # plain iterations (timing) and the accelerated iteration to convergence,
    # after one untimed iteration that allocates the iteration's scratch (an
    # allocation right after large frees can wait while the device clears the
    # freed memory: a one-time cost that is not an iteration's)
    S_w = B.clone()
    v.two_level_solve_batched(G, off, wlam, phi, chi_L, chi_c, B, eps, S_w, max_iter=1, tol=0.0, sweep_dtype=f32,
                              exec_mode=modes[mode_name])
    torch.cuda.synchronize()
    del S_w
    res_it = {}
    for name, acc, cap in (("plain", False, max_iter), ("accelerated", True, accel_iter)):
        if not cap:
            continue
        S_L = B.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, its, hist = v.two_level_solve_batched(G, off, wlam, phi, chi_L, chi_c, B, eps, S_L, max_iter=cap,
                                                  tol=1e-3, sweep_dtype=f32, exec_mode=modes[mode_name],
                                                  accel=acc)
        torch.cuda.synchronize()
        total_s = time.perf_counter() - t1
        n_iter = int(np.max(its))
        it_ms = total_s * 1e3 / max(n_iter, 1)
        # each atmosphere's change at its own last iteration (the history holds -1 after it stopped)
        last = np.array([hist[its[a] - 1, a] for a in range(len(its))]) if n_iter else np.zeros(0)
        res_it[name] = {"ms_per_iteration": round(it_ms, 3), "iterations": {"min": int(np.min(its)), "max": n_iter,
                                                                              "median": float(np.median(its)),
                                                                              "cap": cap},
                        "converged": bool(st == v.VRT_OK),
                        "atmospheres_converged": int(np.sum(last < 1e-3)),
                        "final_change": {"min": float(np.min(last)), "max": float(np.max(last))},
                        "solve_s": round(total_s, 3)}
        log(f"{workload} {name} iteration: status {st}, iterations {np.min(its)}..{n_iter}, {it_ms:.3f} ms per "
            f"iteration, {total_s:.2f} s")
    out = {
        "workload": (f"two-level Lambda iteration, " +
                     (f"{U.n} sites" if n_atm == 1 else f"{n_atm} atmospheres, {U.n} sites in total") +
                     f", {nl} line wavelengths, {R} rays, eps {eps}, FP32 sweeps, FP64 update"),
        "sites": U.n, "atmospheres": n_atm, "wavelengths": nl, "rays": R, "levels_max": info["max_levels"],
        "formal_solution_ms": round(fs_ms, 3), "updates_per_s": upd_s, "launch_mode": mode_name,
        "formal_solution_ms_by_mode": {k: round(t, 3) for k, t in fs_by_mode.items()},
        "tuning": tuning["chosen"] if tuning else None,
        "layout": {k: layout.get(k) for k in LAMBDA_LAYOUT_KEYS},
        "roofline": {
            "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "whole_solution": {"bytes_per_update": round(whole_bpu, 3),
                               "achieved": round(upd_s * whole_bpu / 1e9, 1),
                               "frac": round(upd_s * whole_bpu / 1e9 / HBM_PEAK_GBS, 4)},
            "sweep_kernel": {"kernel": sweep_kernel_names(mode_name, layout, 32),
                             "bytes_per_update": round(sweep_bpu, 3), "sweep_ms": round(sweep_ms, 3),
                             "launches": launches, "achieved": round(sweep_gbs, 1),
                             "frac": round(sweep_gbs / HBM_PEAK_GBS, 4),
                             "traffic": None if traffic is None else round(traffic),
                             "traffic_over_algorithmic": None if traffic is None else
                             round(traffic / (sweep_bpu * updates), 3)},
            "j_quadrature_ms": round(jr_one, 3)},
        "formal_solution_share": (round(fs_ms / res_it["plain"]["ms_per_iteration"], 3) if "plain" in res_it
                                  else None),
        "iteration": res_it,
        "inputs_build_s": round(build_s, 1), "setup_s": round(setup_s, 3),
    }
    G.close()
    ctx.close()
    del phi, chi_L, chi_c, B
    torch.cuda.empty_cache()
    return out


def run_lambda(args):
    """The c2 / c3 workloads alone: one JSON line with the block's figures."""
    out = lambda_block(args.workload, max_iter=args.max_iter or (20 if args.workload == "c2" else 10),
                       accel_iter=0 if args.no_accel else (1000 if args.workload == "c2" else 200),
                       mode_pref="auto" if args.mode == "auto" else args.mode, interleave=args.interleave,
                       pipeline=args.pipeline, workers=args.workers, cache_dir=args.inputs_cache,
                       shared_levels=args.shared_levels, rows=args.rows)
    line = {"metric": "site*ray*lambda updates/s of the formal solution inside the two-level Lambda iteration",
            "value": out["updates_per_s"], "unit": "site*ray*lambda updates/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32",
            "data": "synthetic (seeded Bifrost-like stratified atmospheres, rejection-sampled Voronoi sites)",
            "config": {"workload": out["workload"], "sites": out["sites"], "atmospheres": out["atmospheres"]}}
    line.update(out)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
