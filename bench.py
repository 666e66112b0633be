#!/usr/bin/env python3
"""Benchmark of the Newton iteration of the polymer-flooding simulator on one
MI355X.

A bench "step" is one scheduled timestep of the workload: a sequence of
Newton iterations, each one pass of the whole hot path (accumulation
snapshot, residual + Jacobian assembly with wells, convergence norms, CPR
set-up, CPR-preconditioned FGMRES, chopped update).  The metric is
cell-Newton iterations per second: N_cells x (Newton iterations in the timed
steps) / timed wall time, inputs resident in HBM before timing starts.

Default workload: the 300x300x300 lognormal polymer flood (27M cells, 100
wells, 10-day steps), FP64 CPR-FGMRES; the same schedule is then run with the
mixed-precision preconditioner and reported beside it with its per-field
difference from the FP64 states.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell and launch of the timed kernels (FP64)
KERNEL_BYTES = {
    "assemble": ("PF_K_ASSEMBLE", 1, 552),        # x 24 + Mn 24 + T 24 + PVr 8 in; R 24 + J 448 out (8 of 9 entries per block)
    # the (oil, C) entry of every block of J is zero and not read: 8 of 9 entries per block
    "spmv": ("PF_K_SPMV", 2, 496),                # J 448 + x 24 in; y 24 out (x FP32 in mixed: 484)
    "zline": ("PF_K_ZLINE", 3, None),             # level-0 half-sweep, per active column set (below)
    "ilu": ("PF_K_ILU", 6, None),
    # last ILU phase with the red rows of w = J z (which equal v there): Lc 384 + inverse diagonal 72 + z 24
    # + p 8 + black z 24 + v 24 in, z 24 + w 24 out, per red cell (half the cells)
    "red_spmv": ("PF_K_RED_SPMV", 8, (384 + 72 + 24 + 8 + 24 + 24 + 24 + 24) // 2),
    # black rows of w = J z: Lc 384 + J diagonal 64 + z 24 + p 8 + red z 24 in, z (P plane) 8 + w 24 out,
    # per black cell
    "black_spmv": ("PF_K_BLACK_SPMV", 9, (384 + 64 + 24 + 8 + 24 + 8 + 24) // 2),
    # FP64 stage residual of the red rows with the first ILU phase, from the colour-split copies of J:
    # J_rr P-column 24 + off-diagonal P-columns 144 + v 24 + p 8 + border map 4 + D_r^{-1} 72 in, z 24 out,
    # per red cell (the black rows' residual is formed in the forward black phase)
    "stage_resid": ("PF_K_STAGE_RESID", 7, (24 + 144 + 24 + 8 + 4 + 72 + 24) // 2),
}


# committed counter summaries (rocprofv3 FETCH_SIZE / WRITE_SIZE passes) per
# timed kernel: file (named for the 1.12M-cell workload; the same name with
# another workload's tag covers that one), source file and device functions
# whose text they cover
TRAFFIC_FILES = {
    "spmv": ("profiles/k_spmv_c2_fp64_hbm_counters.md",
             [("paper_1807_05298_amd/csrc/k_linalg.hip", "k_spmv_d"),
              ("paper_1807_05298_amd/csrc/k_linalg.hip", "jld"),
              ("paper_1807_05298_amd/csrc/pf_internal.h", "xcd_block")]),
    "red_spmv": ("profiles/k_ilu_red_spmv_c2_fp64_hbm_counters.md",
                 [("paper_1807_05298_amd/csrc/k_cpr.hip", "k_ilu_red_spmv_d"),
                  ("paper_1807_05298_amd/csrc/k_cpr.hip", "strip_slot"),
                  ("paper_1807_05298_amd/csrc/pf_internal.h", "strip_order"),
                  ("paper_1807_05298_amd/csrc/k_cpr.hip", "ilu_ld"),
                  ("paper_1807_05298_amd/csrc/k_cpr.hip", "ilu_slot_cell"),
                  ("paper_1807_05298_amd/csrc/pf_internal.h", "xcd_block")]),
    "black_spmv": ("profiles/k_black_spmv_c2_fp64_hbm_counters.md",
                   [("paper_1807_05298_amd/csrc/k_cpr.hip", "k_black_spmv_d"),
                    ("paper_1807_05298_amd/csrc/k_cpr.hip", "strip_slot"),
                    ("paper_1807_05298_amd/csrc/pf_internal.h", "strip_order"),
                    ("paper_1807_05298_amd/csrc/k_cpr.hip", "ilu_ld"),
                    ("paper_1807_05298_amd/csrc/k_cpr.hip", "ilu_slot_cell"),
                    ("paper_1807_05298_amd/csrc/pf_internal.h", "xcd_block")]),
    "stage_resid": ("profiles/k_stage_red_c2_fp64_hbm_counters.md",
                    [("paper_1807_05298_amd/csrc/k_cpr.hip", "k_stage_red_d"),
                     ("paper_1807_05298_amd/csrc/k_cpr.hip", "strip_slot"),
                     ("paper_1807_05298_amd/csrc/pf_internal.h", "strip_order"),
                     ("paper_1807_05298_amd/csrc/k_cpr.hip", "stage_border"),
                     ("paper_1807_05298_amd/csrc/k_cpr.hip", "ilu_ld"),
                     ("paper_1807_05298_amd/csrc/k_cpr.hip", "ilu_slot_cell"),
                     ("paper_1807_05298_amd/csrc/pf_internal.h", "xcd_block")]),
    "assemble": ("profiles/k_assemble_c2_fp64_hbm_counters.md",
                 [("paper_1807_05298_amd/csrc/k_physics.hip", f) for f in
                  ("k_assemble_d", "cell_props", "table_eval", "accumulation", "face_flux", "exp_density", "rcp_nr",
                   "row_scales")]
                 + [("paper_1807_05298_amd/csrc/pf_internal.h", "xcd_block")]),
}


def _function_text(path: str, name: str) -> str:
    """Source text of one device function (with its template line)."""
    import re
    lines = open(os.path.join(ROOT, path)).read().split("\n")
    k = next(i for i, l in enumerate(lines)
             if re.search(r"\b%s\s*\(" % re.escape(name), l) and ("__global__" in l or "__device__" in l))
    if k > 0 and lines[k - 1].startswith("template"):
        k -= 1
    e = next(i for i in range(k, len(lines)) if lines[i] == "}")
    return "\n".join(lines[k:e + 1])


def _traffic(kname: str, workload: str, precision: str):
    """HBM bytes per launch from the committed counter passes, scaled by the
    plain-copy calibration taken in the same runs; None when no summary covers
    this kernel and workload or the kernel's source changed since."""
    import hashlib
    import re
    if kname not in TRAFFIC_FILES or precision != "fp64":
        return None
    path, funcs = TRAFFIC_FILES[kname]
    path = path.replace("_c2_", f"_{workload}_")
    try:
        text = open(os.path.join(ROOT, path)).read()
        rec = json.loads(re.search(r"<!-- traffic: (\{.*\}) -->", text).group(1))
        digest = hashlib.sha256("\n".join(_function_text(p, f) for p, f in funcs).encode()).hexdigest()
    except (OSError, AttributeError, StopIteration, ValueError):
        return None
    if digest != rec["source_sha256"]:
        return None
    kib = rec["copy_bytes"] / 1024.0
    read = rec["fetch_kib"] * (kib / rec["copy_fetch_kib"]) * 1024.0
    write = rec["write_kib"] * (kib / rec["copy_write_kib"]) * 1024.0
    return int(round(read + write))


# solver options a workload needs beyond the defaults: the 27.4M-block model
# starts with fronts crossing many ~1 m^3 cells per day and needs more cuts
WORKLOAD_OPTS = {"p2": dict(max_cuts=12, max_newton=16)}


def _dt_init_days(args) -> float:
    if args.dt_init_days is not None:
        return args.dt_init_days
    return 0.005 if args.workload == "p2" else 0.25


def _workload(name: str):
    from paper_1807_05298_amd import inputs as I
    if name == "c2":
        return I.case_c2(), "60x220x85 layered/channelised polymer flood (1.12M cells), 5 x 5-day wells: 1 rate injector + 4 BHP producers"
    if name == "c1":
        return I.case_c1(), "10x10x3 quarter five-spot (300 cells), daily steps"
    if name == "c3":
        return I.case_c3(), "200x200x50 lognormal field (2M cells), 5x5 line drive, 5-day steps"
    if name == "c5":
        return I.case_c5(), "300x300x300 lognormal field (27M cells), 100 wells on a 10x10 lattice, 10-day steps"
    if name == "p1":
        return I.case_paper_low(), ("95x192x5 (91,200 cells) performance-test reservoir of the paper (Table 3 layers), "
                                    "4 corner injectors with BHP limit + horizontal producer, 10-day steps")
    if name == "p2":
        return I.case_paper_high(), ("951x1920x15 (27,388,800 cells) performance-test reservoir of the paper "
                                     "(Table 3 layers refined), 4 corner injectors with BHP limit + horizontal producer, "
                                     "10-day steps")
    raise SystemExit(f"unknown workload {name}")


def _cpu_sample(case, workload: str):
    """A bounded sample of the benched workload for the oracle: a sub-box of
    the same field and wells, injection per perforated layer as in the full
    model, started from the initial state with the bench's first sub-step."""
    from paper_1807_05298_amd import inputs as I
    if workload == "c5":
        # two lattice wells (injector at (15, 15), producer at (45, 15)) in the top 10 layers
        sample = I.sub_box(case, 0, 60, 0, 30, 0, 10)
        what = "60x30x10 corner sub-box of the 300^3 field (18,000 cells; one injector, one producer, top 10 of 300 layers)"
    elif workload == "c2":
        sample = I.sub_box(case, 0, 60, 0, 220, 0, 3)
        what = "top 3 of the 85 layers of the 60x220x85 field (39,600 cells)"
    else:
        sample = I.case_c1()
        what = "full 10x10x3 case"
    return sample, what


def _oracle_newton_rate(sample, dt, tol_res, tol_upd, max_newton):
    """cells x Newton iterations / s of the oracle on one core."""
    from threadpoolctl import threadpool_limits
    import oracle
    with threadpool_limits(limits=1):
        o = oracle.Oracle(sample)
        x0 = o.initial_state()
        t0 = time.perf_counter()
        _, its, _, _ = o.newton(x0, dt, oracle.NewtonOpts(tol_res=tol_res, tol_upd=tol_upd, max_newton=max_newton))
        el = time.perf_counter() - t0
    return sample.n * its, its, el


def _cpu_worker(a):
    sample, dt, tol_res, tol_upd, max_newton = a
    return _oracle_newton_rate(sample, dt, tol_res, tol_upd, max_newton)


def _cpu_baseline(case, workload: str, tol_res: float, tol_upd: float, dt: float):
    """The oracle (plain FP64 CPU reference: C residual and AD Jacobian,
    sparse direct solve per Newton iteration) timed on a bounded sample of the
    benched workload: its first Newton iterations from the initial state, on
    one core, then as independent copies on every core this process may use
    (at most 16) at once.  Runs before the GPU is touched, so the copies can
    be forked."""
    import multiprocessing as mp
    sample, what = _cpu_sample(case, workload)
    max_newton = 3
    work, its, el = _oracle_newton_rate(sample, dt, tol_res, tol_upd, max_newton)
    one = work / el
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(sample, dt, tol_res, tol_upd, max_newton)] * cores)
    wall = time.perf_counter() - t0
    allc = sum(r[0] for r in res) / wall
    return {"value": round(allc, 1), "unit": "cell-Newton-its/s", "cores": cores, "kind": "oracle",
            "sample": (f"{what}; first {its} Newton iterations of a {dt / 86400.0:g}-day first step, "
                       f"one copy per core on {cores} cores at once ({wall:.1f} s)"),
            "one_core": {"value": round(one, 1), "cores": 1, "seconds": round(el, 2)}}


def _serving(args):
    """Serving workload: realisations of 20k-500k cells (20 steps of 5 d
    each by default) through the continuous-batching server.  First all are
    submitted at once (saturated throughput); then the same set arrives as a
    Poisson stream at 0.8 x the saturated rate."""
    import torch
    from paper_1807_05298_amd import inputs as I
    from paper_1807_05298_amd import polyflood as pf
    n_real, n_steps = args.serving_n, args.serving_steps
    cases = [I.serving_realisation(r) for r in range(n_real)]
    opts = pf.default_opts(tol_res=args.tol_res, tol_upd=args.tol_upd,
                           precision=pf.PREC_MIXED if args.precision == "mixed" else pf.PREC_FP64,
                           dt_init=_dt_init_days(args) * 86400.0)
    sizes = [pf.workspace_size(c, opts) for c in cases]
    arena = int(min(args.serving_arena_gb * (1 << 30), 1.2 * sum(sizes)))
    arena = max(arena, max(sizes) + (1 << 20))

    def run(arrivals, fused):
        slots = args.serving_fused_slots if fused else args.serving_slots
        sv = pf.Server(arena, max_slots=slots, fused=args.serving_groups if fused else 0)
        t0 = time.perf_counter()
        tickets = []
        for k, c in enumerate(cases):
            if arrivals is not None:
                wait = t0 + arrivals[k] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            tickets.append(sv.submit(c, opts, n_steps=n_steps))
        sv.wait()
        wall = time.perf_counter() - t0
        res = [sv.poll(t)[1] for t in tickets]
        info = sv.info()
        sv.close()
        lat = np.concatenate([r["latency"] for r in res])
        cell_its = sum(c.n * int(np.sum(r["newton"])) for c, r in zip(cases, res))
        return dict(wall_s=round(wall, 3), cell_newton_its_per_s=round(cell_its / wall, 1),
                    realisations_per_s=round(len(cases) / wall, 3),
                    step_latency_ms={"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                                     "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
                    peak_running=info["peak_running"], peak_gb=round(info["peak_bytes"] / 2**30, 3))

    modes = {}
    for name in (("fused", "streams") if args.serving_modes == "both" else (args.serving_modes,)):
        fused = name == "fused"
        sat = run(None, fused)
        print(f"serving {name}: saturated {sat}", file=sys.stderr, flush=True)
        rate = 0.8 * sat["realisations_per_s"]
        arrivals = I.serving_arrivals(n_real, rate_per_s=rate)
        poi = run(arrivals, fused)
        print(f"serving {name}: poisson {poi}", file=sys.stderr, flush=True)
        modes[name] = {"slots": args.serving_fused_slots if fused else args.serving_slots,
                       "fusion_groups": args.serving_groups if fused else 0,
                       "saturated": sat, "poisson": dict(poi, rate_per_s=round(rate, 3))}
    head = modes.get("fused") or modes["streams"]
    sat, poi = head["saturated"], head["poisson"]
    out = {
        "metric": "cell-Newton its/s (assemble+CPR-GMRES), serving",
        "value": poi["cell_newton_its_per_s"],
        "unit": "cell-Newton-its/s",
        "n_gpus": 1, "steps": n_steps, "warmup": 0, "ms_per_step": poi["step_latency_ms"]["p50"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (outer) / f32+bf16 (preconditioner)",
        "data": "synthetic",
        "config": {"workload": f"c4: {n_real} realisations of 20k-500k cells, {n_steps} x 5-day steps, "
                               f"{head['slots']} slots, " + ("fused launches" if "fused" in modes else
                                                               "one stream per slot")
                               + f", arena {arena / 2**30:.1f} GB",
                   "cells_total": int(sum(c.n for c in cases))},
        "saturated": sat, "poisson": poi,
        "latency_ms": poi["step_latency_ms"],
        "modes": modes,
    }
    print(json.dumps(out), flush=True)


def _timed_run(sim, case, dts, args, kid):
    """W untimed warm-up steps, then K timed steps; the chosen kernel's
    launches are bracketed by HIP events on the library's stream."""
    import ctypes
    import torch
    from paper_1807_05298_amd import polyflood as pf
    for k in range(args.warmup):
        sim.apply_events(case, k)
        st = sim.step(dts[k])
        print(f"warmup step {k}: newton {st['newton_its']} lin {st['lin_its']} cuts {st['cuts']} "
              f"{st['t_total']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if kid:
        pf._lib.pf_profile_begin(sim.h, kid, 4096)
    lat = []
    newton = lin = cuts = 0
    t_asm = t_lin = 0.0
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        sim.apply_events(case, k)
        ts = time.perf_counter()
        st = sim.step(dts[k])
        lat.append(time.perf_counter() - ts)
        print(f"step {k}: newton {st['newton_its']} lin {st['lin_its']} cuts {st['cuts']} "
              f"{lat[-1]:.3f} s", file=sys.stderr, flush=True)
        newton += st["newton_its"]
        lin += st["lin_its"]
        cuts += st["cuts"]
        # the paper's split: residual/Jacobian assembly with the convergence test ("platform")
        # against the linear solver (CPR set-up and FGMRES, up to the update)
        t_asm += st["t_assemble"]
        t_lin += st["t_setup"] + st["t_solve"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    nl = ctypes.c_int32(0)
    tot = ctypes.c_double(0.0)
    if kid:
        pf._lib.pf_profile_end(sim.h, ctypes.byref(nl), ctypes.byref(tot))
    return dict(wall=t1 - t0, lat=lat, newton=newton, lin=lin, cuts=cuts, launches=nl.value, total_ms=tot.value,
                t_asm=t_asm, t_lin=t_lin)


def _field_diffs(a, b, floor_c):
    """Per field max |a - b| / max(|b|_inf, floor): P, S, C, Pb."""
    out = {}
    for name, x, y, floor in zip(("P", "S", "C", "Pb"), a, b, (1.0, 1.0, floor_c, 1.0)):
        ref = float(np.max(np.abs(y))) if y.size else 0.0
        out[name] = float(np.max(np.abs(x - y)) / max(ref, floor)) if y.size else 0.0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12, help="timed timesteps")
    ap.add_argument("--warmup", type=int, default=2, help="untimed timesteps before timing")
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--smoother", default="rbilu0", choices=["bjac", "rbilu0"])
    ap.add_argument("--order", default="pf", choices=["pf", "fp"])
    ap.add_argument("--profile-kernel", default=None, choices=sorted(KERNEL_BYTES),
                    help="kernel timed for the roofline (default: red_spmv, the last ILU phase with the red rows of w = J z, in FP64 with the ILU(0) smoother in PF order; spmv otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the same schedule (300^3 workload)")
    ap.add_argument("--tol-res", type=float, default=1e-6)
    ap.add_argument("--tol-upd", type=float, default=1e-3)
    ap.add_argument("--mg-cycles", type=int, default=None, help="V-cycles per pressure stage (default: library default)")
    ap.add_argument("--mg-pre", type=int, default=None, help="pre-smoothing sweeps (default: library default)")
    ap.add_argument("--mg-post", type=int, default=None, help="post-smoothing sweeps (default: library default)")
    ap.add_argument("--zline-len", type=int, default=None, help="layers per z-line smoother segment (default: library default)")
    ap.add_argument("--mg-pre-small", type=int, default=None,
                    help="pre-smoothing sweeps on small multigrid levels (default: library default)")
    ap.add_argument("--mg-small-cells", type=int, default=None,
                    help="cell limit of the small multigrid levels (default: library default)")
    ap.add_argument("--dt-init-days", type=float, default=None,
                    help="first sub-step after the initial state (default 0.25 d; 0.005 d for p2, whose 2 m "
                         "cells next to the injectors hold about 1 m^3 of pore volume each)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--serving-n", type=int, default=64)
    ap.add_argument("--serving-steps", type=int, default=20)
    ap.add_argument("--serving-slots", type=int, default=4, help="slots of the one-stream-per-slot server")
    ap.add_argument("--serving-fused-slots", type=int, default=16, help="slots of the fused server")
    ap.add_argument("--serving-groups", type=int, default=4, help="fusion groups of the fused server")
    ap.add_argument("--serving-modes", choices=("both", "fused", "streams"), default="both")
    ap.add_argument("--serving-arena-gb", type=float, default=48.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 5 plain device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.profile_kernel is None:
        fused = args.precision == "fp64" and args.smoother == "rbilu0" and args.order == "pf"
        args.profile_kernel = "red_spmv" if fused else "spmv"

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        _serving(args)
        return

    case, desc = _workload(args.workload)
    dt_init = _dt_init_days(args) * 86400.0
    # the oracle's leg first: its per-core copies are forked before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(case, args.workload, args.tol_res, args.tol_upd, dt_init)
        print(f"cpu baseline: {cpu}", file=sys.stderr, flush=True)

    import torch
    from paper_1807_05298_amd import polyflood as pf

    mg = {k: v for k, v in (("mg_cycles", args.mg_cycles), ("mg_pre", args.mg_pre), ("mg_post", args.mg_post),
                             ("zline_len", args.zline_len), ("mg_pre_small", args.mg_pre_small),
                             ("mg_small_cells", args.mg_small_cells)) if v is not None}
    mg.update(WORKLOAD_OPTS.get(args.workload, {}))

    def make_opts(precision):
        return pf.default_opts(smoother=pf.SMOOTH_RBILU0 if args.smoother == "rbilu0" else pf.SMOOTH_BJAC,
                               cpr_order=pf.CPR_PF if args.order == "pf" else pf.CPR_FP,
                               tol_res=args.tol_res, tol_upd=args.tol_upd, **mg,
                               precision=pf.PREC_MIXED if precision == "mixed" else pf.PREC_FP64,
                               dt_init=dt_init)

    opts = make_opts(args.precision)
    dts = [float(d) for d in case.dts]
    if args.warmup + args.steps > len(dts):
        dts = dts * ((args.warmup + args.steps) // len(dts) + 1)
    kname = args.profile_kernel
    kid = KERNEL_BYTES[kname][1]
    sim = pf.Simulator(case, opts)
    r = _timed_run(sim, case, dts, args, kid)
    n = case.n
    value = n * r["newton"] / r["wall"]

    roof = None
    per_cell = KERNEL_BYTES[kname][2]
    if kname == "spmv" and args.precision == "mixed":
        per_cell -= 12                            # x in FP32
    if r["launches"] > 0 and per_cell is not None:
        avg_s = r["total_ms"] / 1e3 / r["launches"]
        bytes_launch = per_cell * n
        achieved = bytes_launch / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _traffic(kname, args.workload, args.precision), "traffic_unit": "bytes/launch",
                "algorithmic_bytes": bytes_launch,
                "launches": r["launches"], "avg_us": round(avg_s * 1e6, 2),
                "bytes_per_cell": per_cell}

    lat = r["lat"]
    out = {
        "metric": "cell-Newton its/s (assemble+CPR-GMRES)",
        "value": round(value, 1),
        "unit": "cell-Newton-its/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["wall"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (outer) / f32+bf16 (preconditioner)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "cells": n, "wells": len(case.wells),
                   "step_days": dts[args.warmup] / 86400.0, "cpr": f"{args.order.upper()} MG(z-line GS, {opts.mg_cycles} V-cycles, {opts.mg_pre}+{opts.mg_post} sweeps, {opts.mg_pre_small} pre on levels <= max({opts.mg_small_cells}, n0/32) cells of grids of n0 >= {10 * opts.mg_small_cells} cells)+{args.smoother}",
                   "precision": args.precision,
                   "fgmres_restart": opts.restart, "tol_res": args.tol_res, "tol_upd": args.tol_upd,
                   "max_newton": opts.max_newton, "max_cuts": opts.max_cuts,
                   "dt_init_days": _dt_init_days(args)},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
        "newton_its": r["newton"],
        "lin_its": r["lin"],
        "cuts": r["cuts"],
        "time_split_s": {"assembly_and_tests": round(r["t_asm"], 4), "linear_solver": round(r["t_lin"], 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.workload == "c5" and args.precision == "fp64" and not args.no_mixed:
        # the same schedule with the FP32/BF16 preconditioner inside FP64 FGMRES,
        # at the same Newton tolerances; its states against the FP64 run's
        x64 = sim.get_state()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        sim = pf.Simulator(case, make_opts("mixed"))
        rm = _timed_run(sim, case, dts, args, 0)
        xm = sim.get_state()
        sim.close()
        floor_c = max([w.c_inj for w in case.wells if w.injector] + [1.0])
        out["mixed"] = {"value": round(n * rm["newton"] / rm["wall"], 1),
                        "ms_per_step": round(1e3 * rm["wall"] / args.steps, 3),
                        "latency_ms": {"p50": round(1e3 * float(np.percentile(rm["lat"], 50)), 3),
                                       "p99": round(1e3 * float(np.percentile(rm["lat"], 99)), 3)},
                        "newton_its": rm["newton"], "lin_its": rm["lin"], "cuts": rm["cuts"],
                        "dtype": "f64 (outer FGMRES, assembly, wells, Arnoldi) / f32+bf16 (preconditioner)",
                        "field_diff_vs_fp64": _field_diffs(xm, x64, floor_c)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
