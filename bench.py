"""Throughput of the T3S3-DUGKS sweep on one MI355X.

Workload: Taylor-Green vortex on a periodic 2048 x 2048 grid with the D2Q37
velocity set, FP32 storage of the deviation f - w_q rho0 (the 2048^2 / D2Q37 /
FP32-delta member of the Taylor-Green family at 256^2..2048^2, D2Q9 and D2Q37,
FP64 vs FP32-delta).  The same grid in FP64 is timed beside it.  One "step"
is one full T3S3 step (stage A + stage C) over every (cell, velocity) pair.

Prints one JSON line.  Metric: G cell-velocity updates per second (cells * Q *
steps / s / 1e9) plus the HBM-roofline fraction of the dominant kernel.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
METRIC = "G cell\u00b7velocity updates/s per DUGKS step + %HBM peak, FP32-\u03b4f vs FP64"
UNIT = "G cell\u00b7velocity updates/s"
# sources whose change invalidates stored hardware-counter traffic of the sweep kernels
KERNEL_SOURCES = ["sweep_fast.hip", "sweep_common.h", "lattices.h", "launchers.h", "ring.h",
                  "dugks_internal.h", "api.cpp", "../build.py"]   # (build flags shape the code too)
# the same for the any-size kernels
LQ_SOURCES = ["sweep_large.hip", "sweep_common.h", "ring.h", "dugks_internal.h", "api.cpp", "../build.py"]
# the same for the three-dimensional kernels
SOURCES_3D = ["sweep3d.hip", "dugks_internal.h", "../build.py"]
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash(sources=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1709_05458_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_summary_name(n: int, lattice_name: str) -> str:
    """File under profiles/ holding the stage kernels' counter traffic of the
    Taylor-Green workload with n x n cells and the named velocity set."""
    return f"sweep_stages_tgv{n}_{lattice_name.lower()}_fp32delta_traffic.txt"


def stored_traffic(summary: str, kernel_key: str, sources=None):
    """HBM bytes per launch of one kernel from a stored counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the factor the
    same counter shows on a plain copy of known size), or None when the
    summary is missing or was taken on other kernel sources."""
    path = os.path.join(PROFILES, summary)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != kernel_source_hash(sources):
        return None
    try:
        f_fetch = float(kv["fetch_scale"])
        f_write = float(kv["write_scale"])
        fetch = float(kv[f"{kernel_key}.fetch_kib"])
        write = float(kv[f"{kernel_key}.write_kib"])
    except (KeyError, ValueError):
        return None
    return (fetch * f_fetch + write * f_write) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048, help="cells per side")
    ap.add_argument("--lattice", default="d2q37", choices=["d2q9", "d2q37"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tile", default="", help="tile as TXxTY")
    ap.add_argument("--scheme", default="t3s3", choices=["t3s3", "t2s3"],
                    help="time integrator of the Taylor-Green workload (t2s3: the paper's second-order "
                         "comparison scheme, one sweep per step)")
    ap.add_argument("--workload", default="tgv", choices=["tgv", "batched", "rarefied", "adjoint", "cavity", "abc3d"],
                    help="tgv: Taylor-Green (headline); batched: 64 uneven cavities in one graph "
                         "launch per step; rarefied: Newton-Cotes cavity on stretched cells; adjoint: "
                         "gradient of 500 Taylor-Green 256^2 D2Q9 steps (dugks_backward); cavity: "
                         "lid-driven cavity at Re 1000 with bounce-back walls (--n, --lattice, --tile; 16x16 "
                         "by default); abc3d: the three-dimensional sweep on the ABC flow, 128^3 cells, D3Q19 "
                         "(--n3, --lattice3)")
    ap.add_argument("--n3", type=int, default=128, help="cells per side (abc3d)")
    ap.add_argument("--lattice3", default="d3q19", choices=["d3q19", "d3q27"])
    ap.add_argument("--nc", type=int, default=101, help="Newton-Cotes points per axis (rarefied)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters of a profiler against a kernel whose traffic is known."""
    import torch
    n = mib * 1024 * 1024
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 3}))


def make_case(n, lattice):
    from paper_1709_05458_amd import cases as C
    vs = C.d2q37(1.0 / 3.0) if lattice == "d2q37" else C.d2q9(1.0 / 3.0)
    return C.tgv_case(n, vs, steps=1000)


def time_run(case, precision, steps, warmup, tile, scheme=0):
    import torch
    from paper_1709_05458_amd import dugks
    s = dugks.Solver(case, precision, tile=tile, scheme=scheme)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    r0, ux0, uy0 = s.moments()
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    s.prof_begin(2 * steps + 8)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    a_ms, a_n = s.prof_query(dugks.K_STAGE_A)
    c_ms, c_n = s.prof_query(dugks.K_STAGE_C)
    s.prof_end()
    s.sync()   # raises on a non-finite state
    r, ux, uy = s.moments()
    desc = s.describe()
    s.close()
    # checks on the state after warmup + steps: conservation (periodic, moment-
    # exact weights: exact up to rounding) and the viscous decay of the vortex
    # against the analytic factor exp(-2 nu t) (the 1% initial noise decays faster)
    t = (warmup + steps) * case.dt
    mass0, mass = float(r0.sum()), float(r.sum())
    mom0 = (float((r0 * ux0).sum()), float((r0 * uy0).sum()))
    mom = (float((r * ux).sum()), float((r * uy).sum()))
    from paper_1709_05458_amd import cases as C
    _, uxa, uya = C.taylor_green_fields(case.grid.xc, case.grid.yc, t, case.meta["u0"], 1.0, 1.0,
                                        case.meta["nu"], case.vs.RT)
    err = math.sqrt(float(((ux - uxa) ** 2 + (uy - uya) ** 2).sum()) / float((uxa ** 2 + uya ** 2).sum()))
    checks = {"steps_total": warmup + steps, "mass_rel_drift": abs(mass - mass0) / mass0,
              "momentum_drift_over_mass": max(abs(mom[0] - mom0[0]), abs(mom[1] - mom0[1])) / mass0,
              "u_rel_l2_vs_analytic_decay": err}
    return {"ms_per_step": ms_total / steps, "stage_a_ms": a_ms, "stage_c_ms": c_ms,
            "launches": (a_n, c_n), "variant": desc, "u_max": float(max(np.abs(ux).max(), np.abs(uy).max())),
            "mass": float(r.mean()), "checks": checks, "_u": (ux, uy)}


def precision_gap(u32, u64):
    """FP32-delta velocity field against the FP64 one after the same steps from
    the same initial state: max |u32 - u64| / max |u64| and the relative L2
    distance (both components)."""
    d = max(float(np.abs(a - b).max()) for a, b in zip(u32, u64))
    m = max(float(np.abs(b).max()) for b in u64)
    l2 = math.sqrt(sum(float(((a - b) ** 2).sum()) for a, b in zip(u32, u64)) /
                   sum(float((b ** 2).sum()) for b in u64))
    return {"u_max_rel_diff": d / m, "u_rel_l2": l2}


def run_batched(args):
    """64 independent cavities (D2Q9 bounce-back or Newton-Cotes 16^2..40^2
    diffuse walls, 32^2..256^2 cells, Kn log-uniform in [1e-3, 10], seed 4),
    FP32-delta, one graph launch per step, tuned tiles."""
    import torch
    from paper_1709_05458_amd import cases as C, dugks, tune
    cases = C.batch_cases(64, seed=4)
    tiles = tune.tiles_for(cases, dugks.FP32_DELTA)
    b = dugks.BatchSolver(cases, dugks.FP32_DELTA, tiles=tiles)
    for inst, c in zip(b.instances, cases):
        inst.init_equilibrium(c.rho, c.ux, c.uy)
    b.step(args.warmup)
    b.sync()
    torch.cuda.synchronize()
    b.prof_begin(args.steps + 4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    g_ms, g_n = b.prof_query(dugks.K_AUX)
    b.sync()
    pairs = sum(c.grid.nx * c.grid.ny * c.vs.nq for c in cases)
    desc = b.describe()
    b.close()
    gcups = pairs / (ms * 1e-3) / 1e9
    # algorithmic bytes of a step: lattice instances 5 elements per pair (stage A
    # read + write, stage C two reads + write); any-size instances 7 (each stage
    # reads its input twice)
    lat_pairs = sum(c.grid.nx * c.grid.ny * c.vs.nq for c in cases if c.vs.name == "D2Q9")
    step_bytes = 4 * (5 * lat_pairs + 7 * (pairs - lat_pairs))
    achieved = step_bytes / (ms * 1e-3) / 1e9
    return {
        "metric": METRIC,
        "value": round(gcups, 3), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched: 64 lid-driven cavities, 32^2..256^2 cells, D2Q9 or Newton-Cotes "
                               "16^2..40^2, Kn 1e-3..10, seed 4, one graph launch per step",
                   "pairs": pairs, "variant": desc},
        "roofline": {"bound": "hbm", "kernel": "whole step (graph)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": step_bytes, "launch_ms": round(g_ms, 5)},
        "cpu_baseline": None,
    }


def run_rarefied(args):
    """Rarefied lid-driven cavity: 128^2 tanh-stretched cells, Newton-Cotes
    nc x nc velocities on [-4, 4] sqrt(RT), Kn = 1, diffuse walls, FP32-delta."""
    import torch
    from paper_1709_05458_amd import cases as C, dugks
    n = args.n if args.n != 2048 else 128
    vs = C.newton_cotes(args.nc, 0.5)
    case = C.cavity_case(n, vs, wall=C.BC_DIFFUSE, grid=C.tanh_grid(n, n), tau=C.kn_to_tau(1.0, 0.5),
                         lid=0.146, cfl=0.25)
    out = {}
    pairs = n * n * vs.nq
    steps = max(3, args.steps // 10)
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
    for prec, name, elem in ((dugks.FP32_DELTA, "fp32", 4), (dugks.FP64, "fp64", 8)):
        s = dugks.Solver(case, prec, allow_defect=True, tile=tile)
        s.init_equilibrium(case.rho, case.ux, case.uy)
        s.step(2)
        s.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # kernel times in a run of their own: while profiling, each stage's
        # faces and update kernels are timed separately
        s.prof_begin(4 * steps + 8)
        s.step(steps)
        f_ms, f_n = s.prof_query(dugks.K_LQ_FACES)
        u_ms, u_n = s.prof_query(dugks.K_LQ_UPDATE)
        s.prof_end()
        s.sync()
        # algorithmic bytes of the faces kernel: it reads the stage input and
        # writes the x- and y-face values, about three stored elements per pair
        faces_gbs = 3 * elem * pairs / (f_ms * 1e-3) / 1e9
        out[name] = {"value": round(pairs / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 4),
                     "variant": s.describe(), "faces_ms": round(f_ms, 5), "update_ms": round(u_ms, 5),
                     "launches": (f_n, u_n), "faces_GBs": round(faces_gbs, 1),
                     "faces_frac": round(faces_gbs / HBM_PEAK_GBS, 4)}
        s.close()
    r = out["fp32"]
    traffic = stored_traffic(f"any_size_rarefied_cavity{n}_nc{args.nc}_fp32delta_traffic.txt", "lq_faces",
                             LQ_SOURCES)
    return {"metric": METRIC,
            "value": r["value"], "unit": UNIT, "n_gpus": 1,
            "steps": steps, "warmup": 2, "ms_per_step": r["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"rarefied cavity {n}x{n} tanh cells, Newton-Cotes {args.nc}x{args.nc}, "
                                   "Kn 1, diffuse walls",
                       "pairs": pairs, "variant": r["variant"]},
            "fp64": out["fp64"],
            "roofline": {"bound": "hbm", "kernel": "lq_faces (any-size faces kernel, both stages)",
                         "achieved": r["faces_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": r["faces_frac"], "traffic": None if traffic is None else round(traffic),
                         "bytes_per_launch": 3 * 4 * pairs,
                         "launch_ms": r["faces_ms"], "update_ms": r["update_ms"]},
            "cpu_baseline": None}


def run_adjoint(args):
    """Gradient of ||u(T)||^2 after 500 T3S3 steps of the Taylor-Green vortex
    (256^2, D2Q9, per-cell tau field, FP32-delta forward, FP64 adjoint) with
    respect to the initial f and the tau field, checkpoint every 25 steps
    (dugks_backward).  Inputs and outputs stay in device memory."""
    import torch
    from paper_1709_05458_amd import cases as C, dugks
    n, nsteps, ckpt = 256, 500, 25
    case = C.tgv_case(n, C.d2q9(1.0 / 3.0))
    s = dugks.Solver(case, dugks.FP32_DELTA, tau_field=True)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    dev = torch.device("cuda", 0)
    f0 = torch.from_numpy(s.get_state()).to(dev)
    s.step(nsteps)
    _, ux, uy = s.moments()
    seed = torch.from_numpy(2.0 * np.stack([ux, uy])).to(dev)
    s.backward(f0, 50, ckpt, None, seed)   # warm-up (workspace, code paths)
    torch.cuda.synchronize()
    s.prof_begin(nsteps + 8)
    t0 = time.perf_counter()
    gf, gt = s.backward(f0, nsteps, ckpt, None, seed)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    a_ms, a_n = s.prof_query(dugks.K_ADJ_STEP)
    s.prof_end()
    finite = bool(torch.isfinite(gf).all().item() and torch.isfinite(gt).all().item())
    desc = s.describe()
    s.close()
    pairs = n * n * case.vs.nq
    # algorithmic bytes of one reverse step: read the adjoint state and write
    # its predecessor (FP64), read the forward state and the stage-A output it
    # linearises about (FP32-delta)
    per_pair = 8 + 8 + 4 + 4
    achieved = per_pair * pairs / (a_ms * 1e-3) / 1e9
    ms = wall * 1e3 / nsteps
    return {"metric": METRIC,
            "value": round(pairs / (ms * 1e-3) / 1e9, 3), "unit": UNIT, "n_gpus": 1,
            "steps": nsteps, "warmup": 1, "ms_per_step": round(ms, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "adjoint: taylor-green 256x256 D2Q9 with a tau field, 500 steps, checkpoint "
                                   "every 25, FP32-delta forward and FP64 adjoint; value counts each step of "
                                   "the backward call once (forward recompute included)",
                       "pairs": pairs, "variant": desc, "gradients_finite": finite},
            "roofline": {"bound": "hbm", "kernel": "one reverse step (adj_prep, adj_face x2, adj_cellC, adj_cellA)",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                         "bytes_per_launch": per_pair * pairs, "launch_ms": round(a_ms, 5), "launches": a_n},
            "cpu_baseline": None}


def run_cavity(args):
    """Lid-driven cavity (the paper's wall-bounded flow): [0,1]^2, bounce-back walls,
    lid Ma 0.1 against sqrt(3 RT), Re 1000, n x n cells, D2Q9 or D2Q37,
    FP32-delta with FP64 beside it.  Interior tiles run the compile-time-shape
    kernels, tiles touching a wall the general ones."""
    import torch
    from paper_1709_05458_amd import cases as C, dugks
    vs = C.d2q37(1.0 / 3.0) if args.lattice == "d2q37" else C.d2q9(1.0 / 3.0)
    case = C.cavity_case(args.n, vs, re=1000.0)
    pairs = args.n * args.n * vs.nq
    # 16 x 16 tiles: the ring of wall tiles that the general kernel takes is
    # 508 tiles (two rounds of blocks at one block per CU) against 636 for the
    # 32 x 8 default, which is best on periodic grids
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else (16, 16)
    out = {}
    for prec, name, steps in ((dugks.FP32_DELTA, "fp32", args.steps), (dugks.FP64, "fp64", args.steps)):
        s = dugks.Solver(case, prec, tile=tile)
        s.init_equilibrium(case.rho, case.ux, case.uy)
        m0 = float(s.moments()[0].sum())
        s.step(args.warmup)
        s.sync()
        s.prof_begin(2 * steps + 8)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        a_ms, _ = s.prof_query(dugks.K_STAGE_A)
        c_ms, _ = s.prof_query(dugks.K_STAGE_C)
        s.prof_end()
        s.sync()   # raises on a non-finite state
        r, ux, uy = s.moments()
        out[name] = {"value": round(pairs / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 5),
                     "variant": s.describe(), "steps": steps,
                     "mass_rel_drift": abs(float(r.sum()) - m0) / m0,
                     "u_max_over_lid": float(np.abs(ux).max() / case.meta["U"]),
                     "stage_a_ms": a_ms, "stage_c_ms": c_ms, "_u": (ux, uy)}
        s.close()
    gap = precision_gap(out["fp32"].pop("_u"), out["fp64"].pop("_u"))
    r32 = out["fp32"]
    # dominant stage, timed as one record over its launches (the fast kernel
    # on the interior tiles, the general one on the ring of wall tiles);
    # algorithmic bytes as for the periodic flow: 3 stored elements per pair
    # for stage C, 2 for stage A
    dom = "C" if r32["stage_c_ms"] >= r32["stage_a_ms"] else "A"
    dom_ms = r32["stage_c_ms"] if dom == "C" else r32["stage_a_ms"]
    bytes_dom = (3 if dom == "C" else 2) * 4 * pairs
    achieved = bytes_dom / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": f"stage {dom} (sweep_fast on interior tiles + sweep_small on the "
                                          "wall ring, one record)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": bytes_dom, "launch_ms": round(dom_ms, 5),
                "stage_a_ms": round(r32["stage_a_ms"], 5), "stage_c_ms": round(r32["stage_c_ms"], 5)}
    for k in out:
        out[k]["stage_a_ms"] = round(out[k]["stage_a_ms"], 5)
        out[k]["stage_c_ms"] = round(out[k]["stage_c_ms"], 5)
    return {"metric": METRIC,
            "value": r32["value"], "unit": UNIT, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"lid-driven cavity {args.n}x{args.n}, {vs.name}, Re 1000, lid Ma 0.1, "
                                   "bounce-back walls, FP32-delta storage",
                       "pairs": pairs, "variant": r32["variant"]},
            "fp64": out["fp64"],
            "checks": dict({k: {"mass_rel_drift": out[k]["mass_rel_drift"],
                                "u_max_over_lid": out[k]["u_max_over_lid"]} for k in out},
                           fp32_vs_fp64=dict(gap, steps_total=args.warmup + args.steps)),
            "roofline": roofline, "cpu_baseline": None}


def run_abc3d(args):
    """Three-dimensional sweep on the Arnold-Beltrami-Childress flow: a
    triply periodic box of n^3 uniform cells on [0, 2 pi]^3, D3Q19 or D3Q27,
    nu = 0.01, Ma 0.05, CFL 0.5; FP32-delta with FP64 beside it, the same
    steps from the same equilibrium start."""
    import torch
    from paper_1709_05458_amd import cases as C, dugks
    vs = getattr(C, args.lattice3)(1.0 / 3.0)
    case = C.abc_case(args.n3, vs, nu=0.01, ma=0.05, cfl=0.5)
    pairs = case.ncell * vs.nq
    out = {}
    for prec, name in ((dugks.FP32_DELTA, "fp32"), (dugks.FP64, "fp64")):
        s = dugks.Solver3D(case, prec)
        s.init_equilibrium(case.rho, case.u)
        r0, u0 = s.moments()
        s.step(args.warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(args.steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        a_ms, c_ms = s.step_timed(10)   # kernel time per stage, HIP events on the library's stream
        r, u = s.moments()
        if not np.isfinite(r).all():
            raise RuntimeError("non-finite state")
        out[name] = {"value": round(pairs / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 5),
                     "stage_a_ms": round(a_ms, 5), "stage_c_ms": round(c_ms, 5),
                     "mass_rel_drift": abs(float(r.sum()) - float(r0.sum())) / float(r0.sum()),
                     "_u": tuple(u)}
        s.close()
    gap = precision_gap(out["fp32"].pop("_u"), out["fp64"].pop("_u"))
    r32 = out["fp32"]
    # dominant stage; algorithmic bytes as for the two-dimensional sweep: stage
    # C reads fhat and tilde f and writes fhat (3 stored elements per pair),
    # stage A reads fhat and writes tilde f (2).  The kernels also move the
    # transformed states B of both stages (design traffic, not counted).
    dom = "C" if r32["stage_c_ms"] >= r32["stage_a_ms"] else "A"
    dom_ms = r32["stage_c_ms"] if dom == "C" else r32["stage_a_ms"]
    bytes_dom = (3 if dom == "C" else 2) * 4 * pairs
    achieved = bytes_dom / (dom_ms * 1e-3) / 1e9
    traffic = stored_traffic(f"sweep3d_abc{args.n3}_{vs.name.lower()}_fp32delta_traffic.txt",
                             f"stage_{dom.lower()}", SOURCES_3D)
    roofline = {"bound": "hbm", "kernel": f"stage {dom} (k3_stage_lat, STAGE={1 if dom == 'C' else 0})",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(round(traffic)),
                "bytes_per_launch": bytes_dom, "launch_ms": round(dom_ms, 5),
                "stage_a_ms": r32["stage_a_ms"], "stage_c_ms": r32["stage_c_ms"]}
    n = args.n3
    return {"metric": METRIC, "value": r32["value"], "unit": UNIT, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"ABC flow {n}x{n}x{n} periodic, {vs.name}, nu 0.01, Ma 0.05, FP32-delta "
                                   "storage, T3S3 (three-dimensional sweep)", "pairs": pairs},
            "fp64": out["fp64"],
            "checks": {"fp32_mass_rel_drift": r32["mass_rel_drift"],
                       "fp64_mass_rel_drift": out["fp64"]["mass_rel_drift"],
                       "fp32_vs_fp64": dict(gap, steps_total=args.warmup + args.steps + 10)},
            "roofline": roofline, "cpu_baseline": None}


def cpu_baseline(lattice):
    """The oracle as it stands on the host cores, on a bounded sample of the
    same workload (Taylor-Green, same velocity set, 256 x 256, a few steps)."""
    import oracle
    n = 256
    case = make_case(n, lattice)
    o = oracle.Oracle(case)
    fh = o.init_fhat()
    t0 = time.perf_counter()
    o.run(fh, 1)
    t1 = time.perf_counter() - t0
    steps = max(2, min(200, int(math.ceil(15.0 / max(t1, 1e-3)))))   # about 15 s of CPU work
    t0 = time.perf_counter()
    o.run(fh, steps)
    dt = time.perf_counter() - t0
    pairs = n * n * case.vs.nq
    return {"value": pairs * steps / dt / 1e9, "unit": UNIT,
            "cores": o.num_threads(), "kind": "oracle",
            "sample": f"Taylor-Green {n}x{n} {case.vs.name} FP64, {steps} steps ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1709_05458_amd import dugks
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload == "batched":
        print(json.dumps(run_batched(args)))
        return
    if args.workload == "rarefied":
        print(json.dumps(run_rarefied(args)))
        return
    if args.workload == "adjoint":
        print(json.dumps(run_adjoint(args)))
        return
    if args.workload == "cavity":
        print(json.dumps(run_cavity(args)))
        return
    if args.workload == "abc3d":
        print(json.dumps(run_abc3d(args)))
        return
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
    case = make_case(args.n, args.lattice)
    Q = case.vs.nq
    pairs = args.n * args.n * Q
    print(f"# bench: TGV {args.n}^2 {case.vs.name} FP32-delta, {args.steps} steps", file=sys.stderr, flush=True)
    scheme = dugks.T2S3 if args.scheme == "t2s3" else dugks.T3S3
    r32 = time_run(case, dugks.FP32_DELTA, args.steps, args.warmup, tile, scheme)
    u32 = r32.pop("_u")
    print(f"# fp32-delta: {r32}", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        # the same steps from the same initial state, so that the two fields compare
        r64 = time_run(case, dugks.FP64, args.steps, args.warmup, tile, scheme)
        u64 = r64.pop("_u")
        print(f"# fp64: {r64}", file=sys.stderr, flush=True)
    gcups = pairs / (r32["ms_per_step"] * 1e-3) / 1e9
    # dominant kernel (the longer of the two stage kernels).  Algorithmic
    # bytes per launch: stage A reads fhat and writes tilde f (2 stored
    # elements per pair), stage C reads tilde f and fhat and writes the new
    # fhat (3); halo re-reads and per-cell tau are not counted.
    s = 4
    dom = "C" if r32["stage_c_ms"] >= r32["stage_a_ms"] else "A"
    per_pair = 3 if dom == "C" else 2
    bytes_dom = per_pair * s * pairs
    dom_ms = r32["stage_c_ms"] if dom == "C" else r32["stage_a_ms"]
    achieved = bytes_dom / (dom_ms * 1e-3) / 1e9
    traffic = stored_traffic(traffic_summary_name(args.n, case.vs.name), f"stage_{dom.lower()}")
    out = {
        "metric": METRIC,
        "value": round(gcups, 3),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"taylor-green {args.n}x{args.n} periodic, {case.vs.name}, FP32-delta storage, "
                               f"{args.scheme.upper()}",
                   "cells": args.n * args.n, "velocities": Q, "pairs": pairs,
                   "variant": r32["variant"]},
        "roofline": {"bound": "hbm", "kernel": f"stage {dom} (sweep_fast, STAGE={1 if dom == 'C' else 0})",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "bytes_per_launch": bytes_dom, "launch_ms": round(dom_ms, 5),
                     "stage_a_ms": round(r32["stage_a_ms"], 5), "stage_c_ms": round(r32["stage_c_ms"], 5)},
    }
    out["checks"] = {"fp32_delta": r32["checks"], "fp64": r64["checks"] if r64 else None,
                     "fp32_vs_fp64": dict(precision_gap(u32, u64), steps_total=args.warmup + args.steps)
                     if r64 else None}
    if r64:
        g64 = pairs / (r64["ms_per_step"] * 1e-3) / 1e9
        # the same dominant stage as the FP32-delta line (T2S3: its single sweep)
        ms64 = r64["stage_c_ms"] if dom == "C" else r64["stage_a_ms"]
        a64 = per_pair * 8 * pairs / (ms64 * 1e-3) / 1e9
        out["fp64"] = {"value": round(g64, 3), "ms_per_step": round(r64["ms_per_step"], 5),
                       f"stage_{dom.lower()}_GBs": round(a64, 1), "frac": round(a64 / HBM_PEAK_GBS, 4),
                       "stage_a_ms": round(r64["stage_a_ms"], 5), "stage_c_ms": round(r64["stage_c_ms"], 5)}
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline(args.lattice)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
