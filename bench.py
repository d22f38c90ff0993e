#!/usr/bin/env python3
"""Throughput of the ISM pressure solve on one MI355X.

A step is one whole solve of A x = b - mean(b) from x = 0 to a relative FP64 residual of
1e-10 (every kernel of the method: outer FP64 residuals, coarse solves, fused
prolongation + smoothing + restriction cycles, updates, mean removal).  The inputs are
resident in HBM before the timed region starts.  Default workload: the 8192 x 8192 Neumann
cavity grid with the smooth-plus-noise right-hand side, 32h tiles, FP32 inner cycles inside
the FP64 defect-correction loop; the FP64 form on the same grid is measured beside it.

Prints one JSON line.  `value` is Mdof/s = batch * nx * ny / (seconds per solve) / 1e6.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
CYCLE_BYTES = {"mixed": (12, 8), "fp64": (24, 16)}  # per cell: (e read + rhs read + e write, first cycle)
# hardware-counter record of the fused cycle's HBM traffic (rocprofv3 --pmc, calibrated with
# a plain copy); used while the kernel sources it was taken on are unchanged
PROFILE_RECORD = os.path.join(ROOT, "profiles", "k_cycle_cavity8192_mixed.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1309_7128_amd", "csrc", f)
                  for f in ("ism_cycle.h", "ism_device.h")]


def measured_traffic(workload, nu):
    """HBM bytes per cycle launch from the counter record, or None if there is no record for
    this workload and sweep count or the kernel sources changed since it was taken."""
    import hashlib
    import re

    try:
        text = open(PROFILE_RECORD).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(f, "rb").read())
    except OSError:
        return None
    for m in re.finditer(r"^traffic-record: (.*)$", text, re.M):
        kv = dict(item.split("=", 1) for item in m.group(1).split())
        if kv.get("workload") == workload and int(kv.get("nu", -1)) == nu and \
                kv.get("source_sha256") == h.hexdigest():
            return int((float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                        float(kv["write_kib"]) * float(kv["write_scale"])) * 1024)
    return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cavity8192_mixed")
    ap.add_argument("--nu", type=int, default=5, help="sweeps per cycle (FP32 inner cycles)")
    ap.add_argument("--nu-fp64", type=int, default=4, help="sweeps per cycle of the FP64 form")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel event timing")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="time every n-th launch of each kernel class inside the timed region "
                         "(each HIP event record costs the stream a few microseconds)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB, three times (copy "
                         "ceiling and counter calibration)")
    ap.add_argument("--read-gib", type=float, default=0.0,
                    help="only run a plain device read (a sum) of this many GiB, three times "
                         "(counter calibration)")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="jet workload: this many successive warm-started solves per step (the "
                         "time loop); step t's right-hand side is step 0's shifted t cells in x")
    ap.add_argument("--oneshot-table", type=int, default=0,
                    help="only run this many warm-started time steps of the workload with the "
                         "paper's one-shot accommodative cycling, for each tile size and coarse "
                         "criterion of --oneshot-tiles / --oneshot-coarse-tol, one JSON line each")
    ap.add_argument("--oneshot-tiles", default="16,32")
    ap.add_argument("--oneshot-coarse-gs", default="block",
                    help="coarse iteration of the one-shot table: block and/or multicolour")
    ap.add_argument("--oneshot-precision", default="fp64,mixed",
                    help="fine-stage precision of the one-shot table: fp64 and/or mixed (FP32)")
    ap.add_argument("--time-loop", type=int, default=0,
                    help="only run this many projection time steps (predictor, pressure solve, "
                         "correction) of a shear-driven cavity of --time-loop-n cells per side")
    ap.add_argument("--time-loop-n", type=int, default=2048)
    ap.add_argument("--oneshot-coarse-tol", default="1e-2,1e-3,1e-4",
                    help="coarse criteria as fractions of max|b| (fine criterion: 1e-5 max|b|)")
    ap.add_argument("--schemes", action="store_true",
                    help="only compare ISM, the 5-point GMG variant and ACM on the 2048^2 FP64 "
                         "cavity at 16h and 32h: one JSON line each with cycles, kernel launches "
                         "and time per solve")
    ap.add_argument("--projection", action="store_true",
                    help="only time the differentiable projection (forward solve and backward "
                         "adjoint solve through torch.autograd) on the 8 x 1024^2 batch")
    ap.add_argument("--cycles-only", type=int, default=0,
                    help="only run this many fused cycles on the workload grid (short program "
                         "for hardware-counter passes)")
    return ap.parse_args()


# The library's default (ISM_FUSED_AUTO) takes the LDS-tiled cycle kernel up to this many
# cells per launch (include/ism.h), the row walk above.
TILE_CELLS = 1024 * 1024


def cycle_kernel_name(w, cells, nu):
    t = "float" if w.precision == "mixed" else "double"
    if cells <= TILE_CELLS:  # cells of the whole batch
        return f"k_cycle_tile<{t}, {nu}>"
    return f"k_cycle<{t}, {nu}, {w.coarsen.bit_length() - 1}>"


def oneshot_table(w, args):
    """The paper's iteration and synchronization counts (Sec. 4.3, Tables A.1-A.3) on a
    synthetic time loop: step 0 is solved to the workload's tolerance with the default
    cycling, then each step t = 1 .. K solves the right-hand side of step t (the jet's
    perturbation moved t cells) warm-started from step t-1, with one-shot accommodative
    cycling (block or multicolour GS on the coarse grid to the coarse criterion, then fine
    red-black iterations to the fine one).  Per configuration: mean I_c, I_f, NCC_c (I_c for
    block GS, colours x I_c for multicolour GS), NCC_f = 2 I_f, NCC_t and
    N_Lap = NCC_f / 2 + NCC_c / n^2 per step, and wall time."""
    import torch

    from paper_1309_7128_amd import inputs
    from paper_1309_7128_amd.solver import Solver

    u, v = inputs.workload_fields(w.name, 0)
    ref = Solver(w.nx, w.ny, bc_x=w.bc_x, bc_y=w.bc_y, coarsen=w.coarsen, lx=w.lx, ly=w.ly,
                 precision="mixed", rtol=w.rtol)
    b0 = ref.div(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda())
    x0, _ = ref.solve(b0)
    bmax = float(b0.abs().max())
    steps = [torch.roll(b0, t, dims=-1) if w.bc_x == "periodic" else b0
             for t in range(1, args.oneshot_table + 1)]
    configs = [(gs, prec, n, frac) for gs in args.oneshot_coarse_gs.split(",")
               for prec in args.oneshot_precision.split(",")
               for n in [int(a) for a in args.oneshot_tiles.split(",")]
               for frac in [float(a) for a in args.oneshot_coarse_tol.split(",")]]
    for gs, prec, n, frac in configs:
        s = Solver(w.nx, w.ny, bc_x=w.bc_x, bc_y=w.bc_y, coarsen=n, lx=w.lx, ly=w.ly,
                   precision=prec, cycling="oneshot", coarse_tol=frac * bmax,
                   fine_tol=1e-5 * bmax, max_cycles=200000, coarse_gs=gs)
        x = x0.clone()
        ic = fi = syncs = csyncs = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for bt in steps:
            x, st = s.solve(bt, x)
            ic += st["coarse_iters"]
            fi += st["fine_iters"]
            syncs += st["host_syncs"]
            csyncs += st["coarse_syncs"]
        dt = time.perf_counter() - t0
        k = len(steps)
        ncc_c, ncc_f = csyncs / k, 2.0 * fi / k
        print(json.dumps({"workload": w.name, "coarse_gs": gs, "precision": prec, "tile": n,
                          "coarse_tol_frac": frac,
                          "fine_tol_frac": 1e-5, "steps": k, "I_c": ic / k, "I_f": fi / k,
                          "NCC_c": ncc_c, "NCC_f": ncc_f, "NCC_t": ncc_c + ncc_f,
                          "N_Lap": ncc_f / 2.0 + ncc_c / float(n * n),
                          "host_syncs_per_step": syncs / k,
                          "ms_per_step": round(1e3 * dt / k, 2)}), flush=True)


def schemes(args):
    """Configuration 2: ISM against the comparison schemes (the 5-point coarse stencil of
    aggressive-coarsening GMG and additive correction multigrid, Sec. 4.3.1-4.3.2) on the
    2048^2 FP64 cavity, 16h and 32h, each solved from x = 0 to 1e-10."""
    import torch

    from paper_1309_7128_amd import inputs
    from paper_1309_7128_amd.solver import Solver

    w = inputs.WORKLOADS["cavity2048_fp64"]
    u, v = inputs.workload_fields(w.name, 0)
    for n in (16, 32):
        for scheme in ("ism", "gmg5", "acm"):
            s = Solver(w.nx, w.ny, coarsen=n, precision="fp64", rtol=w.rtol, nu=args.nu_fp64,
                       coarse_stencil=scheme)
            b = s.div(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda())
            s.solve(b)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = max(1, args.steps)
            for _ in range(k):
                _, st = s.solve(b)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / k
            print(json.dumps({"workload": w.name, "scheme": scheme, "coarsen": n,
                              "nu": 1 if scheme == "acm" else args.nu_fp64,
                              "cycles": st["cycles"], "launches": st["launches"],
                              "host_syncs": st["host_syncs"], "rel_res_l2": st["rel_res_l2"],
                              "ms_per_solve": round(1e3 * dt, 3),
                              "Mdof_per_s": round(w.nx * w.ny / dt / 1e6, 2)}), flush=True)
            s.close()


def projection(args):
    """Configuration 5: u -> u - G A^+ (D u - mean) through torch.autograd on 8 independent
    1024^2 grids (mixed precision, 1e-10), loss = sum(w u_new) with seeded normal weights; one
    step is the forward solve and the backward adjoint solve.  Mdof/s counts the cells of
    the batch per step."""
    import numpy as np
    import torch

    from paper_1309_7128_amd import inputs
    from paper_1309_7128_amd.autograd import project
    from paper_1309_7128_amd.solver import Solver

    w = inputs.WORKLOADS["batch8x1024_mixed"]
    s = Solver(w.nx, w.ny, batch=w.batch, coarsen=w.coarsen, precision="mixed", rtol=w.rtol,
               nu=args.nu)
    uv = [inputs.workload_fields(w.name, k) for k in range(w.batch)]
    u = torch.from_numpy(np.stack([a for a, _ in uv])).cuda()
    v = torch.from_numpy(np.stack([c for _, c in uv])).cuda()
    wts = [inputs.normal_faces(600 + k, uv[k][0].shape, uv[k][1].shape) for k in range(w.batch)]
    wu = torch.from_numpy(np.stack([a for a, _ in wts])).cuda()
    wv = torch.from_numpy(np.stack([c for _, c in wts])).cuda()

    def step():
        uu = u.clone().requires_grad_(True)
        vv = v.clone().requires_grad_(True)
        un, vn, _ = project(uu, vv, s)
        loss = (wu * un).sum() + (wv * vn).sum()
        loss.backward()
        return uu.grad, vv.grad

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = max(1, args.steps)
    for _ in range(k):
        gu, gv = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / k
    cells = w.batch * w.nx * w.ny
    print(json.dumps({"workload": "batch8x1024_projection", "steps": k,
                      "ms_per_step": round(1e3 * dt, 3), "Mdof_per_s": round(cells / dt / 1e6, 2),
                      "step": "forward solve + backward adjoint solve", "nu": args.nu,
                      "grad_finite": bool(torch.isfinite(gu).all() and torch.isfinite(gv).all())}),
          flush=True)


def time_loop(args):
    """Projection time steps of Goda's scheme (Sec. 2.2) on a shear-driven cavity in the shape
    of Benchmark I (Sec. 4.3.1): unit cells, dt = 1, viscosity 0.1, walls sliding
    counter-clockwise at 0.1, from rest.  Each step is the explicit predictor, the divergence,
    a mixed-precision pressure solve to 1e-8 warm-started from the previous pressure change,
    and the correction.  The first 5 steps are warm-up; the rest are timed."""
    import torch

    from paper_1309_7128_amd.solver import Solver

    n = args.time_loop_n
    U = 0.1
    walls = (-U, U, U, -U)
    s = Solver(n, n, coarsen=32 if n >= 4096 else 16, lx=float(n), precision="mixed", rtol=1e-8,
               nu=args.nu)
    u = torch.zeros(s.u_shape, dtype=torch.float64, device="cuda")
    v = torch.zeros(s.v_shape, dtype=torch.float64, device="cuda")
    p = torch.zeros(s.cell_shape, dtype=torch.float64, device="cuda")
    x = None
    for _ in range(5):
        u, v, p, x, _ = s.step(u, v, p, 1.0, 0.1, walls, x)
    torch.cuda.synchronize()
    cycles = 0
    t0 = time.perf_counter()
    for _ in range(args.time_loop):
        u, v, p, x, st = s.step(u, v, p, 1.0, 0.1, walls, x)
        cycles += st["cycles"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k = args.time_loop
    print(json.dumps({"workload": f"cavity{n}_time_loop", "steps": k,
                      "ms_per_step": round(1e3 * dt / k, 3),
                      "Mdof_per_s": round(n * n * k / dt / 1e6, 2),
                      "solve_cycles_per_step": cycles / k}), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solver is a single-GPU library and this "
              "benchmark has no multi-GPU mode (run it with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1309_7128_amd import inputs
    from paper_1309_7128_amd.solver import Solver

    torch.cuda.set_device(0)
    if args.copy_gib > 0:
        n = int(args.copy_gib * (1 << 30) // 4)
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return
    if args.read_gib > 0:
        n = int(args.read_gib * (1 << 30) // 4)
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        for _ in range(3):
            tot = a.sum()
        torch.cuda.synchronize()
        print(json.dumps({"read_bytes": 4 * n, "sum": float(tot)}))
        return

    w = inputs.WORKLOADS[args.workload]
    if args.cycles_only > 0:
        return cycles_only(w, args)
    if args.oneshot_table > 0:
        return oneshot_table(w, args)
    if args.time_loop > 0:
        return time_loop(args)
    if args.schemes:
        return schemes(args)
    if args.projection:
        return projection(args)
    u, v = inputs.workload_fields(w.name, 0) if w.batch == 1 else (None, None)
    if w.batch > 1:
        uv = [inputs.workload_fields(w.name, k) for k in range(w.batch)]
        u = np.stack([a for a, _ in uv])
        v = np.stack([c for _, c in uv])
        del uv
    cells = w.batch * w.nx * w.ny

    def make(prec):
        nu = args.nu if prec == "mixed" else args.nu_fp64
        return Solver(w.nx, w.ny, batch=w.batch, bc_x=w.bc_x, bc_y=w.bc_y, coarsen=w.coarsen,
                      lx=w.lx, ly=w.ly, precision=prec, nu=nu, rtol=w.rtol)

    s = make(w.precision)
    b = s.div(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda())
    del u, v
    x = torch.zeros(s.cell_shape, dtype=torch.float64, device="cuda")

    def run(solver, steps, profile):
        stats = []
        torch.cuda.synchronize()
        if profile:
            solver.profile(True, every=args.profile_every)
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            if args.time_steps:
                # the jet's perturbation moves one cell per step along the periodic axis; a
                # whole-cell shift commutes with the divergence, so b_t = b_0 rolled by t
                for t in range(args.time_steps):
                    _, st = solver.solve(torch.roll(b, t, dims=-1), x)
                    stats.append(st)
            else:
                _, st = solver.solve(b, x)
                stats.append(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = solver.profile_read() if profile else None
        if profile:
            solver.profile(False)
        return dt, stats, prof

    run(s, args.warmup, False)
    dt, stats, prof = run(s, args.steps, not args.no_profile)
    ms = 1e3 * dt / args.steps
    solves_per_step = max(1, args.time_steps)
    value = cells * solves_per_step / (dt / args.steps) / 1e6
    last = stats[-1]
    status_ok = all(st["status"] == 0 and st["rel_res_l2"] <= w.rtol for st in stats)

    roofline = None
    if prof is not None and prof["cycle"][1] > 0:
        per, first = CYCLE_BYTES[w.precision]
        launches = sum(st["cycles"] for st in stats)  # every cycle launch of the timed region
        firsts = sum(st["outer_iters"] for st in stats)  # an inner solve's first cycle reads no e
        alg = (per * (launches - firsts) + first * firsts) * cells
        timed = prof["cycle"][1]  # the launches the events bracketed (every n-th)
        avg_s = prof["cycle"][0] * 1e-3 / timed
        achieved = alg / launches / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(w.name, args.nu if w.precision == "mixed" else args.nu_fp64),
                    "kernel": cycle_kernel_name(w, cells, args.nu if w.precision == "mixed"
                                                else args.nu_fp64),
                    "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
                    "timed_launches": timed, "bytes_per_launch": int(alg / launches)}

    out = {
        "metric": "Mdof/s solved to 1e-10 rel. residual, ISM mixed vs FP64; smoother HBM GB/s",
        "value": round(value, 2),
        "unit": "Mdof/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if w.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "batch": w.batch,
                   "bc": [w.bc_x, w.bc_y], "coarsen": w.coarsen, "nu": args.nu,
                   "precision": w.precision, "rtol": w.rtol},
        "solve": {"cycles": last["cycles"], "outer_iters": last["outer_iters"],
                  "launches": last["launches"], "host_syncs": last["host_syncs"],
                  "rel_res_l2": last["rel_res_l2"], "converged": status_ok,
                  "solves_per_step": solves_per_step,
                  "cycles_per_solve_mean": round(sum(st["cycles"] for st in stats) / len(stats), 2)},
        "roofline": roofline,
    }
    if prof is not None:
        # mean time of the timed launches of a class times that class's launches per step
        n_cyc = sum(st["cycles"] for st in stats) / args.steps
        counts = {"cycle": n_cyc, "coarse": n_cyc,
                  "outer": sum(st["outer_iters"] + 1 for st in stats) / args.steps}
        out["kernel_ms_per_step"] = {k: round(v[0] / v[1] * counts[k], 3)
                                     for k, v in prof.items() if v[1] and k in counts}

    if not args.no_fp64 and w.precision == "mixed" and not args.time_steps:
        s.close()
        s64 = make("fp64")
        run(s64, 1, False)
        k64 = max(1, min(3, args.steps))
        dt64, st64, _ = run(s64, k64, False)
        out["fp64"] = {"value": round(cells / (dt64 / k64) / 1e6, 2), "unit": "Mdof/s",
                       "nu": args.nu_fp64,
                       "ms_per_step": round(1e3 * dt64 / k64, 3), "steps": k64,
                       "cycles": st64[-1]["cycles"], "rel_res_l2": st64[-1]["rel_res_l2"]}
        out["mixed_over_fp64"] = round(value / out["fp64"]["value"], 3)
        s64.close()

    if not args.no_cpu:
        mean_cycles = sum(st["cycles"] for st in stats) / len(stats)
        mean_outer = sum(st["outer_iters"] for st in stats) / len(stats)
        out["cpu_baseline"] = cpu_baseline(w, b, mean_cycles, mean_outer, args.nu)

    print(json.dumps(out), flush=True)


def cycles_only(w, args):
    """A few fused two-level cycles on the workload grid (no convergence loop)."""
    import torch

    from paper_1309_7128_amd.solver import Solver

    s = Solver(w.nx, w.ny, batch=w.batch, bc_x=w.bc_x, bc_y=w.bc_y, coarsen=w.coarsen, lx=w.lx,
               ly=w.ly, precision=w.precision, nu=args.nu, rtol=w.rtol)
    dt = torch.float32 if w.precision == "mixed" else torch.float64
    g = torch.Generator(device="cuda").manual_seed(5)
    rhs = torch.randn(s.cell_shape, device="cuda", dtype=dt, generator=g)
    e = torch.zeros(s.cell_shape, device="cuda", dtype=dt)
    rc = s.restrict(rhs, e)
    s.cycle(rhs, e, rc, zero_e=True)
    s.profile(True)
    for _ in range(args.cycles_only):
        s.cycle(rhs, e, rc)
    prof = s.profile_read()
    ms, n = prof["cycle"]
    cells = w.batch * w.nx * w.ny
    per = CYCLE_BYTES[w.precision][0]
    print(json.dumps({"cycles": n, "avg_launch_us": 1e3 * ms / max(n, 1),
                      "achieved_GBs": per * cells / (1e-3 * ms / max(n, 1)) / 1e9 if n else None,
                      "coarse_avg_us": 1e3 * prof["coarse"][0] / max(prof["coarse"][1], 1)}))


def _oracle_sample(w, nu, path):
    """One timed sample of the oracle's ISM iteration on the right-hand side stored at path
    (one outer residual and one inner cycle, in the precision form of the workload), on one
    thread.  Returns (seconds per inner cycle, seconds per outer residual)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ism_oracle as O

    b = np.load(path, mmap_mode="r")
    bx, by, n, h = w.bc_x, w.bc_y, w.coarsen, w.h
    with threadpool_limits(limits=1):
        cs = O.CoarseSolver(O.coarse_matrix(O.coarse_stencil_ism(w.nx // n, w.ny // n, n, bx, by), bx, by))
        t0 = time.perf_counter()
        bp = h * h * (b - b.mean())
        x = np.zeros_like(bp)
        r = bp - O.laplacian(x, bx, by)
        t_outer = time.perf_counter() - t0
        ft = np.float32 if w.precision == "mixed" else np.float64
        rT = r.astype(ft)
        Rc = O.restrict_sum(r, n)
        e = np.zeros_like(rT)
        t0 = time.perf_counter()
        E = cs.solve(Rc)
        e = e + O.prolong_bilinear(E, n, bx, by, ft)
        e = O.red_black_gs(e, rT, bx, by, sweeps=nu)
        res = rT - O.laplacian(e, bx, by)
        Rc = O.restrict_sum(res.astype(np.float64), n)
        t_cycle = time.perf_counter() - t0
    return t_cycle, t_outer


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, b_dev, gpu_cycles, gpu_outer, nu):
    """The CPU oracle on the same input, timed on the host: one outer residual and one inner
    cycle of its ISM iteration (in the precision form of the workload), extrapolated to the
    number of cycles and outer steps the GPU solve took.  Measured twice: on one core, and
    on every core of this process's CPU share (capped at 16) as that many independent
    oracle solves running at once, one per worker process (the oracle's array operations
    run on one thread, so independent solves are how it uses more cores); the whole-host
    rate is the sum of the workers' rates."""
    import multiprocessing as mp
    import tempfile

    import numpy as np

    b = b_dev.cpu().numpy()
    if w.batch > 1:
        b = b[0]
    b = np.ascontiguousarray(b.reshape(w.ny, w.nx))
    cells = w.nx * w.ny
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "b.npy")
        np.save(path, b)
        del b
        t_cycle, t_outer = _oracle_sample(w, nu, path)
        one = cells / (gpu_cycles * t_cycle + (gpu_outer + 1) * t_outer) / 1e6
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        with mp.get_context("spawn").Pool(workers) as pool:
            samples = pool.starmap(_oracle_sample, [(w, nu, path)] * workers)
    rates = [cells / (gpu_cycles * tc + (gpu_outer + 1) * to) / 1e6 for tc, to in samples]
    mean_cycle = sum(tc for tc, _ in samples) / workers
    return {"value": round(sum(rates), 5), "unit": "Mdof/s", "cores": workers, "kind": "oracle",
            "one_core": round(one, 5), "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"one inner cycle and one outer residual of the oracle's ISM iteration on grid "
                      f"0 of the same input, per worker: {workers} single-threaded oracle solves at "
                      f"once (inner cycle {mean_cycle:.3g} s each on average; {t_cycle:.3g} s when "
                      f"alone), extrapolated to the GPU solve's {gpu_cycles:g} cycles and "
                      f"{gpu_outer:g} outer steps; the oracle's coarse factorization excluded like "
                      f"the library's set-up"}


if __name__ == "__main__":
    main()
