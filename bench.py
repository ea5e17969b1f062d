#!/usr/bin/env python3
"""Benchmark: s-step GMRES time to 1e-8 relative residual on the 3-D 7-point
convection-diffusion problem -Lap u + 50 (u_x + u_y + u_z) = f, 256^3 interior
grid (N = 16 777 216), s-GMRES(m=40, s=8), FP64, x0 = 0, f = A x_true with
x_true ~ U(-1, 1) (seeded).  One step = one full solve from x0 = 0.

Prints one JSON line.  Also reported: the plain comparator (standard
GMRES(320) = s = 1 on the same GPU and kernels), achieved HBM bandwidth per
kernel class from HIP events recorded by the library on its stream, and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def vec_passes_gmres(blocks_per_cycle, s):
    """Algorithmic vector passes (each vector element read or written once)
    of s-step GMRES cycles with the given numbers of blocks."""
    tot = 0
    for nb in blocks_per_cycle:
        for k in range(1, nb + 1):
            tot += (s + 1)                       # matrix powers: read 1, write s
            if k > 1:
                tot += (k - 1) * s + s           # Gram against previous blocks
                tot += (k - 1) * s + 2 * s       # block update (read, write s)
            tot += 2 * (s + 1)                   # block Gram of [w, y_1..y_s]
            tot += s + 2                         # next start vector + norm
        tot += nb * s + 2 + 3                    # assembly + true residual
    return tot


def flops_gmres(blocks_per_cycle, s, N, ndim):
    """Algorithmic floating-point operations per kernel class of s-step GMRES
    cycles (FP64 or FP32 alike): a (2q-1)-flop stencil row of q points, 2 per
    multiply-add of the Gram and update contractions."""
    st = 2 * (2 * ndim + 1) - 1                  # 13 (7-point) or 9 (5-point)
    fl = dict(mpk=0.0, gram=0.0, update=0.0, resid=0.0, scalar=0.0, vec=0.0)
    fl["vec"] += 2.0 * N                         # ||f||
    fl["resid"] += (st + 3.0) * N                # r = f - A x and ||r||^2, initial
    for nb in blocks_per_cycle:
        for k in range(1, nb + 1):
            fl["mpk"] += st * s * N
            if k > 1:
                fl["gram"] += 2.0 * (k - 1) * s * s * N
                fl["update"] += 2.0 * (k - 1) * s * s * N
            fl["vec"] += (s + 1) * (s + 2) * N   # distinct entries of the block's own Gram
            fl["vec"] += 2.0 * s * N + 2.0 * N   # next start vector and its norm
        fl["vec"] += 2.0 * nb * s * N            # x = x0 + V y
        fl["resid"] += (st + 3.0) * N            # true residual of the cycle
    return fl


KERNEL_SOURCES = ("kernels.hpp", "launch.hpp", "mpk.hpp", "mpk3d.hpp", "gram_self.hpp")


def kernel_source_hash():
    """Hash of the sources that define the N-length kernels and their launch
    shapes (a committed traffic record is valid only for these)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2001_04886_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kind):
    """HBM bytes per launch of the kernel class from the committed rocprofv3
    counter summary, or None when the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "sgmres_256cube_s8m40_fp64_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hash") != kernel_source_hash() or kind not in rec:
        return None
    return rec[kind]["hbm_bytes_per_launch"]


def copy_bandwidth_gbs(torch, nbytes=1 << 30, reps=10):
    """Bytes read + written per second by a device-to-device tensor copy."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def blocks_per_cycle(total_blocks, cycles, m):
    out = []
    left = total_blocks
    for c in range(cycles):
        nb = min(m, left) if c < cycles - 1 else left
        out.append(nb)
        left -= nb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--s", type=int, default=8)
    ap.add_argument("--m", type=int, default=40)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--basis", choices=["monomial", "chebyshev"], default="monomial")
    ap.add_argument("--no-plain", action="store_true", help="skip the GMRES(ms) comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--cpu-blocks", type=int, default=2)
    ap.add_argument("--oracle-n", type=int, default=64,
                    help="grid side on which mixed3d compares every result with the oracle")
    ap.add_argument("--cpu-n", type=int, default=96,
                    help="grid side of the all-core oracle timing (one full restart cycle)")
    ap.add_argument("--workload", choices=["gmres3d", "mixed3d", "omin2d", "small2d", "batched",
                                           "learned", "paper2d"],
                    default="gmres3d")
    ap.add_argument("--nsys", type=int, default=512)
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--omin-iters", type=int, default=600)
    ap.add_argument("--eval-samples", type=int, default=64)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2001_04886_amd import problems as PB
    from paper_2001_04886_amd import sstep as S

    S.load()
    dev = torch.device("cuda:0")
    if args.workload != "gmres3d":
        return OTHER[args.workload](args)
    prob = PB.cube_3d(args.n, seed=0, gamma=50.0)
    A = S.Stencil.from_problem(prob)
    N = prob.N
    xt = torch.from_numpy(prob.x_true()).to(dev)
    f = torch.empty_like(xt)
    S.stencil_apply(A, xt, f)
    basis = S.CHEBYSHEV if args.basis == "chebyshev" else S.MONOMIAL
    wsb = max(S.workspace_bytes(A, S.METHOD_GMRES, args.s, args.m),
              S.workspace_bytes(A, S.METHOD_GMRES, 1, args.s * args.m))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    x = torch.zeros_like(xt)
    torch.cuda.synchronize()

    def solve(profile):
        x.zero_()
        return S.gmres_solve(A, f, x, args.s, args.m, args.tol, basis=basis, workspace=ws,
                             profile=profile)

    for _ in range(args.warmup):
        info = solve(True)
        print(f"# warmup: status={info.status} blocks={info.iters} cycles={info.cycles} "
              f"rel_resid={info.rel_resid:.3e} ms={info.ms_total:.1f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(solve(True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    last = infos[-1]
    ok = all(i.status == 0 and i.rel_resid <= args.tol for i in infos)
    xerr = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
    print(f"# timed: {args.steps} solves, {ms_per_step:.1f} ms/solve, blocks={last.iters} "
          f"cycles={last.cycles} rel_resid={last.rel_resid:.3e} |x-x_true|/|x_true|={xerr:.2e}",
          file=sys.stderr, flush=True)

    # per kernel class over the timed region (library events on its stream)
    classes = {}
    for k in S.KERNEL_CLASSES:
        ms = sum(i.ms[k] for i in infos)
        by = sum(i.bytes[k] for i in infos)
        nl = sum(i.launches[k] for i in infos)
        classes[k] = {"ms": ms / args.steps, "launches": nl // args.steps,
                      "GBs": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None,
                      "bytes": by / args.steps}
    fl = flops_gmres(blocks_per_cycle(last.iters, last.cycles, args.m), args.s, N, 3)
    for k in classes:
        classes[k]["GFLOPs"] = (fl[k] / (classes[k]["ms"] * 1e-3) / 1e9
                                if classes[k]["ms"] > 0 and fl[k] > 0 else None)
    dom = max(("gram", "update", "mpk"), key=lambda k: classes[k]["ms"])
    dom_gbs = classes[dom]["GBs"] or 0.0
    traffic = measured_traffic(dom)
    total_bytes = sum(classes[k]["bytes"] for k in classes)
    out = {
        "metric": "s-step GMRES time to 1e-8 rel. resid + HBM GB/s, 7-pt 256^3, vs plain",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D 7-pt convection-diffusion {args.n}^3 gamma=50, "
                               f"s-step GMRES(m={args.m}, s={args.s}), {args.basis} basis, "
                               f"FP64, tol {args.tol:g}, x0=0, x_true~U(-1,1) seed 0",
                   "N": N, "s": args.s, "m": args.m, "tol": args.tol},
        "converged": ok,
        "blocks": last.iters,
        "cycles": last.cycles,
        "rel_resid": last.rel_resid,
        "x_err_vs_true": xerr,
        "algorithmic_GBs_solve": total_bytes / (ms_per_step * 1e-3) / 1e9,
        "GFLOPs_solve": sum(fl.values()) / (ms_per_step * 1e-3) / 1e9,
        "flop_per_solve": sum(fl.values()),
        "fp64_vector_peak_TFLOPs": 78.6,
        "kernels": classes,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dom_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE)",
                     "algorithmic_bytes_per_launch": classes[dom]["bytes"] / max(classes[dom]["launches"], 1)},
    }

    # the machine's attainable streaming rate: a device-to-device copy of
    # 1 GiB (read + write) timed with events, next to the nominal 8 TB/s
    cp = copy_bandwidth_gbs(torch)
    out["roofline"]["measured_copy_GBs"] = cp
    out["roofline"]["frac_of_copy"] = dom_gbs / cp

    if not args.no_plain:
        x.zero_()
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        pinfo = S.gmres_solve(A, f, x, 1, args.s * args.m, args.tol, workspace=ws, profile=False)
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        out["plain"] = {"method": f"GMRES({args.s * args.m}) (s=1, same kernels)",
                        "s": (tp1 - tp0), "steps": pinfo.iters, "cycles": pinfo.cycles,
                        "status": pinfo.status, "rel_resid": pinfo.rel_resid,
                        "speedup_sstep": (tp1 - tp0) / (ms_per_step / 1e3)}
        print(f"# plain GMRES({args.s * args.m}): {tp1 - tp0:.2f} s, steps={pinfo.iters} "
              f"status={pinfo.status}", file=sys.stderr, flush=True)

    if not args.no_cpu:
        from oracle import timing as OT  # CPU baseline leg only
        del ws
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(OT, args, N, blocks_per_cycle(last.iters, last.cycles,
                                                                          args.m),
                                           0 if basis == S.MONOMIAL else 1)
    print(json.dumps(out), flush=True)


def cpu_baseline(OT, args, N, gpu_cycles, basis):
    """The FP64 oracle timed on the host cores, scaled to the benchmarked
    solve by algorithmic vector passes x points (both legs stream far more
    than the caches hold).  All cores: one full restart cycle (m blocks) of
    the same method on the cpu_n^3 grid, OpenMP timing build.  One core:
    the first cpu_blocks blocks on the benchmarked grid, plain build."""
    cpu = OT.host_cpu()
    full = vec_passes_gmres(gpu_cycles, args.s) * N
    nc = args.cpu_n ** 3
    allc = OT.time_sgmres(3, args.cpu_n, 50.0, args.s, args.m, args.m, basis, threads=cpu["cores"])
    est_all = allc["seconds"] / (vec_passes_gmres([allc["blocks"]], args.s) * nc) * full
    one = OT.time_sgmres(3, args.n, 50.0, args.s, args.m, args.cpu_blocks, basis, threads=1)
    est_one = one["seconds"] / (vec_passes_gmres([one["blocks"]], args.s) * N) * full
    print(f"# cpu oracle: {allc['seconds']:.1f} s for a {args.m}-block cycle at {args.cpu_n}^3 on "
          f"{cpu['cores']} threads, {one['seconds']:.1f} s for {args.cpu_blocks} blocks at "
          f"{args.n}^3 on 1 thread", file=sys.stderr, flush=True)
    return {
        "value": est_all, "unit": "s", "cores": cpu["cores"], "kind": "oracle",
        "cpu_model": cpu["model"],
        "sample": f"oracle s-GMRES(m={args.m}, s={args.s}), OpenMP timing build on all "
                  f"{cpu['cores']} host threads: one full {args.m}-block restart cycle of the "
                  f"{args.cpu_n}^3 problem in {allc['seconds']:.1f} s, scaled by algorithmic vector "
                  f"passes x points to the GPU solve ({len(gpu_cycles)} cycles, "
                  f"{sum(gpu_cycles)} blocks at {args.n}^3)",
        "measured_s": allc["seconds"],
        "single_core": {"value": est_one, "cores": 1, "measured_s": one["seconds"],
                        "sample": f"plain oracle build, first {args.cpu_blocks} blocks of the "
                                  f"{args.n}^3 solve on 1 thread, scaled the same way"},
    }


def _classes(S, infos, steps):
    out = {}
    for k in S.KERNEL_CLASSES:
        ms = sum(i.ms[k] for i in infos)
        by = sum(i.bytes[k] for i in infos)
        out[k] = {"ms": ms / steps, "launches": sum(i.launches[k] for i in infos) // steps,
                  "GBs": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None,
                  "bytes": by / steps}
    return out


def _line(metric, value, unit, hib, ms, args, dtype, workload, extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": hib, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": workload}}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_mixed3d(args):
    """FP32 basis / FP64 Gram, least squares and refinement on the 256^3
    problem, s in {4, 8, 12}, tol 1e-10, against FP64 s-step GMRES."""
    import torch
    from paper_2001_04886_amd import problems as PB
    from paper_2001_04886_amd import sstep as S
    import numpy as np
    import oracle as O
    from oracle import timing as OT
    dev = torch.device("cuda:0")
    prob = PB.cube_3d(args.n, seed=0, gamma=50.0)
    A = S.Stencil.from_problem(prob)
    Ao = O.Operator(prob.ndim, prob.nx, prob.ny, prob.nz, c=prob.c)
    xt_h = prob.x_true()
    f_h = O.apply(Ao, xt_h)   # right-hand side and residual checks by the FP64 oracle operator
    xt = torch.from_numpy(xt_h).to(dev)
    f = torch.from_numpy(f_h).to(dev)
    tol = 1e-10
    wsb = max(S.workspace_bytes(A, S.METHOD_GMRES, 12, args.m),
              S.workspace_bytes(A, S.METHOD_GMRES, 12, args.m, S.MIXED))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    x = torch.zeros_like(xt)
    res = {}
    configs = [("fp64_s8", 8, S.FP64, S.MONOMIAL),
               # like with like: the FP64 solve in the basis the mixed s = 8 solve uses
               ("fp64_s8_chebyshev", 8, S.FP64, S.CHEBYSHEV),
               ("mixed_s4", 4, S.MIXED, S.MONOMIAL),
               ("mixed_s8", 8, S.MIXED, S.CHEBYSHEV),
               ("mixed_s12", 12, S.MIXED, S.CHEBYSHEV),
               # larger s in FP64: the three bases side by side
               ("fp64_s12_monomial", 12, S.FP64, S.MONOMIAL),
               ("fp64_s12_chebyshev", 12, S.FP64, S.CHEBYSHEV),
               ("fp64_s12_newton", 12, S.FP64, S.NEWTON),
               ("mixed_s12_newton", 12, S.MIXED, S.NEWTON)]
    for name, s, prec, basis in configs:
        infos = []
        for rep in range(args.warmup + args.steps):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = S.gmres_solve(A, f, x, s, args.m, tol, precision=prec, basis=basis, workspace=ws,
                                 profile=True)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                infos.append((time.perf_counter() - t0, info))
        t = sum(a for a, _ in infos) / len(infos)
        info = infos[-1][1]
        xerr = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
        xh = x.cpu().numpy()
        r_or = float(np.linalg.norm(f_h - O.apply(Ao, xh)) / np.linalg.norm(f_h))
        res[name] = {"s": t, "blocks": info.iters, "cycles": info.cycles, "status": info.status,
                     "rel_resid": info.rel_resid, "x_err_vs_true": xerr,
                     "oracle_true_rel_resid": r_or,
                     "basis": {S.MONOMIAL: "monomial", S.CHEBYSHEV: "chebyshev",
                               S.NEWTON: "newton"}[basis],
                     "kernels": _classes(S, [i for _, i in infos], len(infos))}
        print(f"# {name}: {t:.3f} s blocks={info.iters} cycles={info.cycles} rel_resid={info.rel_resid:.2e}"
              f" x_err={xerr:.2e}", file=sys.stderr, flush=True)
    # error against the FP64 oracle where it can finish: the oracle's solution
    # of the same problem on 64^3 to 1e-12 (all host cores), every
    # configuration solved on the GPU to 1e-10
    small = PB.cube_3d(args.oracle_n, seed=0, gamma=50.0)
    As = S.Stencil.from_problem(small)
    Aso = O.Operator(small.ndim, small.nx, small.ny, small.nz, c=small.c)
    fs_h = O.apply(Aso, small.x_true())
    fs = torch.from_numpy(fs_h).to(dev)
    xo, ores = OT.solve_sgmres(3, args.oracle_n, 50.0, 8, args.m, 1e-12, 0,
                               threads=OT.host_cpu()["cores"])
    errs = {}
    for name, s, prec, basis in configs:
        xs = torch.zeros(small.N, dtype=torch.float64, device=dev)
        info = S.gmres_solve(As, fs, xs, s, args.m, tol, precision=prec, basis=basis)
        xsh = xs.cpu().numpy()
        errs[name] = {"x_err_vs_oracle": float(np.linalg.norm(xsh - xo) / np.linalg.norm(xo)),
                      "oracle_true_rel_resid": float(np.linalg.norm(fs_h - O.apply(Aso, xsh))
                                                     / np.linalg.norm(fs_h)),
                      "status": info.status}
        print(f"# {args.oracle_n}^3 {name}: |x - x_oracle|/|x_oracle| = "
              f"{errs[name]['x_err_vs_oracle']:.2e}", file=sys.stderr, flush=True)
    v = res["mixed_s8"]["s"]
    upd = res["mixed_s8"]["kernels"]["update"]["GBs"] or 0.0
    _line("mixed-precision s-step GMRES time to 1e-10 rel. resid, 7-pt 256^3", v, "s", False, v * 1e3,
          args, "f32+f64",
          f"3-D 7-pt convection-diffusion {args.n}^3 gamma=50, s-step GMRES(m={args.m}), FP32 basis, "
          f"FP64 Gram/LS/refinement, tol 1e-10 (s=8 headline; s=4, 12, FP64 s=8 and FP64 s=12 "
          f"with monomial / Chebyshev / Newton bases alongside)",
          {"results": res, "speedup_vs_fp64": res["fp64_s8"]["s"] / v,
           "speedup_vs_fp64_same_basis": res["fp64_s8_chebyshev"]["s"] / v,
           "vs_oracle": {"grid": f"{args.oracle_n}^3", "oracle": f"FP64 s-GMRES(m={args.m}, s=8) "
                         f"to 1e-12 ({ores['blocks']} blocks)", "results": errs},
           "roofline": {"bound": "hbm", "kernel": "update", "achieved": upd, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": upd / HBM_PEAK_GBS, "traffic": None}})


def bench_omin2d(args):
    """s-step Orthomin(k=8, s=8) on the 2-D 4096^2 problem, gamma = 50."""
    import torch
    from paper_2001_04886_amd import problems as PB
    from paper_2001_04886_amd import sstep as S
    dev = torch.device("cuda:0")
    n = 4096 if args.n == 256 else args.n
    prob = PB.square_2d_large(n, seed=0, gamma=50.0)
    A = S.Stencil.from_problem(prob)
    xt = torch.from_numpy(prob.x_true()).to(dev)
    f = torch.empty_like(xt)
    S.stencil_apply(A, xt, f)
    ws = S.allocate_workspace(A, S.METHOD_OMIN, 8, 8)
    x = torch.zeros_like(xt)
    infos = []
    for rep in range(args.warmup + args.steps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = S.omin_solve(A, f, x, 8, 8, 1e-8, max_iters=args.omin_iters, workspace=ws, profile=True)
        torch.cuda.synchronize()
        if rep >= args.warmup:
            infos.append((time.perf_counter() - t0, info))
        print(f"# omin rep {rep}: {time.perf_counter() - t0:.2f} s iters={info.iters} "
              f"rel_resid={info.rel_resid:.2e} status={info.status}", file=sys.stderr, flush=True)
    t = sum(a for a, _ in infos) / len(infos)
    info = infos[-1][1]
    cls = _classes(S, [i for _, i in infos], len(infos))
    dom = max(("gram", "update", "mpk"), key=lambda k: cls[k]["ms"])
    g = cls[dom]["GBs"] or 0.0
    per_it = t * 1e3 / max(info.iters, 1)
    _line("s-step Omin(k=8,s=8) time per s-step iteration, 5-pt 4096^2", per_it, "ms/iter", False,
          t * 1e3, args, "f64",
          f"2-D 5-pt convection-diffusion {n}^2 gamma=50, s-step Orthomin(k=8, s=8), FP64, "
          f"tol 1e-8 (cap {args.omin_iters} iterations), x0=0",
          {"iters": info.iters, "status": info.status, "rel_resid": info.rel_resid,
           "converged": info.status == S.OK, "time_to_tol_s": t if info.status == S.OK else None,
           "solve_s": t, "kernels": cls,
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": g, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": g / HBM_PEAK_GBS, "traffic": None}})


def bench_small2d(args):
    """64 x 64, gamma = 10: s-GMRES(m=20, s=4) and s-Omin(k=4, s=4) to 1e-8."""
    import torch
    from paper_2001_04886_amd import problems as PB
    from paper_2001_04886_amd import sstep as S
    dev = torch.device("cuda:0")
    prob = PB.small_2d(0)
    A = S.Stencil.from_problem(prob)
    xt = torch.from_numpy(prob.x_true()).to(dev)
    f = torch.empty_like(xt)
    S.stencil_apply(A, xt, f)
    out = {}
    for name, fn, km in [("gmres", S.gmres_solve, 20), ("omin", S.omin_solve, 4)]:
        ws = S.allocate_workspace(A, S.METHOD_GMRES if name == "gmres" else S.METHOD_OMIN, 4, km)
        x = torch.zeros_like(xt)
        ts = []
        for rep in range(args.warmup + max(args.steps, 5)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = fn(A, f, x, 4, km, 1e-8, workspace=ws)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                ts.append(time.perf_counter() - t0)
        out[name] = {"ms": 1e3 * sorted(ts)[len(ts) // 2], "iters": info.iters,
                     "rel_resid": info.rel_resid, "status": info.status}
    _line("s-step GMRES(20,4) time to 1e-8, 5-pt 64^2", out["gmres"]["ms"] / 1e3, "s", False,
          out["gmres"]["ms"], args, "f64", "2-D 5-pt convection-diffusion 64^2 gamma=10, "
          "s-GMRES(m=20, s=4) and s-Omin(k=4, s=4), FP64, tol 1e-8 (latency bound)", {"results": out})


def bench_paper2d(args):
    """The paper's own problem (Sec. 5, eq. (9), variable coefficients,
    beta = 1, gamma = 50, x0 = 0.05 mod(i, 50)) on n x n grids, n in {64, 128,
    192, 256}, stopped at the paper's rule ||r||_2 < 1e-6, with the four
    settings of its Table 6.1 (Orthomin(4), 2-Orthomin(2), GMRES(10),
    2-GMRES(5)), unpreconditioned and with the paper's ILU(0) right
    preconditioning (Sec. 5).  Iterations of the HIP path and of the oracle
    side by side (unless --no-cpu), the solve times, and the time of one
    preconditioner solve."""
    import numpy as np
    import torch
    from paper_2001_04886_amd import problems as PB
    from paper_2001_04886_amd import sstep as S
    dev = torch.device("cuda:0")
    settings = [("omin", 1, 4), ("omin", 2, 2), ("gmres", 1, 10), ("gmres", 2, 5)]
    rows, cpu, pc_us = [], None, {}
    for n in (64, 128, 192, 256):
        prob = PB.paper_problem(n)
        coef = torch.from_numpy(prob.coef).to(dev)
        A = S.Stencil.from_problem(prob, coef)
        g, x0 = PB.paper_rhs(n), PB.paper_x0(prob.N)
        tol = 1e-6 / float(np.linalg.norm(g))
        gd, x0d = torch.from_numpy(g).to(dev), torch.from_numpy(x0).to(dev)
        x = torch.empty_like(x0d)
        # one preconditioner solve (events around 50 back-to-back launches)
        d = S.ilu0_factor(A)
        z = torch.empty_like(gd)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        S.ilu0_solve(A, d, gd, z)
        e0.record()
        for _ in range(50):
            S.ilu0_solve(A, d, gd, z)
        e1.record()
        torch.cuda.synchronize()
        pc_us[n] = e0.elapsed_time(e1) * 1e3 / 50
        print(f"# paper n={n} ILU(0) solve {pc_us[n]:.1f} us", file=sys.stderr, flush=True)
        for pc in (S.PRECOND_NONE, S.PRECOND_ILU0):
            for method, s, km in settings:
                fn = S.gmres_solve if method == "gmres" else S.omin_solve
                mth = S.METHOD_GMRES if method == "gmres" else S.METHOD_OMIN
                ws = S.allocate_workspace(A, mth, s, km, precond=pc)
                ts = []
                for rep in range(args.warmup + max(args.steps, 3)):
                    x.copy_(x0d)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    # s-GMRES replays each restart cycle from a hipGraph
                    # (short cycles: the host's per-cycle launches dominate)
                    extra_kw = {"graph": True} if method == "gmres" else {}
                    info = fn(A, gd, x, s, km, tol, max_iters=20000, workspace=ws, precond=pc,
                              **extra_kw)
                    torch.cuda.synchronize()
                    if rep >= args.warmup:
                        ts.append(time.perf_counter() - t0)
                xh = x.cpu().numpy()
                row = {"n": n, "precond": "ilu0" if pc else "none", "method": method, "s": s,
                       "k_or_m": km, "iters": info.iters, "cycles": info.cycles,
                       "matvecs": info.matvecs, "status": info.status,
                       "resid_2norm": info.rel_resid * float(np.linalg.norm(g)),
                       "max_err_vs_analytic": float(np.max(np.abs(xh - PB.paper_exact(n)))),
                       "gpu_s": sorted(ts)[len(ts) // 2]}
                if not args.no_cpu:
                    import oracle as O
                    Ao = O.Operator(2, n, n, coef=prob.coef)
                    t0 = time.perf_counter()
                    if method == "gmres":
                        run = O.sgmres_ilu0 if pc else O.sgmres
                        _, res = run(Ao, g, x0, s, km, tol, max_blocks=20000)
                    else:
                        run = O.somin_ilu0 if pc else O.somin
                        _, res = run(Ao, g, x0, s, km, tol, max_iters=20000)
                    row["oracle_iters"], row["oracle_s"] = res.iters, time.perf_counter() - t0
                    if n == 256 and (method, s) == ("gmres", 2) and not pc:
                        cpu = {"value": row["oracle_s"], "unit": "s", "cores": 1,
                               "kind": "oracle",
                               "sample": "the whole 256^2 2-GMRES(5) solve, one host thread"}
                rows.append(row)
                print(f"# paper n={n} {row['precond']} {method} s={s} k/m={km}: iters "
                      f"{info.iters} cycles {info.cycles}"
                      + (f" (oracle {row['oracle_iters']})" if "oracle_iters" in row else "")
                      + f" gpu {row['gpu_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # larger s: s-step Orthomin(1) with and without the A^T A-orthogonal
    # blocks of Sec. 3 (orth = MGS), 256^2, unpreconditioned
    n = 256
    prob = PB.paper_problem(n)
    coef = torch.from_numpy(prob.coef).to(dev)
    A = S.Stencil.from_problem(prob, coef)
    g, x0 = PB.paper_rhs(n), PB.paper_x0(prob.N)
    tol = 1e-6 / float(np.linalg.norm(g))
    gd, x0d = torch.from_numpy(g).to(dev), torch.from_numpy(x0).to(dev)
    x = torch.empty_like(x0d)
    large_s = []
    for s in (4, 8, 12, 16):
        for orth in (S.ORTH_CHOL, S.ORTH_MGS):
            ts = []
            for rep in range(args.warmup + max(args.steps, 3)):
                x.copy_(x0d)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = S.omin_solve(A, gd, x, s, 1, tol, max_iters=20000, orth=orth)
                torch.cuda.synchronize()
                if rep >= args.warmup:
                    ts.append(time.perf_counter() - t0)
            row = {"n": n, "s": s, "k": 1, "orth": "mgs" if orth else "chol",
                   "iters": info.iters, "cycles": info.cycles, "status": info.status,
                   "gpu_s": sorted(ts)[len(ts) // 2]}
            large_s.append(row)
            print(f"# paper n={n} s-Omin s={s} k=1 {row['orth']}: iters {info.iters} restarts "
                  f"{info.cycles - 1} gpu {row['gpu_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    head = next(r for r in rows if r["n"] == 256 and r["method"] == "gmres" and r["s"] == 2
                and r["precond"] == "none")
    extra = {"results": rows, "ilu0_solve_us": pc_us, "omin_large_s": large_s}
    if cpu:
        extra["cpu_baseline"] = cpu
    _line("2-step GMRES(5) time to ||r|| < 1e-6, paper eq. (9) 256^2", head["gpu_s"], "s", False,
          head["gpu_s"] * 1e3, args, "f64",
          "paper eq. (9) 2-D variable-coefficient convection-diffusion, beta=1 gamma=50, "
          "n in {64,128,192,256}, Table 6.1 settings unpreconditioned (and ILU(0) alongside), "
          "x0 = 0.05 mod(i,50), s-GMRES restart cycles replayed from a hipGraph",
          extra)


def bench_batched(args):
    """512 independent 2-D 5-pt systems (side ~ U{32..512}, gamma ~ U(0,100)),
    s = 4, m = 30 blocks, FP64, tol 1e-8, one persistent launch replayed from
    a captured hipGraph, launch shape from the autotuner; compared with the
    same systems solved one after another by the single-system solver."""
    import torch
    from paper_2001_04886_amd import problems as PB
    from paper_2001_04886_amd import sstep as S
    from paper_2001_04886_amd import tune as TU
    dev = torch.device("cuda:0")
    table = PB.batched_table(args.nsys, master_seed=0)
    probs = [PB.convdiff(2, n, g, seed=sd) for n, g, sd in table]
    st = [S.Stencil.from_problem(p) for p in probs]
    xts = [torch.from_numpy(p.x_true()).to(dev) for p in probs]
    fs = []
    for a, xt in zip(st, xts):
        f = torch.empty_like(xt)
        S.stencil_apply(a, xt, f)
        fs.append(f)
    xs = [torch.zeros_like(xt) for xt in xts]
    s, m, tol = 4, 30, 1e-8
    shape = TU.lookup(st, s, m)
    if shape is None or args.retune:
        shape = TU.tune_batched(st, fs, xs, s, m, tol,
                                log=lambda msg: print(msg, file=sys.stderr, flush=True))
    threads, wpc, team, gcols = shape
    ws = torch.empty(S.batch_workspace_bytes(st, s, m, wpc, team), dtype=torch.uint8, device=dev)
    plan = S.BatchPlan(st, fs, xs, s, m, tol, threads=threads, wgs_per_cu=wpc, graph=True,
                       workspace=ws, team=team, gram_cols=gcols)
    times = []
    for rep in range(args.warmup + args.steps):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, infos = plan.execute()
        t = time.perf_counter() - t0
        if rep >= args.warmup:
            times.append(t)
        print(f"# batched rep {rep}: {t:.3f} s status={status}", file=sys.stderr, flush=True)
    plan.close()
    t = sum(times) / len(times)
    ok = all(i.status == 0 and i.rel_resid <= tol for i in infos)
    # algorithmic traffic of the batch from each system's block / cycle counts
    vp_bytes = sum(vec_passes_gmres(blocks_per_cycle(i.iters, i.cycles, m), s) * 8.0 * a.N
                   for i, a in zip(infos, st))
    gbs = vp_bytes / t / 1e9
    xerr = max(float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt)) for x, xt in zip(xs, xts))
    del ws
    torch.cuda.empty_cache()
    # plain comparator: the same systems one after another, single-system solver
    if args.no_plain:
        tseq = None
    else:
        tseq = _sequential(S, st, fs, xs, s, m, tol)
    _line("batched s-step GMRES time to 1e-8 for 512 uneven systems", t, "s", False, t * 1e3, args,
          "f64", f"{len(st)} independent 2-D 5-pt convection-diffusion systems, side ~ U{{32..512}}, "
          f"gamma ~ U(0,100), s-GMRES(m={m}, s={s}), FP64, tol 1e-8, one persistent launch from a "
          f"captured hipGraph, autotuned shape {threads} threads x {wpc} WG/CU, teams of {team} "
          f"workgroups on systems >= {team * 16384} points, Gram tile "
          f"{gcols or (4 if s <= 4 else 2)} columns per wave",
          {"converged_all": ok, "total_unknowns": int(sum(a.N for a in st)),
           "total_blocks": int(sum(i.iters for i in infos)), "max_x_err_vs_true": xerr,
           "algorithmic_GBs": gbs, "sequential_s": tseq,
           "speedup_vs_sequential": (tseq / t) if tseq else None,
           "shape": {"threads": threads, "wgs_per_cu": wpc, "team": team,
                     "gram_cols": gcols or (4 if s <= 4 else 2)},
           "team_systems": int(sum(1 for i in infos if i.matvecs > 1)),
           "roofline": {"bound": "hbm", "kernel": "k_batched_gmres", "achieved": gbs,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "traffic": None}})


def _sequential(S, st, fs, xs, s, m, tol):
    """The batch solved one system after another by the single-system solver."""
    import torch
    big = max(range(len(st)), key=lambda i: st[i].N)
    ws1 = S.allocate_workspace(st[big], S.METHOD_GMRES, s, m)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_blocks = 0
    for a, f, x in zip(st, fs, xs):
        info = S.gmres_solve(a, f, x, s, m, tol, workspace=ws1)
        seq_blocks += info.iters
    torch.cuda.synchronize()
    tseq = time.perf_counter() - t0
    print(f"# sequential single-system solves: {tseq:.2f} s", file=sys.stderr, flush=True)
    return tseq


def bench_learned(args):
    """Learned initial guess on 256^2 variable-coefficient diffusion: s-step
    GMRES(m=30, s=8) to 1e-8 from x0 = 0, from the trained network's guess
    with the fallback rule, and from the raw guess, on held-out seeded fields
    (the trained model is the committed one)."""
    import numpy as np
    import torch
    from paper_2001_04886_amd import learn as LN
    from paper_2001_04886_amd import sstep as S
    dev = torch.device("cuda:0")
    params, out_scale, meta = LN.load_model()
    log = lambda *a: print("#", *a, file=sys.stderr, flush=True)  # noqa: E731
    factor, sweeps = int(meta["coarsen"]), int(meta["sweeps"])
    if args.warmup:
        wds = LN.generate(1, 9000, nstreams=1, log=log)
        LN.evaluate(params, out_scale, wds, factor, sweeps, log=log)
    ds = LN.generate(args.eval_samples, 5000, nstreams=1, log=log)
    res = LN.evaluate(params, out_scale, ds, factor, sweeps, log=log)
    summ = {}
    for mode in LN.MODES:
        r = res[mode]
        summ[mode] = {"mean_s": float(r["seconds"].mean()), "mean_blocks": float(r["blocks"].mean()),
                      "median_blocks": float(np.median(r["blocks"])),
                      "converged_all": bool(np.all(r["status"] == S.OK))}
    fb = float(res["fallback"].mean())
    # what the network adds beyond the Jacobi sweeps its guess goes through
    summ["network_share"] = {
        "blocks_vs_zero": summ["cnn"]["mean_blocks"] / summ["zero"]["mean_blocks"],
        "blocks_vs_jacobi_only": summ["cnn"]["mean_blocks"] / summ["jacobi"]["mean_blocks"],
        "time_vs_zero": summ["cnn"]["mean_s"] / summ["zero"]["mean_s"],
        "time_vs_jacobi_only": summ["cnn"]["mean_s"] / summ["jacobi"]["mean_s"],
        "training_samples": int(meta.get("samples", 0)),
        "training_symmetries": 8 if meta.get("augment", True) else 1}
    # the network's own speed: forward (inference) at batch 32 and one
    # training step, timed with events on the stream the kernels run on
    B, n = 32, LN.GRID
    pdev = torch.as_tensor(params, device=dev)
    lk = ds.logk[:1].expand(B, n, n).contiguous()
    f = ds.f[:1].expand(B, n, n).contiguous()
    x = ds.x[:1].expand(B, n, n).contiguous()
    x0 = torch.empty_like(f)
    wsf = torch.empty(S.cnn_workspace_bytes(B, n, n, False), dtype=torch.uint8, device=dev)
    wst = torch.empty(S.cnn_workspace_bytes(B, n, n, True), dtype=torch.uint8, device=dev)
    g = torch.zeros_like(pdev)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    for _ in range(3):
        S.cnn_forward(pdev, out_scale, lk, f, x0=x0, workspace=wsf)
    e0.record(st)
    for _ in range(reps):
        S.cnn_forward(pdev, out_scale, lk, f, x0=x0, workspace=wsf)
    e1.record(st)
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    e0.record(st)
    for _ in range(reps):
        S.cnn_gradient(pdev, out_scale, lk, f, x, g, workspace=wst)
    e1.record(st)
    e1.synchronize()
    grad_ms = e0.elapsed_time(e1) / reps
    fwd_flop = 2.0 * n * n * 9 * (2 * 32 + 32 * 32 * 2 + 32)  # per sample, all four layers
    tf_fwd = fwd_flop * B / (fwd_ms * 1e-3) / 1e12
    tf_grad = 3.0 * fwd_flop * B / (grad_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        import oracle.cnn as OC
        t0 = time.perf_counter()
        OC.forward(params.astype(np.float64), ds.logk[:1].cpu().numpy(), ds.f[:1].cpu().numpy())
        tcf = time.perf_counter() - t0
        cpu = {"value": tcf, "unit": "s per 256^2 forward", "cores": 1, "kind": "oracle",
               "sample": "FP64 oracle network forward on one held-out 256^2 sample, 1 thread "
                         f"(GPU batch-32 forward: {fwd_ms / B:.4f} ms per sample)"}
    v = summ["cnn"]["mean_s"]
    _line("s-step GMRES(30,8) time to 1e-8 from the learned x0 (with fallback), 256^2 diffusion",
          v, "s", False, v * 1e3, args, "f64+bf16",
          f"2-D 5-pt -div(k grad u)=f, 256^2, log k and f squared-exponential GRFs (length 0.1), "
          f"{args.eval_samples} held-out seeds; s-GMRES(m=30, s=8) FP64 tol 1e-8; network 2-32-32-32-1 "
          f"dilated 3x3, bf16 storage / FP32 accumulation, on {factor}x{factor} block averages "
          f"(bilinear interpolation, {sweeps} Jacobi sweeps), trained on {meta.get('samples')} "
          f"solved systems x 8 grid symmetries",
          {"results": summ, "fallback_rate": fb,
           "blocks_ratio_nofallback": summ["cnn_nofallback"]["mean_blocks"] / summ["zero"]["mean_blocks"],
           "time_ratio_vs_zero": v / summ["zero"]["mean_s"],
           "model": {k: meta.get(k) for k in ("samples", "epochs", "batch", "lr", "steps",
                                                "coarsen", "sweeps")},
           "cnn": {"forward_ms_batch32": fwd_ms, "gradient_ms_batch32": grad_ms,
                   "forward_TFLOPs": tf_fwd, "gradient_TFLOPs": tf_grad},
           "roofline": {"bound": "mfma", "kernel": "network forward, batch 32 (all layers)",
                        "achieved": tf_fwd, "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": tf_fwd / 2500.0, "traffic": None},
           "cpu_baseline": cpu})


OTHER = {"mixed3d": bench_mixed3d, "omin2d": bench_omin2d, "small2d": bench_small2d,
         "paper2d": bench_paper2d,
         "batched": bench_batched, "learned": bench_learned}


if __name__ == "__main__":
    main()
