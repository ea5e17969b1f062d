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
    dom = max(("gram", "update", "mpk"), key=lambda k: classes[k]["ms"])
    dom_gbs = classes[dom]["GBs"] or 0.0
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
        "kernels": classes,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dom_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS, "traffic": None},
    }

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
        import oracle as O  # CPU baseline leg only
        del ws
        torch.cuda.empty_cache()
        Ao = O.Operator(prob.ndim, prob.nx, prob.ny, prob.nz, c=prob.c)
        fh = f.cpu().numpy()
        x0 = np.zeros(N)
        tc0 = time.perf_counter()
        xo, res = O.sgmres(Ao, fh, x0, args.s, args.m, 0.0, max_blocks=args.cpu_blocks,
                           basis=0 if basis == S.MONOMIAL else 1)
        tc1 = time.perf_counter()
        sample_vp = vec_passes_gmres([args.cpu_blocks], args.s)
        full_vp = vec_passes_gmres(blocks_per_cycle(last.iters, last.cycles, args.m), args.s)
        per_vp = (tc1 - tc0) / sample_vp
        out["cpu_baseline"] = {
            "value": per_vp * full_vp, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle s-GMRES(m={args.m}, s={args.s}) on the same {args.n}^3 problem, "
                      f"first {args.cpu_blocks} blocks in {tc1 - tc0:.1f} s on 1 thread, scaled by "
                      f"algorithmic vector passes ({sample_vp} -> {full_vp}) of the GPU solve",
            "measured_s": tc1 - tc0,
        }
        print(f"# cpu oracle sample: {tc1 - tc0:.1f} s for {args.cpu_blocks} blocks", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
