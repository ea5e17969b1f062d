"""Learned initial guess: training-data generation, training and evaluation.

Alg 4.2 (restarted s-step GMRES) starts from an arbitrary x0.  This module
trains the network of ``sstep_cnn_*`` (include/sstep.h) to propose x0 for the
variable-coefficient diffusion family -div(k grad u) = f on a 256 x 256 grid,
with log k and f squared-exponential Gaussian random fields (correlation
length 0.1, unit variance), and measures what the guess buys the solver.

The network sees 31 points in each direction, far less than the domain of a
global elliptic problem, so it runs on a coarse grid: inputs and targets are
block averages over COARSEN x COARSEN cells (32 x 32 coarse points for the
256 x 256 grid, where 31 points span the domain), and the guess is carried
back by bilinear interpolation and SWEEPS damped Jacobi sweeps
(sstep_x0_predict_coarse).

Everything numeric runs in the HIP library: the solves that produce the
training targets (sstep_gmres_solve), the block averages (sstep_grid_pool),
the network's forward/backward/Adam (sstep_cnn_train_step) and the guess with
its fallback test (sstep_x0_predict_coarse).  This module only generates
seeded inputs (through problems.py), moves batches, and keeps the books.

Command line (on a GPU):
    python -m paper_2001_04886_amd.learn --samples 2560 --epochs 300 --out model.npz
"""
from __future__ import annotations

import argparse
import json
import os
import threading
import time

import numpy as np

from . import problems as P
from . import sstep as S

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(_HERE, "tuned", "x0_cnn.npz")
GRID = 256
CORR_LENGTH = 0.1
COARSEN = 8
SOLVE_S, SOLVE_M, SOLVE_TOL = 8, 30, 1e-8


def _log(*a):
    print(*a, flush=True)


class Dataset:
    """Samples on the device: logk float32 [S][n][n], f and x float64."""

    def __init__(self, logk, f, x, blocks, seconds, seed):
        self.logk, self.f, self.x = logk, f, x
        self.blocks, self.seconds, self.seed = blocks, seconds, seed

    def __len__(self):
        return self.logk.shape[0]


def sample_inputs(count, seed, n=GRID, device="cuda:0"):
    """log k (float32) and f (float64) fields for ``count`` samples; the two
    fields of a sample come from independent generator streams."""
    import torch
    logk = P.grf_batch_torch(n, CORR_LENGTH, 2 * seed, count, device=device).to(torch.float32)
    f = P.grf_batch_torch(n, CORR_LENGTH, 2 * seed + 1, count, device=device)
    return logk.contiguous(), f.contiguous()


def stencil_for(logk_sample):
    """Stencil descriptor + its [7][N] coefficient tensor (kept alive by the
    caller) for one log k field."""
    coef = P.diffusion_coef_torch(logk_sample).contiguous()
    n = logk_sample.shape[0]
    return S.Stencil(2, n, n, 1, (0.0,) * 7, coef), coef


def solve_all(logk, f, x, s=SOLVE_S, m=SOLVE_M, tol=SOLVE_TOL, nstreams=4, x0_fn=None,
              log=_log, graph=False):
    """Solve every sample with s-step GMRES(m) on ``nstreams`` concurrent
    streams (one host thread each; the library waits on its own stream).
    x holds the initial guesses on entry (or x0_fn(i, A, stream) fills them)
    and the solutions on return.  Returns per-sample (blocks, status, seconds)."""
    import torch
    count = logk.shape[0]
    n = logk.shape[1]
    blocks = np.zeros(count, dtype=np.int64)
    status = np.zeros(count, dtype=np.int64)
    secs = np.zeros(count)
    done = [0]
    lock = threading.Lock()
    errors = []
    A0, _ = stencil_for(logk[0])
    ws_bytes = S.workspace_bytes(A0, S.METHOD_GMRES, s, m)

    def worker(t):
        try:
            st = torch.cuda.Stream(device=logk.device)
            ws = torch.empty(ws_bytes, dtype=torch.uint8, device=logk.device)
            with torch.cuda.stream(st):
                for i in range(t, count, nstreams):
                    A, coef = stencil_for(logk[i])
                    t0 = time.perf_counter()
                    if x0_fn is not None:
                        x0_fn(i, A, st)
                    info = S.gmres_solve(A, f[i].reshape(-1), x[i].reshape(-1), s, m, tol,
                                         workspace=ws, stream=st, graph=graph)
                    secs[i] = time.perf_counter() - t0
                    blocks[i], status[i] = info.iters, info.status
                    del coef
                    with lock:
                        done[0] += 1
                        if done[0] % 64 == 0 or done[0] == count:
                            log(f"  solved {done[0]}/{count}")
        except Exception as e:  # surfaced after join
            errors.append(e)

    torch.cuda.synchronize()
    threads = [threading.Thread(target=worker, args=(t,)) for t in range(nstreams)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    if errors:
        raise errors[0]
    return blocks, status, secs


def generate(count, seed, n=GRID, nstreams=4, device="cuda:0", log=_log, graph=False):
    """Training/evaluation samples: seeded fields and their s-step GMRES
    solutions to the solver tolerance from x0 = 0 (graph: restart cycles
    replayed from a hipGraph, one launch per cycle instead of ~500)."""
    import torch
    t0 = time.perf_counter()
    logk, f = sample_inputs(count, seed, n, device)
    x = torch.zeros_like(f)
    log(f"generating {count} samples (seed {seed}) on {nstreams} streams")
    blocks, status, secs = solve_all(logk, f, x, nstreams=nstreams, log=log, graph=graph)
    bad = int(np.sum(status != S.OK))
    log(f"generated {count} samples in {time.perf_counter() - t0:.1f} s; "
        f"mean blocks {blocks.mean():.0f}; not converged {bad}")
    return Dataset(logk, f, x, blocks, secs, seed)


def generate_batched(count, seed, n=GRID, chunk=512, device="cuda:0", log=_log, threads=0,
                     wgs_per_cu=0, team=0):
    """generate() through the batched persistent solver: chunks of ``chunk``
    systems solved together in one launch per chunk (sstep_batch_plan_*),
    each to the solver tolerance from x0 = 0.  The per-sample seconds are the
    chunk's wall time divided evenly."""
    import torch
    t0 = time.perf_counter()
    logk, f = sample_inputs(count, seed, n, device)
    x = torch.zeros_like(f)
    blocks = np.zeros(count, dtype=np.int64)
    status = np.zeros(count, dtype=np.int64)
    secs = np.zeros(count)
    log(f"generating {count} samples (seed {seed}) in batches of {chunk}")
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        stc = [stencil_for(logk[i]) for i in range(c0, c1)]
        tc = time.perf_counter()
        plan = S.BatchPlan([a for a, _ in stc], [f[i].reshape(-1) for i in range(c0, c1)],
                           [x[i].reshape(-1) for i in range(c0, c1)], SOLVE_S, SOLVE_M, SOLVE_TOL,
                           graph=False, threads=threads, wgs_per_cu=wgs_per_cu, team=team)
        try:
            _, infos = plan.execute()
        finally:
            plan.close()
        torch.cuda.synchronize()
        dt = time.perf_counter() - tc
        for j, info in enumerate(infos):
            blocks[c0 + j], status[c0 + j] = info.iters, info.status
        secs[c0:c1] = dt / (c1 - c0)
        del stc
        log(f"  solved {c1}/{count} ({dt:.1f} s for {c1 - c0})")
    bad = int(np.sum(status != S.OK))
    log(f"generated {count} samples in {time.perf_counter() - t0:.1f} s; "
        f"mean blocks {blocks.mean():.0f}; not converged {bad}")
    return Dataset(logk, f, x, blocks, secs, seed)


def coarsen(ds, factor):
    """The block-averaged dataset the network trains on (log k kept float32)."""
    import torch
    if factor == 1:
        return ds
    lk = S.grid_pool(ds.logk.double().contiguous(), factor).float().contiguous()
    return Dataset(lk, S.grid_pool(ds.f, factor), S.grid_pool(ds.x, factor), ds.blocks,
                   ds.seconds, ds.seed)


def save_shard(path, ds, factor):
    """Write the block-averaged samples of ``ds`` (the network's training data)
    as float32 arrays, with the fine solves' block counts and seconds."""
    c = coarsen(ds, factor)
    np.savez(path, logk=c.logk.float().cpu().numpy(), f=c.f.float().cpu().numpy(),
             x=c.x.float().cpu().numpy(), blocks=ds.blocks, seconds=ds.seconds,
             meta=np.array(json.dumps({"seed": ds.seed, "factor": factor, "grid": int(ds.logk.shape[1])})))


MAX_BLOCKS = 10000  # the solver's default block cap: a sample that reached it did not converge


def load_shards(paths, device="cuda:0"):
    """Concatenate shards written by save_shard into one (block-averaged)
    Dataset on the device, leaving out samples whose solve reached the block
    cap without converging."""
    import torch
    parts = []
    for p in paths:
        with np.load(p, allow_pickle=False) as z:
            parts.append({k: z[k] for k in ("logk", "f", "x", "blocks", "seconds")})
    cat = {k: np.concatenate([q[k] for q in parts]) for k in parts[0]}
    keep = cat["blocks"] < MAX_BLOCKS
    cat = {k: v[keep] for k, v in cat.items()}
    return Dataset(torch.tensor(cat["logk"], dtype=torch.float32, device=device).contiguous(),
                   torch.tensor(cat["f"], dtype=torch.float64, device=device).contiguous(),
                   torch.tensor(cat["x"], dtype=torch.float64, device=device).contiguous(),
                   cat["blocks"], cat["seconds"], None)


def out_scale_of(ds, nsamp=64):
    """rms over samples of x / rms(f): the output scale that makes the
    regression target O(1) (a model constant)."""
    k = min(nsamp, len(ds))
    x = ds.x[:k].double().cpu().numpy().reshape(k, -1)
    f = ds.f[:k].double().cpu().numpy().reshape(k, -1)
    fr = np.sqrt(np.mean(f * f, axis=1))
    return float(np.sqrt(np.mean((x / fr[:, None]) ** 2)))


def init_params(seed=0):
    """He-normal weights, zero biases, in the flat layout of sstep_cnn_*."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in ((32, 2), (32, 32), (32, 32), (1, 32)):
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == S.cnn_param_count()
    return p


def symmetry(t, g):
    """Element g (0..7) of the symmetry group of the square grid applied to a
    batch [B][n][n]: g % 4 quarter turns, then a transpose when g >= 4.  The
    harmonic-mean diffusion stencil is equivariant under all eight, so a
    solved (k, f, x) maps to another solved sample; so does (k, -f, -x)."""
    import torch
    t = torch.rot90(t, g % 4, dims=(1, 2))
    if g >= 4:
        t = t.transpose(1, 2)
    return t.contiguous()


def train(ds, epochs, batch=32, lr=1e-3, seed=0, val=None, augment=True, log=_log):
    """Adam on the mean-squared error against x / (rms(f) out_scale); each
    batch is drawn under a random grid symmetry and sign (augment=True)."""
    import torch
    dev = ds.logk.device
    n = ds.logk.shape[1]
    out_scale = out_scale_of(ds)
    params = torch.tensor(init_params(seed), device=dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = torch.empty(S.cnn_workspace_bytes(batch, n, n, True), dtype=torch.uint8, device=dev)
    grad = torch.zeros_like(params)
    rng = np.random.default_rng(seed + 1)
    step = 0
    hist = []
    t0 = time.perf_counter()
    nb = len(ds) // batch
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(len(ds))[: nb * batch], device=dev)
        losses = []
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            step += 1
            g = int(rng.integers(8)) if augment else 0
            sign = float(rng.choice((-1.0, 1.0))) if augment else 1.0
            lk, f, x = (symmetry(t[idx], g) for t in (ds.logk, ds.f, ds.x))
            losses.append(S.cnn_train_step(params, m, v, step, lr, out_scale, lk, f * sign,
                                           x * sign, workspace=ws))
        rec = {"epoch": ep + 1, "train_loss": float(np.mean(losses))}
        if val is not None:
            vl = []
            for b in range(0, len(val) - batch + 1, batch):
                vl.append(S.cnn_gradient(params, out_scale, val.logk[b:b + batch].contiguous(),
                                         val.f[b:b + batch].contiguous(),
                                         val.x[b:b + batch].contiguous(), grad, workspace=ws))
            rec["val_loss"] = float(np.mean(vl)) if vl else None
        hist.append(rec)
        log(f"  epoch {ep + 1}/{epochs}: " + ", ".join(
            f"{k} {v_:.4e}" for k, v_ in rec.items() if k != "epoch" and v_ is not None)
            + f"  ({time.perf_counter() - t0:.1f} s)")
    train_s = time.perf_counter() - t0
    return params.cpu().numpy(), out_scale, hist, train_s, step


def save_model(path, params, out_scale, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(params, dtype=np.float32),
             out_scale=np.float64(out_scale), meta=np.array(json.dumps(meta)))


def load_model(path=DEFAULT_MODEL):
    """params, out_scale, meta; meta["coarsen"] / meta["sweeps"] (1 / 0 when
    absent) say how the guess is formed."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        meta.setdefault("coarsen", 1)
        meta.setdefault("sweeps", 0)
        return z["params"].astype(np.float32), float(z["out_scale"]), meta


MODES = ("zero", "jacobi", "cnn", "cnn_nofallback")


def evaluate(params, out_scale, ds, factor=1, sweeps=0, nstreams=1, log=_log, modes=None,
             graph=False):
    """Solve every sample of ``ds`` from x0 = 0 ("zero"); from x0 = 0
    followed by the same ``sweeps`` damped Jacobi sweeps and fallback rule as
    the guess ("jacobi": the guess path with an all-zero network, whose output
    is 0 -- the ablation that isolates what the network itself adds); from the
    network's guess (block averages over ``factor`` cells, ``sweeps`` Jacobi
    sweeps) with the fallback rule ("cnn"); and from the raw guess
    ("cnn_nofallback").  Returns per-sample blocks and wall seconds (guess
    included) for each, and the fallback flags of "cnn" and "jacobi"."""
    import torch
    dev = ds.logk.device
    n = ds.logk.shape[1]
    pdev = torch.as_tensor(params, device=dev)
    pzero = torch.zeros_like(pdev)
    count = len(ds)
    ws = [torch.empty(S.x0_coarse_workspace_bytes(n, n, factor), dtype=torch.uint8, device=dev)
          for _ in range(nstreams)]
    fallback = np.zeros(count, dtype=bool)
    fallback_j = np.zeros(count, dtype=bool)
    res = {}
    for mode in modes or MODES:
        x = torch.zeros_like(ds.f)

        def x0_fn(i, A, st, mode=mode):
            if mode == "zero":
                return
            used = S.x0_predict_coarse(pzero if mode == "jacobi" else pdev, out_scale, factor,
                                       sweeps, A, ds.logk[i].reshape(-1), ds.f[i].reshape(-1),
                                       x[i].reshape(-1), use_fallback=(mode != "cnn_nofallback"),
                                       workspace=ws[i % nstreams], stream=st)
            if mode == "cnn":
                fallback[i] = used
            elif mode == "jacobi":
                fallback_j[i] = used

        blocks, status, secs = solve_all(ds.logk, ds.f, x, nstreams=nstreams, x0_fn=x0_fn,
                                         log=lambda *a: None, graph=graph)
        res[mode] = {"blocks": blocks, "status": status, "seconds": secs}
        log(f"  eval {mode} (factor {factor}, sweeps {sweeps}): mean blocks {blocks.mean():.1f}, "
            f"mean time {secs.mean() * 1e3:.1f} ms, not converged {int(np.sum(status != S.OK))}")
    res["fallback"] = fallback
    res["fallback_jacobi"] = fallback_j
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gen-shard", default=None,
                    help="only generate --samples solved samples (seed --seed) and write their "
                         "block averages to this .npz")
    ap.add_argument("--shards", nargs="+", default=None,
                    help="train on these shards (from --gen-shard) instead of generating")
    ap.add_argument("--graph", action="store_true",
                    help="replay restart cycles from a hipGraph in the data solves")
    ap.add_argument("--samples", type=int, default=2560)
    ap.add_argument("--val", type=int, default=128)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--coarsen", type=int, default=COARSEN)
    ap.add_argument("--sweeps", type=int, nargs="+", default=[0, 32, 128, 512],
                    help="Jacobi sweep counts to evaluate; the fastest (with the fallback rule) "
                         "is stored with the model")
    ap.add_argument("--out", default=DEFAULT_MODEL)
    args = ap.parse_args(argv)
    import torch
    S.load()
    dev = "cuda:0"
    torch.cuda.init()
    if args.gen_shard:
        ds = generate(args.samples, args.seed, nstreams=args.streams, device=dev, graph=args.graph)
        save_shard(args.gen_shard, ds, args.coarsen)
        _log(f"wrote {args.gen_shard}: {len(ds)} samples, mean blocks {ds.blocks.mean():.0f}, "
             f"{ds.seconds.sum():.0f} solver-seconds")
        return
    if args.shards:
        train_c = load_shards(args.shards, dev)
        args.samples = len(train_c)
        data_mean_blocks = float(train_c.blocks.mean())
        data_seconds = float(train_c.seconds.sum())
    else:
        train_ds = generate(args.samples, args.seed, nstreams=args.streams, device=dev,
                            graph=args.graph)
        data_mean_blocks = float(train_ds.blocks.mean())
        data_seconds = float(train_ds.seconds.sum())
        train_c = coarsen(train_ds, args.coarsen)
        del train_ds
    val_ds = generate(args.val, args.seed + 1, nstreams=args.streams, device=dev, graph=args.graph)
    val_c = coarsen(val_ds, args.coarsen)
    params, out_scale, hist, train_s, steps = train(train_c, args.epochs, args.batch, args.lr,
                                                    val=val_c)
    del train_c
    ev_ds = generate(args.eval, args.seed + 2, nstreams=args.streams, device=dev, graph=args.graph)
    evals = {}
    zero = None
    for sw in args.sweeps:
        res = evaluate(params, out_scale, ev_ds, args.coarsen, sw,
                       modes=("jacobi", "cnn", "cnn_nofallback") if zero else None)
        if zero is None:
            zero = res["zero"]
        evals[sw] = {m: {"mean_blocks": float(res[m]["blocks"].mean()),
                         "mean_ms": float(res[m]["seconds"].mean() * 1e3)}
                     for m in ("jacobi", "cnn", "cnn_nofallback")}
        evals[sw]["fallback_rate"] = float(res["fallback"].mean())
    best = min(args.sweeps, key=lambda sw: evals[sw]["cnn"]["mean_ms"])
    summary = {"zero": {"mean_blocks": float(zero["blocks"].mean()),
                        "mean_ms": float(zero["seconds"].mean() * 1e3)},
               "by_sweeps": {str(k): v for k, v in evals.items()}, "chosen_sweeps": best}
    meta = {"grid": GRID, "coarsen": args.coarsen, "sweeps": best, "samples": args.samples,
            "val": args.val, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "seed": args.seed, "steps": steps, "train_seconds": train_s, "history": hist,
            "data_mean_blocks": data_mean_blocks, "data_seconds": data_seconds,
            "data": ("shards " + " ".join(os.path.basename(p) for p in args.shards)
                     if args.shards else f"generated, seed {args.seed}"),
            "eval": summary}
    save_model(args.out, params, out_scale, meta)
    _log(f"saved {args.out} (out_scale {out_scale:.4e}, sweeps {best})")
    _log("EVAL " + json.dumps(summary))


if __name__ == "__main__":
    main()
