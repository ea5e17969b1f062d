"""Autotuner for the batched persistent solver's launch shape.

Candidate shapes (threads per workgroup x resident workgroups per compute
unit x workgroups per team on large systems x the block Gram's column tile,
i.e. stored-block columns per wave and pass) are timed on the actual batch --
two executions of the captured graph each, the faster kept -- and the fastest
is cached in a JSON table keyed by GPU architecture, batch signature (count,
total unknowns, largest system), s and m.  The table lives next to this
module (``tuned/batched.json``) unless a path is given.

A batch with no entry of its own takes the shape of the nearest tuned batch
of the same architecture, s and m: batches are compared by the share of their
unknowns in each power-of-two size class of the systems (what decides which
systems get teams and how the work spreads over the workgroups), plus the
log-ratios of their counts and total unknowns; beyond a distance of
``NEAREST_MAX`` there is no match and the library's defaults apply.
"""
from __future__ import annotations

import json
import os
import time

from . import sstep as S

# (threads, workgroups per CU, team, Gram column tile); tile NARROW is half the
# default one (2 instead of 4 columns per wave for s <= 4, 1 instead of 2 for
# s <= 8), 0 the default
NARROW = -1
CANDIDATES = ((256, 2, 1, 0), (512, 1, 1, 0), (512, 1, 2, 0), (512, 1, 2, NARROW), (512, 1, 4, 0),
              (512, 1, 4, NARROW), (1024, 1, 1, 0), (1024, 1, 2, 0), (1024, 1, 4, 0))


def gram_cols(s, tile):
    """The library's batch_gram_cols value of a candidate tile for this s."""
    if tile == NARROW:
        return 2 if s <= 4 else 1
    return int(tile)


DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "batched.json")


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


NEAREST_MAX = 0.5


def batch_key(stencils, s, m):
    sizes = [a.N for a in stencils]
    return f"{_arch()}|n{len(sizes)}|N{sum(sizes)}|max{max(sizes)}|s{s}|m{m}"


def size_histogram(sizes):
    """Share of the unknowns in each power-of-two size class (class k holds
    systems of 2^k .. 2^(k+1) - 1 points)."""
    tot = float(sum(sizes))
    h = {}
    for n in sizes:
        k = max(0, int(n).bit_length() - 1)
        h[k] = h.get(k, 0.0) + n / tot
    return {str(k): v for k, v in sorted(h.items())}


def signature(sizes, s, m, arch):
    return {"arch": arch, "s": s, "m": m, "n": len(sizes), "N": int(sum(sizes)),
            "hist": size_histogram(sizes)}


def distance(a, b):
    """Distance of two batch signatures (inf across architectures, s or m)."""
    import math
    if (a["arch"], a["s"], a["m"]) != (b["arch"], b["s"], b["m"]):
        return math.inf
    keys = set(a["hist"]) | set(b["hist"])
    l1 = sum(abs(a["hist"].get(k, 0.0) - b["hist"].get(k, 0.0)) for k in keys)
    return l1 + abs(math.log(a["n"] / b["n"])) + abs(math.log(a["N"] / b["N"]))


def nearest(sig, cache):
    """(distance, record) of the tuned entry nearest to ``sig``."""
    best = (float("inf"), None)
    for rec in cache.values():
        if "sig" in rec and "team" in rec:
            d = distance(sig, rec["sig"])
            if d < best[0]:
                best = (d, rec)
    return best


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(stencils, s, m, path=DEFAULT_CACHE):
    """Launch shape (threads, workgroups per CU, team, Gram column tile; tile 0
    = the library default) tuned for this batch, else that of the nearest
    tuned batch (within NEAREST_MAX), else None."""
    cache = load_cache(path)
    rec = cache.get(batch_key(stencils, s, m))
    if not rec or "team" not in rec:
        d, rec = nearest(signature([a.N for a in stencils], s, m, _arch()), cache)
        if rec is None or d > NEAREST_MAX:
            return None
    return rec["threads"], rec["wgs_per_cu"], rec["team"], rec.get("gram_cols", 0)


def tune_batched(stencils, fs, xs, s, m, tol, candidates=CANDIDATES, path=DEFAULT_CACHE,
                 max_iters=0, log=None):
    """Time every candidate shape on this batch; returns (threads, wgs_per_cu,
    team, gram_cols) of the fastest and records all timings in the cache."""
    import torch
    nb = max(S.batch_workspace_bytes(stencils, s, m, c[1], c[2]) for c in candidates)
    ws = torch.empty(nb, dtype=torch.uint8, device=xs[0].device)
    times = {}
    for threads, wpc, team, tile in candidates:
        gc = gram_cols(s, tile)
        plan = S.BatchPlan(stencils, fs, xs, s, m, tol, threads=threads, wgs_per_cu=wpc,
                           graph=True, max_iters=max_iters, workspace=ws, team=team,
                           gram_cols=gc)
        best = None
        for _ in range(2):
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.execute()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        plan.close()
        times[f"{threads}x{wpc}x{team}x{gc}"] = best
        if log:
            log(f"# tune batched: threads={threads} wgs/CU={wpc} team={team} gram cols={gc or 'default'}: "
                f"{best * 1e3:.1f} ms")
    key = min(times, key=times.get)
    threads, wpc, team, gc = (int(v) for v in key.split("x"))
    cache = load_cache(path)
    cache[batch_key(stencils, s, m)] = {"threads": threads, "wgs_per_cu": wpc, "team": team,
                                        "gram_cols": gc,
                                        "ms": {k: v * 1e3 for k, v in times.items()},
                                        "sig": signature([a.N for a in stencils], s, m, _arch())}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    del ws
    return threads, wpc, team, gc
