"""Wall time of the FP64 oracle's s-step GMRES on the host cores (the CPU
baseline of the benchmark; test infrastructure like the rest of oracle/).

Each measurement runs in a child process so that the OpenMP timing build
(``build_omp``) and its thread count stay out of the caller: the child
builds the problem, then times only the solver call."""
from __future__ import annotations

import json
import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)

_CHILD = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as O
from paper_2001_04886_amd import problems as PB
ndim, n, gamma, s, m, blocks, basis = json.loads(sys.argv[2])
prob = PB.convdiff(ndim, n, gamma)
A = O.Operator(prob.ndim, prob.nx, prob.ny, prob.nz, c=prob.c)
f = O.apply(A, prob.x_true())
t0 = time.perf_counter()
x, res = O.sgmres(A, f, np.zeros(prob.N), s, m, 0.0, max_blocks=blocks, basis=basis)
t1 = time.perf_counter()
print(json.dumps({"seconds": t1 - t0, "blocks": res.iters, "cycles": res.cycles,
                  "rel_resid": res.rel_resid}))
"""


def host_cpu() -> dict:
    """Cores this process may run on and the CPU model name."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cores": cores, "model": model}


def time_sgmres(ndim, n, gamma, s, m, blocks, basis=0, threads=1, timeout=900):
    """Seconds the oracle takes for `blocks` s-blocks of s-GMRES(m, s) on the
    convection-diffusion problem (f = A x_true, x0 = 0), on `threads` cores
    (1: the plain build; more: the OpenMP timing build)."""
    import oracle as O
    if threads > 1:
        if not os.path.exists(O.LIB_OMP) or (os.path.getmtime(O.LIB_OMP)
                                             < os.path.getmtime(O._SRC)):
            O.build_omp()
        lib = O.LIB_OMP
    else:
        if not os.path.exists(O._LIB) or os.path.getmtime(O._LIB) < os.path.getmtime(O._SRC):
            O.build()
        lib = O._LIB
    env = dict(os.environ, SSTEP_ORACLE_LIB=lib, OMP_NUM_THREADS=str(threads),
               OMP_PROC_BIND="close")
    r = subprocess.run([sys.executable, "-c", _CHILD, _ROOT,
                        json.dumps([ndim, n, gamma, s, m, blocks, basis])],
                       env=env, capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0:
        raise RuntimeError("oracle timing child failed:\n" + r.stderr[-2000:])
    out = json.loads(r.stdout.strip().splitlines()[-1])
    out["threads"] = threads
    return out


_SOLVE_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as O
from paper_2001_04886_amd import problems as PB
ndim, n, gamma, s, m, tol, basis, out = json.loads(sys.argv[2])
prob = PB.convdiff(ndim, n, gamma)
A = O.Operator(prob.ndim, prob.nx, prob.ny, prob.nz, c=prob.c)
f = O.apply(A, prob.x_true())
x, res = O.sgmres(A, f, np.zeros(prob.N), s, m, tol, basis=basis)
np.save(out, x)
print(json.dumps({"status": res.status, "blocks": res.iters, "cycles": res.cycles,
                  "rel_resid": res.rel_resid}))
"""


def solve_sgmres(ndim, n, gamma, s, m, tol, basis=0, threads=1, timeout=1200):
    """The oracle's s-GMRES(m, s) solution of the convection-diffusion
    problem (f = A x_true, x0 = 0) to the relative tolerance tol, computed in
    a child process on `threads` cores; returns (x, result dict)."""
    import tempfile

    import numpy as np

    import oracle as O
    if threads > 1:
        if not os.path.exists(O.LIB_OMP) or (os.path.getmtime(O.LIB_OMP)
                                             < os.path.getmtime(O._SRC)):
            O.build_omp()
        lib = O.LIB_OMP
    else:
        lib = O._LIB
    env = dict(os.environ, SSTEP_ORACLE_LIB=lib, OMP_NUM_THREADS=str(threads),
               OMP_PROC_BIND="close")
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "x.npy")
        r = subprocess.run([sys.executable, "-c", _SOLVE_CHILD, _ROOT,
                            json.dumps([ndim, n, gamma, s, m, tol, basis, out])],
                           env=env, capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            raise RuntimeError("oracle solve child failed:\n" + r.stderr[-2000:])
        return np.load(out), json.loads(r.stdout.strip().splitlines()[-1])
