"""Rounding spread of the FP64 oracle behind every loosened GPU iterate bound.

For each fixed-work case of ``parity_bounds.CASES`` the oracle runs three
times: as built, with every matrix-vector product perturbed by one ulp in a
seeded direction, and with every inner product summed in reverse order.  The
two changes alter nothing but rounding, so the largest relative distance of
their iterates from the unchanged one is a lower estimate of how far two
correct FP64 implementations (such as the GPU path, which sums in blocks and
contracts multiply-adds) can drift apart on that case.  Each bound must leave
at least a 3x margin above that spread, and may exceed it at most 30x unless
it is the 1e-8 contract itself.  CPU only; the planted changes live in
temporary copies of the oracle source."""
import json
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import parity_bounds as PBND

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sstep_oracle.c")

# one ulp towards +inf or -inf, chosen by a SplitMix64-style hash of (point,
# matvec counter), on every output of the stencil operator
PERTURB = [
    ("#include <string.h>\n", "#include <string.h>\nstatic unsigned long long orc_pert_ctr;\n"),
    ("y[p] = acc + c[0] * x[p];",
     "{ double v_ = acc + c[0] * x[p];"
     " unsigned long long h_ = (unsigned long long)p + 0x9E3779B97F4A7C15ull * ++orc_pert_ctr;"
     " h_ ^= h_ >> 30; h_ *= 0xBF58476D1CE4E5B9ull; h_ ^= h_ >> 27; h_ *= 0x94D049BB133111EBull;"
     " h_ ^= h_ >> 31; y[p] = (h_ >> 63) ? nextafter(v_, INFINITY) : nextafter(v_, -INFINITY); }"),
]
REVERSE = [("for (long long p = 0; p < n; ++p) s += a[p] * b[p];",
            "for (long long p = n - 1; p >= 0; --p) s += a[p] * b[p];")]

RUNNER = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import oracle as O
import parity_bounds as PBND
from paper_2001_04886_amd import problems as PB
case = [c for c in PBND.CASES if c[0] == sys.argv[2]][0]
_, ndim, n, gamma, method, s, km, nb, basis, rhs, bound = case
prob = PB.convdiff(ndim, n, gamma)
A = O.Operator(prob.ndim, prob.nx, prob.ny, prob.nz, c=prob.c)
f = PBND.rhs(rhs, prob, lambda v: O.apply(A, v))
x, res = O.sgmres(A, f, np.zeros(prob.N), s, km, 0.0, max_blocks=nb, basis=basis)
np.save(sys.argv[3], x)
print(json.dumps({"blocks": res.iters, "cycles": res.cycles}))
"""


def _variant(tmp, name, subs):
    src = open(SRC).read()
    for a, b in subs:
        assert a in src, a
        src = src.replace(a, b, 1)
    c = os.path.join(tmp, name + ".c")
    with open(c, "w") as fh:
        fh.write(src)
    lib = os.path.join(tmp, name + ".so")
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-I", os.path.join(ROOT, "oracle"), "-o", lib, c, "-lm"],
                   check=True)
    return lib


@pytest.fixture(scope="module")
def spreads():
    with tempfile.TemporaryDirectory() as tmp:
        libs = {"base": _variant(tmp, "base", []), "perturb": _variant(tmp, "perturb", PERTURB),
                "reverse": _variant(tmp, "reverse", REVERSE)}
        runner = os.path.join(tmp, "run.py")
        with open(runner, "w") as fh:
            fh.write(RUNNER)

        def one(job):
            cid, var = job
            out = os.path.join(tmp, f"{cid}-{var}.npy")
            env = dict(os.environ, SSTEP_ORACLE_LIB=libs[var])
            r = subprocess.run([sys.executable, runner, ROOT, cid, out], env=env,
                               capture_output=True, text=True, timeout=600)
            assert r.returncode == 0, r.stderr[-2000:]
            return job, np.load(out), json.loads(r.stdout.strip().splitlines()[-1])

        jobs = [(c[0], v) for c in PBND.CASES for v in libs]
        with ThreadPoolExecutor(max_workers=6) as ex:
            done = {job: (x, meta) for job, x, meta in ex.map(one, jobs)}
    out = {}
    for c in PBND.CASES:
        xb, mb = done[(c[0], "base")]
        assert mb["blocks"] == c[7]
        out[c[0]] = {v: float(np.linalg.norm(done[(c[0], v)][0] - xb) / np.linalg.norm(xb))
                     for v in ("perturb", "reverse")}
    print("rounding spread per case:", json.dumps(out, indent=1))
    return out


@pytest.mark.parametrize("case", PBND.CASES, ids=[c[0] for c in PBND.CASES])
def test_bound_follows_rounding_spread(spreads, case):
    spread = max(spreads[case[0]].values())
    bound = case[-1]
    assert 3.0 * spread <= bound, (case[0], spread, bound)
    assert bound <= max(PBND.CONTRACT, 30.0 * spread), (case[0], spread, bound)


def test_planted_changes_alter_rounding(spreads):
    # both changes must actually move the iterate of an ill-conditioned case
    s = spreads["3d128-mono-s8m40-b4"]
    assert s["perturb"] > 1e-9 and s["reverse"] > 1e-9, s
