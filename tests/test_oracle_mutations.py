"""The oracle's pins are not vacuous: a copy of the oracle with one plausible
mistake planted in it (a sign, a dropped term, a wrong index, a transposed
operand) is compiled on the CPU and the pin file that covers that part of the
method must fail on it, while the unmodified source compiled the same way
passes.  CPU only; nothing here touches the GPU path."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sstep_oracle.c")

PINS = "tests/test_oracle_pins.py"
ILU = "tests/test_ilu0_oracle.py"
NEWTON = "tests/test_newton_basis_oracle.py"
MGS = "tests/test_omin_mgs_oracle.py"

# name: (text in the oracle, planted replacement, pin file that must fail)
MUTANTS = {
    # Hessenberg column of the s-step GMRES block (Sec. 4, eq. (6)): sign
    "hessenberg_sign": ("gc[rr] -= gi[rr] * t;", "gc[rr] += gi[rr] * t;", PINS),
    # block Gram-Schmidt against the earlier blocks: first block skipped
    "projection_drops_first_block": (
        "for (int i = 0; i < kb; ++i) {\n                const double *Ti = T + (size_t)i * s * (s + 1);\n"
        "                for (int q = 0; q < s; ++q) axpy(N, -Ti",
        "for (int i = 1; i < kb; ++i) {\n                const double *Ti = T + (size_t)i * s * (s + 1);\n"
        "                for (int q = 0; q < s; ++q) axpy(N, -Ti",
        PINS),
    # Chebyshev basis change: half-width not halved
    "chebyshev_half_width": ("B[(j - 1) + j * (s + 1)] = 0.5 * cd;", "B[(j - 1) + j * (s + 1)] = cd;",
                             PINS),
    # s-Omin Scalar2 (Sec. 3): W_j B_j = -C_j sign
    "somin_B_sign": ("Bj[q + l * s] = -c[q];", "Bj[q + l * s] = c[q];", PINS),
    # stencil: south neighbour takes the north coefficient
    "stencil_transposed_neighbour": ("if (j > 0) acc += c[3] * x[p - sy];",
                                     "if (j > 0) acc += c[4] * x[p - sy];", PINS),
    # Givens update of the least-squares right-hand side: sign
    "givens_sign": ("rhs[cj + 1] = -sn[cj] * rhs[cj];", "rhs[cj + 1] = sn[cj] * rhs[cj];", PINS),
    # equilibrated Cholesky solve: scaling dropped
    "cholesky_equilibration": ("for (int i = 0; i < q; ++i) z[i] = F->sc[i] * t[i];",
                               "for (int i = 0; i < q; ++i) z[i] = t[i];", PINS),
    # L-scaled Hessenberg entries: diagonal of L skipped
    "L_scaling_diagonal": ("for (int b = a; b < qi; ++b) acc += Li[a + b * s]",
                           "for (int b = a + 1; b < qi; ++b) acc += Li[a + b * s]", PINS),
    # start vector normalisation nu missing from the Hessenberg column
    "nu_missing": ("gc[c0 + nq] += bl * nu;", "gc[c0 + nq] += bl;", PINS),
    # Orthomin(k) window one direction too short
    "omin_window_off_by_one": ("int j0 = i - k + 1 > 0 ? i - k + 1 : 0;\n            memcpy(APn",
                               "int j0 = i - k + 2 > 0 ? i - k + 2 : 0;\n            memcpy(APn", PINS),
    # standard GMRES modified Gram-Schmidt: wrong basis vector
    "gmres_mgs_index": ("double h = dot(N, Q + (long long)i * N, w);",
                        "double h = dot(N, Q + (long long)(i > 0 ? i - 1 : 0) * N, w);", PINS),
    # ILU(0) (Sec. 5): fill update sign, multiplier not divided by the pivot
    "ilu_update_sign": ("if (ilu_col(A, k, qq) == cj) LU[qj * N + p] -= lpk * LU[qq * N + k];",
                        "if (ilu_col(A, k, qq) == cj) LU[qj * N + p] += lpk * LU[qq * N + k];", ILU),
    "ilu_multiplier_unscaled": ("const double lpk = LU[qk * N + p] / ukk;",
                                "const double lpk = LU[qk * N + p];", ILU),
    # Newton basis: wrong Chebyshev points, Leja start at the smallest point,
    # shifts applied in reverse order
    "newton_points": ("pts[k] = cc + cd * cos((2.0 * k + 1.0) * ORC_PI / (2.0 * s));",
                      "pts[k] = cc + cd * cos((2.0 * k) * ORC_PI / (2.0 * s));", NEWTON),
    "leja_first_point": ("v = fabs(pts[k]);", "v = -fabs(pts[k]);", NEWTON),
    "newton_shift_order": ("yj[p] = (yj[p] - th[j - 1] * yp[p]) / cd;",
                           "yj[p] = (yj[p] - th[s - j] * yp[p]) / cd;", NEWTON),
    # A^T A-orthogonal s-Omin blocks (Sec. 3): P not updated with AP,
    # dependence test removed
    "mgs_P_sign": ("axpy(N, -c, P + (long long)l * N, pq);", "axpy(N, c, P + (long long)l * N, pq);",
                   MGS),
    "mgs_no_dependence_test": ("if (!(w > ORC_RANK_TOL * n0) || !isfinite(w)) {",
                               "if (!isfinite(w)) {", MGS),
}


CNN_SRC = os.path.join(ROOT, "oracle", "cnn_oracle.c")
CNN = "tests/test_cnn_oracle.py"

# the learned-guess network's FP64 oracle: direct convolution loops
CNN_MUTANTS = {
    # data gradient: one tap offset flipped
    "conv_data_grad_offset": ("i - (ty - 1) * d, j - (tx - 1) * d", "i + (ty - 1) * d, j - (tx - 1) * d",
                              CNN),
    # weight gradient stored with the tap indices transposed
    "conv_weight_grad_transposed": ("dw[(((size_t)co * Cin + ci) * 3 + ty) * 3 + tx] = acc",
                                    "dw[(((size_t)co * Cin + ci) * 3 + tx) * 3 + ty] = acc", CNN),
    # forward: bias dropped
    "conv_bias_dropped": ("double acc = bias ? bias[co] : 0.0;", "double acc = 0.0;", CNN),
    # weight gradient: one tap offset flipped
    "conv_weight_grad_offset": (
        "at(xp, H, W, i + (ty - 1) * d, j + (tx - 1) * d);\n                    }\n                    dw",
        "at(xp, H, W, i - (ty - 1) * d, j + (tx - 1) * d);\n                    }\n                    dw", CNN),
}


def _build(src_path, text, out):
    path = out + ".c"
    with open(path, "w") as fh:
        fh.write(text)
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-I", os.path.dirname(src_path), "-o", out, path, "-lm"], check=True)
    return out


def _pins(env_var, lib, pin_file):
    env = dict(os.environ, **{env_var: lib})
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", pin_file,
                        "-p", "no:cacheprovider"], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=600)
    return p.returncode, p.stdout[-300:]


def _check(tmp_path, src_path, env_var, mutants):
    src = open(src_path).read()
    jobs = {}
    for name, (a, b, pin_file) in mutants.items():
        assert src.count(a) == 1, f"{name}: the text to mutate is not unique or not found"
        jobs[name] = (_build(src_path, src.replace(a, b), str(tmp_path / f"mut_{name}.so")), pin_file)
    control = _build(src_path, src, str(tmp_path / "control.so"))
    files = sorted({f for _, f in jobs.values()})
    with ThreadPoolExecutor(max_workers=4) as ex:
        ctl = {f: ex.submit(_pins, env_var, control, f) for f in files}
        res = {n: ex.submit(_pins, env_var, lib, f) for n, (lib, f) in jobs.items()}
        for f, fut in ctl.items():
            rc, out = fut.result()
            assert rc == 0, f"unmodified oracle fails {f}: {out}"
        missed = []
        for n, fut in res.items():
            rc, out = fut.result()
            if rc != 1:         # 1: tests ran and at least one failed
                missed.append((n, rc, out))
    assert not missed, missed


def test_every_planted_mistake_fails_a_pin(tmp_path):
    _check(tmp_path, SRC, "SSTEP_ORACLE_LIB", MUTANTS)


def test_every_planted_mistake_in_the_network_oracle_fails_a_pin(tmp_path):
    _check(tmp_path, CNN_SRC, "SSTEP_CNN_ORACLE_LIB", CNN_MUTANTS)
