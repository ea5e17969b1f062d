"""The block update writes its outputs with non-temporal stores.

The compiler can drop the non-temporal bit of an inlined store without any
diagnostic (a plain ``global_store`` is emitted), which costs the block update
3-9% of its streaming rate.  This compiles ``k_update`` for every output width
and type combination the library instantiates and counts the non-temporal
16-byte stores in the gfx950 assembly.  Host-only: hipcc cross-compiles.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_04886_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")

# (basis TV, base TB, output TO, arithmetic TA): FP64, FP32, FP32 basis into FP64
COMBOS = [("double", "double", "double", "double"),
          ("float", "float", "float", "float"),
          ("float", "double", "double", "double")]
SIZE = {"double": 8, "float": 4}
MANGLE = {"double": "d", "float": "f"}
# The one-column update of an FP32 basis into FP64 outputs (the mixed-precision
# solution assembly, once per restart cycle) still compiles to plain stores.
KNOWN_PLAIN = {("float", "double", "double", "double", 1)}


def _ppt(tv, tb, to):
    return max(16 // SIZE[tv], 16 // SIZE[tb], 16 // SIZE[to])


def test_update_output_stores_are_nontemporal(tmp_path):
    lines = ['#include "kernels.hpp"', "namespace sstep {"]
    cases = []
    for tv, tb, to, ta in COMBOS:
        for k in range(1, 17):
            for norm in ((False, True) if k == 1 else (False,)):
                # 16-wave workgroups: FP64 updates of 4 or more outputs
                for ut in ((256, 1024) if (k >= 4 and tv == "double") else (256,)):
                    nb = "true" if norm else "false"
                    lines.append(
                        f"template __global__ void k_update<{tv}, {tb}, {to}, {ta}, {k}, {nb}, {ut}>("
                        f"long long, const {tb}*, long long, const {tv}*, long long, int, const int*, "
                        f"const double*, {to}*, long long, double*, const int*);")
                    cases.append((tv, tb, to, ta, k, norm, ut))
    lines.append("}")
    src = tmp_path / "update_inst.hip"
    src.write_text("\n".join(lines) + "\n")
    asm = tmp_path / "update_inst.s"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-I", CSRC, "--cuda-device-only", "-S", "-o", str(asm), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    text = asm.read_text()
    bodies = {}
    for m in re.finditer(r"^(_ZN5sstep8k_update\S+):", text, re.M):
        end = text.index(".Lfunc_end", m.end())
        bodies[m.group(1)] = text[m.end():end]
    checked = 0
    for tv, tb, to, ta, k, norm, ut in cases:
        key = f"I{MANGLE[tv]}{MANGLE[tb]}{MANGLE[to]}{MANGLE[ta]}Li{k}ELb{int(norm)}ELi{ut}E"
        names = [n for n in bodies if key in n]
        assert len(names) == 1, (key, names)
        stores = re.findall(r"global_store_dwordx4[^\n]*", bodies[names[0]])
        nt = sum(1 for s in stores if re.search(r"\bnt\b", s))
        # one 16-byte store per output column per 16 bytes of a thread's points
        want = k * _ppt(tv, tb, to) * SIZE[to] // 16
        if (tv, tb, to, ta, k) in KNOWN_PLAIN:
            continue
        assert nt >= want, f"{names[0]}: {nt} non-temporal 16-byte stores, want {want}"
        checked += 1
    assert checked == len(cases) - 2
