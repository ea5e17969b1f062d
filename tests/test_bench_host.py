"""Host logic of bench.py that needs no GPU: the one-GPU guard, the guard on
the committed HBM-traffic record, and the cycle bookkeeping behind the
algorithmic byte counts."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (defines functions only; main() runs under __main__)


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, env=e,
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_record_guarded_by_kernel_hash(monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "sgmres_256cube_s8m40_fp64_traffic.json")))
    # the committed record was taken on the current kernels
    assert rec["kernels_hash"] == bench.kernel_source_hash()
    for kind in ("update", "gram"):
        t = bench.measured_traffic(kind)
        assert t == rec[kind]["hbm_bytes_per_launch"]
        # HBM bytes within a few percent of the algorithmic bytes: no re-reads
        assert 0.99 <= t / rec[kind]["algorithmic_bytes_per_launch"] <= 1.05
    assert bench.measured_traffic("no_such_kernel") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("update") is None


def test_blocks_per_cycle():
    # 110 blocks in 3 restart cycles of m = 40: two full cycles, then the rest
    assert bench.blocks_per_cycle(110, 3, 40) == [40, 40, 30]
    assert bench.blocks_per_cycle(40, 1, 40) == [40]
    assert bench.blocks_per_cycle(7, 2, 5) == [5, 2]
    assert sum(bench.blocks_per_cycle(123, 4, 40)) == 123


def test_vector_pass_model_is_additive_and_grows_with_the_basis():
    # each block k of a cycle projects against the (k-1) s earlier columns
    # twice (Gram and update), so consecutive blocks differ by 2 s passes
    s = 8
    one = bench.vec_passes_gmres([1], s)
    assert bench.vec_passes_gmres([1, 1], s) == 2 * one
    d = [bench.vec_passes_gmres([k + 1], s) - bench.vec_passes_gmres([k], s) for k in range(1, 6)]
    assert all(b - a == 2 * s for a, b in zip(d, d[1:]))
    assert bench.vec_passes_gmres([40, 40, 30], s) == sum(bench.vec_passes_gmres([n], s)
                                                          for n in (40, 40, 30))


def test_flop_model_closed_forms():
    # per cycle of m blocks on N points: the Gram and the update each contract
    # (k-1)s basis columns with s columns for k = 2..m, 2 flops per
    # multiply-add, i.e. m(m-1)s^2 N flops; matrix powers take 13 flops per
    # point and power for the 7-point stencil, 9 for the 5-point one
    s, m, N = 8, 40, 1000
    fl = bench.flops_gmres([m], s, N, 3)
    assert fl["gram"] == fl["update"] == m * (m - 1) * s * s * N
    assert fl["mpk"] == 13 * s * m * N
    assert bench.flops_gmres([m], s, N, 2)["mpk"] == 9 * s * m * N
    two = bench.flops_gmres([m, 3], s, N, 3)
    assert two["gram"] == fl["gram"] + 3 * 2 * s * s * N
