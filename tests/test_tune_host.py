"""The batched solver's tuning table without a GPU: exact keys, the nearest
tuned batch for a batch of its own (same size distribution, other seeds), and
no match for batches whose systems are distributed differently or that use
another s, m or architecture."""
import pytest

from paper_2001_04886_amd import problems as PB
from paper_2001_04886_amd import tune as TU


class _A:
    def __init__(self, n):
        self.N = n


def _batch(nsys, seed, lo=32, hi=512):
    import numpy as np
    rng = np.random.default_rng(seed)
    return [_A(int(n) ** 2) for n in rng.integers(lo, hi + 1, nsys)]


@pytest.fixture(autouse=True)
def _gfx950(monkeypatch):
    monkeypatch.setattr(TU, "_arch", lambda: "gfx950")


def test_exact_entry_of_the_benchmarked_batch():
    st = [_A(n * n) for n, _, _ in PB.batched_table(512, master_seed=0)]
    assert TU.lookup(st, 4, 30)[:3] == (512, 1, 2)


def test_histogram_is_the_share_of_unknowns_per_size_class():
    h = TU.size_histogram([1024, 1500, 4096])
    assert set(h) == {"10", "12"}
    assert abs(sum(h.values()) - 1.0) < 1e-12
    assert abs(h["12"] - 4096 / (1024 + 1500 + 4096)) < 1e-12


def test_nearest_entry_for_a_batch_of_the_same_distribution():
    # another draw of side ~ U{32..512}: no exact entry, the committed one is near
    st = _batch(480, 7)
    d, rec = TU.nearest(TU.signature([a.N for a in st], 4, 30, "gfx950"), TU.load_cache())
    assert d < TU.NEAREST_MAX
    assert TU.lookup(st, 4, 30)[:3] == (512, 1, 2)


def test_no_match_for_other_distributions_or_parameters():
    small = _batch(512, 3, lo=32, hi=64)          # only small systems
    assert TU.lookup(small, 4, 30) is None
    st = _batch(512, 7)
    assert TU.lookup(st, 8, 30) is None           # another s
    assert TU.lookup(st, 4, 20) is None           # another m
