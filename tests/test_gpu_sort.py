"""The stable bucket sort (Alg. 1, distribute loop) on its own: keys given by
the test, the permutation compared with numpy's stable argsort element by
element.  Sizes span one tile (4096 keys), ragged tails, many tiles (the
workgroups wait on their predecessors' digit counts) and the largest particle
count the filter accepts in one sort; key sets include every key equal (a
converged filter), a few distinct keys, and keys using all 32 bits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2404_16370_amd import megapf as M


def _check(keys, bits):
    ko, order = M.debug_sort_u32(keys, bits)
    ref = np.argsort(keys, kind="stable")
    assert np.array_equal(order, ref.astype(np.int32))
    assert np.array_equal(ko, keys[ref])


@pytest.mark.parametrize("n", [2, 3, 4095, 4096, 4097, 50_000, 1_048_576 + 37])
@pytest.mark.parametrize("bits", [8, 12, 24, 32])
def test_sort_random_keys(n, bits):
    rng = np.random.default_rng(n * 64 + bits)
    keys = rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)
    print("random keys n=%d bits=%d" % (n, bits), flush=True)
    _check(keys, bits)


@pytest.mark.parametrize("n", [300_001, 1_048_576])
def test_sort_equal_and_few_keys(n):
    rng = np.random.default_rng(n)
    print("equal keys n=%d" % n, flush=True)
    _check(np.full(n, 0xABCDEF, np.uint32), 24)
    print("few keys n=%d" % n, flush=True)
    _check(rng.choice(rng.integers(0, 1 << 24, 7, dtype=np.uint64), n).astype(np.uint32), 24)
    # long runs of equal keys in input order (a histogram thread sees whole runs)
    print("runs n=%d" % n, flush=True)
    _check(np.repeat(rng.integers(0, 1 << 20, n // 1000 + 1, dtype=np.uint64), 1000)[:n].astype(np.uint32), 20)


def test_sort_largest_filter():
    # 2^26 keys: the largest particle count of one filter
    n = 1 << 26
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 1 << 24, n, dtype=np.uint64).astype(np.uint32)
    print("random keys n=%d bits=24" % n, flush=True)
    _check(keys, 24)


def test_sort_rejects():
    with pytest.raises(M.MegaPFError):
        M.debug_sort_u32(np.zeros(4, np.uint32), 0)
    with pytest.raises(M.MegaPFError):
        M.debug_sort_u32(np.zeros(4, np.uint32), 33)
