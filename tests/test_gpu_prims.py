"""The device sort and de-duplication (rt_keys_sort) against NumPy's: keys
of one and two words, sizes from empty to millions (both the one-workgroup
path and the many-workgroup path, on both sides of the boundary between
them), bit ranges, stability of equal keys, and unique against np.unique."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_13034_amd import risrt
    c = risrt.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _u64(a):
    return np.asarray(a, np.uint64)


def _gpu(ctx, keys, **kw):
    import torch
    t = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    n = ctx.keys_sort(t, **kw)
    return t.cpu().numpy().view(np.uint64)[:n]


@pytest.mark.parametrize("n", [0, 1, 2, 5, 1023, 1024, 1025, 8191, 8192, 8193, 20_000, 300_001, 2_000_000])
def test_sort_one_word(ctx, n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n).astype(np.uint64)
    _say("case sort 1 word n", n)
    assert np.array_equal(_gpu(ctx, keys), np.sort(keys))
    # many duplicates, 21-bit fields like the candidate keys, then unique
    keys = rng.integers(1, 40, size=(n, 3)).astype(np.uint64)
    packed = keys[:, 0] | (keys[:, 1] << np.uint64(21)) | (keys[:, 2] << np.uint64(42))
    assert np.array_equal(_gpu(ctx, packed, end_bit=63, unique=True), np.unique(packed))
    assert sorted(set(packed.tolist())) == _gpu(ctx, packed, end_bit=63, unique=True).tolist()


@pytest.mark.parametrize("n", [3, 4095, 4096, 4097, 50_000, 1_000_003])
def test_sort_two_words_and_stability(ctx, n):
    rng = np.random.default_rng(100 + n)
    lo = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).astype(np.uint64)
    hi = rng.integers(0, 1 << 41, size=n, dtype=np.int64).astype(np.uint64)
    keys = np.stack([lo, hi], axis=1)
    _say("case sort 2 words n", n)
    got = _gpu(ctx, keys).reshape(-1, 2)
    order = np.lexsort((lo, hi))
    assert np.array_equal(got, keys[order])
    # sort by the high word only (bits 64..127): equal high words keep their input order
    hi_small = rng.integers(0, 300, size=n).astype(np.uint64)
    keys = np.stack([np.arange(n, dtype=np.uint64), hi_small], axis=1)
    got = _gpu(ctx, keys, begin_bit=64, end_bit=128).reshape(-1, 2)
    assert np.array_equal(got, keys[np.argsort(hi_small, kind="stable")])
    # unique of two-word keys with duplicates
    base = np.stack([rng.integers(1, 50, size=n).astype(np.uint64), rng.integers(0, 3, size=n).astype(np.uint64)], 1)
    got = _gpu(ctx, base, unique=True).reshape(-1, 2)
    ref = np.unique(base[:, 0] + (base[:, 1] << np.uint64(32)))
    assert np.array_equal(got[:, 0] + (got[:, 1] << np.uint64(32)), ref)


def test_sort_bit_range_one_word(ctx):
    """Only bits [8, 40) decide the order; the others ride along (stable)."""
    rng = np.random.default_rng(9)
    n = 70_000
    keys = rng.integers(0, 2 ** 62, size=n, dtype=np.int64).astype(np.uint64)
    field = (keys >> np.uint64(8)) & np.uint64((1 << 32) - 1)
    got = _gpu(ctx, keys, begin_bit=8, end_bit=40)
    assert np.array_equal(got, keys[np.argsort(field, kind="stable")])


@pytest.mark.parametrize("n", [2, 1000, 8192])
def test_sort_skips_shared_digits_stably(ctx, n):
    """Keys whose 8-bit digits are partly the same in every key (those passes
    are skipped), all-equal keys, and the receiver-order keys of the
    per-element kernel (cost above bit 32, the index below, sorted on the
    cost bits alone): stable results equal to NumPy's."""
    rng = np.random.default_rng(7 + n)
    _say("case sort shared digits n", n)
    keys = (np.uint64(0xAB) << np.uint64(56)) | (rng.integers(0, 256, size=n).astype(np.uint64) << np.uint64(16)) \
        | np.uint64(0x3C00)
    keys = keys | np.arange(n, dtype=np.uint64) % np.uint64(3)   # low digit varies a little
    assert np.array_equal(_gpu(ctx, keys), np.sort(keys))
    same = np.full(n, np.uint64(0x1234_5678_9ABC_DEF0))
    assert np.array_equal(_gpu(ctx, same), same)
    cost = rng.integers(1, 40, size=n).astype(np.uint64)
    rk = ((np.uint64(0xFFFFF) - cost) << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    got = _gpu(ctx, rk, begin_bit=32, end_bit=52)
    assert np.array_equal(got, rk[np.argsort(rk >> np.uint64(32), kind="stable")])
    assert np.array_equal(got, np.sort(rk))   # the same order as a sort of every bit
    two = np.stack([np.arange(n, dtype=np.uint64), np.full(n, np.uint64(5))], axis=1)
    got = _gpu(ctx, two, begin_bit=0, end_bit=128).reshape(-1, 2)
    assert np.array_equal(got, two)
