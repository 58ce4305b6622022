"""Host checks of two arithmetic arguments the counting kernels rely on (no GPU).

* A streamline's close splits pair q of its (new rows) x (distinct labels) product into row q / nU
  and label q % nU with a float32 quotient, q * fl32(1 / nU), truncated and raised by one where
  (r + 1) * nU <= q.  The kernel relies on this being exact for every q < 4096 and 1 <= nU <= 64:
  checked here exhaustively in float32.
* The fallback finds the streamline holding point p (the last s with offsets[s] <= p) by testing
  256 evenly spaced offsets per round and narrowing [lo, hi) by the count of those at or below p.
  Over nondecreasing offsets, with runs of empty streamlines, this must give the serial search's
  answer: checked here against numpy's searchsorted on random offsets.
* Large calls split their points into ranges that taper from 1.5x to 0.5x the mean, in exact
  integer arithmetic: checked here for the sizes of the benchmark subjects and small corner cases.
* A batched plan transposes all subjects' copies of C in one grid of 64x64 tiles, numbered subject
  after subject; each tile finds its subject by a binary search over the subjects' first tiles and
  its corner from its local number.  Every entry of every subject must be written by exactly one
  tile: checked here for ragged N and M.
"""
import numpy as np
import pytest


def test_float_quotient_is_exact_for_the_close_products():
    q = np.arange(4096, dtype=np.int64)
    qf = q.astype(np.float32)
    for nu in range(1, 65):
        rcp = np.float32(1.0) / np.float32(nu)
        r = (qf * rcp).astype(np.float32).astype(np.int64)   # float32 product, truncated
        r = r + ((r + 1) * nu <= q)
        np.testing.assert_array_equal(r, q // nu, err_msg=f"nU = {nu}")
        np.testing.assert_array_equal(q - r * nu, q % nu, err_msg=f"nU = {nu}")


def _search_by_counts(offsets, p, width=256):
    S = len(offsets) - 1
    lo, hi = 0, S
    while hi - lo > 1:
        step = (hi - lo + width - 1) // width
        idx = lo + np.arange(width, dtype=np.int64) * step
        passing = (np.arange(width) > 0) & (idx < hi)
        passing[passing] = offsets[idx[passing]] <= p
        lo += int(passing.sum()) * step
        hi = min(hi, lo + step)
    return lo


@pytest.mark.parametrize("seed", range(8))
def test_count_search_finds_the_streamline_of_a_point(seed):
    rng = np.random.default_rng(seed)
    S = int(rng.choice([1, 2, 255, 256, 257, 70_000, 5_000_000]))
    lengths = rng.integers(0, 400, S)
    lengths[rng.random(S) < 0.2] = 0   # runs of empty streamlines share their start
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    P = int(offsets[-1])
    if P == 0:
        return
    points = rng.integers(0, P, 200)
    for p in points:
        want = int(np.searchsorted(offsets, p, side="right")) - 1   # last s with offsets[s] <= p
        got = _search_by_counts(offsets, int(p))
        assert got == want, (S, int(p), got, want)
        assert offsets[got] <= p < offsets[got + 1]


@pytest.mark.parametrize("P,n", [(1_097_713_418, 28_672), (112_532_461, 14_336), (1000, 7), (5, 9), (0, 4)])
def test_tapering_range_targets(P, n):
    # range i of the flat-stream partition starts at point P * g(i / n), g(x) = 1.5 x - 0.5 x^2, in
    # exact integer arithmetic: targets start at 0, end at P, never decrease, and the ranges shrink
    # linearly from 1.5x to 0.5x the mean (up to rounding)
    i = np.arange(n + 1, dtype=object)
    t = np.array([(P * k * (3 * n - k)) // (2 * n * n) for k in i], dtype=object)
    assert t[0] == 0 and t[-1] == P
    sizes = np.diff(t).astype(np.float64)
    assert (sizes >= 0).all()
    want = (1.5 - (np.arange(n) + 0.5) / n) * P / n   # the mean of g' over range i, times P / n
    assert np.abs(sizes - want).max() <= 1.0 + 1e-9 * P


@pytest.mark.parametrize("seed", range(4))
def test_transpose_tiles_cover_every_entry_once(seed):
    T = 64
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(64, 700)), int(rng.integers(2, 200))) for _ in range(int(rng.integers(1, 9)))]
    shapes += [(64, 2), (65, 64), (128, 65)]
    first, total = [], 0
    for N, M in shapes:
        first.append(total)
        total += ((N + T - 1) // T) * ((M + T - 1) // T)
    hits = [np.zeros((N, M), np.int64) for N, M in shapes]
    for t in range(total):
        lo, hi = 0, len(shapes)
        while hi - lo > 1:
            mid = (lo + hi) >> 1
            if first[mid] <= t:
                lo = mid
            else:
                hi = mid
        N, M = shapes[lo]
        local = t - first[lo]
        tn = (N + T - 1) // T
        i0, m0 = (local % tn) * T, (local // tn) * T
        assert i0 < N and m0 < M
        hits[lo][i0:min(i0 + T, N), m0:min(m0 + T, M)] += 1
    for h in hits:
        assert (h == 1).all()
