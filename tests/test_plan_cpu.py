"""Host logic of the convolution's work plan, on the CPU (no GPU calls): the
item lists cover every (row, m1 chunk, cell group, k3 range) exactly once,
the XCD slices carry equal work, each slice runs heaviest first, mixed
launches give every XCD its share of every mesh, and the row windows
partition the rows within their byte limit.
"""
import numpy as np
import pytest

import paper_1301_4195_amd as bz

XCDS = 8


def _mcount(N, k):
    return min(k + N // 2, N - 1) - max(k - N // 2 + 1, 0) + 1


def _klo(N, m):
    return max(m - N // 2, 0)


def _khi(N, m):
    return min(m + N // 2 - 1, N - 1)


def _kept_lines(N, r, S, s):
    """Kept lines (m1, m2) of row r in chunk s of S: the first half of the
    mirrored line set, m1 range cut into S chunks."""
    c1, c2 = _mcount(N, r // N), _mcount(N, r % N)
    h = (c1 + 1) // 2
    per = -(-h // S)
    n = 0
    for a1 in range(s * per, min(h, (s + 1) * per)):
        n += (c2 + 1) // 2 if (c1 % 2 and a1 == c1 // 2) else c2
    return n


def _range_pairs(N, KH, q):
    kb, ke = q * (N // KH), (q + 1) * (N // KH)
    return sum(max(0, min(_khi(N, m), ke - 1) - max(_klo(N, m), kb) + 1) for m in range(N))


def _cost(N, S, KH, it):
    return (1 + _kept_lines(N, it[0], S, it[1])) * _range_pairs(N, KH, it[3])


@pytest.fixture(scope="module")
def lib():
    bz.load()  # loads libbz.so; the plan calls never touch the device
    return bz


@pytest.mark.parametrize("N,ncells,S,KH", [(8, 1, 1, 1), (16, 256, 4, 1), (16, 200, 3, 2), (24, 130, 6, 4),
                                           (32, 65, 4, 2)])
def test_items_cover_everything_once(lib, N, ncells, S, KH):
    it = lib.bz_plan_items(N, ncells, S, KH)
    G = -(-ncells // 64)
    assert it.shape[0] % XCDS == 0
    real = it[it[:, 0] >= 0]
    want = {(r, s, g, q) for r in range(N * N) for s in range(S) for g in range(G) for q in range(KH)}
    got = [tuple(x[:4]) for x in real]
    assert len(got) == len(set(got)) == len(want)
    assert set(got) == want
    assert np.all(real[:, 4] == 0)


@pytest.mark.parametrize("N,ncells,S,KH", [(16, 256, 4, 1), (24, 1024, 3, 2), (32, 512, 4, 2)])
def test_xcd_slices_balanced_and_heaviest_first(lib, N, ncells, S, KH):
    it = lib.bz_plan_items(N, ncells, S, KH)
    costs = np.array([_cost(N, S, KH, x) if x[0] >= 0 else 0 for x in it])
    per = costs.reshape(-1, XCDS)  # column x = XCD x's slice in launch order
    tot = per.sum(axis=0)
    assert tot.max() - tot.min() <= costs.max()  # equal cost up to one item
    for x in range(XCDS):
        col = per[:, x]
        col = col[col > 0]
        assert np.all(np.diff(col) <= 0)  # longest processing time first
    # each slice works on few cell groups: contiguous group ranges
    for x in range(XCDS):
        g = it[x::XCDS, 2][it[x::XCDS, 0] >= 0]
        assert np.unique(g).size <= -(-(-(-ncells // 64)) // XCDS) + 1


def test_row_range_items(lib):
    N, S, KH = 32, 2, 2
    it = lib.bz_plan_items(N, 128, S, KH, row0=100, row1=357)
    real = it[it[:, 0] >= 0]
    assert real[:, 0].min() == 100 and real[:, 0].max() == 356
    assert len(real) == (357 - 100) * S * 2 * KH


def test_mixed_items_every_op_on_every_xcd(lib):
    Ns, ncells, chunks = [8, 16, 24, 32], [1667, 1206, 812, 411], [2, 3, 6, 6]
    it = lib.bz_plan_mixed_items(Ns, ncells, chunks, f64=False)
    real = it[it[:, 0] >= 0]
    for j, (N, n, S) in enumerate(zip(Ns, ncells, chunks)):
        KH = 1 if N <= 16 else 2
        mine = real[real[:, 4] == j]
        G = -(-n // 64)
        want = {(r, s, g, q) for r in range(N * N) for s in range(S) for g in range(G) for q in range(KH)}
        got = [tuple(x[:4]) for x in mine]
        assert len(got) == len(set(got)) and set(got) == want, N
        for x in range(XCDS):  # every XCD holds part of every mesh
            col = it[x::XCDS]
            assert np.any(col[:, 4][col[:, 0] >= 0] == j), (N, x)
    # an op without cells contributes nothing
    it2 = lib.bz_plan_mixed_items([8, 16], [0, 100], [2, 2], f64=True)
    assert np.all(it2[it2[:, 0] >= 0][:, 4] == 1)


def _stored(N):
    """Packed weights of each output row (kept lines x 3N^2/4 pairs)."""
    out = []
    for r in range(N * N):
        c1, c2 = _mcount(N, r // N), _mcount(N, r % N)
        out.append(((c1 // 2) * c2 + ((c2 + 1) // 2 if c1 % 2 else 0)) * 3 * N * N // 4)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("N,dt,mb", [(32, bz.BZ_F64, 512), (32, bz.BZ_F32, 512), (32, bz.BZ_F64, 256),
                                     (24, bz.BZ_F64, 512), (16, bz.BZ_F64, 1), (8, bz.BZ_F32, 1),
                                     (48, bz.BZ_F32, 256)])
def test_windows_partition_rows(lib, N, dt, mb):
    cap = mb << 20
    b = lib.bz_plan_windows(N, dt, cap)
    elem = 8 if dt == bz.BZ_F64 else 4
    rows = _stored(N)
    assert b[0] == 0 and b[-1] == N * N and np.all(np.diff(b) > 0)
    for j in range(len(b) - 1):
        assert rows[b[j]:b[j + 1]].sum() * elem <= cap
        if j + 1 < len(b) - 1:  # greedy: the next row would not have fitted
            assert rows[b[j]:b[j + 1] + 1].sum() * elem > cap
    total = rows.sum() * elem
    assert len(b) - 1 >= -(-total // cap)


def _fill_rows(ncells, S, KH):
    return -(-8192 // (-(-ncells // 64) * S * KH))


def test_window_sizes_of_the_stored_tables(lib):
    """Stored tables above 512 MiB are convolved in windows that each keep
    enough rows to fill the chip: N = 32 with 512 cells in four (FP64) or two
    (FP32) launches, N <= 24 in one; small batches in fewer, larger ones."""
    assert len(lib.bz_plan_windows(32, bz.BZ_F64, 512 << 20, _fill_rows(512, 4, 2))) - 1 == 4
    assert len(lib.bz_plan_windows(32, bz.BZ_F32, 512 << 20, _fill_rows(512, 4, 2))) - 1 == 2
    assert len(lib.bz_plan_windows(24, bz.BZ_F64, 512 << 20, _fill_rows(1024, 4, 1))) - 1 == 1
    assert len(lib.bz_plan_windows(32, bz.BZ_F64, 512 << 20, _fill_rows(65, 4, 2))) - 1 == 1
    w48 = lib.bz_plan_windows(48, bz.BZ_F64, 512 << 20, _fill_rows(128, 4, 4))
    assert np.all(np.diff(w48) >= _fill_rows(128, 4, 4)) and len(w48) - 1 <= 48 * 48 // _fill_rows(128, 4, 4)


@pytest.mark.parametrize("min_rows", [1, 7, 100, 5000])
def test_window_merging(lib, min_rows):
    base = lib.bz_plan_windows(32, bz.BZ_F64, 64 << 20)
    w = lib.bz_plan_windows(32, bz.BZ_F64, 64 << 20, min_rows)
    assert w[0] == 0 and w[-1] == 32 * 32 and set(w) <= set(base)  # merged from the byte slabs
    if len(w) > 2:
        assert np.all(np.diff(w) >= min_rows)


def test_plan_argument_errors(lib):
    for args in ((12, 10, 1, 1), (16, 0, 1, 1), (16, 10, 0, 1), (16, 10, 99, 1), (16, 10, 1, 3)):
        with pytest.raises(bz.BzError) as e:
            lib.bz_plan_items(*args)
        assert e.value.code == bz.BZ_EINVAL
    with pytest.raises(bz.BzError):
        lib.bz_plan_items(16, 10, 1, 1, row0=5, row1=5)
    with pytest.raises(bz.BzError):  # below one row's weights
        lib.bz_plan_windows(32, bz.BZ_F64, 1000)


@pytest.mark.parametrize("N", [8, 16, 24, 32, 48])
def test_small_batch_plan(lib, N):
    """The small-batch form: blocks of a power of two of cells (at most 8,
    4 at N = 24 and 32, 2 at N = 48) that tile the batch inside one padded
    group of 64, three chunks for one block and fewer for more (a single
    cell at N <= 16, which the one-cell kernel takes: two), the default form
    up to the measured crossover (32 cells at N <= 16, 16 above)."""
    cap = 8 if N <= 16 else (4 if N <= 32 else 2)
    maxc = (N // 2 + 2) // 2
    for n in range(1, 65):
        cb, nb, ch, dflt = lib.bz_plan_small_batch(N, n)
        assert cb in (1, 2, 4, 8) and cb <= cap
        assert cb == min(cap, 1 << (n - 1).bit_length())  # smallest power of two >= n, capped
        assert nb == -(-n // cb) and (nb - 1) * cb < n <= nb * cb <= 64
        if n == 1 and N <= 16:
            assert ch == 2
        else:
            assert 1 <= ch <= min(3, maxc) and ch == max(1, min(-(-3 // nb), maxc))
        assert dflt == (n <= (32 if N <= 16 else 16))
    for bad in ((12, 1), (16, 0), (16, 65)):
        with pytest.raises(bz.BzError):
            lib.bz_plan_small_batch(*bad)
