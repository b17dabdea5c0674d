"""Host check of the lane-exchange sorting networks that the K-best, hybrid
and parallel-SD kernels use (sort_lanes, merge_lanes, bitonic_sort and the
truncating merges in the selection), simulated lane by lane with numpy: the
mirror-form stages (lane ^ 3, ^ 7, ^ 15 within rows, then half cleaners),
the odd rows reversed before the 32-lane merge, the upper half sorted as
complements before the 64-lane merge, the pair stages across rows, the
descending variant, the two-register top-64 merge and the multi-register
sort.  The GPU parity tests check the HIP code itself; this checks that the
network it implements sorts."""
import numpy as np
import pytest

L = np.arange(64)
FULL = np.uint64(0xFFFFFFFFFFFFFFFF)


def _before(x, y, desc):
    return (y < x) if desc else (x < y)


def _keep(key, p, m, desc):
    """Lane bit m clear: the key that goes first of key and partner p."""
    upper = (L & m) != 0
    return np.where(_before(p, key, desc) != upper, p, key)


def _pair(key, j, desc):
    """Stage lane ^ j (16 or 32) from one row swap: both keys of the pair."""
    a = key[L & ~j]
    b = key[L | j]
    upper = (L & j) != 0
    return np.where(_before(b, a, desc) != upper, b, a)


def _rev_odd_rows(key):
    out = key.copy()
    for r in (1, 3):
        out[16 * r:16 * r + 16] = key[16 * r:16 * r + 16][::-1]
    return out


def _clean16(key, desc):
    for j in (8, 4, 2, 1):
        key = _keep(key, key[L ^ j], j, desc)
    return key


def sort_lanes(key, lim, desc=False):
    cm = np.where(((L & 32) != 0) & (lim == 64), FULL, np.uint64(0))
    key = key ^ cm
    for pj, m in ((1, 1), (3, 2), (1, 1), (7, 4), (2, 2), (1, 1), (15, 8), (4, 4), (2, 2), (1, 1)):
        key = _keep(key, key[L ^ pj], m, desc)
    if lim >= 32:
        key = _clean16(_pair(_rev_odd_rows(key), 16, desc), desc)
    if lim == 64:
        key = _clean16(_pair(_pair(key ^ cm, 32, desc), 16, desc), desc)
    return key


def merge_lanes(key, desc=False):
    return _clean16(_pair(_pair(key, 32, desc), 16, desc), desc)


def _keys(rng, n, pads):
    k = (rng.integers(0, 1 << 20, n).astype(np.uint64) << np.uint64(32)) | rng.permutation(1 << 16)[:n].astype(
        np.uint64)
    if pads:
        k[rng.random(n) < 0.3] = FULL
    return k


@pytest.mark.parametrize("lim", [16, 32, 64])
@pytest.mark.parametrize("desc", [False, True])
def test_sort_lanes_sorts_every_group(lim, desc):
    rng = np.random.default_rng(lim + 7 * desc)
    for t in range(300):
        k = _keys(rng, 64, t % 2)
        s = sort_lanes(k, lim, desc)
        for g in range(0, 64, lim):
            want = np.sort(k[g:g + lim])
            assert np.array_equal(s[g:g + lim], want[::-1] if desc else want)


def test_top64_of_two_registers():
    """The selection's top-64: first 64 keys sorted ascending, the rest (c1 of
    them) complemented, sorted in the top 16, 32 or 64 lanes and complemented
    back (descending over the wave), the lane-wise minimum merged."""
    rng = np.random.default_rng(3)
    for t in range(500):
        k0 = _keys(rng, 64, False)
        c1 = int(rng.integers(1, 65))
        lim = 16 if c1 <= 16 else (32 if c1 <= 32 else 64)
        rest = _keys(rng, c1, False)
        k1 = np.zeros(64, np.uint64)
        k1[64 - lim:64 - lim + c1] = ~rest
        k1 = ~sort_lanes(k1, lim)
        assert np.all(np.diff(k1.astype(object)) <= 0)
        m = merge_lanes(np.minimum(sort_lanes(k0, 64), k1))
        assert np.array_equal(m, np.sort(np.concatenate([k0, rest]))[:64])


@pytest.mark.parametrize("E", [2, 4, 8])
def test_block_merge_select(E):
    """All blocks sorted (even ascending, odd descending), then pairs merged
    with truncation: block 0 ends with the 64 smallest, ascending."""
    rng = np.random.default_rng(E)
    for t in range(200):
        keys = [_keys(rng, 64, t % 2) for _ in range(E)]
        kk = [sort_lanes(keys[e], 64, bool(e & 1)) for e in range(E)]
        w = 1
        while w < E:
            for e in range(0, E, 2 * w):
                kk[e] = merge_lanes(np.minimum(kk[e], kk[e + w]), bool((e // (2 * w)) & 1))
            w *= 2
        assert np.array_equal(kk[0], np.sort(np.concatenate(keys))[:64])


@pytest.mark.parametrize("E", [1, 2, 4])
def test_multi_register_sort(E):
    """bitonic_sort over 64 E keys: registers sorted alternately, register
    stages compare whole registers, lane stages are merge_lanes."""
    rng = np.random.default_rng(10 + E)
    for t in range(200):
        keys = [_keys(rng, 64, t % 2) for _ in range(E)]
        kk = [sort_lanes(keys[e], 64, E > 1 and bool(e & 1)) for e in range(E)]
        size = 128
        while size <= 64 * E:
            j = size // 2
            while j >= 64:
                je = j // 64
                for e in range(E):
                    pe = e ^ je
                    if pe > e:
                        asc = ((e * 64) & size) == 0
                        a, b = kk[e], kk[pe]
                        sw = (a > b) if asc else (a < b)
                        kk[e], kk[pe] = np.where(sw, b, a), np.where(sw, a, b)
                j //= 2
            kk = [merge_lanes(kk[e], ((e * 64) & size) != 0) for e in range(E)]
            size *= 2
        assert np.array_equal(np.concatenate(kk), np.sort(np.concatenate(keys)))
