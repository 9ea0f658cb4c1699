"""The fill keeps a tile's cube starts in LDS as 16-bit values: start - t0 + 1
clamped to [0, tile + 2].  This models a lane's use of them (binary search
for its first cube, the head test, the next cube's start compared with each
of its samples and with its end) and checks every outcome against the
unclamped starts, on cube sizes from n_min = 2 up to cubes much longer than
a tile."""
import numpy as np
import pytest


def lane_view(start, h_lo, nst_load, t0, k0, k1, tile, clamp):
    st = np.array(start[h_lo:h_lo + nst_load], dtype=np.int64)
    if clamp:
        st = np.clip(st - t0 + 1, 0, tile + 2)
        key = k0 - t0 + 1
    else:
        key = k0
    lo, hi = 0, nst_load - 1
    while hi - lo > 1:
        mid = (lo + hi) >> 1
        if st[mid] <= key:
            lo = mid
        else:
            hi = mid
    nxt = int(st[lo + 1]) + (t0 - 1 if clamp else 0)
    head = bool(st[lo] < key)
    hits = tuple(k for k in range(k0, k1) if k == nxt)
    return lo, head, hits, nxt > k1


@pytest.mark.parametrize("seed", range(6))
def test_clamped_starts_keep_every_outcome(seed):
    rng = np.random.default_rng(seed)
    tile = int(rng.choice([1024, 4096, 32768]))
    per_lane = tile // 1024
    # cube sizes: mostly small (n_min = 2 and up), a few far longer than a tile
    sizes = rng.integers(2, 12, 20000)
    sizes[rng.integers(0, sizes.size, 30)] = rng.integers(tile, 5 * tile, 30)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n_eval = int(start[-1])
    n_tiles = (n_eval + tile - 1) // tile
    # random tiles, and the tiles around the long cubes (a tile inside one,
    # and the tiles where one begins or ends)
    long_h = np.nonzero(sizes >= tile)[0]
    picks = list(rng.integers(0, n_tiles, 8))
    for h in long_h[:6]:
        picks += [start[h] // tile, (start[h] + tile) // tile, (start[h + 1] - 1) // tile]
    for t in sorted(set(int(p) for p in picks if 0 <= p < n_tiles)):
        t0 = int(t) * tile
        t1 = min(t0 + tile, n_eval)
        h_lo = int(np.searchsorted(start, t0, side="right") - 1)
        h_nx = int(np.searchsorted(start, min(t1, n_eval - 1), side="right") - 1)
        h_top = min(h_nx, sizes.size - 1)
        nst_load = h_top - h_lo + 2
        assert nst_load <= tile // 2 + 4
        for lane in list(range(0, 1024, 7)) + [1021, 1022, 1023]:
            k0 = t0 + lane * per_lane
            k1 = min(k0 + per_lane, t1)
            if k0 >= k1:
                continue
            a = lane_view(start, h_lo, nst_load, t0, k0, k1, tile, clamp=False)
            b = lane_view(start, h_lo, nst_load, t0, k0, k1, tile, clamp=True)
            assert a == b, (t0, lane)
