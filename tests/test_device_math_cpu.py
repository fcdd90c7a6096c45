"""Host-side checks of arithmetic identities the gfx950 kernels rely on."""
import numpy as np


def test_reciprocal_small_division_is_exact():
    """The kernels' small integer division floor(a / b) is computed as
    (float(a) + 0.5) * rcp(b) truncated; it must equal a // b for every
    0 <= a <= 4096, 1 <= b <= 256 even when the hardware reciprocal is off by
    up to two ulps of float32."""
    a = np.arange(0, 4097, dtype=np.float32)
    want_all = np.arange(0, 4097)
    for b in range(1, 257):
        r0 = np.float32(1.0) / np.float32(b)
        cands = [r0]
        for direction in (np.float32(np.inf), np.float32(-np.inf)):
            r = r0
            for _ in range(2):
                r = np.nextafter(r, direction)
                cands.append(r)
        want = want_all // b
        for r in cands:
            q = np.floor((a + np.float32(0.5)) * r).astype(np.int64)
            assert np.array_equal(q, want), (b, r)


def _pairs_like_kernel(c, threads):
    """The scaled box update's pair walk: pair q of c*floor((c-1)/2) +
    (c even ? c/2 : 0) is (q mod c, (q mod c + q div c + 1) mod c); each
    thread starts at q = t and steps by `threads` with an incremental
    (d, i) update in place of a division."""
    total = c * ((c - 1) // 2) + (0 if c & 1 else c // 2)
    out = []
    for t in range(min(threads, total)):
        d, i = t // c, t % c
        sd, si = threads // c, threads % c
        q = t
        while q < total:
            j = i + d + 1
            if j >= c:
                j -= c
            assert 0 <= i < c and 0 <= j < c
            out.append((i, j))
            i += si
            d += sd
            if i >= c:
                i -= c
                d += 1
            q += threads
    return out


def test_pair_walk_visits_every_unordered_pair_once():
    for threads, cs in ((1024, list(range(1, 70)) + [511, 512, 1023, 1024, 1025, 2049]),
                        (64, list(range(1, 70)) + [129]), (7, list(range(1, 40)))):
        for c in cs:
            got = _pairs_like_kernel(c, threads)
            assert len(got) == c * (c - 1) // 2, (c, threads)
            keys = {(min(i, j), max(i, j)) for i, j in got}
            assert len(keys) == len(got), (c, threads)
            assert all(i != j for i, j in got)


def _items_like_kernel(c, threads, slices, K=4):
    """The passes' blocked walk over items split into `slices` contiguous
    ranges: item t < G*c (G = ceil(floor((c-1)/2) / K)) is point i = t mod c
    with the distances 1 + K*g .. K*(g+1) below c/2 (g = t div c); for even
    c, item G*c + i (i < c/2) is the pair (i, i + c/2).  Each thread of a
    slice starts at its item and steps by `threads` with an incremental
    (g, i) update."""
    if c < 2:
        return []
    df = (c - 1) // 2
    gc = -(-df // K) * c
    items = gc + (0 if c & 1 else c // 2)
    out = []
    for s in range(slices):
        t0, t1 = items * s // slices, items * (s + 1) // slices
        for th in range(threads):
            t = t0 + th
            if t >= t1:
                break
            g, i = t // c, t % c
            sg, si = threads // c, threads % c
            while t < t1:
                if t < gc:
                    d0 = g * K
                    j = i + d0 + 1
                    if j >= c:
                        j -= c
                    for k in range(K):
                        if d0 + k < df:
                            assert 0 <= i < c and 0 <= j < c
                            out.append((i, j))
                        j += 1
                        if j >= c:
                            j -= c
                else:
                    ih = t - gc
                    assert 0 <= ih < c // 2
                    out.append((ih, ih + c // 2))
                i += si
                g += sg
                if i >= c:
                    i -= c
                    g += 1
                t += threads
    return out


def test_blocked_pair_walk_visits_every_unordered_pair_once():
    for threads, slices, cs in ((1024, 1, list(range(0, 70)) + [511, 512, 1023, 1024, 1025, 2049]),
                                (1024, 64, list(range(0, 40)) + [257, 1000, 1001]),
                                (1024, 12, [2, 3, 400, 401]),
                                (64, 3, list(range(0, 70)) + [129]), (7, 5, list(range(0, 40)))):
        for c in cs:
            got = _items_like_kernel(c, threads, slices)
            assert len(got) == c * (c - 1) // 2, (c, threads, slices)
            keys = {(min(i, j), max(i, j)) for i, j in got}
            assert len(keys) == len(got), (c, threads, slices)
            assert all(i != j for i, j in got)
