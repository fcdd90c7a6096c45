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
