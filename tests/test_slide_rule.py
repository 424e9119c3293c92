"""The sliding rule of the median's later windows (host logic, checked on the CPU).

A median block sorts its union by (value, position) and answers a thread's
first window with the wavelet matrix; each next window of the thread is the
previous one moved by one position.  Stated in Python here: the element that
leaves and the one that enters are compared with the old median in that
order, and the new median is the old one or the nearest element above or
below it in sorted order whose position lies in the new window (Eq. "running
median": the h-th smallest of the window's W values).  Checked against the
plain definition on random unions with many ties, including the walk's
bounds: the element it stops at always exists on the side it walks to.  The
kernel itself is checked against the oracle by the GPU parity tests.
"""
import numpy as np
import pytest


def slide(x, sw, W, h, ap, m, a):
    """The sorted index of the median of window [a, a + W) from that (m) of
    [ap, ap + W), a = ap + 1; sw maps sorted index to position."""
    def before(p, q):
        return (x[p], p) < (x[q], q)
    pm, po, pi = sw[m], ap, ap + W
    if po == pm:
        step = -1 if before(pi, pm) else 1
    else:
        ob, ib = before(po, pm), before(pi, pm)
        step = 0 if ob == ib else (1 if ob else -1)
    c, walked = m, 0
    if step:
        while True:
            c += step
            walked += 1
            assert 0 <= c < len(sw)
            if a <= sw[c] < a + W:
                break
    return c, walked


@pytest.mark.parametrize("seed", range(6))
def test_sliding_median_matches_the_definition(seed):
    rng = np.random.default_rng(seed)
    longest = 0
    for _ in range(60):
        M = int(rng.integers(3, 300))
        W = int(rng.integers(1, M + 1)) | 1
        if W > M:
            W -= 2
        h = (W - 1) // 2
        levels = int(rng.integers(1, 40))
        x = rng.integers(0, levels, size=M).astype(np.float64)        # many equal values
        if rng.random() < 0.3:
            x += np.arange(M) * rng.choice([-1.0, 1.0]) * 0.5          # a trend
        sw = sorted(range(M), key=lambda p: (x[p], p))
        rank = {p: i for i, p in enumerate(sw)}

        def median(a):
            return sorted(range(a, a + W), key=lambda p: (x[p], p))[h]

        m = rank[median(0)]
        for a in range(1, M - W + 1):
            m, walked = slide(x, sw, W, h, a - 1, m, a)
            longest = max(longest, walked)
            assert sw[m] == median(a)
    assert longest >= 1
