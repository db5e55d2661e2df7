"""A CPU model of one merge level of the merge scheme (the Step 3 count of
Sec. 3.2 as a merge of sorted runs), step by step as a lane takes it: the
padded row (4 pad slots after every 64 keys, the first one holding the
sentinel), the merge-path search for the lane's first output, loads clamped
to the pad slot after the run, and the count formed from the running sum of
the right run's head position.  Checked against brute force: the lanes'
outputs concatenated are the merged run, and their counts sum to the number
of (left, right) pairs with the left key strictly larger.  It checks the
design, not the GPU code (which the GPU parity tests compare with the
oracle)."""
import numpy as np
import pytest

SENTINEL = 0xFFFF


def padded(p):
    return p + ((p >> 6) << 2)


def padded_byte(i2):
    return i2 + ((i2 >> 7) << 3)


def make_row(keys, NR):
    """keys (NR of them) in the padded layout as uint16, pads = sentinel."""
    row = np.full(padded(NR - 1) + 1 + 4, SENTINEL, np.int64)
    for p in range(NR):
        row[padded(p)] = keys[p]
    return row


def lane_segment(row, l0, s, lenA, lenB, diag, K):
    at = lambda p: int(row[padded(l0 + p)])
    lo = diag - lenB if diag > lenB else 0
    hi = diag if diag < lenA else lenA
    while lo < hi:
        mid = (lo + hi) >> 1
        if at(mid) <= at(s + diag - 1 - mid):
            lo = mid + 1
        else:
            hi = mid
    limA = padded_byte(2 * (l0 + lenA - 1)) + 2
    limB = padded_byte(2 * (l0 + s + lenB - 1)) + 2

    def load(i2, lim):
        o = min(padded_byte(i2), lim)
        assert o % 2 == 0
        return int(row[o // 2])

    ia2, ib2 = 2 * (l0 + lo), 2 * (l0 + s + diag - lo)
    ib0 = ib2
    a, b = load(ia2, limA), load(ib2, limB)
    heads, out, tb = 0, [], False
    for t in range(K):
        heads += ib2
        tb = b < a
        out.append(b if tb else a)
        if t + 1 < K:
            nxt = (ib2 if tb else ia2) + 2
            if tb:
                ib2 = nxt
            else:
                ia2 = nxt
            nv = load(nxt, limB if tb else limA)
            if tb:
                b = nv
            else:
                a = nv
    nb = (ib2 - ib0) // 2 + (1 if tb else 0)
    sum_nb = (heads - K * ib0) // 2
    sum_t = nb * (K - 1) - sum_nb
    cnt = nb * (lenA - lo) - sum_t + nb * (nb - 1) // 2
    return out, cnt


@pytest.mark.parametrize("K,s,lenB,seed", [(32, 2048, 2048, 1), (64, 4096, 4096, 2),
                                           (64, 4096, 1024, 3), (32, 2048, 64 * 32, 4),
                                           (64, 8192, 4096, 5), (32, 4096, 2048, 6)])
def test_merge_level_counts_cross_inversions(K, s, lenB, seed):
    rng = np.random.default_rng(seed)
    lenA = s
    for trial in range(3):
        hi = [40, 2 * (lenA + lenB), 0xFFFE][trial]      # many ties, few, any
        A = np.sort(rng.integers(0, hi // 2 + 1, lenA) * 2)
        B = np.sort(rng.integers(0, hi // 2 + 1, lenB) * 2)
        if trial == 0:
            B[-lenB // 4:] = 0xFFFE                       # padding keys at the end
        l0 = 2 * s                                        # the second run pair of a row
        NR = l0 + s + lenB
        keys = np.concatenate([rng.integers(0, 100, l0) * 2, A, B])
        row = make_row(keys, NR)
        merged, total = [], 0
        for diag in range(0, lenA + lenB, K):
            out, cnt = lane_segment(row, l0, s, lenA, lenB, diag, K)
            merged += out
            total += cnt
        assert merged == sorted(np.concatenate([A, B]).tolist())
        brute = int(np.sum(A[:, None] > B[None, :]))
        assert total == brute, (trial, total, brute)


def test_sentinel_read_stays_in_the_run_pad():
    # a head one past its run reads the first pad slot after the run's last block
    for end in (64, 128, 4096, 4096 + 64):
        lim = padded_byte(2 * (end - 1)) + 2
        assert lim == 2 * (padded(end - 1) + 1)
        assert padded_byte(2 * end) > lim and padded_byte(2 * (end - 1)) < lim
