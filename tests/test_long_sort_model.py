"""A CPU model of the long-row pre-pass sort: the row's sort words in blocks
of H (the LDS sort width), each block sorted in LDS in the direction the
next merge level wants (a block with fewer than H samples sorts only the
smallest power of two of words that holds them and is padded on the side
that keeps its direction), then the upper merge levels with their stages of
distance H and more over the whole row and the rest per block.  Checked
against a plain sort for every row length from H + 1 to 4 H, with a small
H; the GPU parity tests run the kernel itself against the oracle."""
import numpy as np

PAD = np.inf


def stages(s, cnt, base, k_first, k_last, j_first):
    k = k_first
    while k <= k_last:
        j = j_first if k == k_first else k >> 1
        while j > 0:
            for i in range(cnt):
                p = i ^ j
                if p > i:
                    up = ((base + i) & k) == 0
                    if (s[i] > s[p]) == up:
                        s[i], s[p] = s[p], s[i]
            j >>= 1
        k <<= 1


def sort_long(x, H):
    n = len(x)
    npow2 = 2 * H
    while npow2 < n:
        npow2 <<= 1
    g = [PAD] * npow2
    for b in range(npow2 // H):
        r = n - b * H
        P = H
        if r < H:
            P = 1
            while P < r:
                P <<= 1
        s = [x[b * H + i] if b * H + i < n else PAD for i in range(P)]
        desc = b % 2 == 1
        stages(s, P, P if desc else 0, 2, P, 1)
        off = H - P if desc else 0
        for i in range(H):
            q = i - off
            g[b * H + i] = s[q] if 0 <= q < P else PAD
    k = 2 * H
    while k <= npow2:
        j = k >> 1
        while j >= H:
            for i in range(npow2):
                p = i ^ j
                if p > i and (g[i] > g[p]) == ((i & k) == 0):
                    g[i], g[p] = g[p], g[i]
            j >>= 1
        for b in range(npow2 // H):
            s = g[b * H:(b + 1) * H]
            stages(s, H, b * H, k, k, H >> 1)
            g[b * H:(b + 1) * H] = s
        k <<= 1
    return g


def test_block_sort_with_partial_last_blocks():
    rng = np.random.default_rng(7)
    H = 16
    for n in range(H + 1, 4 * H + 1):
        x = rng.standard_normal(n).tolist()
        g = sort_long(x, H)
        assert g[:n] == sorted(x), n
        assert all(v == PAD for v in g[n:]), n
