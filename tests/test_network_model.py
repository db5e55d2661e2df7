"""A CPU model of the half-precision counting network (the pair kernels'
Step 3 for groups of up to one wave), element by element, against a brute
force inversion count: the key layout (rank above a field of tag bits), the
tag epochs, the ascending in-half levels with mirrored first stages, the
level-0 direct count, and from the half stage on the sign patterns and
orientations.  It checks the design, not the GPU code (which the GPU parity
tests compare with the oracle); inputs are small so that the model runs in
seconds."""
import numpy as np
import pytest

BIAS = 0x0400
MAX_FINITE = 0x7BFF


def ilog2(v):
    return v.bit_length() - 1


def half_tag_bits(N):
    # the most tag bits (up to 5) for which padding at rank N with a full
    # field is still a finite half-precision pattern
    t = 1
    while t < 5 and (N + 1) * (2 << t) + BIAS - 1 <= MAX_FINITE:
        t += 1
    return t


class Shape:
    def __init__(self, K, G):
        self.K, self.G = K, G
        self.KV = K // 2
        self.LOGK, self.LOGKV, self.LOGN = ilog2(K), ilog2(K // 2), ilog2(K * G)
        self.N = K * G
        self.T = half_tag_bits(self.N)
        self.kW = 12

    def patterned(self, k):
        # element lane bit lb is physical lane bit lb: bits 0-4 exchange by
        # swizzles under a sign pattern, bit 5 (whole waves) by permlane swaps
        # with plain signs
        return k == self.LOGKV or (k >= self.LOGK and k - self.LOGK != 5)

    def plain(self, k):
        return k >= self.LOGK and not self.patterned(k)

    def epoch_start(self, L):
        if L in (1, self.LOGKV):
            return True
        return (L - 1) % self.T == 0 if L < self.LOGKV else (L - self.LOGKV) % self.T == 0

    def epoch_of(self, L):
        while not self.epoch_start(L):
            L -= 1
        return L

    def pos(self, lane, j, h):
        return (lane << self.LOGK) | (h << self.LOGKV) | j

    def bit(self, lane, j, h, b):
        return (self.pos(lane, j, h) >> b) & 1

    def field(self, S, lane, j, h):
        return (self.pos(lane, j, h) >> S) & ((1 << self.T) - 1)

    def pattern(self, lane, b):
        if b < 0:
            return (0, 0)
        if b == self.LOGKV:
            return (0, 1)
        x = (lane >> (b - self.LOGK)) & 1
        return (x, x)

    def sign_start(self, L, lane, j, h):
        desc = self.bit(lane, j, h, L + 1) if L + 1 < self.LOGN else 0
        return desc ^ (self.bit(lane, j, h, L) if self.patterned(L) else 0)

    def sign_end(self, L, lane, j, h):
        desc = self.bit(lane, j, h, L + 1) if L + 1 < self.LOGN else 0
        return desc ^ h


def value(p):
    mag = p & 0x7FFF
    assert mag <= MAX_FINITE
    return -mag if p & 0x8000 else mag


def fmin(a, b):
    return a if value(a) <= value(b) else b


def fmax(a, b):
    return a if value(a) >= value(b) else b


def network_count(sh, keys, top):
    """Inversions of keys (2 rank, padding 0xFFFE, element e = lane K + r) as
    the network counts them; without the top level, the first half's keys
    must end as BIAS + rank 2^T once field and sign are cleared."""
    K, KV, G, T = sh.K, sh.KV, sh.G, sh.T
    FM = (1 << T) - 1
    # v[lane][j] = [low half, high half]
    v = [[[0, 0] for _ in range(KV)] for _ in range(G)]
    for p in range(G):
        for j in range(KV):
            for h in range(2):
                g = min(int(keys[p * K + h * KV + j]), 2 * sh.N)
                in_half = ((j >> 1) & ((1 << min(T, sh.LOGKV - 1)) - 1)) if sh.LOGKV > 1 else 0
                v[p][j][h] = g * (1 << (T - 1)) + BIAS + in_half
    total = 0
    for p in range(G):                       # level 0: counted, then exchanged
        for j in range(0, KV, 2):
            for h in range(2):
                a, b = v[p][j][h], v[p][j + 1][h]
                total += a > b
                v[p][j][h], v[p][j + 1][h] = min(a, b), max(a, b)
    for L in range(1, sh.LOGN if top else sh.LOGN - 1):
        S = sh.epoch_of(L)
        if L < sh.LOGKV:
            if S == L and L != 1:
                for p in range(G):
                    for j in range(KV):
                        f = (j >> S) & ((1 << min(T, sh.LOGKV - S)) - 1)
                        for h in range(2):
                            v[p][j][h] = (v[p][j][h] & ~FM) | f
            m = (2 << L) - 1
            for p in range(G):
                for j in range(KV):              # mirrored first stage
                    if not (j >> L) & 1:
                        for h in range(2):
                            a, b = v[p][j][h], v[p][j ^ m][h]
                            v[p][j][h], v[p][j ^ m][h] = min(a, b), max(a, b)
                for k in range(L - 1, -1, -1):
                    for j in range(KV):
                        if not (j >> k) & 1:
                            q = j | (1 << k)
                            for h in range(2):
                                a, b = v[p][j][h], v[p][q][h]
                                v[p][j][h], v[p][q][h] = min(a, b), max(a, b)
            acc = 0
            for p in range(G):
                for j in range(KV):
                    for h in range(2):
                        acc += ((v[p][j][h] >> (L - S)) & 1) * (j & m)
            total -= acc
            continue
        for p in range(G):                   # into level L: field and signs
            for j in range(KV):
                for h in range(2):
                    if L == sh.LOGKV:
                        c = sh.field(S, p, j, h) | (sh.sign_start(L, p, j, h) << 15)
                        v[p][j][h] = (v[p][j][h] & ~FM) ^ c
                    else:
                        flip = sh.sign_end(L - 1, p, j, h) ^ sh.sign_start(L, p, j, h)
                        if S == L:
                            v[p][j][h] = (v[p][j][h] & ~FM) ^ (sh.field(S, p, j, h) | flip << 15)
                        else:
                            v[p][j][h] ^= flip << 15
        cur = L if sh.patterned(L) else -1
        for k in range(L, -1, -1):
            want = k if sh.patterned(k) else (-1 if sh.plain(k) else cur)
            if want != cur:
                for p in range(G):
                    a, b = sh.pattern(p, cur), sh.pattern(p, want)
                    for j in range(KV):
                        for h in range(2):
                            v[p][j][h] ^= (a[h] ^ b[h]) << 15
            if k < sh.LOGKV:
                for p in range(G):
                    for j in range(KV):
                        if not (j >> k) & 1:
                            q = j | (1 << k)
                            for h in range(2):
                                a, b = v[p][j][h], v[p][q][h]
                                v[p][j][h], v[p][q][h] = fmin(a, b), fmax(a, b)
            elif k == sh.LOGKV:
                for p in range(G):
                    old = [list(x) for x in v[p]]
                    for j in range(KV):
                        lo, hi = old[j]
                        plo, phi = old[KV - 1 - j]
                        v[p][j] = [fmin(lo, phi ^ 0x8000), fmin(hi, plo ^ 0x8000)]
            else:
                lb = k - sh.LOGK
                old = [[list(x) for x in row] for row in v]
                for p in range(G):
                    q = p ^ (1 << lb)
                    for j in range(KV):
                        for h in range(2):
                            a, b = old[p][j][h], old[q][j][h]
                            if sh.patterned(k):
                                v[p][j][h] = fmin(a, b ^ 0x8000)
                            else:
                                assert (a ^ b) & 0x8000 == 0
                                v[p][j][h] = fmin(a, b) if not (p >> lb) & 1 else fmax(a, b)
            cur = want
        m2s = (2 << L) - 1
        for p in range(G):
            acc = 0
            for j in range(KV):
                t = [(v[p][j][h] >> (L - S)) & 1 for h in range(2)]
                acc += t[0] * (j + (1 << sh.kW)) + t[1] * ((K - 1 - j) + (1 << sh.kW))
            base = (p & ((1 << (L + 1 - sh.LOGK)) - 1)) << sh.LOGK
            rsum, nraw = acc & ((1 << sh.kW) - 1), acc >> sh.kW
            desc = (p >> (L + 1 - sh.LOGK)) & 1 if L + 1 < sh.LOGN else 0
            total -= (m2s - base) * nraw - rsum if desc else base * nraw + rsum
    const = 0
    for L in range(1, sh.LOGN):
        s = 1 << L
        const += (sh.N // (2 * s)) * (s * s + s * (s - 1) // 2)
    if not top:
        s = sh.N // 2
        const -= s * s + s * (s - 1) // 2
        got = sorted(((v[p][j][h] & ~(FM | 0x8000)) - BIAS) >> T
                     for p in range(G // 2) for j in range(KV) for h in range(2))
        assert got == sorted(min(int(k), 2 * sh.N) // 2 for k in keys[:sh.N // 2])
    return total + const


def brute(keys, top):
    x = np.asarray(keys, dtype=np.int64)
    inv = sum(int(np.sum(x[i] > x[i + 1:])) for i in range(len(x)))
    if not top:
        h = len(x) // 2
        inv -= sum(int(np.sum(x[:h] > b)) for b in x[h:])
    return inv


def test_tag_bits():
    assert [half_tag_bits(N) for N in (128, 512, 1024, 2048, 4096, 8192)] == [5, 5, 4, 3, 2, 1]


@pytest.mark.parametrize("K,G", [(4, 8), (8, 8), (16, 8), (8, 4), (16, 16), (32, 8), (4, 64),
                                 (8, 32), (8, 64)])
def test_network_counts_inversions(K, G):
    sh = Shape(K, G)
    N = K * G
    rng = np.random.default_rng(K * 1000 + G)
    for trial in range(4):
        n = N if trial == 0 else int(rng.integers(N // 2 + 1, N + 1))
        if trial == 3:
            r = np.zeros(n, np.int64)                       # one tie group
        else:
            r = rng.integers(0, max(2, n // 3 if trial == 2 else n), n)
        keys = np.full(N, 0xFFFE, np.int64)
        keys[:n] = 2 * r
        for top in (True, False):
            assert network_count(sh, keys, top) == brute(keys, top), (K, G, n, top)
