"""CPU emulation of the integer bookkeeping of the period-blocked
missing-value kernel's history split (uint32 numpy arithmetic, the kernel's
formulas): each share of the history blocks counts its observations per phase
(W_r), sums their block indices per phase (Q_r, packed above W_r in one word),
and keeps the sum over observed rows of the squared block index by parts
(before block b, (2b - 1) times the count so far); the shares are then added in
order, each with the cross term (count of the earlier shares) x ((b1 - 1)^2 -
(b0 - 1)^2) for its blocks [b0, b1).  The result must equal the direct sums
(Eq. 5-6 need W_r, Q_r and sum w_t b_t^2 exactly) for every split, including
histories that end inside a block and shares with no observation."""
import numpy as np
import pytest

COUNT_BITS = 12


def shares(nblk, split):
    return [(nblk * w // split, nblk * (w + 1) // split) for w in range(split)]


def share_sums(ok, F, n, b0, b1):
    """One wave's share: packed per-phase words, count, squared-index sum by parts."""
    P = ok.shape[1]
    acc = np.zeros((F, P), dtype=np.uint32)
    cnt = np.zeros(P, dtype=np.uint32)
    zs = np.zeros(P, dtype=np.uint32)
    for b in range(b0, b1):
        if b > 0:
            zs += np.uint32(2 * b - 1) * cnt
        inc = np.uint32(1 + (b << COUNT_BITS))
        for u in range(F):
            t = b * F + u
            if t >= n:
                break
            o = ok[t].astype(np.uint32)
            acc[u] += o * inc
            cnt += o
    return acc, cnt, zs


def combined(ok, F, n, split):
    nblk = (n + F - 1) // F
    acc = np.zeros((F, ok.shape[1]), dtype=np.uint32)
    cnt = np.zeros(ok.shape[1], dtype=np.uint32)
    zs = np.zeros(ok.shape[1], dtype=np.uint32)
    for b0, b1 in shares(nblk, split):
        a, c, z = share_sums(ok, F, n, b0, b1)
        bw0 = np.uint32(b0 - 1 if b0 > 0 else 0)
        bw1 = np.uint32(b1 - 1)
        weight = bw1 * bw1 - bw0 * bw0
        acc += a
        zs += z + cnt * weight
        cnt += c
    blast = np.uint32((n - 1) // F)
    zsum = blast * blast * cnt - zs  # modulo 2^32, exact below it
    return acc, cnt, zsum


def direct(ok, F, n):
    t = np.arange(n)
    b, u = t // F, t % F
    W = np.stack([ok[u == r].sum(0) for r in range(F)])
    Q = np.stack([(ok[u == r] * b[u == r, None]).sum(0) for r in range(F)])
    Z = (ok * (b[:, None] ** 2)).sum(0)
    return W, Q, ok.sum(0), Z


@pytest.mark.parametrize("F", [12, 23, 24])
@pytest.mark.parametrize("n,miss", [(200, 0.25), (199, 0.4), (97, 0.1), (400, 0.0), (1000, 0.6)])
def test_split_sums_equal_direct_sums(F, n, miss):
    rng = np.random.default_rng(F * 1000 + n)
    P = 257
    ok = rng.random((n, P)) >= miss
    ok[:, 0] = False                      # a pixel with no observation
    ok[: n // 2, 1] = False               # one with none in the first shares
    ok[n // 2:, 2] = False                # one with none in the last shares
    W, Q, C, Z = direct(ok.astype(np.int64), F, n)
    nblk = (n + F - 1) // F
    for split in (1, 2, 4, 8):
        if split > nblk:
            continue
        acc, cnt, zsum = combined(ok, F, n, split)
        np.testing.assert_array_equal(acc & np.uint32((1 << COUNT_BITS) - 1), W)
        np.testing.assert_array_equal(acc >> np.uint32(COUNT_BITS), Q)
        np.testing.assert_array_equal(cnt, C)
        np.testing.assert_array_equal(zsum, Z)


def test_cross_term_is_needed():
    """Without the cross term a split gets the squared-index sum wrong (a
    mutant of the bookkeeping above fails)."""
    F, n = 23, 200
    ok = np.ones((n, 4), dtype=bool)
    nblk = (n + F - 1) // F
    acc = np.zeros((F, 4), dtype=np.uint32)
    cnt = np.zeros(4, dtype=np.uint32)
    zs = np.zeros(4, dtype=np.uint32)
    for b0, b1 in shares(nblk, 4):
        a, c, z = share_sums(ok, F, n, b0, b1)
        acc += a
        zs += z
        cnt += c
    blast = np.uint32((n - 1) // F)
    _, _, _, Z = direct(ok.astype(np.int64), F, n)
    assert not np.array_equal(blast * blast * cnt - zs, Z)
