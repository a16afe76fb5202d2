"""Host check of the bucket ranking that the FP32 one-wave IECM path uses for
its first division (by U): the map floor((U - U_min) * (64 / (U_max - U_min)))
in binary32, clamped to 63 and 0 for a zero or non-finite scale, never
decreases with U, so the rank of a key is the start of its bucket plus its
rank among the bucket's (key, id) words.  Restated here in NumPy binary32 and
compared with the plain (key, id) rank count on ties, signed zeros, subnormal
values and spreads at the limits of the format.  Parity of the kernel itself
is in test_gpu_iecm.py."""
import numpy as np
import pytest

F32 = np.float32
NB = 64


def ordkey(v):
    b = int(np.array([F32(v) + F32(0.0)], dtype=np.float32).view(np.uint32)[0])
    return (~b & 0xFFFFFFFF) if b & 0x80000000 else (b | 0x80000000)


def rank_plain(u, ids):
    k = [(ordkey(x) << 32) | int(i) for x, i in zip(u, ids)]
    return [sum(kk < m for kk in k) for m in k]


def rank_buckets(u, ids):
    n = len(u)
    k = [(ordkey(x) << 32) | int(i) for x, i in zip(u, ids)]
    lo, hi = F32(np.min(u)), F32(np.max(u))
    with np.errstate(all="ignore"):
        scale = F32(F32(NB) / F32(hi - lo))
    if not scale <= np.finfo(np.float32).max:
        scale = F32(0.0)
    b = []
    for x in u:
        with np.errstate(all="ignore"):
            bb = int(F32(F32(F32(x) - lo) * scale)) if scale > 0 else 0
        b.append(min(bb, NB - 1))
    cnt = [0] * NB
    within = []
    for bb in b:
        within.append(cnt[bb])
        cnt[bb] += 1
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    arr = [None] * n
    for i in range(n):
        arr[start[b[i]] + within[i]] = k[i]
    out = []
    for i in range(n):
        s0 = int(start[b[i]])
        out.append(s0 + sum(arr[r] < k[i] for r in range(s0, s0 + cnt[b[i]])))
    return out


def _cases():
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 17, 64, 65, 100, 128):
        yield rng.standard_normal(n).astype(np.float32)
        yield np.full(n, F32(0.5))
        yield rng.choice(np.array([-0.0, 0.0, 1.0, -1.0], dtype=np.float32), n)
        yield (rng.standard_normal(n) * 1e-42).astype(np.float32)  # subnormal
        yield rng.choice(np.array([-3e38, 3e38, 0.0, 1.0], dtype=np.float32), n)  # the spread overflows
        yield (1 + rng.integers(0, 3, n) * F32(1.2e-7)).astype(np.float32)  # neighbours one ulp apart
        yield np.sort(rng.standard_normal(n)).astype(np.float32)[::-1].copy()


@pytest.mark.parametrize("u", list(_cases()), ids=lambda u: f"n{len(u)}")
def test_bucket_rank_equals_plain_rank(u):
    ids = np.random.default_rng(len(u)).permutation(1000)[: len(u)]
    r = rank_buckets(u, ids)
    assert r == rank_plain(u, ids)
    assert sorted(r) == list(range(len(u)))


def test_bucket_map_is_monotone():
    """Consecutive binary32 values across several binades never step back."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        lo, hi = np.sort(rng.standard_normal(2).astype(np.float32) * F32(10.0 ** rng.integers(-3, 4)))
        if hi == lo:
            continue
        scale = F32(F32(NB) / F32(hi - lo))
        x = np.sort(rng.uniform(lo, hi, 4000).astype(np.float32))
        b = np.minimum((((x - lo).astype(np.float32)) * scale).astype(np.float32).astype(np.int64), NB - 1)
        assert np.all(np.diff(b) >= 0)
