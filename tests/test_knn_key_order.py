"""The neighbour search's list keys (csrc/orca_kernels.hip, knn_offer): a
candidate's key is the 64-bit pattern (bits(d2) + 2^20) << 32 | (id + 1), with
d2 its float32 squared distance, and two keys are compared as float64 values
(v_min_f64 / v_max_f64 on the patterns).  This pins the arithmetic fact the
search rests on: for every d2 the search can admit (finite, >= 0) and every id
below 2^32 - 1, the pattern is a positive normal double, and comparing the
doubles orders keys exactly by (d2, id).  The empty-slot pattern (+infinity)
is above every key and the padding key 0.0 below, and the minimum / maximum of
two keys is one of the two patterns, bit for bit."""
import numpy as np

BIAS = np.uint64(1 << 20)
EMPTY = np.uint64(0x7FF0000000000000)


def keys(d2, ids):
    hi = d2.astype(np.float32).view(np.uint32).astype(np.uint64) + BIAS
    return (hi << np.uint64(32)) | (ids.astype(np.uint64) + np.uint64(1))


def as_f64(k):
    return np.ascontiguousarray(k, np.uint64).view(np.float64)


def sample_d2(rng, n):
    # squared distances across the whole float32 range a search can admit:
    # zeros, subnormals, ordinary values, values next to the largest finite
    parts = [
        np.zeros(8, np.float32),
        rng.integers(1, 1 << 23, 64, dtype=np.uint32).view(np.float32),  # subnormals
        rng.uniform(0, 50, n).astype(np.float32),
        (rng.uniform(0, 1, 64) * np.float32(3.0e38)).astype(np.float32),
        np.array([np.finfo(np.float32).max, np.finfo(np.float32).tiny], np.float32),
    ]
    d2 = np.concatenate(parts)
    # exact ties in d2 with different ids
    return np.concatenate([d2, d2[: n // 4]])


def test_keys_are_positive_normal_and_ordered_like_tuples():
    rng = np.random.default_rng(3)
    d2 = sample_d2(rng, 4000)
    ids = rng.integers(0, 2**32 - 2, d2.size, dtype=np.uint64)
    k = keys(d2, ids)
    f = as_f64(k)
    assert np.all(np.isfinite(f)) and np.all(f > 0)
    assert np.all(np.abs(f) >= np.finfo(np.float64).tiny)  # no subnormal key
    # order as doubles == order by (d2, id)
    by_double = np.argsort(f, kind="stable")
    by_tuple = np.lexsort((ids, d2.astype(np.float32)))
    assert np.array_equal(f[by_double], f[by_tuple])
    # and the patterns order the same way as unsigned integers
    assert np.array_equal(np.sort(k), k[by_tuple])


def test_empty_and_padding_keys_bracket_every_key():
    rng = np.random.default_rng(4)
    d2 = sample_d2(rng, 500)
    f = as_f64(keys(d2, rng.integers(0, 2**32 - 2, d2.size, dtype=np.uint64)))
    assert np.all(f < as_f64(np.array([EMPTY]))[0])
    assert np.all(f > 0.0)
    assert as_f64(np.array([EMPTY]))[0] == np.inf


def test_min_max_select_an_operand_bit_for_bit():
    rng = np.random.default_rng(5)
    d2 = sample_d2(rng, 1000)
    k = keys(d2, rng.integers(0, 2**32 - 2, d2.size, dtype=np.uint64))
    a, b = k, np.roll(k, 7)
    lo = np.minimum(as_f64(a), as_f64(b)).view(np.uint64)
    hi = np.maximum(as_f64(a), as_f64(b)).view(np.uint64)
    assert np.all((lo == a) | (lo == b)) and np.all((hi == a) | (hi == b))
    assert np.array_equal(lo, np.minimum(a, b)) and np.array_equal(hi, np.maximum(a, b))


def test_insertion_by_min_max_keeps_the_k_smallest():
    """The list update slot_k <- max(slot_{k-1}, min(key, slot_k)), slot 0 <-
    min(key, slot 0), applied to every offered key from a list of +infinity
    (with leading 0.0 padding for K < KMAX), leaves the K smallest keys in
    order in the last K slots."""
    rng = np.random.default_rng(6)
    for kmax, kk in ((16, 16), (16, 5), (10, 10), (10, 1)):
        for _ in range(40):
            n = int(rng.integers(0, 60))
            d2 = rng.uniform(0, 9, n).astype(np.float32)
            if n:
                d2[: n // 5] = d2[0]  # exact ties, ordered by id
            ids = rng.permutation(n).astype(np.uint64)
            f = as_f64(keys(d2, ids)) if n else np.zeros(0)
            best = np.full(kmax, np.inf)
            best[: kmax - kk] = 0.0
            for key in f:
                for s in range(kmax - 1, 0, -1):
                    best[s] = max(best[s - 1], min(key, best[s]))
                best[0] = min(key, best[0])
            want = np.sort(f)[:kk]
            got = best[kmax - kk:]
            got = got[np.isfinite(got)]
            assert np.array_equal(got, want)
            assert np.all(best[: kmax - kk] == 0.0)
