"""Every (read, window) pair of length m <= 5 over ACGT, e = 0..4, through the
C oracle's batch driver: invariants P1, P2, P3, P7, P8 hold everywhere, and
the decision at e = 0 is exactly string equality.  Also reports exact
false-accept / false-reject counts over the whole space."""
import itertools

import numpy as np
import pytest

import oracle


def all_pairs(m):
    words = np.array([list(t) for t in itertools.product(b"ACGT", repeat=m)], dtype=np.uint8)
    n = len(words)
    reads = words.reshape(-1)
    read_off = np.arange(n + 1, dtype=np.uint64) * m
    ref = words.reshape(-1)                    # window j sits at j*m
    ri, wi = np.meshgrid(np.arange(n, dtype=np.uint32), np.arange(n, dtype=np.uint32),
                         indexing="ij")
    return words, reads, read_off, ref, ri.reshape(-1), (wi.reshape(-1) * m).astype(np.uint32)


def rev_index(m):
    """Index of the reversed word for every word index (base-4 digits reversed)."""
    idx = np.arange(4 ** m)
    digits = [(idx // 4 ** k) % 4 for k in range(m)]
    return sum(digits[k] * 4 ** (m - 1 - k) for k in range(m))


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_exhaustive(m):
    words, reads, read_off, ref, pr, pos = all_pairs(m)
    n = len(words)
    threads = 8
    res, est = {}, {}
    for e in range(0, 5):
        a, s = oracle.filter_batch(reads, read_off, ref, pr, pos, e, n_threads=threads)
        assert set(np.unique(a)) <= {0, 1}
        res[e], est[e] = a.reshape(n, n), s.reshape(n, n).astype(np.int64)
        a2, s2 = oracle.filter_batch(reads, read_off, ref, pr, pos, e, flags=oracle.NO_REFINE,
                                     n_threads=threads)
        # P7
        assert np.all(est[e] >= s2.reshape(n, n))
        assert np.all(a2.reshape(n, n)[res[e] == 1] == 1)
    eye = np.eye(n, dtype=bool)
    # P1 and the e = 0 decision
    for e in range(5):
        assert np.all(est[e][eye] == 0) and np.all(res[e][eye] == 1)
    assert np.array_equal(res[0] == 1, eye)
    # P2
    for e in range(4):
        assert np.all(est[e + 1] <= est[e])
    # P8
    for e in range(m, 5):
        assert np.all(res[e] == 1)
    # P3: reversing both strings
    rv = rev_index(m)
    for e in range(5):
        assert np.array_equal(est[e], est[e][np.ix_(rv, rv)])


def test_exhaustive_accuracy_m4():
    """Exact false accepts / rejects against Levenshtein over all 4^4 x 4^4
    pairs (reported; the only hard facts asserted are the ones the method
    guarantees: no false reject at lev = 0, no false accept at e = 0)."""
    m = 4
    words, reads, read_off, ref, pr, pos = all_pairs(m)
    lev = oracle.levenshtein_batch(reads, read_off, ref, pr, pos, cap=m, n_threads=8)
    for e in range(0, 4):
        a, _ = oracle.filter_batch(reads, read_off, ref, pr, pos, e, n_threads=8)
        fa = int(np.sum((a == 1) & (lev > e)))
        fr = int(np.sum((a == 0) & (lev <= e)))
        if e == 0:
            assert fa == 0 and fr == 0
        assert np.all(a[lev == 0] == 1)
        print(f"m={m} e={e}: FA={fa} FR={fr} of {len(a)}")
