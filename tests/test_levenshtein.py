"""Ground-truth edit distance: full DP, banded DP, brute force."""
import functools
import itertools
import random

import pytest

import oracle


def brute_force(a, b):
    """Textbook recursive definition (memoised), unit costs."""
    @functools.lru_cache(maxsize=None)
    def d(i, j):
        if i == 0:
            return j
        if j == 0:
            return i
        return min(d(i - 1, j) + 1, d(i, j - 1) + 1, d(i - 1, j - 1) + (a[i - 1] != b[j - 1]))
    return d(len(a), len(b))


def test_known_values():
    assert oracle.levenshtein("", "") == 0
    assert oracle.levenshtein("ACGT", "") == 4
    assert oracle.levenshtein("", "AC") == 2
    assert oracle.levenshtein("ACGT", "ACGT") == 0
    assert oracle.levenshtein("ACGT", "AGT") == 1
    assert oracle.levenshtein("ACGT", "TGCA") == 4
    assert oracle.levenshtein("AAAA", "TTTT") == 4
    assert oracle.levenshtein("GATTACA", "GCATGCT") == 4


@pytest.mark.parametrize("n", range(0, 6))
def test_full_dp_exhaustive_tiny(n):
    strs = ["".join(t) for t in itertools.product("ACG", repeat=n)]
    others = ["".join(t) for k in range(0, 5) for t in itertools.product("AC", repeat=k)]
    for a in strs:
        for b in others:
            assert oracle.levenshtein(a, b) == brute_force(a, b)


def test_banded_matches_full():
    rnd = random.Random(3)
    for _ in range(3000):
        n = rnd.randint(0, 60)
        a = "".join(rnd.choice("ACGT") for _ in range(n))
        b = list(a)
        for _ in range(rnd.randint(0, 12)):
            op = rnd.random()
            if op < 0.5 and b:
                b[rnd.randrange(len(b))] = rnd.choice("ACGT")
            elif op < 0.75:
                b.insert(rnd.randint(0, len(b)), rnd.choice("ACGT"))
            elif b:
                del b[rnd.randrange(len(b))]
        b = "".join(b)
        full = oracle.levenshtein(a, b)
        for cap in (0, 1, 2, 3, 5, 8, 13, 100):
            assert oracle.levenshtein(a, b, cap) == min(full, cap + 1), (a, b, cap)
