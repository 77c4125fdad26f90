"""Invariants of the filter that hold for every input (checked on random
pairs with hypothesis).  Each pins part of the oracle to a fact that follows
from the method itself rather than from the oracle's code:

P1 identical pair -> estimate 0, accepted for every e
P2 the estimate never grows with e (each extra k only ANDs more masks)
P3 reversing both strings leaves the estimate unchanged (deletion and
   insertion masks swap; vacated fill, amendment and edges are symmetric)
P4 estimate <= 1s in the amended Hamming mask <= m
P5 a read equal to the window moved by delta bases (|delta| <= e) scores at
   most |delta| (the mask for that shift is 0 except its refined positions)
P6 s <= e substitutions pairwise >= 4 apart score at most s (amendment cannot
   bridge a run of >= 3 zeros), so the pair is accepted
P7 refinement only raises bits: estimate with refinement >= estimate without,
   and an accept with refinement implies an accept without
P8 e >= m -> accepted
"""
import random

from hypothesis import given, settings, strategies as st

import oracle

dna = lambda lo, hi: st.text(alphabet="ACGT", min_size=lo, max_size=hi)


@settings(max_examples=400, deadline=None)
@given(dna(1, 120), st.integers(0, 40))
def test_p1_identical(s, e):
    assert oracle.filter_pair(s, s, 0, e) == (oracle.ACCEPT, 0)


@st.composite
def pair(draw, lo=1, hi=80):
    m = draw(st.integers(lo, hi))
    r = draw(dna(m, m))
    mode = draw(st.integers(0, 2))
    if mode == 0:
        g = draw(dna(m, m))
    else:                                   # a few point changes of r
        g = list(r)
        for _ in range(draw(st.integers(0, 4))):
            i = draw(st.integers(0, m - 1))
            g[i] = draw(st.sampled_from("ACGT"))
        g = "".join(g)
    return r, g


@settings(max_examples=300, deadline=None)
@given(pair(), st.integers(0, 12))
def test_p2_monotone_in_e(rg, e):
    r, g = rg
    a0, est0 = oracle.filter_pair(r, g, 0, e)
    a1, est1 = oracle.filter_pair(r, g, 0, e + 1)
    assert est1 <= est0
    if a0 == oracle.ACCEPT:
        assert a1 == oracle.ACCEPT


@settings(max_examples=300, deadline=None)
@given(pair(), st.integers(0, 12))
def test_p3_reversal(rg, e):
    r, g = rg
    assert oracle.filter_pair(r, g, 0, e) == oracle.filter_pair(r[::-1], g[::-1], 0, e)


@settings(max_examples=300, deadline=None)
@given(pair(), st.integers(0, 12))
def test_p4_dominated_by_hamming(rg, e):
    r, g = rg
    _, est, masks = oracle.filter_trace(r, g, 0, e)
    h = sum(masks[0][oracle.STAGE_AMENDED])
    assert est <= h <= len(r)
    # and the estimate is the count of 1s in the AND of the refined masks
    fin = [1] * len(r)
    for slot in masks:
        fin = [a & b for a, b in zip(fin, slot[oracle.STAGE_REFINED])]
    assert est == sum(fin)


@settings(max_examples=300, deadline=None)
@given(st.integers(1, 100), st.integers(-12, 12), st.integers(0, 4), st.randoms())
def test_p5_shift_only(m, delta, extra_e, rnd):
    ref = "".join(rnd.choice("ACGT") for _ in range(m + 40))
    p = 20
    read = ref[p + delta:p + delta + m]
    e = abs(delta) + extra_e
    res, est = oracle.filter_pair(read, ref, p, e)
    assert est <= abs(delta)
    assert res == oracle.ACCEPT


@settings(max_examples=300, deadline=None)
@given(st.integers(1, 150), st.integers(0, 8), st.randoms())
def test_p6_sparse_substitutions(m, s, rnd):
    g = [rnd.choice("ACGT") for _ in range(m)]
    r = list(g)
    positions = []
    for i in rnd.sample(range(m), m):
        if len(positions) == s:
            break
        if all(abs(i - j) >= 4 for j in positions):
            positions.append(i)
    for i in positions:
        r[i] = rnd.choice([b for b in "ACGT" if b != g[i]])
    s_real = len(positions)
    for e in range(s_real, s_real + 3):
        res, est = oracle.filter_pair("".join(r), "".join(g), 0, e)
        assert est <= s_real
        assert res == oracle.ACCEPT


@settings(max_examples=300, deadline=None)
@given(pair(), st.integers(0, 12))
def test_p7_refinement_dominates_gatekeeper(rg, e):
    r, g = rg
    a_gpu, est_gpu = oracle.filter_pair(r, g, 0, e)
    a_gk, est_gk = oracle.filter_pair(r, g, 0, e, oracle.NO_REFINE)
    assert est_gpu >= est_gk
    if a_gpu == oracle.ACCEPT:
        assert a_gk == oracle.ACCEPT


@settings(max_examples=200, deadline=None)
@given(pair(1, 40), st.integers(0, 10))
def test_p8_threshold_at_least_length(rg, extra):
    r, g = rg
    assert oracle.filter_pair(r, g, 0, len(r) + extra)[0] == oracle.ACCEPT


def test_p3_reversal_long_reads():
    rnd = random.Random(11)
    for _ in range(200):
        m = rnd.randint(100, 512)
        r = "".join(rnd.choice("ACGT") for _ in range(m))
        g = list(r)
        for _ in range(rnd.randint(0, 30)):
            g[rnd.randrange(m)] = rnd.choice("ACGT")
        g = "".join(g)
        e = rnd.randint(0, 40)
        assert oracle.filter_pair(r, g, 0, e) == oracle.filter_pair(r[::-1], g[::-1], 0, e)


@settings(max_examples=400, deadline=None)
@given(pair(), st.integers(0, 12), st.sampled_from([0, oracle.NO_REFINE]))
def test_hamming_fastpath_variant(rg, e, base):
    """The Hamming fast path (a variant outside the paper) decides exactly the
    pairs whose count of differing bases is at most e, accepting them with
    that count; every other pair keeps its result without the fast path."""
    r, g = rg
    hd = sum(a != b for a, b in zip(r, g))
    fast = oracle.filter_pair(r, g, 0, e, base | oracle.HAMMING_FASTPATH)
    plain = oracle.filter_pair(r, g, 0, e, base)
    if hd <= e:
        assert fast == (oracle.ACCEPT, hd)
        assert plain[0] == oracle.ACCEPT or plain[1] > hd
    else:
        assert fast == plain
