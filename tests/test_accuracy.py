"""Accuracy of the filter against edit distance on config 0 (all 10,000
pairs), as the FA/FR definitions of Sec. 4.4 count it: the directions the
method fixes must hold."""
import numpy as np
import pytest

import gen
import oracle

NO_REFINE = 1


@pytest.fixture(scope="module")
def c0():
    ref = gen.c0_reference()
    return ref, gen.c0_pairs(ref)


def counts(ref, ps, e, flags=0):
    a, est = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, e,
                                 flags=flags, n_threads=gen.default_threads())
    lev = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos, e,
                                   n_threads=gen.default_threads()).astype(np.int64)
    return a, est.astype(np.int64), lev


def test_exact_threshold_has_no_errors(c0):
    """e = 0 accepts exactly the pairs with edit distance 0 (read == window)."""
    ref, ps = c0
    a, _, lev = counts(ref, ps, 0)
    assert np.array_equal(a == 1, lev == 0)
    assert np.sum(lev == 0) > 100


@pytest.mark.parametrize("e", [1, 2, 3, 5])
def test_refinement_trades_accepts_for_rejects(c0, e):
    """Refinement only raises estimates (Sec. 3.4): never more false accepts,
    never fewer false rejects than without it, and strictly fewer false
    accepts on this workload."""
    ref, ps = c0
    a, est, lev = counts(ref, ps, e)
    a0, est0, _ = counts(ref, ps, e, NO_REFINE)
    assert np.all(est >= est0)
    fa, fa0 = np.sum((a == 1) & (lev > e)), np.sum((a0 == 1) & (lev > e))
    fr, fr0 = np.sum((a == 0) & (lev <= e)), np.sum((a0 == 0) & (lev <= e))
    assert fa < fa0 and fr >= fr0


@pytest.mark.parametrize("e", [1, 2, 3, 5])
def test_sparse_substitutions_are_accepted(c0, e):
    """The estimate is at most the amended Hamming count, and every pair whose
    read equals its window, or differs only by substitutions at least 4
    positions apart numbering at most e, is accepted (no false reject)."""
    ref, ps = c0
    a, est, lev = counts(ref, ps, e)
    for i in range(0, ps.n_pairs, 7):
        r = np.frombuffer(ps.read(int(ps.pair_read[i])), np.uint8)
        p = int(ps.cand_pos[i])
        g = ref[p:p + len(r)]
        diff = np.nonzero(r != g)[0]
        assert est[i] <= len(r)
        if len(diff) <= e and (len(diff) < 2 or np.min(np.diff(diff)) >= 4):
            assert a[i] == 1 and est[i] <= len(diff), i


@pytest.mark.parametrize("e", [1, 2, 3, 5])
def test_hamming_fastpath_adds_no_false_accept(c0, e):
    """Edit distance never exceeds Hamming distance for equal lengths, so the
    Hamming fast path (a variant outside the paper) cannot add a false accept;
    it only turns rejects into accepts, so it never adds a false reject."""
    ref, ps = c0
    a, _, lev = counts(ref, ps, e)
    ah, _, _ = counts(ref, ps, e, oracle.HAMMING_FASTPATH)
    assert np.sum((ah == 1) & (lev > e)) == np.sum((a == 1) & (lev > e))
    assert np.sum((ah == 0) & (lev <= e)) <= np.sum((a == 0) & (lev <= e))
    assert np.all(ah[a == 1] == 1)
