"""Oracle unit behaviour: amendment, codes, unknown bases, limits, edges."""
import itertools
import re

import pytest

import oracle


def amend_by_pattern(bits):
    """Second characterisation of amendment: a 0-run of length 1 or 2 that is
    immediately preceded and followed by a 1 (a regular-expression match on
    the unamended string) becomes 1s."""
    s = "".join(map(str, bits))
    return [int(c) for c in re.sub(r"(?<=1)(0{1,2})(?=1)", lambda mo: "1" * len(mo.group(1)), s)]


@pytest.mark.parametrize("m", range(1, 13))
def test_amend_all_masks(m):
    for bits in itertools.product((0, 1), repeat=m):
        assert oracle.amend(list(bits)) == amend_by_pattern(bits), bits


def test_amend_never_clears_and_is_idempotent_on_results():
    for bits in itertools.product((0, 1), repeat=10):
        a = oracle.amend(list(bits))
        assert all(x >= y for x, y in zip(a, bits))


def test_lowercase_is_same_base():
    assert oracle.filter_pair("acgtacgt", "ACGTACGT", 0, 0) == (oracle.ACCEPT, 0)
    assert oracle.filter_pair("ACGTACGT", "acgtaCGT", 0, 1) == (oracle.ACCEPT, 0)


@pytest.mark.parametrize("bad", ["N", "n", "X", "-", "U", "."])
def test_unknown_base_in_read_or_window_passes(bad):
    read = "ACGT" + bad + "ACG"
    assert oracle.filter_pair(read, "ACGTAACG", 0, 0) == (oracle.UNDEFINED, oracle.EST_NONE)
    assert oracle.filter_pair("ACGTAACG", "ACGT" + bad + "ACG", 0, 3) == (oracle.UNDEFINED,
                                                                          oracle.EST_NONE)


def test_unknown_base_outside_window_is_ignored():
    ref = "NNACGTACGTNN"
    assert oracle.filter_pair("ACGTACGT", ref, 2, 0) == (oracle.ACCEPT, 0)
    assert oracle.filter_pair("ACGTACGT", ref, 1, 0)[0] == oracle.UNDEFINED


def test_window_past_end_is_undefined():
    ref = "ACGTACGTAC"
    assert oracle.filter_pair("GTAC", ref, 6, 0) == (oracle.ACCEPT, 0)     # ends exactly at the end
    assert oracle.filter_pair("GTACG", ref, 6, 0) == (oracle.UNDEFINED, oracle.EST_NONE)
    assert oracle.filter_pair("A", ref, 10, 0) == (oracle.UNDEFINED, oracle.EST_NONE)
    assert oracle.filter_pair("A", ref, 11, 0) == (oracle.UNDEFINED, oracle.EST_NONE)


def test_length_limits():
    ref = "A" * 1200
    assert oracle.filter_pair("", ref, 0, 0) == (oracle.INVALID, oracle.EST_NONE)
    assert oracle.filter_pair("A" * 512, ref, 0, 0) == (oracle.ACCEPT, 0)
    assert oracle.filter_pair("A" * 513, ref, 0, 0) == (oracle.INVALID, oracle.EST_NONE)


def test_length_one():
    assert oracle.filter_pair("A", "A", 0, 0) == (oracle.ACCEPT, 0)
    assert oracle.filter_pair("A", "C", 0, 0) == (oracle.REJECT, 1)
    # e >= m: masks with shift >= m are all ones after refinement, H stays
    assert oracle.filter_pair("A", "C", 0, 1) == (oracle.ACCEPT, 1)


def test_e_zero_is_string_equality():
    """With e = 0 the decision reduces to exact matching (textbook string
    equality), whatever amendment does to the Hamming mask."""
    import random
    rnd = random.Random(5)
    for _ in range(3000):
        m = rnd.randint(1, 20)
        r = "".join(rnd.choice("ACGT") for _ in range(m))
        g = r if rnd.random() < 0.3 else "".join(rnd.choice("ACGT") for _ in range(m))
        res, est = oracle.filter_pair(r, g, 0, 0)
        assert (res == oracle.ACCEPT) == (r == g)
        assert (est == 0) == (r == g)


def test_vacated_positions_compare_with_A():
    """Reading: a logical shift of the encoded read fills code 00 ('A'), so a
    vacated position is a mismatch iff the window base there is not 'A'."""
    _, _, m = oracle.filter_trace("CCCC", "ACGT", 0, 1)
    # deletion mask: position 0 vacated, window[0] = 'A' -> 0
    assert m[1][oracle.STAGE_RAW][0] == 0
    # insertion mask: position 3 vacated, window[3] = 'T' -> 1
    assert m[2][oracle.STAGE_RAW][3] == 1


def test_refinement_only_on_shifted_masks():
    _, _, masks = oracle.filter_trace("AAAAAAAA", "AAAAAAAA", 0, 3)
    assert masks[0][oracle.STAGE_REFINED] == [0] * 8                # H never refined
    for k in range(1, 4):
        d = masks[2 * k - 1][oracle.STAGE_REFINED]
        i = masks[2 * k][oracle.STAGE_REFINED]
        assert d == [1] * k + [0] * (8 - k)
        assert i == [0] * (8 - k) + [1] * k


def test_no_refine_flag_keeps_amended_masks():
    _, _, masks = oracle.filter_trace("AAAAAAAA", "AAAAAAAA", 0, 3, oracle.NO_REFINE)
    for slot in range(7):
        assert masks[slot][oracle.STAGE_REFINED] == masks[slot][oracle.STAGE_AMENDED]
