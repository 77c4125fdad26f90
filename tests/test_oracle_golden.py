"""Oracle against hand-derived worked examples (tests/golden/)."""
import pytest

import oracle
from conftest import golden_rows


@pytest.mark.parametrize("row", golden_rows("gk_examples.txt"), ids=lambda r: f"{r[0]}-e{r[4]}-f{r[5]}")
def test_examples(row):
    name, read, ref, pos, e, flags, accept, est = row
    res, got_est = oracle.filter_pair(read, ref, int(pos), int(e), int(flags))
    assert (res, got_est) == (int(accept), int(est)), name


@pytest.mark.parametrize("row", golden_rows("gk_masks.txt"), ids=lambda r: f"{r[0]}-slot{r[5]}")
def test_masks(row):
    name, read, ref, pos, e, slot, raw, amended, refined = row
    _, _, masks = oracle.filter_trace(read, ref, int(pos), int(e))
    got = masks[int(slot)]
    as_str = lambda bits: "".join(str(b) for b in bits)
    assert as_str(got[oracle.STAGE_RAW]) == raw
    assert as_str(got[oracle.STAGE_AMENDED]) == amended
    assert as_str(got[oracle.STAGE_REFINED]) == refined


@pytest.mark.parametrize("row", golden_rows("amend_cases.txt"), ids=lambda r: r[0])
def test_amend_cases(row):
    src, want = row
    got = oracle.amend([int(c) for c in src])
    assert "".join(str(b) for b in got) == want


def test_examples_levenshtein():
    """The Levenshtein distances quoted in the example comments."""
    assert oracle.levenshtein("AACAGGTT", "AACCGGTT") == 1
    assert oracle.levenshtein("GCGTTGCC", "ACGTTGCA") == 2
    assert oracle.levenshtein("ACTGTCAAGT", "ACTGGTCAAG") == 2
    assert oracle.levenshtein("ACGATCCA", "ACGTTGCA") == 2
