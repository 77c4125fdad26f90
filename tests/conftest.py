import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def golden_rows(name):
    """Non-comment, non-empty rows of a fixture file, split on whitespace."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def gkctx():
    """A libgk context on cuda:0 (GPU tests only; fails loudly without a GPU)."""
    import torch
    from paper_2103_14978_amd import gk
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    torch.cuda.init()
    ctx = gk.gk_create(0)
    yield ctx
    gk.gk_destroy(ctx)
