"""Cross-check: the C oracle against a second writing in plain Python."""
import random

import pytest

import oracle
import pyoracle


@pytest.mark.parametrize("seed", range(6))
def test_cross_random(seed):
    rnd = random.Random(seed)
    for _ in range(500):
        m = rnd.choice([rnd.randint(1, 12), rnd.randint(1, 70), rnd.randint(90, 160)])
        r = "".join(rnd.choice("ACGT") for _ in range(m))
        if rnd.random() < 0.5:
            g = list(r)
            for _ in range(rnd.randint(0, 6)):
                op = rnd.random()
                if not g:
                    break
                i = rnd.randrange(len(g))
                if op < 0.6:
                    g[i] = rnd.choice("ACGT")
                elif op < 0.8:
                    g.insert(i, rnd.choice("ACGT"))
                else:
                    del g[i]
            g = "".join(g)
            g = (g + "".join(rnd.choice("ACGT") for _ in range(m)))[:m]
        else:
            g = "".join(rnd.choice("ACGT") for _ in range(m))
        e = rnd.randint(0, min(m + 2, 20))
        refine = rnd.random() < 0.8
        got = oracle.filter_pair(r, g, 0, e, 0 if refine else oracle.NO_REFINE)
        want = pyoracle.gatekeeper_gpu(r, g, e, refine)
        assert got == want, (r, g, e, refine)
