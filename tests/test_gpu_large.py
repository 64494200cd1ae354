"""Full-size parity on the largest explicit workload: R-MAT scale 26, edge
factor 16 (about 1.07e9 edges).  Generation and the sequential oracle take
about a minute each, so this test has its own time limit."""
import pytest

import graphgen as gg
from gpu_common import check_all, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


@pytest.mark.timeout(900)
def test_config2_explicit_full(ctx):
    say("  generating R-MAT scale 26 ...")
    g = gg.config2_explicit()
    say(f"  rmat26 n={g.n} m={g.m}; oracle and AC-6 ...")
    check_all(ctx, g, algos=(6,), name="rmat26")
