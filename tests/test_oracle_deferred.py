"""Pins of the oracle's AC-6 with late support registration (AC-3 rounds with
the edge_index cursor first, Sections 4.1 and 8, then the AC-6 propagation of
Section 6.1 from the vertices still live): a hand-worked example, the special
cases that reduce to AC-3 and to plain AC-6, and the literal run against its
closed form on random and deep graphs."""
import numpy as np
import pytest


# 4 -> 0 -> 1 -> 2 (a sink), 3 -> 3 (a self-loop), 4 -> 3.  Levels: 2 at
# step 1, 1 at step 2, 0 at step 3; 3 and 4 stay.  2 has no successor, so it
# is removed before round 1.  Worked by hand:
#   R = 2: round 1 checks 0->1, 1->2, 3->3, 4->0 (4): 1 finds 2 removed and
#          is removed; round 2 re-checks the cursors of 0, 3 and 4 (3
#          re-checks): 0 finds 1 removed and is removed, 3 and 4 join the
#          sets of 3 and 0; taking 0 from Q hands 4 back, which checks 4->3
#          and joins 3 (1).  Total 8, 2 rounds, 3 re-checks.
#   R = 3: rounds 1 and 2 as above without joins (7 checks); round 3
#          re-checks 3->3 and 4->0, finds 0 removed, checks 4->3 (3).  It
#          removes nothing: total 10, 3 rounds, 5 re-checks.
#   R >= 4: round 3 removes nothing, so that is the fixed point, reached by
#          the rounds alone: total 10, 3 rounds, 5 re-checks.
# In every case total - re-checks = 5 = T6 (1 + 1 + 0 checks of the removed
# vertices, 1 + 2 of the live ones).
HAND = [[1], [2], [], [3], [0, 3]]
HAND_WANT = {2: (8, 2, 3), 3: (10, 3, 5), 4: (10, 3, 5), 5: (10, 3, 5), 100: (10, 3, 5)}


@pytest.mark.parametrize("R", sorted(HAND_WANT))
def test_hand_example(orc, gen, R):
    g = gen.from_adjacency(HAND)
    d = orc.ac6_deferred(g, R)
    assert list(d.live) == [0, 0, 0, 1, 1]
    assert (d.edges, d.rounds, d.rechecks) == HAND_WANT[R]
    assert orc.counts_deferred(g, orc.peel(g), R) == HAND_WANT[R]
    assert d.edges - d.rechecks == orc.ac6_seq(g)[1] == 5


def _graphs(gen):
    for seed in range(4):
        for n, m in ((30, 40), (300, 450), (2000, 2600), (3000, 9000)):
            yield gen.uniform(n, m, seed=200 + seed, drop_self=bool(seed % 2))
    # deep: a chain of 400 below a random core, so alpha exceeds every R used
    adj = [[v + 1] for v in range(399)] + [[]]
    rng = np.random.default_rng(5)
    for v in range(400, 700):
        adj.append([int(x) for x in rng.integers(0, 700, 3)])
    yield gen.from_adjacency(adj)


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 8, 33])
def test_literal_run_against_closed_form_and_other_algorithms(orc, gen, R):
    """The literal run keeps the live set of the peeling; its total equals the
    closed form and the AC-6 total after removing the re-checks.  Once R
    reaches alpha it is the Jacobi AC-3 run with the vertices without
    successors removed up front: one round fewer (alpha), and every vertex
    with successors takes part in one round fewer, so one check fewer."""
    for g in _graphs(gen):
        r = orc.peel(g)
        d = orc.ac6_deferred(g, R)
        assert (d.live == r.live).all()
        live6, t6, _ = orc.ac6_seq(g)
        if R <= 1:
            assert (d.edges, d.rechecks) == (t6, 0)
            continue
        assert (d.edges, d.rounds, d.rechecks) == orc.counts_deferred(g, r, R)
        assert d.edges - d.rechecks == t6
        live3, t3, rounds3 = orc.ac3(g, jacobi=True)
        with_succ = int((np.diff(g.row_off) > 0).sum())
        if R >= r.alpha and r.alpha >= 1:
            assert (d.edges, d.rounds) == (t3 - with_succ, rounds3 - 1)
        else:
            assert d.rounds == min(R, max(r.alpha, 1)) and t6 <= d.edges <= t3


def test_no_removal_and_empty(orc, gen):
    # a cycle: round 1 removes nothing, so the run stops after one round
    g = gen.from_adjacency([[1], [2], [0]])
    d = orc.ac6_deferred(g, 5)
    assert (d.edges, d.rounds, d.rechecks) == (3, 1, 0) and list(d.live) == [1, 1, 1]
    # only sinks: all removed before round 1, which finds nothing left
    g = gen.from_adjacency([[], [], []])
    d = orc.ac6_deferred(g, 5)
    assert (d.edges, d.rounds, d.rechecks) == (0, 1, 0) and list(d.live) == [0, 0, 0]
    assert orc.counts_deferred(g, orc.peel(g), 5) == (0, 1, 0)
    # a path into a sink: levels 4, 3, 2, 1; rounds 1, 2, 3 remove 2, 1, 0,
    # round 4 finds the list empty and removes nothing
    g = gen.from_adjacency([[1], [2], [3], []])
    assert orc.counts_deferred(g, orc.peel(g), 8) == (1 + 2 + 3, 4, 0 + 1 + 2)
    d = orc.ac6_deferred(g, 8)
    assert (d.edges, d.rounds, d.rechecks) == (6, 4, 3)
