"""Host-side counters the benchmark compares with the GPU statistics, checked
against plain per-vertex loops written from their definitions."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_sweep_counts_by_loop(gen):
    import bench
    for seed in range(3):
        g = gen.uniform(2000, 2600, seed=seed + 20)
        deg = np.diff(g.row_off)
        checks = joins = cas = members = 0
        for v in range(g.n):
            succ = g.col[g.row_off[v]:g.row_off[v + 1]]
            if succ.size == 0:
                continue
            k = next((i for i, w in enumerate(succ) if deg[w] > 0), -1)
            if k < 0:
                checks += succ.size
                cas += 1
            else:
                checks += k + 1
                joins += 1
                members += k == succ.size - 1
        assert bench.sweep_counts(g) == (checks, joins, cas, members)
        # the chunked count is the same for any chunk size
        assert bench.sweep_counts(g, chunk=97) == (checks, joins, cas, members)


def test_two_sided_sweep_counts_by_loop(gen):
    import bench
    for seed in range(3):
        g = gen.uniform(3000, 3600, seed=seed)
        rro, rcol = gen.transpose(g)
        deg, indeg = np.diff(g.row_off), np.diff(rro)
        alive0 = (deg > 0) & (indeg > 0)
        checks = joins = cas = members = 0
        for v in range(g.n):
            if not alive0[v]:
                continue
            out = g.col[g.row_off[v]:g.row_off[v + 1]]
            k = next((i for i, w in enumerate(out) if alive0[w]), -1)
            if k < 0:
                checks += out.size
                cas += 1
                continue
            checks += k + 1
            joins += 1
            ins = rcol[rro[v]:rro[v + 1]]
            k2 = next((i for i, u in enumerate(ins) if alive0[u]), -1)
            if k2 < 0:
                checks += ins.size
                cas += 1
                continue
            checks += k2 + 1
            joins += 1
            members += k == out.size - 1
        assert bench.two_sided_sweep_counts(g, rro, rcol) == (checks, joins, cas, members,
                                                               int(alive0.sum()))


def test_step_stats():
    import bench
    st = bench.step_stats([1.0, 2.0, 3.0, 4.0])
    assert st["n"] == 4 and st["median_ms"] == 2.5 and st["mean_ms"] == 2.5
    lo, hi = st["ci95_ms"]
    assert lo < 2.5 < hi and abs((hi - lo) / 2 - 1.96 * np.std([1, 2, 3, 4], ddof=1) / 2) < 1e-12
