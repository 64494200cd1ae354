/*
 * oracle.c -- plain, slow, sequential CPU reference for graph trimming.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU baseline
 * of the benchmark use it.  It shares no code with the GPU path.
 *
 * Paper: "Efficient Parallel Graph Trimming by Arc-Consistency"
 * (arXiv 2107.12720).  Section references below are to that paper.
 *
 * Conventions: status LIVE = 1 / DEAD = 0 (stored in `live`), levels are
 * 1-based peeling steps (0 for vertices that stay live).
 *
 *   or_peel        the trimmed graph (Def. Trimmed Graph, Section 2) and the
 *                  peeling step of every removed vertex (Def. of alpha,
 *                  Section 2.4), by out-degree counters over G^T as in the
 *                  sequential AC-4-based algorithm (Section 5.1), with the
 *                  counters taken from CSR offsets (AC4Trim*, Section 9.3),
 *                  processing one peeling step after the other (FIFO).
 *   or_ac6_seq     the sequential AC-6-based algorithm (Section 6.1) run
 *                  literally, counting every status check of a successor.
 *   or_ac3_jacobi  the AC-3-based algorithm (Section 4.1) with the
 *                  edge_index cursor of Section 8, statuses read as they were
 *                  at the start of each repetition (round).
 *   or_ac3_inplace the same with statuses updated in place during a sweep
 *                  (the literal sequential schedule, vertices in id order).
 *   or_ac6_deferred  AC-3 rounds first, then AC-6 from the vertices still
 *                  LIVE (supporting sets registered only for them), run
 *                  literally; or_counts_deferred its totals in closed form.
 *   or_counts      closed forms of the traversed-edge totals for AC-6,
 *                  AC-4 (with and without the * initialisation) and AC-3.
 *   or_implicit_csr  materialises the hash-generated graph (Section 2.1,
 *                  implicit graphs) with this file's own SplitMix64.
 *   or_batch_peel  or_peel on every graph of a packed batch, one graph per
 *                  thread.
 *   or_peel_preset / or_counts_preset  or_peel and or_counts with some
 *                  vertices set to DEAD before trimming starts (the vertex
 *                  sampling of the scalability experiments, Section 9).
 *   or_peel2       two-sided trimming: the improvement of Section 4.1 that
 *                  also requires at least one live predecessor (the in-degree
 *                  check over G^T), by two counters per vertex.
 *   or_counts2     traversed-edge totals of the two-sided AC-4 algorithm and
 *                  the schedule-independent part of the two-sided AC-6 one.
 *   or_ac3_jacobi2 / or_counts3two  the AC-3 rounds with the same two-sided
 *                  constraint, run literally, and the closed form of their
 *                  traversed-edge total from or_peel2's levels.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ----------------------------------------------------------------- peel */
/*
 * Removes, one peeling step after the other, every vertex whose live
 * out-degree is zero.  cnt[v] starts at |v.post| (CSR offsets, duplicates and
 * self-loops included).  A removed w decrements cnt[u] once per edge u->w,
 * found through this function's own transposed graph.  A self-loop keeps
 * cnt[v] >= 1, so such a v is never removed.
 *
 * Outputs: live[v] (1 LIVE, 0 DEAD), level[v] (peeling step, 0 if live),
 * order[0 .. n_dead) (removal order: non-decreasing level).
 * stats[0] = alpha (max level), stats[1] = n_live, stats[2] = reverse edges
 * traversed during propagation.  Returns n_dead, or -1 on allocation failure.
 */
int64_t or_peel(int32_t n, const int32_t *row_off, const int32_t *col, uint8_t *live,
                int32_t *level, int32_t *order, int64_t *stats) {
    int64_t m = row_off[n];
    int64_t *pre_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *pre = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *cnt = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!pre_off || !pre || !fill || !cnt) {
        free(pre_off); free(pre); free(fill); free(cnt);
        return -1;
    }
    /* G^T by counting the in-degree of every vertex */
    for (int64_t e = 0; e < m; ++e) pre_off[col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) pre_off[v + 1] += pre_off[v];
    memcpy(fill, pre_off, ((size_t)n + 1) * sizeof(int64_t));
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) pre[fill[col[e]]++] = u;

    int64_t qh = 0, qt = 0;
    for (int32_t v = 0; v < n; ++v) {
        cnt[v] = row_off[v + 1] - row_off[v];
        live[v] = 1;
        level[v] = 0;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (cnt[v] == 0) {
            live[v] = 0;
            level[v] = 1;
            order[qt++] = v;
        }
    }
    int64_t rev = 0;
    int32_t alpha = qt > 0 ? 1 : 0;
    while (qh < qt) {
        int32_t w = order[qh++];
        for (int64_t k = pre_off[w]; k < pre_off[w + 1]; ++k) {
            int32_t u = pre[k];
            ++rev;
            cnt[u] -= 1;
            if (cnt[u] == 0 && live[u]) {
                live[u] = 0;
                level[u] = level[w] + 1;
                if (level[u] > alpha) alpha = level[u];
                order[qt++] = u;
            }
        }
    }
    stats[0] = alpha;
    stats[1] = n - qt;
    stats[2] = rev;
    free(pre_off); free(pre); free(fill); free(cnt);
    return qt;
}

/* ------------------------------------------------------------ AC-6 (seq) */
/*
 * Sequential AC-6-based trimming (Section 6.1).  Each vertex keeps a cursor
 * into its successor list; DoPost(v) checks successors from the cursor on,
 * and the first LIVE one w becomes v's support: v joins w.S and the cursor
 * moves past w (the edge is removed from v.post).  With no LIVE successor v
 * becomes DEAD and enters Q; each w taken from Q hands every member of w.S
 * back to DoPost.  Every status check of a successor counts as one traversed
 * edge.  S sets are singly linked lists (sh = head, sn = next).
 *
 * stats[0] = traversed edges, stats[1] = n_live, stats[2] = |Q| high-water.
 */
static int64_t ac6_dopost(int32_t v, const int32_t *row_off, const int32_t *col, uint8_t *live,
                          int64_t *cur, int32_t *sh, int32_t *sn, int32_t *Q, int64_t *qt) {
    int64_t checked = 0;
    int64_t end = row_off[v + 1];
    while (cur[v] < end) {
        int32_t w = col[cur[v]];
        cur[v] += 1;
        checked += 1;
        if (live[w]) {
            sn[v] = sh[w];
            sh[w] = v;
            return checked;
        }
    }
    live[v] = 0;
    Q[(*qt)++] = v;
    return checked;
}

int64_t or_ac6_seq(int32_t n, const int32_t *row_off, const int32_t *col, uint8_t *live,
                   int64_t *stats) {
    int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *sh = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *sn = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *Q = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!cur || !sh || !sn || !Q) {
        free(cur); free(sh); free(sn); free(Q);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) {
        live[v] = 1;
        sh[v] = -1;
        cur[v] = row_off[v];
    }
    int64_t edges = 0, hw = 0, n_dead = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t qh = 0, qt = 0;
        edges += ac6_dopost(v, row_off, col, live, cur, sh, sn, Q, &qt);
        while (qh < qt) {
            if (qt - qh > hw) hw = qt - qh;
            int32_t w = Q[qh++];
            n_dead += 1;
            while (sh[w] >= 0) {
                int32_t u = sh[w];
                sh[w] = sn[u];               /* w.S := w.S \ {u} */
                edges += ac6_dopost(u, row_off, col, live, cur, sh, sn, Q, &qt);
            }
        }
    }
    stats[0] = edges;
    stats[1] = n - n_dead;
    stats[2] = hw;
    free(cur); free(sh); free(sn); free(Q);
    return edges;
}

/* ------------------------------------------------------------ AC-3 (seq) */
/*
 * AC-3-based trimming (Section 4.1) with the edge_index cursor (Section 8):
 * repeat rounds until no vertex changes.  In a round every LIVE vertex v
 * scans from its cursor; a successor that is DEAD is skipped for good (the
 * cursor moves past it), the first non-DEAD successor ends the scan and is
 * checked again next round.  A vertex whose scan reaches the end becomes
 * DEAD.  Every successor check counts as one traversed edge.
 *
 * or_ac3_jacobi reads the status every vertex had at the start of the round
 * (dround[w] < r means "removed in an earlier round"), or_ac3_inplace reads
 * the current status (vertices in id order, removals visible at once).
 * stats[0] = traversed edges, stats[1] = rounds, stats[2] = n_live.
 */
static int64_t ac3_run(int32_t n, const int32_t *row_off, const int32_t *col, uint8_t *live,
                       int64_t *stats, int jacobi) {
    int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *dround = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!cur || !dround) { free(cur); free(dround); return -1; }
    const int64_t NEVER = INT64_MAX;
    for (int32_t v = 0; v < n; ++v) {
        live[v] = 1;
        cur[v] = row_off[v];
        dround[v] = NEVER;
    }
    int64_t edges = 0, rounds = 0, n_live = n;
    int change = 1;
    while (change) {
        change = 0;
        rounds += 1;
        for (int32_t v = 0; v < n; ++v) {
            if (!live[v]) continue;
            int64_t end = row_off[v + 1];
            int found = 0;
            while (cur[v] < end) {
                int32_t w = col[cur[v]];
                edges += 1;
                int dead = jacobi ? (dround[w] < rounds) : !live[w];
                if (!dead) { found = 1; break; }
                cur[v] += 1;
            }
            if (!found) {
                live[v] = 0;
                dround[v] = rounds;
                n_live -= 1;
                change = 1;
            }
        }
    }
    stats[0] = edges;
    stats[1] = rounds;
    stats[2] = n_live;
    free(cur); free(dround);
    return edges;
}
int64_t or_ac3_jacobi(int32_t n, const int32_t *row_off, const int32_t *col, uint8_t *live,
                      int64_t *stats) {
    return ac3_run(n, row_off, col, live, stats, 1);
}
int64_t or_ac3_inplace(int32_t n, const int32_t *row_off, const int32_t *col, uint8_t *live,
                       int64_t *stats) {
    return ac3_run(n, row_off, col, live, stats, 0);
}

/* ------------------------------------------- AC-6, supports registered late */
/*
 * A combination of the two algorithms above, for graphs that are shallow
 * (small alpha): the first R-1 repetitions are AC-3 rounds with the
 * edge_index cursor (statuses as at the start of each round, as in
 * or_ac3_jacobi), in which no vertex joins a supporting set.  Vertices
 * without successors are DEAD before the first round (as during the first
 * DoPost sweep of the AC-6 algorithm, which the first round is), so a vertex
 * of peeling level l >= 2 is removed in round l - 1.  If a round removes
 * nothing, the fixed point is reached and the run stops there.
 * Otherwise round R is one more such round in which every vertex still LIVE
 * re-checks its cursor, scans on past successors removed before round R, and
 * joins the supporting set of the successor it stops at (Section 6.1) -- or
 * becomes DEAD and enters Q if there is none.  From then on the AC-6
 * propagation runs as in or_ac6_seq: every w taken from Q hands the members
 * of w.S back to DoPost, which resumes after their cursor.  R <= 1 is the
 * plain AC-6 algorithm.
 *
 * stats[0] = traversed edges (every status check of a successor, the
 * cursor re-checks of rounds 2.. included), stats[1] = rounds run,
 * stats[2] = n_live, stats[3] = cursor re-checks = entries of the live lists
 * of rounds 2.. (vertices still LIVE at the start of such a round).
 */
int64_t or_ac6_deferred(int32_t n, const int32_t *row_off, const int32_t *col, int32_t R,
                        uint8_t *live, int64_t *stats) {
    int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *dround = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *sh = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *sn = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *Q = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!cur || !dround || !sh || !sn || !Q) {
        free(cur); free(dround); free(sh); free(sn); free(Q);
        return -1;
    }
    const int64_t NEVER = INT64_MAX;
    int64_t edges = 0, rechecks = 0, rounds = 0, n_live = n;
    for (int32_t v = 0; v < n; ++v) {
        live[v] = 1;
        cur[v] = row_off[v];
        dround[v] = NEVER;
        sh[v] = -1;
        if (row_off[v + 1] == row_off[v]) {   /* removed before round 1 */
            live[v] = 0;
            dround[v] = 0;
            n_live -= 1;
        }
    }
    if (R < 1) R = 1;
    int change = 1;
    /* rounds 1 .. R-1: no supporting sets */
    while (change && rounds < R - 1) {
        change = 0;
        rounds += 1;
        for (int32_t v = 0; v < n; ++v) {
            if (!live[v]) continue;
            if (rounds > 1) rechecks += 1;
            int64_t end = row_off[v + 1];
            int found = 0;
            while (cur[v] < end) {
                edges += 1;
                if (dround[col[cur[v]]] >= rounds) { found = 1; break; }
                cur[v] += 1;
            }
            if (!found) {
                live[v] = 0;
                dround[v] = rounds;
                n_live -= 1;
                change = 1;
            }
        }
    }
    if (change) {
        /* round R: the same check, and the survivors join */
        rounds += 1;
        int64_t qh = 0, qt = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (!live[v]) continue;
            if (rounds > 1) rechecks += 1;
            int64_t end = row_off[v + 1];
            int found = 0;
            while (cur[v] < end) {
                int32_t w = col[cur[v]];
                edges += 1;
                if (dround[w] >= rounds) {
                    sn[v] = sh[w];
                    sh[w] = v;
                    found = 1;
                    break;
                }
                cur[v] += 1;
            }
            if (!found) Q[qt++] = v;   /* removed in round R */
        }
        /* statuses of round R's removals change only now, so that round R
           read those of its start */
        for (int64_t i = 0; i < qt; ++i) {
            live[Q[i]] = 0;
            dround[Q[i]] = rounds;
            n_live -= 1;
        }
        /* the AC-6 propagation: a member handed back resumes after its
           cursor with the current statuses */
        while (qh < qt) {
            int32_t w = Q[qh++];
            while (sh[w] >= 0) {
                int32_t u = sh[w];
                sh[w] = sn[u];
                int64_t end = row_off[u + 1];
                int found = 0;
                for (cur[u] += 1; cur[u] < end; cur[u] += 1) {
                    int32_t x = col[cur[u]];
                    edges += 1;
                    if (live[x]) {
                        sn[u] = sh[x];
                        sh[x] = u;
                        found = 1;
                        break;
                    }
                }
                if (!found) {
                    live[u] = 0;
                    n_live -= 1;
                    Q[qt++] = u;
                }
            }
        }
    }
    stats[0] = edges;
    stats[1] = rounds;
    stats[2] = n_live;
    stats[3] = rechecks;
    free(cur); free(dround); free(sh); free(sn); free(Q);
    return edges;
}

/* --------------------------------------------------------- closed forms */
/*
 * Traversed-edge totals from the final live set and the peeling levels
 * (alpha = max level).  fl(v) = index of the first LIVE successor of a live v.
 *   out[0] T6   = sum_dead deg(v) + sum_live (fl(v) + 1)
 *   out[1] T4*  = sum_dead indeg(w)          (propagation over G^T)
 *   out[2] T4   = m + T4*                    (counters found by traversal)
 *   out[3] T3J  = sum_dead (deg(v) + level(v) - 1) + sum_live (fl(v) + alpha + 1)
 *   out[4] rounds of the Jacobi AC-3 = alpha + 1
 *   out[5] T6min = sum_dead deg(v) + n_live  (no successor order does better)
 *   out[6] m, out[7] n_live
 * Returns 0, or -(v+1) for a live vertex without a live successor.
 */
int64_t or_counts(int32_t n, const int32_t *row_off, const int32_t *col, const uint8_t *live,
                  const int32_t *level, int32_t alpha, int64_t *out) {
    int64_t m = row_off[n];
    int64_t *indeg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!indeg) return -1;
    for (int64_t e = 0; e < m; ++e) indeg[col[e]]++;
    int64_t t6 = 0, t4s = 0, t3 = 0, t6min = 0, n_live = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = row_off[v], e = row_off[v + 1], deg = e - b;
        if (live[v]) {
            int64_t fl = -1;
            for (int64_t k = b; k < e; ++k)
                if (live[col[k]]) { fl = k - b; break; }
            if (fl < 0) { free(indeg); return -((int64_t)v + 1); }
            t6 += fl + 1;
            t3 += fl + (int64_t)alpha + 1;
            t6min += 1;
            n_live += 1;
        } else {
            t6 += deg;
            t4s += indeg[v];
            t3 += deg + (int64_t)level[v] - 1;
            t6min += deg;
        }
    }
    out[0] = t6;
    out[1] = t4s;
    out[2] = m + t4s;
    out[3] = t3;
    out[4] = (int64_t)alpha + 1;
    out[5] = t6min;
    out[6] = m;
    out[7] = n_live;
    free(indeg);
    return 0;
}

/*
 * Closed form of or_ac6_deferred's totals for R >= 2, from the final live
 * set and the peeling levels.  Vertices without successors (level 1) are
 * removed before round 1 and check nothing.  In round r a vertex's cursor
 * moves past the successors of level <= r, so a vertex of level l >= 2 takes
 * part in k(v) = min(R, l - 1) rounds: it checks its cursor edge once in
 * each and every other edge once, deg(v) + k(v) - 1 edges; a live one takes
 * part in all rounds run, K = min(R, max(alpha, 1)), and checks
 * fl(v) + K edges:
 *   out[0] T = sum_{dead, deg > 0} (deg(v) + k(v) - 1) + sum_live (fl(v) + K)
 *   out[1] rounds = K
 *   out[2] re-checks = sum_{dead, deg > 0} (k(v) - 1) + sum_live (K - 1)
 * so that T - re-checks is the AC-6 total T6.
 * Returns 0, or -(v+1) for a live vertex without a live successor.
 */
int64_t or_counts_deferred(int32_t n, const int32_t *row_off, const int32_t *col,
                           const uint8_t *live, const int32_t *level, int32_t alpha, int32_t R,
                           int64_t *out) {
    const int64_t a = alpha > 1 ? alpha : 1;
    const int64_t rounds = a < R ? a : R;
    int64_t t = 0, re = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = row_off[v], e = row_off[v + 1];
        if (live[v]) {
            int64_t fl = -1;
            for (int64_t k = b; k < e; ++k)
                if (live[col[k]]) { fl = k - b; break; }
            if (fl < 0) return -((int64_t)v + 1);
            t += fl + rounds;
            re += rounds - 1;
        } else if (e > b) {
            int64_t k = (int64_t)level[v] - 1 < R ? (int64_t)level[v] - 1 : R;
            t += (e - b) + k - 1;
            re += k - 1;
        }
    }
    out[0] = t;
    out[1] = rounds;
    out[2] = re;
    return 0;
}

/* ------------------------------------------------------ implicit graphs */
/*
 * The hash-generated graph G = (V, POST): n = 2^log2n, fin() is the
 * SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA 2014).
 *   deg(v) = 0                       if fin(seed ^ TZ ^ (v<<8)) < zero_thr
 *          = 1 + #{j<255 : fin(seed ^ TD ^ (v<<8)) >= table[j]}   otherwise
 *   POST(v)[i] = fin(seed ^ TN ^ ((v<<8) | i)) & (n-1),  0 <= i < deg(v)
 * Pass col == NULL to fill row_off only.  Returns m.
 */
static inline uint64_t or_fin(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}
uint64_t or_fin64(uint64_t z) { return or_fin(z); }

#define OR_TZ 0x5A45524F00000000ULL
#define OR_TD 0x4445470000000000ULL
#define OR_TN 0x4E42520000000000ULL

int32_t or_implicit_deg(uint64_t seed, uint64_t zero_thr, const uint64_t *table, uint64_t v) {
    if (or_fin(seed ^ OR_TZ ^ (v << 8)) < zero_thr) return 0;
    uint64_t u = or_fin(seed ^ OR_TD ^ (v << 8));
    int32_t d = 1;
    for (int j = 0; j < 255; ++j)
        if (u >= table[j]) d += 1;
    return d;
}
int32_t or_implicit_nbr(uint64_t seed, int log2n, uint64_t v, uint64_t i) {
    uint64_t mask = (log2n >= 64) ? ~0ULL : ((1ULL << log2n) - 1);
    return (int32_t)(or_fin(seed ^ OR_TN ^ ((v << 8) | i)) & mask);
}

/* Three plain passes: every degree (one thread per vertex range), the
 * offsets by a running sum, then every successor list.  The passes only
 * split the loop over v between threads; each value is the formula above. */
int64_t or_implicit_csr(int log2n, uint64_t seed, uint64_t zero_thr, const uint64_t *table,
                        int32_t *row_off, int32_t *col) {
    int64_t n = (int64_t)1 << log2n;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v)
        row_off[v + 1] = or_implicit_deg(seed, zero_thr, table, (uint64_t)v);
    int64_t e = 0;
    row_off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        e += row_off[v + 1];
        row_off[v + 1] = (int32_t)e;
    }
    if (col) {
        #pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < n; ++v)
            for (int32_t i = 0; i < row_off[v + 1] - row_off[v]; ++i)
                col[row_off[v] + i] = or_implicit_nbr(seed, log2n, (uint64_t)v, (uint64_t)i);
    }
    return e;
}

/* --------------------------------------------------------------- batches */
/*
 * or_peel on each graph of a packed batch: graph g owns vertices
 * [vbase[g], vbase[g+1]); row_off is absolute into col; col holds graph-local
 * ids.  live is indexed by global vertex id.  out[g] = n_live of graph g,
 * out[G + g] = alpha of graph g.  One graph per thread.
 */
int64_t or_batch_peel(int64_t G, const int64_t *vbase, const int32_t *row_off, const int32_t *col,
                      uint8_t *live, int64_t *out, int nthreads) {
    int64_t fail = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    (void)nthreads;
#endif
    #pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(+ : fail)
    for (int64_t g = 0; g < G; ++g) {
        int32_t n = (int32_t)(vbase[g + 1] - vbase[g]);
        const int32_t *ro = row_off + vbase[g];
        int32_t e0 = ro[0];
        int32_t *lro = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
        int32_t *lv = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
        int32_t *ord = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
        if (!lro || !lv || !ord) { fail += 1; free(lro); free(lv); free(ord); continue; }
        for (int32_t v = 0; v <= n; ++v) lro[v] = ro[v] - e0;
        int64_t st[3];
        if (or_peel(n, lro, col + e0, live + vbase[g], lv, ord, st) < 0) fail += 1;
        out[g] = st[1];
        out[G + g] = st[0];
        free(lro); free(lv); free(ord);
    }
    return fail ? -1 : 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------- two-sided */
/*
 * Two-sided trimming (Section 4.1, first improvement: with G^T in memory a
 * vertex must also keep an incoming edge from a live vertex).  Removes, one
 * peeling step after the other, every vertex whose live out-degree or live
 * in-degree is zero.  cout[v] starts at |v.post|, cin[v] at |v.pre| (both
 * counted from offsets; duplicates and self-loops included).  A removed w
 * decrements cout[u] once per edge u->w and cin[x] once per edge w->x.
 *
 * Outputs as for or_peel; stats[0] = number of peeling steps, stats[1] =
 * n_live, stats[2] = edges walked during propagation (both directions).
 */
int64_t or_peel2(int32_t n, const int32_t *row_off, const int32_t *col, uint8_t *live,
                 int32_t *level, int32_t *order, int64_t *stats) {
    int64_t m = row_off[n];
    int64_t *pre_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *pre = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *cout = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *cin = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!pre_off || !pre || !fill || !cout || !cin) {
        free(pre_off); free(pre); free(fill); free(cout); free(cin);
        return -1;
    }
    for (int64_t e = 0; e < m; ++e) pre_off[col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) pre_off[v + 1] += pre_off[v];
    memcpy(fill, pre_off, ((size_t)n + 1) * sizeof(int64_t));
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) pre[fill[col[e]]++] = u;

    int64_t qh = 0, qt = 0;
    for (int32_t v = 0; v < n; ++v) {
        cout[v] = row_off[v + 1] - row_off[v];
        cin[v] = pre_off[v + 1] - pre_off[v];
        live[v] = 1;
        level[v] = 0;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (cout[v] == 0 || cin[v] == 0) {
            live[v] = 0;
            level[v] = 1;
            order[qt++] = v;
        }
    }
    int64_t walked = 0;
    int32_t steps = qt > 0 ? 1 : 0;
    while (qh < qt) {
        int32_t w = order[qh++];
        /* w no longer supports its predecessors ... */
        for (int64_t k = pre_off[w]; k < pre_off[w + 1]; ++k) {
            int32_t u = pre[k];
            ++walked;
            cout[u] -= 1;
            if (cout[u] == 0 && live[u]) {
                live[u] = 0;
                level[u] = level[w] + 1;
                if (level[u] > steps) steps = level[u];
                order[qt++] = u;
            }
        }
        /* ... nor its successors */
        for (int64_t k = row_off[w]; k < row_off[w + 1]; ++k) {
            int32_t x = col[k];
            ++walked;
            cin[x] -= 1;
            if (cin[x] == 0 && live[x]) {
                live[x] = 0;
                level[x] = level[w] + 1;
                if (level[x] > steps) steps = level[x];
                order[qt++] = x;
            }
        }
    }
    stats[0] = steps;
    stats[1] = n - qt;
    stats[2] = walked;
    free(pre_off); free(pre); free(fill); free(cout); free(cin);
    return qt;
}

/*
 * Totals of the two-sided algorithms for a given final live set, with G^T as
 * (rrow_off, rcol) in the order the in-side scans use.  fl_out(v) / fl_in(v)
 * = index of the first LIVE successor / predecessor of a live v.
 *   out[0] live part of two-sided AC-6 = sum_live (fl_out + 1 + fl_in + 1):
 *          a live vertex's final supports are its first finally-live
 *          neighbours on each side, whatever the schedule
 *   out[1] least checks of the removed vertices = sum over removed vertices
 *          with both degrees positive of min(deg, indeg): such a vertex dies
 *          only after one side's scan has passed its whole list
 *   out[2] most checks of the removed vertices = the same sum of deg + indeg
 *   out[3] two-sided AC-4 = sum_dead (deg + indeg): every removed vertex
 *          walks both of its lists once
 *   out[4] n_live
 * Returns 0, or -(v+1) for a live vertex without a live neighbour on a side.
 */
int64_t or_counts2(int32_t n, const int32_t *row_off, const int32_t *col,
                   const int32_t *rrow_off, const int32_t *rcol, const uint8_t *live,
                   int64_t *out) {
    int64_t t_live = 0, lo = 0, hi = 0, t4 = 0, n_live = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = row_off[v], e = row_off[v + 1], rb = rrow_off[v], re = rrow_off[v + 1];
        int64_t deg = e - b, indeg = re - rb;
        if (live[v]) {
            int64_t fo = -1, fi = -1;
            for (int64_t k = b; k < e; ++k)
                if (live[col[k]]) { fo = k - b; break; }
            for (int64_t k = rb; k < re; ++k)
                if (live[rcol[k]]) { fi = k - rb; break; }
            if (fo < 0 || fi < 0) return -((int64_t)v + 1);
            t_live += fo + 1 + fi + 1;
            n_live += 1;
        } else {
            t4 += deg + indeg;
            if (deg > 0 && indeg > 0) {
                lo += deg < indeg ? deg : indeg;
                hi += deg + indeg;
            }
        }
    }
    out[0] = t_live;
    out[1] = lo;
    out[2] = hi;
    out[3] = t4;
    out[4] = n_live;
    return 0;
}

/* ------------------------------------------------------ preset removals */
/*
 * or_peel with the vertices marked in preset[] (1 = DEAD from the start)
 * removed before the first step: they get level 0, are propagated first
 * (their predecessors lose them as successors), and are not in order[].
 * Every other vertex follows or_peel: a vertex left without a live successor
 * is removed at 1 + the largest level among its successors.
 * stats[0] = alpha (max level of the vertices removed by trimming), stats[1]
 * = n_live, stats[2] = reverse edges traversed (preset vertices included).
 * Returns the number of vertices removed by trimming (not counting preset).
 */
int64_t or_peel_preset(int32_t n, const int32_t *row_off, const int32_t *col,
                       const uint8_t *preset, uint8_t *live, int32_t *level, int32_t *order,
                       int64_t *stats) {
    int64_t m = row_off[n];
    int64_t *pre_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *pre = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *cnt = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *q = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!pre_off || !pre || !fill || !cnt || !q) {
        free(pre_off); free(pre); free(fill); free(cnt); free(q);
        return -1;
    }
    for (int64_t e = 0; e < m; ++e) pre_off[col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) pre_off[v + 1] += pre_off[v];
    memcpy(fill, pre_off, ((size_t)n + 1) * sizeof(int64_t));
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) pre[fill[col[e]]++] = u;

    int64_t qh = 0, qt = 0, nd = 0;
    for (int32_t v = 0; v < n; ++v) {
        cnt[v] = row_off[v + 1] - row_off[v];
        live[v] = 1;
        level[v] = 0;
    }
    /* the preset removals first (level 0), then the out-degree-0 vertices */
    for (int32_t v = 0; v < n; ++v)
        if (preset[v]) {
            live[v] = 0;
            q[qt++] = v;
        }
    for (int32_t v = 0; v < n; ++v)
        if (!preset[v] && cnt[v] == 0) {
            live[v] = 0;
            level[v] = 1;
            q[qt++] = v;
            order[nd++] = v;
        }
    int64_t rev = 0;
    int32_t alpha = nd > 0 ? 1 : 0;
    while (qh < qt) {
        int32_t w = q[qh++];
        for (int64_t k = pre_off[w]; k < pre_off[w + 1]; ++k) {
            int32_t u = pre[k];
            ++rev;
            cnt[u] -= 1;
            if (cnt[u] == 0 && live[u]) {
                live[u] = 0;
                level[u] = level[w] + 1;
                if (level[u] > alpha) alpha = level[u];
                q[qt++] = u;
                order[nd++] = u;
            }
        }
    }
    stats[0] = alpha;
    stats[1] = n - qt;
    stats[2] = rev;
    free(pre_off); free(pre); free(fill); free(cnt); free(q);
    return nd;
}

/*
 * or_counts for a run with preset removals: preset vertices make no checks
 * of their own (they never run DoPost or a sweep), and a successor that is
 * preset counts as removed from the start.
 *   out[0] T6  = sum_{removed by trimming} deg + sum_live (fl + 1)
 *   out[1] T4* = sum_{all removed, preset included} indeg
 *   out[2] T4  = m + T4*
 *   out[3] T3J = sum_{removed by trimming} (deg + level - 1)
 *                + sum_live (fl + alpha + 1)
 *   out[4] rounds = alpha + 1, out[5] T6min, out[6] m, out[7] n_live
 */
int64_t or_counts_preset(int32_t n, const int32_t *row_off, const int32_t *col,
                         const uint8_t *preset, const uint8_t *live, const int32_t *level,
                         int32_t alpha, int64_t *out) {
    int64_t m = row_off[n];
    int64_t *indeg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!indeg) return -1;
    for (int64_t e = 0; e < m; ++e) indeg[col[e]]++;
    int64_t t6 = 0, t4s = 0, t3 = 0, t6min = 0, n_live = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = row_off[v], e = row_off[v + 1], deg = e - b;
        if (live[v]) {
            int64_t fl = -1;
            for (int64_t k = b; k < e; ++k)
                if (live[col[k]]) { fl = k - b; break; }
            if (fl < 0) { free(indeg); return -((int64_t)v + 1); }
            t6 += fl + 1;
            t3 += fl + (int64_t)alpha + 1;
            t6min += 1;
            n_live += 1;
        } else {
            t4s += indeg[v];
            if (!preset[v]) {
                t6 += deg;
                t3 += deg + (int64_t)level[v] - 1;
                t6min += deg;
            }
        }
    }
    out[0] = t6;
    out[1] = t4s;
    out[2] = m + t4s;
    out[3] = t3;
    out[4] = (int64_t)alpha + 1;
    out[5] = t6min;
    out[6] = m;
    out[7] = n_live;
    free(indeg);
    return 0;
}

/* ------------------------------------------------------ two-sided AC-3 */
/*
 * The AC-3 rounds (Section 4.1) with the constraint that also asks for a live
 * predecessor: two edge_index cursors per vertex (Section 8), one over its
 * successors and one over its predecessors, G^T given as rrow_off / rcol in
 * the order its scans use.  Rounds read the statuses of their start: w counts
 * as removed in round r iff it was removed in an earlier round.  In a round a
 * LIVE vertex scans its successors first and, only if it finds one, its
 * predecessors; a vertex that finds no successor, or then no predecessor, is
 * removed in this round.  Every check of a neighbour counts as one traversed
 * edge.  Outputs live[] and level[] (the removal round, 0 for live vertices);
 * stats[0] = traversed edges, stats[1] = rounds, stats[2] = n_live.  Returns
 * the edges, or -1 on allocation failure.
 */
int64_t or_ac3_jacobi2(int32_t n, const int32_t *row_off, const int32_t *col,
                       const int32_t *rrow_off, const int32_t *rcol, uint8_t *live,
                       int32_t *level, int64_t *stats) {
    int64_t *co = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *ci = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *dround = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!co || !ci || !dround) { free(co); free(ci); free(dround); return -1; }
    const int64_t NEVER = INT64_MAX;
    for (int32_t v = 0; v < n; ++v) {
        live[v] = 1;
        level[v] = 0;
        co[v] = row_off[v];
        ci[v] = rrow_off[v];
        dround[v] = NEVER;
    }
    int64_t edges = 0, rounds = 0, n_live = n;
    int change = 1;
    while (change) {
        change = 0;
        rounds += 1;
        for (int32_t v = 0; v < n; ++v) {
            if (!live[v]) continue;
            int found = 0;
            for (int64_t end = row_off[v + 1]; co[v] < end; co[v] += 1) {
                edges += 1;
                if (dround[col[co[v]]] >= rounds) { found = 1; break; }
            }
            if (found) {
                found = 0;
                for (int64_t end = rrow_off[v + 1]; ci[v] < end; ci[v] += 1) {
                    edges += 1;
                    if (dround[rcol[ci[v]]] >= rounds) { found = 1; break; }
                }
            }
            if (!found) {
                live[v] = 0;
                level[v] = (int32_t)rounds;
                dround[v] = rounds;
                n_live -= 1;
                change = 1;
            }
        }
    }
    stats[0] = edges;
    stats[1] = rounds;
    stats[2] = n_live;
    free(co); free(ci); free(dround);
    return edges;
}

/*
 * Closed form of or_ac3_jacobi2's total from the two-sided peeling levels
 * (or_peel2): alpha is the largest level and the rounds number R = alpha + 1.
 * A vertex is alive at the start of round k iff it is live or its level is at
 * least k.  fo(v, k) and fi(v, k) are the indices of v's first successor and
 * first predecessor alive at the start of round k.  A vertex removed at level
 * L failed on its successors iff none is alive at the start of round L, else
 * on its predecessors.  Its cursors then account for:
 *   failed on successors:   deg + L - 1 successor checks, and L - 1 +
 *                           fi(v, L - 1) predecessor checks (none if L = 1);
 *   failed on predecessors: L + fo(v, L) successor checks, indeg + L - 1
 *                           predecessor checks;
 *   live:                   R + fo(v, R) and R + fi(v, R).
 * (A cursor checked in k rounds has checked k entries plus the ones it passed;
 * one that ran off its list has checked every entry once and its last round's
 * entry no second time.)  out[0] = total, out[1] = R.  Returns 0, or -(v+1)
 * for a vertex whose levels are inconsistent with the graph.
 */
static int64_t first_alive(const int32_t *adj, int64_t b, int64_t e, const uint8_t *live,
                           const int32_t *level, int64_t k) {
    for (int64_t p = b; p < e; ++p)
        if (live[adj[p]] || level[adj[p]] >= k) return p - b;
    return -1;
}
int64_t or_counts3two(int32_t n, const int32_t *row_off, const int32_t *col,
                      const int32_t *rrow_off, const int32_t *rcol, const uint8_t *live,
                      const int32_t *level, int64_t *out) {
    int64_t alpha = 0, total = 0;
    for (int32_t v = 0; v < n; ++v)
        if (!live[v] && level[v] > alpha) alpha = level[v];
    const int64_t R = alpha + 1;
    for (int32_t v = 0; v < n; ++v) {
        const int64_t b = row_off[v], e = row_off[v + 1], rb = rrow_off[v], re = rrow_off[v + 1];
        if (live[v]) {
            const int64_t fo = first_alive(col, b, e, live, level, R);
            const int64_t fi = first_alive(rcol, rb, re, live, level, R);
            if (fo < 0 || fi < 0) return -((int64_t)v + 1);
            total += R + fo + R + fi;
            continue;
        }
        const int64_t L = level[v];
        if (L < 1) return -((int64_t)v + 1);
        const int64_t fo = first_alive(col, b, e, live, level, L);
        if (fo < 0) {   /* no successor left at the start of round L */
            total += (e - b) + L - 1;
            if (L > 1) {
                const int64_t fi = first_alive(rcol, rb, re, live, level, L - 1);
                if (fi < 0) return -((int64_t)v + 1);
                total += L - 1 + fi;
            }
        } else {
            if (first_alive(rcol, rb, re, live, level, L) >= 0) return -((int64_t)v + 1);
            total += L + fo + (re - rb) + L - 1;
        }
    }
    out[0] = total;
    out[1] = R;
    return 0;
}
