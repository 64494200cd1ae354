/*
 * sanitize_main.c -- drives every routine of oracle/oracle.c and of the input
 * generators (graphgen/graphgen.c) on small graphs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitize.py).
 * Host code only.  Besides running clean under the sanitizers, the results
 * must agree across the oracle's routines: the same live set from every
 * algorithm, and the literal AC-6 / AC-3 runs equal to the closed forms.
 * Exit status 0 = all checks passed.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* graphgen.c */
int64_t gg_core_tail(int32_t n, int32_t n_core, int32_t n_sink, int32_t core_fixed_deg,
                     double lam_core, double lam_tail, uint64_t seed, int drop_self,
                     int32_t *row_off, int32_t *col);
void gg_uniform_edges(int32_t n, int64_t m0, uint64_t seed, int32_t *src, int32_t *dst);
void gg_rmat_edges(int scale, int64_t m0, uint64_t seed, double a, double b, double c,
                   int32_t *src, int32_t *dst, int nthreads);
int gg_chain_ids(int32_t n, int32_t L, uint64_t seed, int32_t *chain);
int64_t gg_csr(int32_t n, int64_t m0, const int32_t *src, const int32_t *dst, int drop_self,
               const uint8_t *drop_src, int64_t n_extra, const int32_t *extra_src,
               const int32_t *extra_dst, int32_t *row_off, int32_t *col, int nthreads);
void gg_transpose(int32_t n, const int32_t *row_off, const int32_t *col, int32_t *rrow_off,
                  int32_t *rcol);
void gg_zipf_table(double s, int cap, uint64_t *thr);
void gg_batch_params(uint64_t seed, int64_t g, double n_lo, double n_hi, double d_lo, double d_hi,
                     double f_lo, double f_hi, int32_t *n_out, double *d_out, double *f_out,
                     uint64_t *gseed);
/* oracle.c */
int64_t or_peel(int32_t, const int32_t *, const int32_t *, uint8_t *, int32_t *, int32_t *,
                int64_t *);
int64_t or_ac6_seq(int32_t, const int32_t *, const int32_t *, uint8_t *, int64_t *);
int64_t or_ac3_jacobi(int32_t, const int32_t *, const int32_t *, uint8_t *, int64_t *);
int64_t or_ac3_inplace(int32_t, const int32_t *, const int32_t *, uint8_t *, int64_t *);
int64_t or_counts(int32_t, const int32_t *, const int32_t *, const uint8_t *, const int32_t *,
                  int32_t, int64_t *);
int64_t or_implicit_csr(int, uint64_t, uint64_t, const uint64_t *, int32_t *, int32_t *);
int64_t or_batch_peel(int64_t, const int64_t *, const int32_t *, const int32_t *, uint8_t *,
                      int64_t *, int);
int64_t or_peel_preset(int32_t, const int32_t *, const int32_t *, const uint8_t *, uint8_t *,
                       int32_t *, int32_t *, int64_t *);
int64_t or_counts_preset(int32_t, const int32_t *, const int32_t *, const uint8_t *,
                         const uint8_t *, const int32_t *, int32_t, int64_t *);
int64_t or_peel2(int32_t, const int32_t *, const int32_t *, uint8_t *, int32_t *, int32_t *,
                 int64_t *);
int64_t or_counts2(int32_t, const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                   const uint8_t *, int64_t *);
int64_t or_ac3_jacobi2(int32_t, const int32_t *, const int32_t *, const int32_t *,
                       const int32_t *, uint8_t *, int32_t *, int64_t *);
int64_t or_counts3two(int32_t, const int32_t *, const int32_t *, const int32_t *,
                      const int32_t *, const uint8_t *, const int32_t *, int64_t *);

static int failures = 0;
#define CHECK(c, ...)                                                  \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);      \
            fprintf(stderr, __VA_ARGS__);                              \
            fputc('\n', stderr);                                       \
            failures++;                                                \
        }                                                              \
    } while (0)

typedef struct {
    int32_t n;
    int32_t *row_off, *col;
} graph;

static void *xmalloc(size_t k) {
    void *p = malloc(k ? k : 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

static graph from_edges(int32_t n, int64_t m0, const int32_t *src, const int32_t *dst,
                        int drop_self, const uint8_t *drop_src, int64_t nx, const int32_t *xs,
                        const int32_t *xd) {
    graph g;
    g.n = n;
    g.row_off = xmalloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t m = gg_csr(n, m0, src, dst, drop_self, drop_src, nx, xs, xd, g.row_off, NULL, 1);
    g.col = xmalloc((size_t)m * sizeof(int32_t));
    gg_csr(n, m0, src, dst, drop_self, drop_src, nx, xs, xd, g.row_off, g.col, 1);
    return g;
}

static graph uniform(int32_t n, int64_t m0, uint64_t seed, int drop_self) {
    int32_t *s = xmalloc((size_t)m0 * 4), *d = xmalloc((size_t)m0 * 4);
    gg_uniform_edges(n, m0, seed, s, d);
    graph g = from_edges(n, m0, s, d, drop_self, NULL, 0, NULL, NULL);
    free(s);
    free(d);
    return g;
}

static graph core_tail(int32_t n, uint64_t seed) {
    graph g;
    g.n = n;
    int32_t nc = (int32_t)(0.7 * n), ns = n / 100;
    g.row_off = xmalloc(((size_t)n + 1) * 4);
    int64_t m = gg_core_tail(n, nc, ns, 8, 0.0, 3.0, seed, 1, g.row_off, NULL);
    g.col = xmalloc((size_t)m * 4);
    gg_core_tail(n, nc, ns, 8, 0.0, 3.0, seed, 1, g.row_off, g.col);
    return g;
}

/* R-MAT with a planted chain c_0 -> ... -> c_{L-1} (the last one a sink). */
static graph rmat_chain(int scale, int ef, int32_t L, uint64_t seed) {
    int32_t n = 1 << scale;
    int64_t m0 = (int64_t)ef * n;
    int32_t *s = xmalloc((size_t)m0 * 4), *d = xmalloc((size_t)m0 * 4);
    gg_rmat_edges(scale, m0, seed, 0.57, 0.19, 0.19, s, d, 1);
    int32_t *ch = xmalloc((size_t)L * 4);
    CHECK(gg_chain_ids(n, L, seed, ch) == 0, "chain ids");
    uint8_t *drop = calloc((size_t)n, 1);
    for (int32_t i = 0; i < L; ++i) drop[ch[i]] = 1;
    graph g = from_edges(n, m0, s, d, 1, drop, L - 1, ch, ch + 1);
    free(s); free(d); free(ch); free(drop);
    return g;
}

static void free_graph(graph *g) {
    free(g->row_off);
    free(g->col);
}

static int same(const uint8_t *a, const uint8_t *b, int32_t n) {
    return n == 0 || memcmp(a, b, (size_t)n) == 0;
}

/* Every oracle routine on one graph, cross-checked. */
static void run_all(const char *name, const graph *g) {
    const int32_t n = g->n;
    const size_t N = (size_t)n + 1;
    uint8_t *live = xmalloc(N), *l6 = xmalloc(N), *l3 = xmalloc(N), *l3i = xmalloc(N);
    int32_t *level = xmalloc(N * 4), *order = xmalloc(N * 4);
    int64_t st[3], c[8];
    int64_t nd = or_peel(n, g->row_off, g->col, live, level, order, st);
    CHECK(nd >= 0 && st[1] + nd == n, "%s: peel", name);
    CHECK(or_counts(n, g->row_off, g->col, live, level, (int32_t)st[0], c) == 0, "%s: counts",
          name);
    int64_t s6[3], s3[3], s3i[3];
    int64_t t6 = or_ac6_seq(n, g->row_off, g->col, l6, s6);
    int64_t t3 = or_ac3_jacobi(n, g->row_off, g->col, l3, s3);
    int64_t t3i = or_ac3_inplace(n, g->row_off, g->col, l3i, s3i);
    CHECK(same(live, l6, n) && same(live, l3, n) && same(live, l3i, n), "%s: live sets", name);
    CHECK(t6 == c[0], "%s: T6 %lld vs %lld", name, (long long)t6, (long long)c[0]);
    CHECK(t3 == c[3] && s3[1] == c[4], "%s: T3J", name);
    CHECK(c[0] <= t3i && t3i <= c[3], "%s: in-place AC-3 bounds", name);
    CHECK(st[2] == c[1], "%s: T4*", name);

    /* preset: every third vertex removed before trimming */
    uint8_t *pre = xmalloc(N), *lp = xmalloc(N);
    for (int32_t v = 0; v < n; ++v) pre[v] = v % 3 == 1;
    int64_t stp[3], cp[8];
    int64_t ndp = or_peel_preset(n, g->row_off, g->col, pre, lp, level, order, stp);
    CHECK(ndp >= 0, "%s: peel preset", name);
    CHECK(or_counts_preset(n, g->row_off, g->col, pre, lp, level, (int32_t)stp[0], cp) == 0,
          "%s: counts preset", name);
    for (int32_t v = 0; v < n; ++v) CHECK(!(pre[v] && lp[v]), "%s: preset vertex live", name);

    /* two-sided */
    int64_t m = g->row_off[n];
    int32_t *rro = xmalloc(N * 4), *rcol = xmalloc((size_t)m * 4 + 4);
    gg_transpose(n, g->row_off, g->col, rro, rcol);
    uint8_t *l2 = xmalloc(N), *l23 = xmalloc(N);
    int32_t *lev2 = xmalloc(N * 4), *lev23 = xmalloc(N * 4);
    int64_t st2[3], c2[5], st23[3], c3t[2];
    CHECK(or_peel2(n, g->row_off, g->col, l2, lev2, order, st2) >= 0, "%s: peel2", name);
    CHECK(or_counts2(n, g->row_off, g->col, rro, rcol, l2, c2) == 0, "%s: counts2", name);
    CHECK(c2[3] == st2[2], "%s: two-sided AC-4 total", name);
    CHECK(or_ac3_jacobi2(n, g->row_off, g->col, rro, rcol, l23, lev23, st23) >= 0,
          "%s: ac3 two-sided", name);
    CHECK(same(l2, l23, n), "%s: two-sided live sets", name);
    CHECK(or_counts3two(n, g->row_off, g->col, rro, rcol, l2, lev2, c3t) == 0,
          "%s: counts3two", name);
    CHECK(c3t[0] == st23[0] && c3t[1] == st23[1], "%s: two-sided AC-3 total", name);
    for (int32_t v = 0; v < n; ++v)
        CHECK(!l2[v] || live[v], "%s: two-sided live %d not one-sided live", name, v);

    free(live); free(l6); free(l3); free(l3i); free(level); free(order);
    free(pre); free(lp); free(rro); free(rcol); free(l2); free(l23); free(lev2); free(lev23);
}

int main(void) {
    graph g;
    /* degenerate graphs */
    {
        int32_t ro0[1] = {0};
        graph e0 = {0, ro0, NULL};
        run_all("empty", &e0);
        int32_t ro1[2] = {0, 1}, c1[1] = {0};
        graph e1 = {1, ro1, c1};
        run_all("self-loop", &e1);
        int32_t ro3[4] = {0, 0, 0, 0};
        graph e3 = {3, ro3, NULL};
        run_all("edgeless", &e3);
    }
    for (uint64_t seed = 0; seed < 4; ++seed) {
        g = uniform(300, 900, seed, (int)(seed & 1));
        run_all("uniform 300", &g);
        free_graph(&g);
        g = uniform(2000, 2500, seed + 10, 0);
        run_all("uniform 2000", &g);
        free_graph(&g);
    }
    g = core_tail(4096, 0);
    run_all("core+tail", &g);
    free_graph(&g);
    g = rmat_chain(12, 8, 500, 3);
    run_all("rmat+chain", &g);
    free_graph(&g);

    /* implicit graph, materialised by the oracle */
    {
        uint64_t tab[256];
        gg_zipf_table(2.1, 256, tab);
        const int log2n = 12;
        const int32_t n = 1 << log2n;
        graph h;
        h.n = n;
        h.row_off = xmalloc(((size_t)n + 1) * 4);
        int64_t m = or_implicit_csr(log2n, 5, 0x3333333333333333ULL, tab, h.row_off, NULL);
        h.col = xmalloc((size_t)m * 4);
        CHECK(or_implicit_csr(log2n, 5, 0x3333333333333333ULL, tab, h.row_off, h.col) == m,
              "implicit m");
        run_all("implicit 2^12", &h);
        free_graph(&h);
    }

    /* a packed batch of core+tail graphs */
    {
        const int64_t G = 8;
        int64_t *vbase = xmalloc((G + 1) * 8);
        int32_t ns[8];
        uint64_t gs[8];
        int64_t N = 0, M = 0;
        for (int64_t i = 0; i < G; ++i) {
            double d, f;
            gg_batch_params(1, i, 100, 3000, 1, 8, 0.1, 0.6, &ns[i], &d, &f, &gs[i]);
            vbase[i] = N;
            N += ns[i];
            M += gg_core_tail(ns[i], (int32_t)(ns[i] * (1 - f)), ns[i] / 100 > 0 ? ns[i] / 100 : 1,
                              -1, d, d, gs[i], 1, NULL, NULL);
        }
        vbase[G] = N;
        int32_t *ro = xmalloc(((size_t)N + 1) * 4), *col = xmalloc((size_t)M * 4 + 4);
        int64_t e = 0;
        for (int64_t i = 0; i < G; ++i) {
            double d, f;
            gg_batch_params(1, i, 100, 3000, 1, 8, 0.1, 0.6, &ns[i], &d, &f, &gs[i]);
            int32_t *lro = xmalloc(((size_t)ns[i] + 1) * 4);
            int64_t mi = gg_core_tail(ns[i], (int32_t)(ns[i] * (1 - f)),
                                      ns[i] / 100 > 0 ? ns[i] / 100 : 1, -1, d, d, gs[i], 1, lro,
                                      col + e);
            for (int32_t v = 0; v < ns[i]; ++v) ro[vbase[i] + v] = (int32_t)(lro[v] + e);
            e += mi;
            free(lro);
        }
        ro[N] = (int32_t)e;
        uint8_t *live = xmalloc((size_t)N);
        int64_t *out = xmalloc((size_t)(2 * G) * 8);
        CHECK(or_batch_peel(G, vbase, ro, col, live, out, 1) == 0, "batch peel");
        free(vbase); free(ro); free(col); free(live); free(out);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitized oracle and generators: all checks passed\n");
    return 0;
}
