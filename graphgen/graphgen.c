/*
 * graphgen.c -- seeded synthetic input graphs for the trimming workloads.
 *
 * This module only builds inputs (CSR arrays, the Zipf threshold table used by
 * the implicit graph, packed batches).  It contains none of the trimming
 * arithmetic: both the GPU library and the CPU oracle consume what it writes.
 *
 * Every random draw is counter based: draw(key, i) is the i-th output of a
 * SplitMix64 stream (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) whose state starts at `key`.  Results therefore do
 * not depend on the thread count.
 *
 * Graph storage is CSR (Section 2.1 of the paper): row_off[n+1] and col[m],
 * int32, successors of v in col[row_off[v] .. row_off[v+1]) in generation
 * order (the paper only says successors are ordered).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t fin64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return fin64(seed + GOLDEN) ^ fin64((tag + 1) * GOLDEN);
}
static inline uint64_t draw(uint64_t key, uint64_t i) {
    return fin64(key + (i + 1) * GOLDEN);
}
/* uniform integer in [0, k) from the top 32 bits (multiply-shift) */
static inline uint32_t below(uint64_t u, uint32_t k) {
    return (uint32_t)(((u >> 32) * (uint64_t)k) >> 32);
}
static inline double unit(uint64_t u) { return (double)(u >> 11) * (1.0 / 9007199254740992.0); }

uint64_t gg_fin64(uint64_t z) { return fin64(z); }
uint64_t gg_draw(uint64_t seed, uint64_t tag, uint64_t i) { return draw(stream_key(seed, tag), i); }

/* Stream tags. */
enum { TAG_RMAT = 1, TAG_CHAIN = 2, TAG_DEG = 3, TAG_NBR = 4, TAG_BATCH = 5, TAG_RAND = 6 };

static int nthreads_or_default(int nt) {
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#else
    nt = 1;
#endif
    return nt < 1 ? 1 : nt;
}

/* ---------------------------------------------------------------- Poisson */
/* Inverse-CDF thresholds: deg = #{k : u >= thr[k]}, thr[k] = floor(P(X<=k) * 2^64). */
static int poisson_table(double lam, uint64_t *thr, int cap) {
    double p = exp(-lam), cdf = 0.0;
    int k;
    for (k = 0; k < cap; ++k) {
        cdf += p;
        double t = cdf * 18446744073709551616.0;
        thr[k] = t >= 18446744073709551615.0 ? UINT64_MAX : (uint64_t)t;
        if (thr[k] == UINT64_MAX) { ++k; break; }
        p *= lam / (double)(k + 1);
    }
    return k;
}
static inline int inv_cdf(const uint64_t *thr, int len, uint64_t u) {
    int d = 0;
    while (d < len && u >= thr[d]) ++d;
    return d;
}

/* --------------------------------------------------------------- core+tail */
/*
 * Random core plus DAG tail.  Vertices [0, n_core) form the core: out-degree
 * core_fixed_deg (or Poisson(lam_core) when core_fixed_deg < 0), targets
 * uniform in the core.  Vertices [n_core, n - n_sink) form the tail: out-degree
 * Poisson(lam_tail), targets uniform among the higher ids (v, n-1].  The last
 * n_sink vertices have out-degree 0.  Self-loops are dropped when drop_self.
 * Pass col == NULL to only fill row_off; returns m.
 */
int64_t gg_core_tail(int32_t n, int32_t n_core, int32_t n_sink, int32_t core_fixed_deg,
                     double lam_core, double lam_tail, uint64_t seed, int drop_self,
                     int32_t *row_off, int32_t *col) {
    uint64_t tc[128], tt[128];
    int lc = core_fixed_deg < 0 ? poisson_table(lam_core, tc, 128) : 0;
    int lt = poisson_table(lam_tail, tt, 128);
    uint64_t kdeg = stream_key(seed, TAG_DEG), knbr = stream_key(seed, TAG_NBR);
    int64_t e = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (row_off) row_off[v] = (int32_t)e;
        int deg;
        if (v < n_core) deg = core_fixed_deg >= 0 ? core_fixed_deg : inv_cdf(tc, lc, draw(kdeg, (uint64_t)v));
        else if (v < n - n_sink) deg = inv_cdf(tt, lt, draw(kdeg, (uint64_t)v));
        else deg = 0;
        for (int i = 0; i < deg; ++i) {
            uint64_t u = draw(knbr, ((uint64_t)v << 16) | (uint64_t)i);
            int32_t w;
            if (v < n_core) w = (int32_t)below(u, (uint32_t)n_core);
            else w = v + 1 + (int32_t)below(u, (uint32_t)(n - 1 - v));
            if (drop_self && w == v) continue;
            if (col) col[e] = w;
            ++e;
        }
    }
    if (row_off) row_off[n] = (int32_t)e;
    return e;
}

/* -------------------------------------------------------------- uniform */
/* m0 uniform random edges (self-loops and duplicates possible), for tests. */
void gg_uniform_edges(int32_t n, int64_t m0, uint64_t seed, int32_t *src, int32_t *dst) {
    uint64_t k = stream_key(seed, TAG_RAND);
    for (int64_t e = 0; e < m0; ++e) {
        uint64_t u = draw(k, (uint64_t)e);
        src[e] = (int32_t)below(u, (uint32_t)n);
        dst[e] = (int32_t)below(u << 32, (uint32_t)n);
    }
}

/* ---------------------------------------------------------------- R-MAT */
/*
 * m0 R-MAT edges on 2^scale vertices.  At each of the `scale` bit levels a
 * 32-bit draw picks a quadrant against the integer thresholds a, a+b, a+b+c
 * (scaled by 2^32); no noise and no relabelling.  Two levels per 64-bit draw.
 */
void gg_rmat_edges(int scale, int64_t m0, uint64_t seed, double a, double b, double c,
                   int32_t *src, int32_t *dst, int nthreads) {
    const uint64_t two32 = 4294967296ULL;
    const uint32_t tA = (uint32_t)(a * (double)two32);
    const uint32_t tAB = (uint32_t)((a + b) * (double)two32);
    const uint32_t tABC = (uint32_t)((a + b + c) * (double)two32);
    const uint64_t key = stream_key(seed, TAG_RMAT);
    const int per_edge = (scale + 1) / 2;
    nthreads = nthreads_or_default(nthreads);
    #pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t e = 0; e < m0; ++e) {
        uint32_t s = 0, d = 0;
        int level = 0;
        for (int j = 0; j < per_edge; ++j) {
            uint64_t u = draw(key, (uint64_t)e * (uint64_t)per_edge + (uint64_t)j);
            for (int h = 0; h < 2 && level < scale; ++h, ++level) {
                uint32_t r = (uint32_t)(h ? (u >> 32) : u);
                uint32_t sb, db;
                if (r < tA) { sb = 0; db = 0; }
                else if (r < tAB) { sb = 0; db = 1; }
                else if (r < tABC) { sb = 1; db = 0; }
                else { sb = 1; db = 1; }
                s = (s << 1) | sb;
                d = (d << 1) | db;
            }
        }
        src[e] = (int32_t)s;
        dst[e] = (int32_t)d;
    }
}

/* L distinct vertex ids in [0, n), in draw order (rejection on repeats). */
int gg_chain_ids(int32_t n, int32_t L, uint64_t seed, int32_t *chain) {
    if (L > n) return -1;
    uint8_t *used = (uint8_t *)calloc((size_t)n, 1);
    if (!used) return -2;
    uint64_t key = stream_key(seed, TAG_CHAIN);
    uint64_t i = 0;
    for (int32_t k = 0; k < L; ++i) {
        int32_t v = (int32_t)(((draw(key, i) >> 32) * (uint64_t)n) >> 32);
        if (used[v]) continue;
        used[v] = 1;
        chain[k++] = v;
    }
    free(used);
    return 0;
}

/*
 * CSR from an edge list by a stable counting sort on src.  Edges whose src is
 * flagged in `drop_src` (may be NULL) are removed, and self-loops are removed
 * when drop_self.  The n_extra edges (extra_src, extra_dst) are appended after
 * the generated ones of the same source.  Pass col == NULL to only fill
 * row_off.  Returns m, or a negative value on allocation failure.
 */
int64_t gg_csr(int32_t n, int64_t m0, const int32_t *src, const int32_t *dst, int drop_self,
               const uint8_t *drop_src, int64_t n_extra, const int32_t *extra_src,
               const int32_t *extra_dst, int32_t *row_off, int32_t *col, int nthreads) {
    int T = nthreads_or_default(nthreads);
    int64_t blk = (m0 + T - 1) / T;
    if (blk == 0) blk = 1;
    int64_t *hist = (int64_t *)calloc((size_t)T * (size_t)n + 1, sizeof(int64_t));
    int64_t *xs = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!hist || !xs) { free(hist); free(xs); return -1; }
    #pragma omp parallel for num_threads(T) schedule(static, 1)
    for (int t = 0; t < T; ++t) {
        int64_t *h = hist + (size_t)t * (size_t)n;
        int64_t lo = (int64_t)t * blk, hi = lo + blk < m0 ? lo + blk : m0;
        for (int64_t e = lo; e < hi; ++e) {
            int32_t s = src[e];
            if ((drop_self && s == dst[e]) || (drop_src && drop_src[s])) continue;
            h[s]++;
        }
    }
    for (int64_t k = 0; k < n_extra; ++k) xs[extra_src[k]]++;
    int64_t run = 0;
    for (int32_t v = 0; v < n; ++v) {
        row_off[v] = (int32_t)run;
        for (int t = 0; t < T; ++t) {
            int64_t *h = hist + (size_t)t * (size_t)n;
            int64_t c = h[v];
            h[v] = run;
            run += c;
        }
        int64_t c = xs[v];
        xs[v] = run;
        run += c;
    }
    row_off[n] = (int32_t)run;
    if (col) {
        #pragma omp parallel for num_threads(T) schedule(static, 1)
        for (int t = 0; t < T; ++t) {
            int64_t *h = hist + (size_t)t * (size_t)n;
            int64_t lo = (int64_t)t * blk, hi = lo + blk < m0 ? lo + blk : m0;
            for (int64_t e = lo; e < hi; ++e) {
                int32_t s = src[e];
                if ((drop_self && s == dst[e]) || (drop_src && drop_src[s])) continue;
                col[h[s]++] = dst[e];
            }
        }
        for (int64_t k = 0; k < n_extra; ++k) col[xs[extra_src[k]]++] = extra_dst[k];
    }
    free(hist);
    free(xs);
    return run;
}

/*
 * Transposed CSR (Section 2): rrow_off/rcol list the predecessors of each
 * vertex, in increasing order of the source's CSR position.  Input
 * preparation for the AC-4 form, which takes G^T as an input.
 */
void gg_transpose(int32_t n, const int32_t *row_off, const int32_t *col, int32_t *rrow_off,
                  int32_t *rcol) {
    int64_t m = row_off[n];
    int32_t *cur = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    for (int64_t e = 0; e < m; ++e) cur[col[e]]++;
    int64_t run = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t c = cur[v];
        rrow_off[v] = (int32_t)run;
        cur[v] = (int32_t)run;
        run += c;
    }
    rrow_off[n] = (int32_t)run;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_off[v]; e < row_off[v + 1]; ++e) rcol[cur[col[e]]++] = v;
    free(cur);
}

/* -------------------------------------------------------------- Zipf table */
/*
 * Inverse-CDF thresholds for min(K, cap) with P(K = k) = k^-s / zeta(s),
 * k >= 1: thr[j] = floor(P(K <= j+1) * 2^64) for j = 0 .. cap-2, and
 * thr[cap-1] = UINT64_MAX.  A draw u maps to 1 + #{j < cap-1 : u >= thr[j]}.
 * zeta(s) is summed directly to 10^6 terms plus the Euler-Maclaurin tail.
 */
void gg_zipf_table(double s, int cap, uint64_t *thr) {
    const int64_t K = 1000000;
    double z = 0.0;
    for (int64_t k = K; k >= 1; --k) z += pow((double)k, -s);
    double Kd = (double)K;
    z += pow(Kd, 1.0 - s) / (s - 1.0) - 0.5 * pow(Kd, -s) + s / 12.0 * pow(Kd, -s - 1.0);
    double cdf = 0.0;
    for (int j = 0; j < cap - 1; ++j) {
        cdf += pow((double)(j + 1), -s) / z;
        double t = cdf * 18446744073709551616.0;
        thr[j] = t >= 18446744073709551615.0 ? UINT64_MAX : (uint64_t)t;
    }
    thr[cap - 1] = UINT64_MAX;
}

/* ----------------------------------------------------------------- batches */
/*
 * Parameters of graph g of a batch: n log-uniform in [n_lo, n_hi], mean
 * out-degree d uniform in [d_lo, d_hi], tail fraction f uniform in
 * [f_lo, f_hi].  Stream key for the graph itself is returned in *gseed.
 */
void gg_batch_params(uint64_t seed, int64_t g, double n_lo, double n_hi, double d_lo, double d_hi,
                     double f_lo, double f_hi, int32_t *n_out, double *d_out, double *f_out,
                     uint64_t *gseed) {
    uint64_t k = stream_key(seed, TAG_BATCH);
    double u0 = unit(draw(k, (uint64_t)g * 4 + 0));
    double u1 = unit(draw(k, (uint64_t)g * 4 + 1));
    double u2 = unit(draw(k, (uint64_t)g * 4 + 2));
    double ln = log(n_lo) + u0 * (log(n_hi) - log(n_lo));
    int32_t n = (int32_t)floor(exp(ln));
    if (n < (int32_t)n_lo) n = (int32_t)n_lo;
    if (n > (int32_t)n_hi) n = (int32_t)n_hi;
    *n_out = n;
    *d_out = d_lo + u1 * (d_hi - d_lo);
    *f_out = f_lo + u2 * (f_hi - f_lo);
    *gseed = draw(k, (uint64_t)g * 4 + 3);
}
