// order.hip -- per-edge preprocessing (in-degrees, edge sources) and the
// reordering of successor lists by a per-edge key.
//
// AC-6 checks a vertex's successors in list order and keeps the first live
// one (Section 6.1), so reordering the lists changes the traversed edges but
// never the live set.  These kernels are edge-parallel: the edge array is cut
// into tiles of kTileE edges, one workgroup per tile, so a tile's work does
// not depend on how its edges fall into lists (a hub's list spreads over many
// tiles, a tile may hold thousands of short lists).
//
// Source of each edge of a tile: the source of the tile's first edge comes
// from a per-tile table; every later list that starts inside the tile stamps
// its vertex id at its start in LDS, and a prefix maximum fills the gaps.
//
// Reorder: a stable counting sort of every list into kBuckets levels, larger
// keys first.  With P(x, q) = number of edges before position x (over the
// whole edge array) at level q, edge p of list u = [s, e) at level k moves to
//   s + sum_{q<k} (P(e, q) - P(s, q)) + (P(p, k) - P(s, k)).
// P is an exclusive scan of per-tile level counts plus in-tile prefixes kept
// in LDS; a list start or end outside the tile costs one partial count over
// the tile it lies in (at most two per tile).
#include "trim_device.h"
#include "trim_internal.h"

namespace trim {

namespace {

constexpr int kTileT = 256;                 // threads of a tile workgroup
constexpr int kPerT = kTileE / kTileT;      // consecutive edges per thread
constexpr int kTileWaves = kTileT / kWave;
constexpr int kBuckets = 16;
static_assert(kPerT == 16, "in-tile prefixes assume 16 edges per thread");

// Level of edge p: 0 for keys at hi (placed first) .. kBuckets-1 at lo.
struct Levels {
    const float* key;
    float hi, scale;
    __device__ __forceinline__ int operator()(long long p) const {
        const int k = (int)((hi - key[p]) * scale);
        return k < 0 ? 0 : (k >= kBuckets ? kBuckets - 1 : k);
    }
};

// kBuckets counters of 16 bits in four words (a count never exceeds kTileE).
struct Packed {
    uint64_t w[4];
    __device__ __forceinline__ void clear() { w[0] = w[1] = w[2] = w[3] = 0; }
    __device__ __forceinline__ void add_one(int k) {
        const uint64_t inc = 1ull << (16 * (k & 3));
        const int h = k >> 2;
        w[0] += h == 0 ? inc : 0;
        w[1] += h == 1 ? inc : 0;
        w[2] += h == 2 ? inc : 0;
        w[3] += h == 3 ? inc : 0;
    }
    __device__ __forceinline__ int get(int k) const {
        const int h = k >> 2;
        const uint64_t x = h == 0 ? w[0] : h == 1 ? w[1] : h == 2 ? w[2] : w[3];
        return (int)((x >> (16 * (k & 3))) & 0xFFFFu);
    }
};

__device__ __forceinline__ uint64_t shfl_up64(uint64_t x, int d) {
    const unsigned lo = __shfl_up((unsigned)x, d), hi = __shfl_up((unsigned)(x >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

// Exclusive scan of x over the workgroup; *total gets the sum.  `wtot` holds
// kTileWaves entries of LDS.
__device__ Packed block_exscan(const Packed& x, Packed* wtot, Packed* total) {
    const int l = lane_id(), wv = threadIdx.x / kWave;
    Packed inc = x;
    for (int d = 1; d < kWave; d <<= 1) {
        for (int i = 0; i < 4; ++i) {
            const uint64_t y = shfl_up64(inc.w[i], d);
            if (l >= d) inc.w[i] += y;
        }
    }
    __syncthreads();
    if (l == kWave - 1) wtot[wv] = inc;
    __syncthreads();
    Packed pre, tot;
    pre.clear();
    tot.clear();
    for (int w = 0; w < kTileWaves; ++w)
        for (int i = 0; i < 4; ++i) {
            if (w < wv) pre.w[i] += wtot[w].w[i];
            tot.w[i] += wtot[w].w[i];
        }
    *total = tot;
    Packed ex;
    for (int i = 0; i < 4; ++i) ex.w[i] = inc.w[i] - x.w[i] + pre.w[i];
    return ex;
}

__device__ Packed block_total(const Packed& x, Packed* wtot) {
    Packed tot;
    (void)block_exscan(x, wtot, &tot);
    return tot;
}

// tinfo[t] = (u, row_off[u], row_off[u + 1]) for the source u of edge
// t * kTileE: the list that holds the tile's first edge.
__global__ void tile_first(const int* row_off, int n, int* tinfo) {
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const int b = row_off[u], e = row_off[u + 1];
        for (long long t = (b + (long long)kTileE - 1) / kTileE; t * kTileE < e; ++t) {
            tinfo[3 * t] = u;
            tinfo[3 * t + 1] = b;
            tinfo[3 * t + 2] = e;
        }
    }
}

// owner[j] = source of edge t0 + j for j < len; uf = source of edge t0.
__device__ void tile_owners(const int* row_off, int n, long long t0, int len, int uf, int* owner,
                            int* wmax) {
    for (int j = threadIdx.x; j < kTileE; j += kTileT) owner[j] = -1;
    __syncthreads();
    if (threadIdx.x == 0) owner[0] = uf;
    // lists after uf start after t0 (uf's own list reaches past t0)
    for (int u = uf + 1 + threadIdx.x; u < n; u += kTileT) {
        const long long x = row_off[u] - t0;
        if (x >= len) break;
        atomicMax(owner + x, u);
    }
    __syncthreads();
    const int l = lane_id(), wv = threadIdx.x / kWave;
    int run = -1;
    for (int i = 0; i < kPerT; ++i) run = max(run, owner[threadIdx.x * kPerT + i]);
    int inc = run;
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(inc, d);
        if (l >= d) inc = max(inc, y);
    }
    if (l == kWave - 1) wmax[wv] = inc;
    __syncthreads();
    int m = __shfl_up(inc, 1);
    if (l == 0) m = -1;
    for (int w = 0; w < wv; ++w) m = max(m, wmax[w]);
    for (int i = 0; i < kPerT; ++i) {
        m = max(m, owner[threadIdx.x * kPerT + i]);
        owner[threadIdx.x * kPerT + i] = m;
    }
    __syncthreads();
}

__device__ __forceinline__ int clamp_vertex(int u, int n) { return u < 0 ? 0 : (u >= n ? n - 1 : u); }

// src[e] = source of edge e.
__global__ __launch_bounds__(kTileT) void tile_sources(const int* row_off, int n, long long m,
                                                       const int* tinfo, int* src) {
    __shared__ int owner[kTileE];
    __shared__ int wmax[kTileWaves];
    const long long T = (m + kTileE - 1) / kTileE;
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        const long long t0 = t * kTileE;
        const int len = (int)(m - t0 < kTileE ? m - t0 : kTileE);
        tile_owners(row_off, n, t0, len, clamp_vertex(tinfo[3 * t], n), owner, wmax);
        for (int j = threadIdx.x; j < len; j += kTileT) src[t0 + j] = owner[j];
        __syncthreads();
    }
}

// In-degrees.  Device-wide atomics on one array are slow and serialise on
// hubs; instead every XCD counts into its own copy with workgroup-scope
// atomics, which its L2 executes (no other XCD touches that copy), and
// sum_copies adds the copies at the end.  A wave on an unexpected XCD id adds
// to indeg directly with device-wide atomics.
__global__ void in_degrees_xcd(const int* col, long long m, int n, int* copies, int* indeg) {
    const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);   // XCC_ID[3:0]
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < m;
         e += (long long)gridDim.x * blockDim.x) {
        const int w = col[e];
        if (copies && xcc < kXcdCopies)
            __hip_atomic_fetch_add(copies + (long long)xcc * n + w, 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            atomicAdd(indeg + w, 1);
    }
}

__global__ void sum_copies(const int* copies, int n, int* indeg) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int s = indeg[v];
        for (int x = 0; x < kXcdCopies; ++x) s += copies[(long long)x * n + v];
        indeg[v] = s;
    }
}

__global__ void zero_ints(int* a, long long k) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < k;
         i += (long long)gridDim.x * blockDim.x)
        a[i] = 0;
}

// Keys for the reference orders: 0 = log1p(outdeg w) (larger first), 1 = a hash
// of (seed, e) (a random order).
__global__ void edge_keys(const int* row_off, const int* col, long long m, int kind, uint64_t seed,
                          float* key) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < m;
         e += (long long)gridDim.x * blockDim.x) {
        if (kind == 0) {
            const int w = col[e];
            key[e] = log1pf((float)(row_off[w + 1] - row_off[w]));
        } else {
            key[e] = (float)(mix64(seed ^ (uint64_t)e) >> 40) * (1.f / 16777216.f);
        }
    }
}

// tcnt[t][q] = edges of tile t at level q.
__global__ __launch_bounds__(kTileT) void order_count(long long m, Levels level, int* tcnt) {
    __shared__ Packed wtot[kTileWaves];
    const long long T = (m + kTileE - 1) / kTileE;
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        const long long t0 = t * kTileE;
        const int len = (int)(m - t0 < kTileE ? m - t0 : kTileE);
        Packed c;
        c.clear();
        for (int j = threadIdx.x; j < len; j += kTileT) c.add_one(level(t0 + j));
        const Packed tot = block_total(c, wtot);
        if (threadIdx.x < kBuckets) tcnt[t * kBuckets + threadIdx.x] = tot.get(threadIdx.x);
        __syncthreads();
    }
}

// Exclusive scan of the tile counts, in place: tcnt[t][q] <- the sum of
// tcnt[t'][q] over t' < t, for t = 0..T (row T gets the totals; its input is
// ignored).  Rows are taken kScanRows at a time: scan_reduce sums each chunk,
// scan_rows scans the chunk sums (one workgroup), scan_apply rescans each
// chunk from its offset.
constexpr int kScanRows = 64;
constexpr int kScanT = 1024;

__device__ __forceinline__ int row_val(const int* a, long long rows_in, long long r, int q) {
    return r < rows_in ? a[r * kBuckets + q] : 0;
}

// 64 threads: thread (g, q) covers rows g*16 .. g*16+15 of the chunk, level q.
__global__ __launch_bounds__(kWave) void scan_reduce(const int* tcnt, long long T, int* csum) {
    __shared__ int part[4][kBuckets];
    const int q = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long long r0 = blockIdx.x * (long long)kScanRows + g * 16;
    int acc = 0;
    for (int i = 0; i < 16; ++i) acc += row_val(tcnt, T, r0 + i, q);
    part[g][q] = acc;
    __syncthreads();
    if (g == 0) csum[blockIdx.x * kBuckets + q] = part[0][q] + part[1][q] + part[2][q] + part[3][q];
}

// One workgroup: the same exclusive scan over `rows` rows of a (the input of
// row `rows_in` and later is taken as 0).
__global__ __launch_bounds__(kScanT) void scan_rows(int* a, long long rows_in, long long rows) {
    __shared__ int wsum[kScanT / kWave][kBuckets];
    const int l = lane_id(), wv = threadIdx.x / kWave;
    const long long per = (rows + kScanT - 1) / kScanT;
    const long long r0 = threadIdx.x * per;
    const long long r1 = r0 + per < rows ? r0 + per : rows;
    int acc[kBuckets];
    for (int q = 0; q < kBuckets; ++q) acc[q] = 0;
    for (long long r = r0; r < r1; ++r)
        for (int q = 0; q < kBuckets; ++q) acc[q] += row_val(a, rows_in, r, q);
    int ex[kBuckets];
    for (int q = 0; q < kBuckets; ++q) {
        int inc = acc[q];
        for (int d = 1; d < kWave; d <<= 1) {
            const int y = __shfl_up(inc, d);
            if (l >= d) inc += y;
        }
        if (l == kWave - 1) wsum[wv][q] = inc;
        ex[q] = inc - acc[q];
    }
    __syncthreads();
    for (int w = 0; w < wv; ++w)
        for (int q = 0; q < kBuckets; ++q) ex[q] += wsum[w][q];
    for (long long r = r0; r < r1; ++r)
        for (int q = 0; q < kBuckets; ++q) {
            const int c = row_val(a, rows_in, r, q);
            a[r * kBuckets + q] = ex[q];
            ex[q] += c;
        }
}

__global__ __launch_bounds__(kWave) void scan_apply(int* tcnt, long long T, const int* csum) {
    __shared__ int part[4][kBuckets];
    const int q = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long long r0 = blockIdx.x * (long long)kScanRows + g * 16;
    int v[16];
    int acc = 0;
    for (int i = 0; i < 16; ++i) {
        v[i] = row_val(tcnt, T, r0 + i, q);
        acc += v[i];
    }
    part[g][q] = acc;
    __syncthreads();
    int run = csum[blockIdx.x * kBuckets + q];
    for (int h = 0; h < g; ++h) run += part[h][q];
    for (int i = 0; i < 16; ++i) {
        if (r0 + i > T) break;
        tcnt[(r0 + i) * kBuckets + q] = run;
        run += v[i];
    }
}

// Edge j of the tile (position t0 + j) of list [s, e) at level k goes to
//   s + Lb(e, k) - Lb(s, k + 1) + (Lb(j, k + 1) - Lb(j, k)),
// where Lb(x, k) counts the tile's edges before t0 + x with level < k (the
// tile's scan entry cancels out of every difference).  One lane per edge: the
// tile is 64 chunks of 64 edges, and for every chunk the workgroup keeps, in
// LDS, the lane masks of "level < k" for k = 0..16 (from ballots) and the
// counts of such edges in the chunks before it, so Lb at any in-tile position
// is one mask, one count and a popcount.  A list's bounds come from the tile
// alone: starts of lists after the first are stamped as bits, the first list
// starts at row_off of the tile's first source, and the last one ends where
// the list holding the tile's last edge ends.  A start before the tile or an
// end after it uses counts over the part of the list outside the tile.
constexpr int kChunks = kTileE / kWave;             // 64
constexpr int kChunksPerWave = kChunks / kTileWaves;   // 16
static_assert(kChunks == kWave, "chunk prefixes are scanned one chunk per lane");

__device__ __forceinline__ uint64_t lanes_lt(int l) { return (1ull << l) - 1ull; }

__global__ __launch_bounds__(kTileT, 4) void order_place(const int* row_off, int n, long long m,
                                                      const int* col, Levels level,
                                                      const int* tinfo, const int* tpre,
                                                      int* col_out) {
    __shared__ int8_t lvl[kTileE];                      // level of each edge, -1 past the end
    __shared__ int cols[kTileE];
    __shared__ uint64_t fm[kChunks];                    // bit = a list other than the first starts
    __shared__ uint64_t cm[kChunks][kBuckets + 1];      // lanes of the chunk with level < k
    __shared__ int cpre[kChunks + 1][kBuckets + 1];     // edges of earlier chunks with level < k
    __shared__ int lastst[kChunks], firstst[kChunks];   // last start before / first after the chunk
    __shared__ int wpart[kTileWaves][kBuckets];
    __shared__ int lout[2][kBuckets];
    __shared__ int loutc[2][kBuckets + 1];              // cumulative lout: level < k
    const int l = lane_id(), wv = threadIdx.x / kWave;
    const long long T = (m + kTileE - 1) / kTileE;
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        const long long t0 = t * kTileE;
        const int len = (int)(m - t0 < kTileE ? m - t0 : kTileE);
        const long long t1 = t0 + len;
        for (int i = 0; i < kChunksPerWave; ++i) {
            const int j = (wv * kChunksPerWave + i) * kWave + l;
            cols[j] = j < len ? col[t0 + j] : 0;
            lvl[j] = (int8_t)(j < len ? level(t0 + j) : -1);
        }
        if (threadIdx.x < kChunks) fm[threadIdx.x] = 0;
        const int uf = clamp_vertex(tinfo[3 * t], n);
        const long long sf = tinfo[3 * t + 1];
        long long el = t1;   // end of the list that holds edge t1 - 1
        if (t + 1 < T && tinfo[3 * t + 4] < t1) el = tinfo[3 * t + 5];
        __syncthreads();
        for (int u = uf + 1 + threadIdx.x; u < n; u += kTileT) {
            const long long x = row_off[u] - t0;
            if (x >= len) break;
            atomicOr((unsigned long long*)&fm[x >> 6], 1ull << (x & 63));
        }
#pragma unroll 1
        for (int i = 0; i < kChunksPerWave; ++i) {   // a wave reads back only its own chunks
            const int c = wv * kChunksPerWave + i;
            const int k = lvl[c * kWave + l];
            uint64_t below = 0;
            for (int q = 0; q < kBuckets; ++q) {
                if (l == 0) cm[c][q] = below;
                below |= ballot(k == q);
            }
            if (l == 0) cm[c][kBuckets] = below;
        }
        __syncthreads();
        for (int k = wv; k <= kBuckets; k += kTileWaves) {   // lane = chunk
            const int cnt = popc(cm[l][k]);
            int inc = cnt;
            for (int d = 1; d < kWave; d <<= 1) {
                const int y = __shfl_up(inc, d);
                if (l >= d) inc += y;
            }
            cpre[l][k] = inc - cnt;
            if (l == kWave - 1) cpre[kChunks][k] = inc;
        }
        if (wv == 0) {   // lane = chunk
            const uint64_t f = fm[l];
            int lastv = f ? l * kWave + 63 - __clzll((long long)f) : 0;
            int firstv = f ? l * kWave + __ffsll((unsigned long long)f) - 1 : len;
            for (int d = 1; d < kWave; d <<= 1) {
                const int yl = __shfl_up(lastv, d), yf = __shfl_down(firstv, d);
                if (l >= d) lastv = max(lastv, yl);
                if (l + d < kWave) firstv = min(firstv, yf);
            }
            int ls = __shfl_up(lastv, 1), fs = __shfl_down(firstv, 1);
            if (l == 0) ls = 0;
            if (l == kWave - 1) fs = len;
            lastst[l] = ls;
            firstst[l] = fs;
        }
        __syncthreads();
        // The first list's start before the tile, the last list's end after
        // it: counted over the shorter of "from that position's tile start"
        // (with that tile's scan entry) or "between it and this tile".
        for (int side = 0; side < 2; ++side) {
            const long long x = side == 0 ? sf : el;
            if (side == 0 ? x >= t0 : x <= t1) continue;   // uniform over the workgroup
            const long long tx = x / kTileE;
            const long long fwd = x - tx * kTileE, near = side == 0 ? t0 - x : x - t1;
            const bool use_near = near < fwd;
            const long long p0 = use_near ? (side == 0 ? x : t1) : tx * kTileE;
            const long long p1 = use_near ? (side == 0 ? t0 : x) : x;
            int cq[kBuckets];
            for (int q = 0; q < kBuckets; ++q) cq[q] = 0;
            for (long long p = p0 + wv * kWave; p < p1; p += kTileT) {
                const int k = p + l < p1 ? level(p + l) : -1;
                for (int q = 0; q < kBuckets; ++q) cq[q] += popc(ballot(k == q));
            }
            if (l == 0)
                for (int q = 0; q < kBuckets; ++q) wpart[wv][q] = cq[q];
            __syncthreads();
            if (threadIdx.x < kBuckets) {
                const int q = threadIdx.x;
                int part = 0;
                for (int w = 0; w < kTileWaves; ++w) part += wpart[w][q];
                int v;
                if (!use_near) v = tpre[tx * kBuckets + q] - tpre[t * kBuckets + q] + part;
                else if (side == 0) v = -part;
                else v = cpre[kChunks][q + 1] - cpre[kChunks][q] + part;
                lout[side][q] = v;
            }
            __syncthreads();
            if (threadIdx.x <= kBuckets) {
                int acc = 0;
                for (int q = 0; q < (int)threadIdx.x; ++q) acc += lout[side][q];
                loutc[side][threadIdx.x] = acc;
            }
        }
        __syncthreads();
        auto Lb = [&](int x, int kk) {
            if (x >= len) return cpre[kChunks][kk];
            const int c = x >> 6;
            return cpre[c][kk] + popc(cm[c][kk] & lanes_lt(x & 63));
        };
#pragma unroll 2
        for (int i = 0; i < kChunksPerWave; ++i) {
            const int c = wv * kChunksPerWave + i;
            const int j = c * kWave + l;
            if (j < len) {
                const int k = lvl[j];
                const uint64_t f = fm[c];
                const uint64_t upto = f & (lanes_lt(l) | (1ull << l));
                const uint64_t after = f & ~(lanes_lt(l) | (1ull << l));
                const int s = upto ? c * kWave + 63 - __clzll((long long)upto) : lastst[c];
                const int e = after ? c * kWave + __ffsll((unsigned long long)after) - 1 : firstst[c];
                const long long sg = s == 0 ? sf : t0 + s;
                const long long eg = e == len ? el : t0 + e;
                const int lbe = eg > t1 ? loutc[1][k] : Lb(e, k);
                const int lbs = sg < t0 ? loutc[0][k + 1] : Lb(s, k + 1);
                const long long pos = sg + lbe - lbs + (Lb(j, k + 1) - Lb(j, k));
                if (pos >= sg && pos < eg) col_out[pos] = cols[j];
            }
        }
        __syncthreads();
    }
}

inline int grid_for(long long n, int block, int max_blocks) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

inline int tile_grid(long long m) {
    const long long T = (m + kTileE - 1) / kTileE;
    return (int)(T < (1 << 20) ? (T < 1 ? 1 : T) : (1 << 20));
}

}  // namespace

hipError_t mlp_prepare(const int* row_off, const int* col, int n, long long m, int* indeg,
                       int* src, int* tinfo, int* copies, hipStream_t s) {
    hipLaunchKernelGGL(zero_ints, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, indeg,
                       (long long)n);
    if (m > 0) {
        if (copies)
            hipLaunchKernelGGL(zero_ints, dim3(grid_for((long long)n * kXcdCopies, 256, 16384)),
                               dim3(256), 0, s, copies, (long long)n * kXcdCopies);
        hipLaunchKernelGGL(in_degrees_xcd, dim3(grid_for(m, 256, 16384)), dim3(256), 0, s, col,
                           m, n, copies, indeg);
        if (copies)
            hipLaunchKernelGGL(sum_copies, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, copies,
                               n, indeg);
        hipLaunchKernelGGL(tile_first, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, row_off, n,
                           tinfo);
        hipLaunchKernelGGL(tile_sources, dim3(tile_grid(m)), dim3(kTileT), 0, s, row_off, n, m,
                           tinfo, src);
    }
    return hipGetLastError();
}

hipError_t edge_keys_launch(const int* row_off, const int* col, long long m, int kind,
                            uint64_t seed, float* key, hipStream_t s) {
    if (m > 0)
        hipLaunchKernelGGL(edge_keys, dim3(grid_for(m, 256, 16384)), dim3(256), 0, s, row_off,
                           col, m, kind, seed, key);
    return hipGetLastError();
}

hipError_t order_launch(const int* row_off, const int* col, int n, long long m, const float* key,
                        float lo, float hi, int* col_out, int* tinfo, int* tcnt,
                        hipStream_t s) {
    if (m <= 0) return hipGetLastError();
    const Levels lv{key, hi, hi > lo ? (float)kBuckets / (hi - lo) : 0.f};
    const long long T = (m + kTileE - 1) / kTileE;
    hipLaunchKernelGGL(tile_first, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, row_off, n,
                       tinfo);
    hipLaunchKernelGGL(order_count, dim3(tile_grid(m)), dim3(kTileT), 0, s, m, lv, tcnt);
    const long long B = (T + 1 + kScanRows - 1) / kScanRows;   // chunks of rows 0..T
    int* csum = tcnt + (T + 1) * kBuckets;
    hipLaunchKernelGGL(scan_reduce, dim3((unsigned)B), dim3(kWave), 0, s, tcnt, T, csum);
    hipLaunchKernelGGL(scan_rows, dim3(1), dim3(kScanT), 0, s, csum, B, B);
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)B), dim3(kWave), 0, s, tcnt, T, csum);
    hipLaunchKernelGGL(order_place, dim3(tile_grid(m)), dim3(kTileT), 0, s, row_off, n, m, col,
                       lv, tinfo, tcnt, col_out);
    return hipGetLastError();
}

}  // namespace trim
